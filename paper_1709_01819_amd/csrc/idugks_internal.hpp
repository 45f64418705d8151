// Internal data layout shared by the host orchestration and the HIP kernels.
//
// HBM layout (all arrays carved from the caller's workspace, 256-byte aligned):
//   f    [nc][2][nvp]  S   transformed distributions G~, H~, velocity innermost
//   d1   [nc][2][nvp]  S   flux sum M -> forward-sweep increment -> final increment
//   tab  [nc][nvx+nvy] S   factored Maxwellian of the cell records:
//                          E(ix,iy) = tab[ix] * tab[nvx+iy]
//   tabs [nc][nvx+nvy] S   same for the predicted records
//   tabf [nf][nvx+nvy] S   same for the face records
//   rec, recs [nc], recf [nf]   FP64 equilibrium records
//   fv   [nf][2][nvp]  S   reconstructed phi-bar at every face (Eq. 13-14)
//   raw  [nc][NM]      FP64 raw moments of the stored state
// S is double (FP64 form) or float (FP32-mixed form).  nvp = nv rounded up to 64.
#pragma once

#include <stdint.h>

namespace idugks {

enum FaceType : int { FT_INTERIOR = 0, FT_SELF = 1, FT_WALL = 2, FT_FAR = 3 };

constexpr int NM_BGK = 4;      // raw moments: 1, xi, eta, (|xi|^2 G + H)/2
constexpr int NM_SHAKHOV = 12; // + xi^2, xi eta, eta^2, xi|xi|^2, eta|xi|^2 (G); 1, xi, eta (H)
constexpr int NM_MAX = 12;
constexpr int VPAD = 64;

// One side of one cell (i-, i+, j-, j+ on a structured mesh; the edge from node s to node
// s+1 on an unstructured one, where the absent fourth side of a triangle has type FT_SELF,
// no neighbour and zero length).
struct CellSide {
    int nb;        // neighbour cell, -1 at a boundary (may be the cell itself: self-periodic)
    int face;      // face index
    int type;      // FaceType
    int tie;       // 1 if this cell is upwind for xi.n_out == 0 (R end of interior, far field)
    int wside;     // boundary-condition slot (0..3) of wall / far-field faces
    int pad0, pad1, pad2;
    double nx, ny; // outward unit normal
    double S;      // face length
    double dx, dy; // face midpoint (own frame) minus own centroid
    double ndx, ndy; // neighbour image centroid minus own centroid
    double ax, ay; // least-squares gradient weights of the neighbour (Eq. 15)
};

struct Face {
    int L, R;      // cells (R = -1 at a boundary; L = R for self-periodic faces)
    int sL, sR;    // side index of the face in L and in R
    int type, wside, pad0, pad1;
    double nx, ny, S; // unit normal from L to R (outward of L at a boundary)
};

// Equilibrium record.  With cx = xi - U, cy = eta - V, c2 = cx^2 + cy^2,
// P = kqx cx + kqy cy and E = tab[ix] * tab[nvx + iy]:
//   G_eq = E (c0 + c1 cx + c2c cy + c3 c2 + P (c2 iRT - 4))
//   H_eq = KRT E (c0 + c1 cx + c2c cy + c3 c2 + P (c2 iRT - 2))
struct Rec {
    double rho, U, V, RT, tau;
    double qx, qy;           // Shakhov heat flux entering the equilibrium
    double c0, c1, c2c, c3;  // discrete-conservation correction (central basis)
    double kqx, kqy;         // (1 - Pr)/(5 p RT) * q
    double iRT, KRT;
    double ab, bb;           // cells: phi-bar-plus = ab phi~ + bb phi_eq (Eq. 10, 12)
    double alpha;            // faces: 2 tau / (2 tau + h) (Eq. 18)
    double rw;               // wall faces: density of the reflected Maxwellian
};

// Velocities per block of the flux kernel: all of them up to 8192, else the fewest equal
// chunks of at most 8192 (rounded up to a multiple of 64), blocks ordered chunk by chunk,
// so that a cell's upwind neighbours are read while their slice of the reconstruction is
// still in L2.  Each block first stages its four faces' records and factored Maxwellians,
// which smaller chunks repeat more often (at 101^2 velocities two chunks beat 2048-wide
// ones by a fifth).  (The face-partial kernel takes all velocities per block: its 4 x NM
// sums per block would cost more than the reuse saves.)
inline int vel_chunk(int nv) {
    const int n = nv > 8192 ? (nv + 8191) / 8192 : 1;
    return ((nv + n - 1) / n + 63) & ~63;
}

// Records in the state precision, per cell (current step) and per face: U, V, c0, c1, c2c,
// c3, kqx, kqy, iRT, KRT, ab, bb, alpha, rw (two spare), read in the per-velocity loops
// with scalar loads and no conversions.
constexpr int RT_N = 16;

constexpr int SG_N = 16, SR_N = 12;
// macro row: M_W (dW* after the forward sweep) [4], 1/D, packed side codes, the cell's W [4]
// and sound speed, then per side nx, ny, S
constexpr int MH_SIDE = 11, MH_SN = 3, MH_N = MH_SIDE + 4 * MH_SN, MH_CODE_BITS = 4;
// spare rows after the last cell of the hyperplane-ordered arrays (beyond min(ni, nj)): the
// staging waves read whole passes past the last cell of a hyperplane
constexpr int HP_SPARE = 48;

// Static per-cell data of the micro sweeps (built on the host), per cell side: nx S and
// ny S (0 on a self-periodic side, which has no flux) and the coupling weights of the
// forward and the backward sweep (1 if the neighbour has a lower / higher index, else 0).
// Side code bits (the host builds them for these weights, the macro prep for its rows):
// SG_DIAG the side counts in the diagonal (not self-periodic), SG_LOWER / SG_UPPER the
// neighbour has a lower / higher index.  With periodic directions of 1 or at least 3
// cells, a side couples in one sweep direction only and to one place: sides i- and j- in
// the forward sweep to the adjacent hyperplane, i+ and j+ to the copy kept at a periodic
// seam; the other way round in the backward sweep.
enum SweepCode : int { SG_DIAG = 1, SG_LOWER = 2, SG_UPPER = 4 };
// Row of a position in the level-scheduled sweeps:
//   GR_CELL      the cell;
//   GR_MASK      bit s (bit 4 + s) set if side s couples in the forward (backward) sweep,
//                bit 8 + s if side s is a wall, bit 12 + s if the coupled neighbour of
//                side s is read from the micro sweeps' LDS ring, bit 16 if no cell reads
//                this cell's backward-sweep increment from d1;
//   GR_SRC + s   where the micro sweeps find side s: the neighbour's position if bit
//                12 + s is set, else the value of GR_NB + s;
//   GR_NB + s    the neighbour code of side s: its cell, -1 - t on a boundary side of
//                boundary-condition slot t, the cell itself on a side without flux;
//   GR_NPOS + s  the neighbour's position (the own position where there is none).
// The micro sweeps need only the first eight values.
enum GRow : int { GR_CELL = 0, GR_MASK = 1, GR_SRC = 2, GR_NB = 8, GR_NPOS = 12, GR_N = 16 };
// Positions in the LDS ring of recent increments of the level-scheduled micro sweeps
// (128 KiB per block in either precision).
constexpr int gs_ring_positions(bool fp32) { return fp32 ? 256 : 128; }
// Row of a position in the state precision for the level-scheduled micro sweeps: side
// geometry nx S (4), ny S (4) (static), the predicted record as in srec (12, written with
// it) and the wall ghost increment per side (4, written with sdrho).
enum GRowT : int { GT_GEO = 0, GT_REC = 8, GT_DRHO = 20, GT_N = 24 };
// Scalars kept on the device (FP64).
enum Scalar : int { SC_SCALE = 0, SC_RES = 1, SC_MASS = 2, SC_FLAG = 3, SC_NUM = 8 };

struct Params {
    int ni, nj, nc, nf, nv, nvp, nvx, nvy, K, model, limiter, closed, nm, nwall;
    int vch, nch;            // velocities per chunk of the flux kernel, chunks
    int prep_in_flux;        // the flux kernel (one chunk) also writes the macro rows
    int per_i, per_j;        // the mesh is periodic in i / in j
    int predictor, relax_sweeps; // macro prediction: 0 LU-SGS, 1 point relaxation (sweeps)
    double dt, h, Pr, mu_ref, omega, cfl_imp, M0, gam;
    // velocity set
    const double *xi, *eta, *w;
    const double *x1, *wx1, *y1, *wy1;  // 1D nodes and weights
    const int16_t *vix, *viy;
    // geometry
    const double *area;
    const CellSide *cs;      // [nc][4]
    const Face *faces;       // [nf]
    const int *wall_faces;   // [nwall]
    // boundary distributions
    const double *gw;        // [4][nvp] G of the wall Maxwellian at unit density
    const double *wKRT;      // [4] K RT of each wall side
    const double *ginf, *hinf; // [nvp] free-stream equilibrium
    const double *wden;      // [nf] sum over incoming v of w (xi.n) gw
    const double *bhalf;     // [nf][NM] moments of the incoming half of the ghost distribution
    // state and work (S-typed arrays as void*)
    void *f, *d1, *tab, *tabs, *tabf;
    void *recT, *recfT;      // [nc][RT_N], [nf][RT_N] records in the state precision
    void *fv;                // [nf][2][nvp] reconstructed phi-bar at each face (Eq. 13-14, from the
                             // upwind cell; written by the face-partial kernel for every
                             // velocity whose upwind side is a cell)
    Rec *rec, *recs, *recf;
    double *fields;          // [nc][8] cell fields returned by idugks_moments
    double *raw, *Wc, *MW, *dW, *DWd, *dtimp, *rho_old, *drho, *scal;
    double *MWc;             // [nc][nch][4] per-chunk sums of MW (nch > 1)
    double *dWr;             // [nc][4] second increment buffer of the point relaxation
    // per-cell data of the sweeps stored in i+j hyperplane order (position hp_pos[c]), so
    // that the cells of one hyperplane are contiguous and can be staged into LDS at once
    const int *hp_off;       // [nh+1] first position of each hyperplane (of each level)
    const int *hp_pos;       // [nc] position of each cell
    // level-scheduled sweeps (unstructured meshes, or on request): the positions hold the
    // cells level by level of the sweep order's dependency graph (hp_off has nlev + 1
    // entries); grow holds per position the cell, per side its neighbour cell (-1 - t on a
    // boundary side of boundary-condition slot t, the cell itself on a side without flux),
    // the coupling masks and per side the neighbour's position (GR_* below)
    int graph, gmacro, nlev;  // micro / macro sweeps by levels (else by hyperplanes)
    const int *grow;         // [nc][GR_N]
    void *growT;             // [nc][GT_N] S
    const double *sgeo;      // [nc][SG_N] nx S[4], ny S[4], w_lower[4], w_upper[4] (static)
    double *srec;            // [nc][SR_N] U, V, c0, c1, c2c, c3, kqx, kqy, iRT, KRT, cst, base
    double *sdrho;           // [nc][4] wall ghost density increment per cell side
    double *mh;              // [nc][MH_N] macro rows in hyperplane order
    // sensitivities (BGK, no limiter, FP64 state; null otherwise)
    double Kn, wall_u[4], wall_v[4];
    const double *lam;       // [nc][2][nvp] adjoint weights the VJP is taken with
    double *fbar;            // [nc][2][nvp] VJP output (d/d phi~)
    double *agr;             // [nc][6][nvp] per cell the face adjoints gathered where the cell
                             //   is upwind: direct G, H; sigma-bar x G, y G, x H, y H
    double *fadj;            // [nf][FA_N] face adjoint record
    double *cadj;            // [nc][CA_N] cell adjoint record
    const double *dgw;       // [2][4][nvp] d(wall Maxwellian)/d(u_w), /d(T_w) per wall side
    const double *dwden;     // [2][nf] d(wden)/d(u_w), /d(T_w) per wall face
    double *jacc, *jacf;     // [nc][32], [nf][32] record Jacobians d(rho,U,V,RT,c0..c3)/dW
    double *red;             // [RED_N] partial sums of the fixed-order reductions
};

// face adjoint record: W-bar (4), rho_w-bar, theta-bar (3: lid speed, wall T, Kn), J part
enum FaceAdj : int { FA_WB = 0, FA_RHOW = 4, FA_TH = 5, FA_J = 8, FA_N = 9 };
// cell adjoint record: W-bar (4), theta-bar Kn
enum CellAdj : int { CA_WB = 0, CA_TH = 4, CA_N = 5 };
constexpr int RED_N = 4096;

}  // namespace idugks
