// C ABI of the MI355X implicit DUGKS solver: configuration checks, mesh geometry,
// discrete velocity set, boundary distributions, workspace carving and the kernel
// sequence of one explicit or implicit step.  Method: arXiv:1709.01819, Section 2.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/idugks.h"
#include "idugks_internal.hpp"
#include "idugks_kernels.hpp"

using namespace idugks;

namespace {

thread_local std::string g_err;

idugks_status fail(idugks_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(IDUGKS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------------------
// velocity quadrature (Section 2.2, last paragraph)
// ---------------------------------------------------------------------------------------

// Number of eigenvalues below x of the Jacobi matrix of the Hermite weight exp(-x^2)
// (zero diagonal, off-diagonal sqrt(k/2)) by the Sturm count of its LDL^T pivots.
int sturm_count(int n, double x) {
    int cnt = 0;
    double d = -x;
    if (d < 0) ++cnt;
    for (int k = 1; k < n; ++k) {
        const double b2 = 0.5 * k;
        if (d == 0.0) d = 1e-300;
        d = -x - b2 / d;
        if (d < 0) ++cnt;
    }
    return cnt;
}

// Orthonormal Hermite functions psi_n(x) and psi_{n-1}(x).
void hermite_pair(int n, double x, double &pn, double &pn1) {
    double a = 0.0, b = pow(M_PI, -0.25) * exp(-0.5 * x * x);
    for (int k = 0; k < n; ++k) {
        const double c = sqrt(2.0 / (k + 1)) * x * b - sqrt((double)k / (k + 1)) * a;
        a = b;
        b = c;
    }
    pn = b;
    pn1 = a;
}

// Gauss-Hermite nodes (eigenvalues of the Jacobi matrix by Sturm bisection, then Newton
// on psi_n) and total weights W_i = w_i exp(x_i^2) = 1 / (n psi_{n-1}(x_i)^2).
bool gauss_hermite(int n, std::vector<double> &x, std::vector<double> &W) {
    x.assign(n, 0.0);
    W.assign(n, 0.0);
    const double R = sqrt(2.0 * n + 1.0) + 1.0;
    for (int k = 0; k < n; ++k) {
        double lo = -R, hi = R;
        for (int it = 0; it < 200 && hi - lo > 1e-15 * (1.0 + fabs(lo)); ++it) {
            const double mid = 0.5 * (lo + hi);
            if (sturm_count(n, mid) > k) hi = mid; else lo = mid;
        }
        double r = 0.5 * (lo + hi);
        for (int it = 0; it < 3; ++it) {
            double pn, pn1;
            hermite_pair(n, r, pn, pn1);
            const double dp = sqrt(2.0 * n) * pn1 - r * pn;
            if (dp == 0.0) break;
            const double step = pn / dp;
            if (!(fabs(step) < 1e-3)) break;
            r -= step;
        }
        x[k] = r;
    }
    for (int k = 0; k < n / 2; ++k) {
        const double a = 0.5 * (x[n - 1 - k] - x[k]);
        x[k] = -a;
        x[n - 1 - k] = a;
    }
    if (n & 1) x[n / 2] = 0.0;
    for (int k = 0; k < n; ++k) {
        double pn, pn1;
        hermite_pair(n, x[k], pn, pn1);
        W[k] = 1.0 / (n * pn1 * pn1);
        if (!std::isfinite(W[k]) || !(W[k] > 0)) return false;
    }
    return true;
}

// Composite Newton-Cotes on [-vmax, vmax] with m = n-1 intervals: Boole if 4 | m,
// Simpson 3/8 if 3 | m, Simpson if 2 | m, else trapezoid.
bool newton_cotes(int n, double vmax, std::vector<double> &x, std::vector<double> &W) {
    const int m = n - 1;
    const double h = 2.0 * vmax / m;
    x.resize(n);
    W.assign(n, 0.0);
    for (int k = 0; k < n; ++k) x[k] = -vmax + h * k;
    int panel;
    std::vector<double> c;
    if (m % 4 == 0) { panel = 4; c = {14.0 / 45, 64.0 / 45, 24.0 / 45, 64.0 / 45, 14.0 / 45}; }
    else if (m % 3 == 0) { panel = 3; c = {3.0 / 8, 9.0 / 8, 9.0 / 8, 3.0 / 8}; }
    else if (m % 2 == 0) { panel = 2; c = {1.0 / 3, 4.0 / 3, 1.0 / 3}; }
    else { panel = 1; c = {0.5, 0.5}; }
    for (int s = 0; s < m; s += panel)
        for (int k = 0; k <= panel; ++k) W[s + k] += c[k] * h;
    return true;
}

// ---------------------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------------------
struct Layout {
    static constexpr int N = 80;
    size_t off[N], sz[N];
    size_t bytes = 0;
    int n = 0;
    size_t add(size_t b) {
        bytes = (bytes + 255) & ~size_t(255);
        off[n] = bytes;
        sz[n] = b;
        bytes += b;
        return n++;
    }
    size_t size(int r) const { return sz[r]; }
};

enum KernelId {
    KID_RECORDS, KID_PARTIALS, KID_FACE_RECORDS, KID_FLUX, KID_MACRO_PREP, KID_MACRO, KID_RECORDS_PRED,
    KID_LOWER, KID_WALL_GHOST, KID_UPPER, KID_EXPLICIT, KID_RAW, KID_FINALIZE, KID_MACRO_RELAX,
    KID_COUNT
};
const char *kKernelNames[KID_COUNT] = {
    "records", "face_partials", "face_records", "flux", "macro_prep", "macro_lusgs", "records_pred",
    "sweep_lower", "wall_ghost", "sweep_upper", "explicit_update", "raw_moments", "finalize",
    "macro_relax"};

}  // namespace

struct idugks_ctx {
    idugks_config cfg;
    Params p;
    bool fp32;
    SweepShape sweep;
    bool adj;                           // sensitivities available
    double *lt, *gJ, *ybuf, *adjs;      // adjoint iterate, dJ/df, projection, device scalars
    hipStream_t st;
    std::vector<double> area_h, xi_h, eta_h, w_h;
    double *stage;  // [nc][nvp] FP64 staging of one canonical species
    int64_t iters;
    double cfl_start, cfl_growth;  // start-up ramp of the implicit CFL (0: none)
    int64_t imp_iters;             // implicit iterations since init or set_state (its n)
    // profiling: one event pair per launch, read after the stream drains
    bool prof;
    std::vector<hipEvent_t> evs;
    std::vector<int> ev_kid;
    size_t ev_used;
    double ms[KID_COUNT];
    int64_t cnt[KID_COUNT];
    uint32_t prof_mask;  // kernels timed while prof is set (bit k: kernel k)
    int scratch_dev;     // device whose static scratch array is the workspace (-1: the caller's)
};

namespace {

// How the two sweeps walk the cell order (idugks_config.sweep_order): by levels of the
// order's dependency graph or by i+j hyperplanes.  The level-scheduled micro sweeps take
// one workgroup per slice of 64 velocities, so they pay off from about 128 slices (8192
// velocities) on, where the hyperplane kernel's slices of 8 velocities re-read their
// staged rows; the one-block hyperplane macro sweep keeps its fronts in LDS and stays the
// faster one on structured meshes.
struct SweepPlan {
    bool micro_levels, macro_levels;  // the sweeps of an implicit iteration
    bool hyper_micro_fits, hyper_macro_fits;
};

SweepPlan sweep_plan(const idugks_config *c) {
    SweepPlan sp{};
    if (c->cell_nodes) {
        sp.micro_levels = sp.macro_levels = true;
        return sp;
    }
    const bool per_i = c->bc[0] == IDUGKS_BC_PERIODIC, per_j = c->bc[2] == IDUGKS_BC_PERIODIC;
    const bool small = std::min(c->ni, c->nj) <= 280;
    const MacroShape m = macro_shape(c->ni, c->nj, per_i, per_j);
    sp.hyper_macro_fits = small && m.lds <= 150 * 1024 && m.threads <= 1024;
    sp.hyper_micro_fits = small && sweep_shape(c->ni, c->nj, 1, 8).vb > 0;
    const int64_t nv = (int64_t)c->nvx * c->nvy, slices = (nv + VPAD - 1) / VPAD;
    if (c->sweep_order == IDUGKS_SWEEPS_LEVELS) {
        sp.micro_levels = sp.macro_levels = true;
    } else if (c->sweep_order == IDUGKS_SWEEPS_AUTO) {
        sp.micro_levels = slices >= 128 || !sp.hyper_micro_fits;
        sp.macro_levels = !sp.hyper_macro_fits;
    }
    return sp;
}

idugks_status validate(const idugks_config *c) {
    if (!c) return fail(IDUGKS_E_INVALID, "null config");
    if (c->struct_size != sizeof(idugks_config)) return fail(IDUGKS_E_INVALID, "struct_size mismatch");
    const bool um = c->cell_nodes != nullptr;
    if (c->sweep_order < IDUGKS_SWEEPS_AUTO || c->sweep_order > IDUGKS_SWEEPS_HYPERPLANES)
        return fail(IDUGKS_E_INVALID, "sweep_order must be IDUGKS_SWEEPS_AUTO, _LEVELS or _HYPERPLANES");
    if (c->diverge_iters < 0) return fail(IDUGKS_E_INVALID, "diverge_iters must be >= 0");
    if (um) {
        if (c->ncells < 1 || c->nnodes < 3 || !c->side_tag)
            return fail(IDUGKS_E_INVALID, "unstructured mesh needs ncells >= 1, nnodes >= 3 and side_tag");
        for (int s = 0; s < 4; ++s)
            if (c->bc[s] == IDUGKS_BC_PERIODIC)
                return fail(IDUGKS_E_INVALID, "no periodic boundary conditions on an unstructured mesh");
        if (c->sweep_order == IDUGKS_SWEEPS_HYPERPLANES)
            return fail(IDUGKS_E_INVALID, "i+j hyperplanes need a structured mesh");
    } else {
        if (c->ni < 1 || c->nj < 1) return fail(IDUGKS_E_INVALID, "mesh needs ni, nj >= 1");
        if ((int64_t)c->ni * c->nj >= ((int64_t)1 << 31)) return fail(IDUGKS_E_INVALID, "too many cells");
        const SweepPlan sp = sweep_plan(c);
        if (c->sweep_order == IDUGKS_SWEEPS_HYPERPLANES && !(sp.hyper_micro_fits && sp.hyper_macro_fits))
            return fail(IDUGKS_E_INVALID, "mesh too large for the LDS-resident sweep fronts of the hyperplane "
                                          "sweeps (sweep_order AUTO or LEVELS has no such limit)");
    }
    if (!c->xn || !c->yn) return fail(IDUGKS_E_INVALID, "missing node coordinates");
    if (c->predictor != 0 && c->predictor != 1) return fail(IDUGKS_E_INVALID, "unknown predictor");
    if (c->relax_sweeps < 0 || c->relax_sweeps > 64)
        return fail(IDUGKS_E_INVALID, "relax_sweeps must be 0..64");
    if (!(c->cfl_start >= 0) || (c->cfl_start > 0 && !(c->cfl_growth >= 1 && c->cfl_growth < 1e3)))
        return fail(IDUGKS_E_INVALID, "CFL ramp needs cfl_start >= 0 and 1 <= cfl_growth < 1000");
    if (c->nvx < 2 || c->nvy < 2) return fail(IDUGKS_E_INVALID, "need nv >= 2 per direction");
    if (c->nvx > 4096 || c->nvy > 4096) return fail(IDUGKS_E_INVALID, "velocity grid too large");
    {
        // the sweeps index the state [nc][2][nvp] with 32-bit element offsets
        const int64_t nv = (int64_t)c->nvx * c->nvy, nvp = (nv + VPAD - 1) / VPAD * VPAD;
        const int64_t nc = um ? (int64_t)c->ncells : (int64_t)c->ni * c->nj;
        if (nc * 2 * nvp >= ((int64_t)1 << 31))
            return fail(IDUGKS_E_INVALID, "state too large (nc x 2 x padded nv must stay below 2^31)");
    }
    if (!(c->Kn > 0)) return fail(IDUGKS_E_INVALID, "Kn must be positive");
    if (!(c->Pr > 0)) return fail(IDUGKS_E_INVALID, "Pr must be positive");
    if (c->K < 0) return fail(IDUGKS_E_INVALID, "K must be >= 0");
    if (c->model != IDUGKS_BGK && c->model != IDUGKS_SHAKHOV) return fail(IDUGKS_E_INVALID, "unknown model");
    if (c->model == IDUGKS_SHAKHOV && c->K != 1)
        return fail(IDUGKS_E_INVALID, "the Shakhov model is implemented for K = 1");
    if (c->quad != IDUGKS_GAUSS_HERMITE && c->quad != IDUGKS_NEWTON_COTES)
        return fail(IDUGKS_E_INVALID, "unknown quadrature");
    if (c->quad == IDUGKS_NEWTON_COTES && !(c->vmax > 0))
        return fail(IDUGKS_E_INVALID, "Newton-Cotes needs vmax > 0");
    if (!(c->cfl_phys > 0) || !(c->cfl_imp > 0)) return fail(IDUGKS_E_INVALID, "CFL numbers must be positive");
    if (c->limiter != 0 && c->limiter != 1) return fail(IDUGKS_E_INVALID, "unknown limiter");
    if (c->precision != IDUGKS_FP64 && c->precision != IDUGKS_FP32_MIXED)
        return fail(IDUGKS_E_INVALID, "unknown precision");
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] < 0 || c->bc[s] > 2) return fail(IDUGKS_E_INVALID, "unknown boundary type");
    if ((c->bc[0] == IDUGKS_BC_PERIODIC) != (c->bc[1] == IDUGKS_BC_PERIODIC) ||
        (c->bc[2] == IDUGKS_BC_PERIODIC) != (c->bc[3] == IDUGKS_BC_PERIODIC))
        return fail(IDUGKS_E_INVALID, "periodic sides must come in pairs");
    if (!um && c->bc[0] == IDUGKS_BC_PERIODIC && c->ni == 2) return fail(IDUGKS_E_INVALID, "periodic ni must be 1 or >= 3");
    if (!um && c->bc[2] == IDUGKS_BC_PERIODIC && c->nj == 2) return fail(IDUGKS_E_INVALID, "periodic nj must be 1 or >= 3");
    for (int s = 0; s < 4; ++s) {
        if (c->bc[s] == IDUGKS_BC_WALL && !(c->wall_T[s] > 0)) return fail(IDUGKS_E_INVALID, "wall T must be positive");
        if (c->bc[s] == IDUGKS_BC_FARFIELD && (!(c->far_rho > 0) || !(c->far_T > 0)))
            return fail(IDUGKS_E_INVALID, "far-field state must be positive");
    }
    if (!(c->init_rho > 0) || !(c->init_T > 0)) return fail(IDUGKS_E_INVALID, "initial state must be positive");
    if (!(c->omega >= 0) || !std::isfinite(c->omega)) return fail(IDUGKS_E_INVALID, "bad omega");
    return IDUGKS_OK;
}

// Host-side problem description built from the configuration.
struct Built {
    int ni, nj, nc, nf, nv, nvp, nvx, nvy, nwall, closed;
    double dt;
    std::vector<double> x1, wx1, y1, wy1, xi, eta, w;
    std::vector<int16_t> vix, viy;
    std::vector<double> area, xc, yc;
    std::vector<CellSide> cs;
    std::vector<int> hp_off, hp_pos;  // hyperplanes (structured) or levels (graph sweeps)
    int nlev;
    std::vector<int> grow;            // per position: [GR_N] row of the level sweeps
    std::vector<double> sgeo;
    std::vector<Face> faces;
    std::vector<int> wall_faces;
    std::vector<double> gw, wKRT, ginf, hinf, wden, bhalf, eq0;
    std::vector<double> dgw, dwden;  // [2][4][nvp], [2][nf]: d/d(wall speed), d/d(wall T)
};

// Number with two tangents (derivatives of the wall Maxwellian with respect to the wall
// speed and temperature).
struct HD {
    double v, d[2];
};
inline HD hd(double a, double d0 = 0.0, double d1 = 0.0) { return HD{a, {d0, d1}}; }
inline HD operator+(HD a, HD b) { return HD{a.v + b.v, {a.d[0] + b.d[0], a.d[1] + b.d[1]}}; }
inline HD operator-(HD a, HD b) { return HD{a.v - b.v, {a.d[0] - b.d[0], a.d[1] - b.d[1]}}; }
inline HD operator*(HD a, HD b) { return HD{a.v * b.v, {a.d[0] * b.v + a.v * b.d[0], a.d[1] * b.v + a.v * b.d[1]}}; }
inline HD operator/(HD a, HD b) {
    const double q = a.v / b.v;
    return HD{q, {(a.d[0] - q * b.d[0]) / b.v, (a.d[1] - q * b.d[1]) / b.v}};
}
inline HD exp(HD a) { const double e = std::exp(a.v); return HD{e, {e * a.d[0], e * a.d[1]}}; }
inline double val(double a) { return a; }
inline double val(HD a) { return a.v; }
template <class R> inline R num(double a) { return R(a); }
template <> inline HD num<HD>(double a) { return hd(a); }

// Equilibrium G with exact discrete conserved moments for a state at rest in its own
// frame (no heat flux): G = G_M (1 + beta.psi(c)) (Eq. 2, Eq. 5; H = K RT G).
template <class R>
void host_equilibrium_g(const Built &b, R rho, R U, R V, R T, R *G) {
    using std::exp;
    const R RT = num<R>(0.5) * T, lam = num<R>(0.5) / RT, A0 = rho * lam / num<R>(M_PI);
    R A[4][4], r[4] = {rho, num<R>(0.0), num<R>(0.0), rho * RT};
    for (int a = 0; a < 4; ++a)
        for (int c = 0; c < 4; ++c) A[a][c] = num<R>(0.0);
    std::vector<R> gm(b.nv);
    for (int v = 0; v < b.nv; ++v) {
        const R cx = num<R>(b.xi[v]) - U, cy = num<R>(b.eta[v]) - V, c2 = cx * cx + cy * cy;
        gm[v] = A0 * exp(num<R>(0.0) - lam * c2);
        const R ps[4] = {num<R>(1.0), cx, cy, num<R>(0.5) * c2};
        for (int a = 0; a < 4; ++a) {
            r[a] = r[a] - num<R>(b.w[v]) * ps[a] * gm[v];
            for (int c = 0; c < 4; ++c) A[a][c] = A[a][c] + num<R>(b.w[v]) * ps[a] * ps[c] * gm[v];
        }
    }
    // Gaussian elimination with partial pivoting
    for (int k = 0; k < 4; ++k) {
        int pv = k;
        for (int i = k + 1; i < 4; ++i)
            if (fabs(val(A[i][k])) > fabs(val(A[pv][k]))) pv = i;
        std::swap(A[k], A[pv]);
        std::swap(r[k], r[pv]);
        for (int i = k + 1; i < 4; ++i) {
            const R m = A[i][k] / A[k][k];
            for (int c = k; c < 4; ++c) A[i][c] = A[i][c] - m * A[k][c];
            r[i] = r[i] - m * r[k];
        }
    }
    for (int k = 3; k >= 0; --k) {
        R s = r[k];
        for (int c = k + 1; c < 4; ++c) s = s - A[k][c] * r[c];
        r[k] = s / A[k][k];
    }
    for (int v = 0; v < b.nv; ++v) {
        const R cx = num<R>(b.xi[v]) - U, cy = num<R>(b.eta[v]) - V;
        G[v] = gm[v] * (num<R>(1.0) + r[0] + r[1] * cx + r[2] * cy + num<R>(0.5) * r[3] * (cx * cx + cy * cy));
    }
}

void host_equilibrium(const Built &b, int K, double rho, double U, double V, double T,
                      double *G, double *H) {
    host_equilibrium_g<double>(b, rho, U, V, T, G);
    for (int v = 0; v < b.nv; ++v) H[v] = K * 0.5 * T * G[v];
}

// Normal speed with velocities tangent to the face (within 1e-12 of their speed) snapped
// to exactly 0; the device kernels classify with the same rule.
double normal_speed(double x, double y, double nx, double ny) {
    const double un = x * nx + y * ny;
    return fabs(un) <= 1e-12 * (fabs(x) + fabs(y)) ? 0.0 : un;
}

// 12 raw moments (the set accumulated on the device) of a pair over a subset of v.
void raw12(const Built &b, const double *G, const double *H, const std::vector<char> &use,
           double *m) {
    for (int a = 0; a < 12; ++a) m[a] = 0.0;
    for (int v = 0; v < b.nv; ++v) {
        if (!use[v]) continue;
        const double x = b.xi[v], y = b.eta[v], q2 = x * x + y * y;
        const double wG = b.w[v] * G[v], wH = b.w[v] * H[v];
        m[0] += wG; m[1] += wG * x; m[2] += wG * y; m[3] += 0.5 * (wG * q2 + wH);
        m[4] += wG * x * x; m[5] += wG * x * y; m[6] += wG * y * y;
        m[7] += wG * x * q2; m[8] += wG * y * q2;
        m[9] += wH; m[10] += wH * x; m[11] += wH * y;
    }
}

// Structured mesh: cells (i, j) -> i + j ni, faces, cell sides and the i+j hyperplane order.
idugks_status build_structured(const idugks_config *c, Built &b) {
    const int ni = c->ni, nj = c->nj;
    // cells: shoelace area and centroid
    auto X = [&](int i, int j) { return c->xn[i + j * (ni + 1)]; };
    auto Y = [&](int i, int j) { return c->yn[i + j * (ni + 1)]; };
    b.area.resize(b.nc);
    b.xc.resize(b.nc);
    b.yc.resize(b.nc);
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            const double px[4] = {X(i, j), X(i + 1, j), X(i + 1, j + 1), X(i, j + 1)};
            const double py[4] = {Y(i, j), Y(i + 1, j), Y(i + 1, j + 1), Y(i, j + 1)};
            double a = 0, sx = 0, sy = 0;
            for (int k = 0; k < 4; ++k) {
                const int l = (k + 1) & 3;
                const double cr = px[k] * py[l] - px[l] * py[k];
                a += cr;
                sx += (px[k] + px[l]) * cr;
                sy += (py[k] + py[l]) * cr;
            }
            a *= 0.5;
            if (!(a > 0)) return fail(IDUGKS_E_INVALID, "non-positive cell area (check node order)");
            const int cidx = i + j * ni;
            b.area[cidx] = a;
            b.xc[cidx] = sx / (6.0 * a);
            b.yc[cidx] = sy / (6.0 * a);
        }
    // faces: i-faces (i, j) at index j*(ni+1)+i, then j-faces (i, j) at nfi + j*ni + i
    const bool pi = c->bc[0] == IDUGKS_BC_PERIODIC, pj = c->bc[2] == IDUGKS_BC_PERIODIC;
    const int nfi = (ni + 1) * nj, nfj = ni * (nj + 1);
    b.nf = nfi + nfj;
    b.faces.assign(b.nf, Face{});
    for (auto &F : b.faces) { F.type = FT_SELF; F.L = F.R = -1; }
    auto set_face = [&](int k, int L, int sL, int R, int sR, int type, int side, double ax, double ay,
                        double bx, double by, bool plus_i) {
        Face &F = b.faces[k];
        const double tx = bx - ax, ty = by - ay, S = sqrt(tx * tx + ty * ty);
        double nx = plus_i ? ty / S : -ty / S, ny = plus_i ? -tx / S : tx / S;
        if (R < 0 && (side == 0 || side == 2)) { nx = -nx; ny = -ny; }  // outward at i- / j-
        F.L = L; F.sL = sL; F.R = R; F.sR = sR; F.type = type; F.wside = side;
        F.nx = nx; F.ny = ny; F.S = S;
    };
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i <= ni; ++i) {
            const int k = j * (ni + 1) + i;
            const double ax = X(i, j), ay = Y(i, j), bx = X(i, j + 1), by = Y(i, j + 1);
            if (i > 0 && i < ni) set_face(k, i - 1 + j * ni, 1, i + j * ni, 0, FT_INTERIOR, -1, ax, ay, bx, by, true);
            else if (pi) {
                if (i == ni) set_face(k, ni - 1 + j * ni, 1, j * ni, 0, ni == 1 ? FT_SELF : FT_INTERIOR, -1, ax, ay, bx, by, true);
            } else {
                const int side = i == 0 ? 0 : 1, cell = i == 0 ? j * ni : ni - 1 + j * ni;
                set_face(k, cell, side, -1, -1, c->bc[side] == IDUGKS_BC_WALL ? FT_WALL : FT_FAR, side, ax, ay, bx, by, true);
            }
        }
    for (int j = 0; j <= nj; ++j)
        for (int i = 0; i < ni; ++i) {
            const int k = nfi + j * ni + i;
            const double ax = X(i, j), ay = Y(i, j), bx = X(i + 1, j), by = Y(i + 1, j);
            if (j > 0 && j < nj) set_face(k, i + (j - 1) * ni, 3, i + j * ni, 2, FT_INTERIOR, -1, ax, ay, bx, by, false);
            else if (pj) {
                if (j == nj) set_face(k, i + (nj - 1) * ni, 3, i, 2, nj == 1 ? FT_SELF : FT_INTERIOR, -1, ax, ay, bx, by, false);
            } else {
                const int side = j == 0 ? 2 : 3, cell = j == 0 ? i : i + (nj - 1) * ni;
                set_face(k, cell, side, -1, -1, c->bc[side] == IDUGKS_BC_WALL ? FT_WALL : FT_FAR, side, ax, ay, bx, by, false);
            }
        }
    // cell sides
    b.cs.assign((size_t)4 * b.nc, CellSide{});
    b.closed = 1;
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] == IDUGKS_BC_FARFIELD) b.closed = 0;
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            const int cidx = i + j * ni;
            for (int s = 0; s < 4; ++s) {
                CellSide &q = b.cs[(size_t)4 * cidx + s];
                // own edge, counter-clockwise orientation of the cell
                double ax, ay, bx, by;
                if (s == 0) { ax = X(i, j + 1); ay = Y(i, j + 1); bx = X(i, j); by = Y(i, j); }
                else if (s == 1) { ax = X(i + 1, j); ay = Y(i + 1, j); bx = X(i + 1, j + 1); by = Y(i + 1, j + 1); }
                else if (s == 2) { ax = X(i, j); ay = Y(i, j); bx = X(i + 1, j); by = Y(i + 1, j); }
                else { ax = X(i + 1, j + 1); ay = Y(i + 1, j + 1); bx = X(i, j + 1); by = Y(i, j + 1); }
                const double tx = bx - ax, ty = by - ay, S = sqrt(tx * tx + ty * ty);
                q.nx = ty / S;  // outward normal of a counter-clockwise edge
                q.ny = -tx / S;
                q.S = S;
                q.dx = 0.5 * (ax + bx) - b.xc[cidx];
                q.dy = 0.5 * (ay + by) - b.yc[cidx];
                // face and neighbour
                int fi, fj, ni2 = i, nj2 = j;
                double shx = 0.0, shy = 0.0;
                bool has = true;
                if (s == 0) {
                    fi = j * (ni + 1) + i;
                    if (i > 0) ni2 = i - 1;
                    else if (pi) { ni2 = ni - 1; fi = j * (ni + 1) + ni; shx = -(X(ni, j) - X(0, j)); shy = -(Y(ni, j) - Y(0, j)); }
                    else has = false;
                } else if (s == 1) {
                    fi = j * (ni + 1) + i + 1;
                    if (i < ni - 1) ni2 = i + 1;
                    else if (pi) { ni2 = 0; shx = X(ni, j) - X(0, j); shy = Y(ni, j) - Y(0, j); }
                    else has = false;
                } else if (s == 2) {
                    fi = nfi + j * ni + i;
                    if (j > 0) nj2 = j - 1;
                    else if (pj) { nj2 = nj - 1; fi = nfi + nj * ni + i; shx = -(X(i, nj) - X(i, 0)); shy = -(Y(i, nj) - Y(i, 0)); }
                    else has = false;
                } else {
                    fi = nfi + (j + 1) * ni + i;
                    if (j < nj - 1) nj2 = j + 1;
                    else if (pj) { nj2 = 0; shx = X(i, nj) - X(i, 0); shy = Y(i, nj) - Y(i, 0); }
                    else has = false;
                }
                (void)fj;
                q.face = fi;
                const Face &F = b.faces[fi];
                q.type = F.type;
                q.wside = s;
                if (has) {
                    q.nb = ni2 + nj2 * ni;
                    q.ndx = b.xc[q.nb] + shx - b.xc[cidx];
                    q.ndy = b.yc[q.nb] + shy - b.yc[cidx];
                    q.tie = (F.type == FT_INTERIOR && F.R == cidx && F.sR == s) ? 1 : 0;
                } else {
                    q.nb = -1;
                    q.tie = F.type == FT_FAR ? 1 : 0;
                }
            }
            // least-squares weights (Eq. 15) over the neighbours (periodic images included)
            double a11 = 0, a12 = 0, a22 = 0;
            for (int s = 0; s < 4; ++s) {
                const CellSide &q = b.cs[(size_t)4 * cidx + s];
                if (q.nb < 0) continue;
                a11 += q.ndx * q.ndx; a12 += q.ndx * q.ndy; a22 += q.ndy * q.ndy;
            }
            const double det = a11 * a22 - a12 * a12;
            if (!(det > 0)) return fail(IDUGKS_E_INVALID, "degenerate least-squares stencil");
            for (int s = 0; s < 4; ++s) {
                CellSide &q = b.cs[(size_t)4 * cidx + s];
                if (q.nb < 0) continue;
                q.ax = (a22 * q.ndx - a12 * q.ndy) / det;
                q.ay = (a11 * q.ndy - a12 * q.ndx) / det;
            }
        }
    // i+j hyperplane ordering of the cells (the levels of the sweeps' dependency graph)
    const int nh = ni + nj - 1;
    b.hp_off.assign(nh + 1, 0);
    b.hp_pos.assign(b.nc, 0);
    for (int s = 0, pos = 0; s < nh; ++s) {
        b.hp_off[s] = pos;
        const int lo = std::max(0, s - nj + 1), hi = std::min(ni - 1, s);
        for (int i = lo; i <= hi; ++i) b.hp_pos[i + (s - i) * ni] = pos++;
        b.hp_off[s + 1] = pos;
    }
    b.nlev = nh;
    return IDUGKS_OK;
}

// Unstructured mesh of quadrilaterals and triangles: cells from their nodes, faces from
// the edges two cells share (the lower cell index is L; faces numbered by their sorted
// node pair) or that lie on the boundary (tagged with a boundary-condition slot), one
// zero-length face of type FT_SELF at the end for the absent fourth side of every
// triangle, and the levels of the sweep order (cell index order): a cell's level is one
// more than the highest level of the lower-indexed neighbours it couples to.
idugks_status build_unstructured(const idugks_config *c, Built &b) {
    const int nc = c->ncells, nn = c->nnodes;
    const int32_t *cn = c->cell_nodes, *tag = c->side_tag;
    auto corners = [&](int cell) { return cn[4 * cell + 3] < 0 ? 3 : 4; };
    auto node = [&](int cell, int k) { return cn[4 * cell + k % corners(cell)]; };
    b.area.resize(nc);
    b.xc.resize(nc);
    b.yc.resize(nc);
    for (int cell = 0; cell < nc; ++cell) {
        if (cn[4 * cell + 3] < -1) return fail(IDUGKS_E_INVALID, "bad fourth node (use -1 for a triangle)");
        double a = 0, sx = 0, sy = 0;
        for (int k = 0; k < corners(cell); ++k) {
            const int i0 = node(cell, k), i1 = node(cell, k + 1);
            if (i0 < 0 || i0 >= nn || i1 < 0 || i1 >= nn) return fail(IDUGKS_E_INVALID, "node index out of range");
            const double cr = c->xn[i0] * c->yn[i1] - c->xn[i1] * c->yn[i0];
            a += cr;
            sx += (c->xn[i0] + c->xn[i1]) * cr;
            sy += (c->yn[i0] + c->yn[i1]) * cr;
        }
        a *= 0.5;
        if (!(a > 0)) return fail(IDUGKS_E_INVALID, "non-positive cell area (cells must be counter-clockwise)");
        b.area[cell] = a;
        b.xc[cell] = sx / (6.0 * a);
        b.yc[cell] = sy / (6.0 * a);
    }
    // edges keyed by their sorted node pair, then the cell and side
    struct Edge { int a, b, cell, side; };
    std::vector<Edge> e;
    e.reserve((size_t)4 * nc);
    for (int cell = 0; cell < nc; ++cell)
        for (int k = 0; k < corners(cell); ++k) {
            const int i0 = node(cell, k), i1 = node(cell, k + 1);
            if (i0 == i1) return fail(IDUGKS_E_INVALID, "degenerate edge");
            e.push_back(Edge{std::min(i0, i1), std::max(i0, i1), cell, k});
        }
    std::sort(e.begin(), e.end(), [](const Edge &u, const Edge &v) {
        if (u.a != v.a) return u.a < v.a;
        if (u.b != v.b) return u.b < v.b;
        if (u.cell != v.cell) return u.cell < v.cell;
        return u.side < v.side;
    });
    b.cs.assign((size_t)4 * nc, CellSide{});
    b.faces.clear();
    b.closed = 1;
    for (int t = 0; t < 4; ++t)
        if (c->bc[t] == IDUGKS_BC_FARFIELD) b.closed = 0;
    // the cell's own counter-clockwise edge of side k: outward normal, length, midpoint
    auto side_geo = [&](int cell, int k, CellSide &q) {
        const int i0 = node(cell, k), i1 = node(cell, k + 1);
        const double tx = c->xn[i1] - c->xn[i0], ty = c->yn[i1] - c->yn[i0], S = sqrt(tx * tx + ty * ty);
        q.nx = ty / S;
        q.ny = -tx / S;
        q.S = S;
        q.dx = 0.5 * (c->xn[i0] + c->xn[i1]) - b.xc[cell];
        q.dy = 0.5 * (c->yn[i0] + c->yn[i1]) - b.yc[cell];
    };
    for (size_t i = 0; i < e.size();) {
        size_t j = i + 1;
        while (j < e.size() && e[j].a == e[i].a && e[j].b == e[i].b) ++j;
        if (j - i > 2) return fail(IDUGKS_E_INVALID, "an edge shared by more than two cells");
        const int k = (int)b.faces.size();
        const Edge &L = e[i];
        CellSide &qL = b.cs[(size_t)4 * L.cell + L.side];
        side_geo(L.cell, L.side, qL);
        Face F{};
        F.L = L.cell;
        F.sL = L.side;
        F.nx = qL.nx;
        F.ny = qL.ny;
        F.S = qL.S;
        qL.face = k;
        if (j - i == 2) {
            const Edge &R = e[i + 1];
            if (R.cell == L.cell) return fail(IDUGKS_E_INVALID, "a cell sharing an edge with itself");
            CellSide &qR = b.cs[(size_t)4 * R.cell + R.side];
            side_geo(R.cell, R.side, qR);
            F.R = R.cell;
            F.sR = R.side;
            F.type = FT_INTERIOR;
            F.wside = -1;
            qR.face = k;
            qL.type = qR.type = FT_INTERIOR;
            qL.nb = R.cell;
            qR.nb = L.cell;
            qL.ndx = b.xc[R.cell] - b.xc[L.cell];
            qL.ndy = b.yc[R.cell] - b.yc[L.cell];
            qR.ndx = -qL.ndx;
            qR.ndy = -qL.ndy;
            qL.tie = 0;
            qR.tie = 1;  // the R end is upwind for xi.n = 0
            qL.wside = qR.wside = 0;
        } else {
            const int t = tag[4 * L.cell + L.side];
            if (t < 0 || t > 3) return fail(IDUGKS_E_INVALID, "boundary side without a tag 0..3");
            F.R = -1;
            F.sR = -1;
            F.type = c->bc[t] == IDUGKS_BC_WALL ? FT_WALL : FT_FAR;
            F.wside = t;
            qL.type = F.type;
            qL.nb = -1;
            qL.tie = F.type == FT_FAR ? 1 : 0;
            qL.wside = t;
        }
        b.faces.push_back(F);
        i = j;
    }
    // the absent fourth side of the triangles
    {
        const int k = (int)b.faces.size();
        Face F{};
        F.L = F.R = 0;
        F.sL = F.sR = 3;
        F.type = FT_SELF;
        F.wside = -1;
        b.faces.push_back(F);
        for (int cell = 0; cell < nc; ++cell) {
            if (corners(cell) == 4) continue;
            CellSide &q = b.cs[(size_t)4 * cell + 3];
            q = CellSide{};
            q.nb = -1;
            q.face = k;
            q.type = FT_SELF;
        }
    }
    b.nf = (int)b.faces.size();
    // least-squares weights (Eq. 15)
    for (int cell = 0; cell < nc; ++cell) {
        double a11 = 0, a12 = 0, a22 = 0;
        for (int sd = 0; sd < 4; ++sd) {
            const CellSide &q = b.cs[(size_t)4 * cell + sd];
            if (q.nb < 0) continue;
            a11 += q.ndx * q.ndx; a12 += q.ndx * q.ndy; a22 += q.ndy * q.ndy;
        }
        const double det = a11 * a22 - a12 * a12;
        if (!(det > 0)) return fail(IDUGKS_E_INVALID, "degenerate least-squares stencil");
        for (int sd = 0; sd < 4; ++sd) {
            CellSide &q = b.cs[(size_t)4 * cell + sd];
            if (q.nb < 0) continue;
            q.ax = (a22 * q.ndx - a12 * q.ndy) / det;
            q.ay = (a11 * q.ndy - a12 * q.ndx) / det;
        }
    }
    // levels of the sweep order and the positions (by level, then cell index)
    std::vector<int> lev(nc, 0);
    int nlev = 0;
    for (int cell = 0; cell < nc; ++cell) {
        int l = 0;
        for (int sd = 0; sd < 4; ++sd) {
            const CellSide &q = b.cs[(size_t)4 * cell + sd];
            if (q.type != FT_SELF && q.nb >= 0 && q.nb < cell) l = std::max(l, lev[q.nb] + 1);
        }
        lev[cell] = l;
        nlev = std::max(nlev, l + 1);
    }
    b.nlev = nlev;
    b.hp_off.assign(nlev + 1, 0);
    for (int cell = 0; cell < nc; ++cell) ++b.hp_off[lev[cell] + 1];
    for (int l = 0; l < nlev; ++l) b.hp_off[l + 1] += b.hp_off[l];
    b.hp_pos.assign(nc, 0);
    std::vector<int> fill(b.hp_off.begin(), b.hp_off.end() - 1);
    for (int cell = 0; cell < nc; ++cell) b.hp_pos[cell] = fill[lev[cell]]++;
    return IDUGKS_OK;
}

idugks_status build(const idugks_config *c, Built &b) {
    const bool um = c->cell_nodes != nullptr;
    b.ni = um ? c->ncells : c->ni;
    b.nj = um ? 1 : c->nj;
    b.nc = b.ni * b.nj;
    b.nvx = c->nvx;
    b.nvy = c->nvy;
    b.nv = c->nvx * c->nvy;
    b.nvp = (b.nv + VPAD - 1) / VPAD * VPAD;
    // velocity set
    bool ok = c->quad == IDUGKS_GAUSS_HERMITE
                  ? gauss_hermite(c->nvx, b.x1, b.wx1) && gauss_hermite(c->nvy, b.y1, b.wy1)
                  : newton_cotes(c->nvx, c->vmax, b.x1, b.wx1) && newton_cotes(c->nvy, c->vmax, b.y1, b.wy1);
    if (!ok) return fail(IDUGKS_E_INVALID, "quadrature construction failed");
    b.xi.assign(b.nvp, 0.0);
    b.eta.assign(b.nvp, 0.0);
    b.w.assign(b.nvp, 0.0);
    b.vix.assign(b.nvp, 0);
    b.viy.assign(b.nvp, 0);
    for (int ix = 0; ix < b.nvx; ++ix)
        for (int iy = 0; iy < b.nvy; ++iy) {
            const int v = ix * b.nvy + iy;
            b.xi[v] = b.x1[ix];
            b.eta[v] = b.y1[iy];
            b.w[v] = b.wx1[ix] * b.wy1[iy];
            b.vix[v] = (int16_t)ix;
            b.viy[v] = (int16_t)iy;
        }
    const idugks_status gs = um ? build_unstructured(c, b) : build_structured(c, b);
    if (gs != IDUGKS_OK) return gs;
    // Per position of the sweep order the index row (GRow): the cell; per side the
    // neighbour cell, or -1 - t on a boundary side with boundary-condition slot t, or the
    // cell itself (a side without flux); the coupling masks; the neighbours' positions.
    // A coupled neighbour is read from the micro sweeps' LDS ring of RN positions when no
    // level exceeds RN cells, it lies on an earlier level (forward sweep) or a later one
    // (backward sweep) than the reading cell, and fewer than RN positions separate it from
    // the far end of the reading cell's level, so that its slot (position mod RN) has been
    // written in this sweep and not reused since.  (A cell that couples to itself, across
    // a periodic direction one cell wide, reads its forward-sweep increment from d1.)
    b.grow.assign((size_t)GR_N * b.nc, 0);
    const int RN = gs_ring_positions(c->precision == IDUGKS_FP32_MIXED);
    int lev_max = 0;
    std::vector<int> lev_of_pos(b.nc);
    for (int l = 0; l < b.nlev; ++l) {
        lev_max = std::max(lev_max, b.hp_off[l + 1] - b.hp_off[l]);
        for (int pos = b.hp_off[l]; pos < b.hp_off[l + 1]; ++pos) lev_of_pos[pos] = l;
    }
    for (int cidx = 0; cidx < b.nc; ++cidx) {
        const int pos = b.hp_pos[cidx];
        int *g = &b.grow[(size_t)GR_N * pos];
        const int l = lev_of_pos[pos], lo = b.hp_off[l], hi = b.hp_off[l + 1];
        g[GR_CELL] = cidx;
        int mask = 0;
        for (int sd = 0; sd < 4; ++sd) {
            const CellSide &q = b.cs[(size_t)4 * cidx + sd];
            g[GR_NB + sd] = q.type == FT_SELF ? cidx : q.nb >= 0 ? q.nb : -1 - q.wside;
            g[GR_SRC + sd] = g[GR_NB + sd];
            const bool coupled = q.type != FT_SELF && q.nb >= 0;
            if (coupled) mask |= q.nb < cidx ? 1 << sd : 1 << (4 + sd);
            if (q.type == FT_WALL) mask |= 1 << (8 + sd);
            g[GR_NPOS + sd] = coupled ? b.hp_pos[q.nb] : pos;
            if (coupled && lev_max <= RN) {
                const int qp = b.hp_pos[q.nb];
                if (q.nb < cidx ? qp < lo && qp + RN >= hi : qp >= hi && qp < lo + RN) {
                    mask |= 1 << (12 + sd);
                    g[GR_SRC + sd] = qp;
                }
            }
        }
        g[GR_MASK] = mask;
    }
    // bit 16: every cell that reads this cell's increment in the backward sweep takes it
    // from the ring, so the backward sweep need not leave it in d1
    {
        std::vector<char> from_d1(b.nc, 0);
        for (int cidx = 0; cidx < b.nc; ++cidx) {
            const int *g = &b.grow[(size_t)GR_N * b.hp_pos[cidx]];
            for (int sd = 0; sd < 4; ++sd)
                if (((g[GR_MASK] >> (4 + sd)) & 1) && !((g[GR_MASK] >> (12 + sd)) & 1))
                    from_d1[g[GR_NB + sd]] = 1;
        }
        for (int cidx = 0; cidx < b.nc; ++cidx)
            if (!from_d1[cidx]) b.grow[(size_t)GR_N * b.hp_pos[cidx] + GR_MASK] |= 1 << 16;
    }
    b.sgeo.assign((size_t)b.nc * SG_N, 0.0);
    for (int cidx = 0; cidx < b.nc; ++cidx)
        for (int s = 0; s < 4; ++s) {
            const CellSide &q = b.cs[(size_t)4 * cidx + s];
            double *g = &b.sgeo[(size_t)b.hp_pos[cidx] * SG_N];
            int code = 0;
            if (q.type != FT_SELF) {
                code |= SG_DIAG;
                if (q.nb >= 0) code |= q.nb < cidx ? SG_LOWER : SG_UPPER;
            }
            const bool flux = code & SG_DIAG;
            g[s] = flux ? q.nx * q.S : 0.0;  // xi.n S = xi nxS + eta nyS
            g[4 + s] = flux ? q.ny * q.S : 0.0;
            g[8 + s] = (code & SG_LOWER) ? 1.0 : 0.0;
            g[12 + s] = (code & SG_UPPER) ? 1.0 : 0.0;
        }
    // physical time step
    double hmin = 1e300, smax = 0.0;
    for (int cidx = 0; cidx < b.nc; ++cidx) {
        double d = 1e300;
        for (int s = 0; s < 4; ++s) {
            const CellSide &q = b.cs[(size_t)4 * cidx + s];
            if (q.S == 0.0) continue;  // the absent side of a triangle
            d = std::min(d, fabs(q.dx * q.nx + q.dy * q.ny));
        }
        hmin = std::min(hmin, 2.0 * d);
    }
    for (int v = 0; v < b.nv; ++v) smax = std::max(smax, sqrt(b.xi[v] * b.xi[v] + b.eta[v] * b.eta[v]));
    b.dt = c->cfl_phys * hmin / smax;
    // boundary distributions
    b.gw.assign((size_t)4 * b.nvp, 0.0);
    b.wKRT.assign(4, 0.0);
    std::vector<double> tmpH(b.nvp, 0.0);
    for (int s = 0; s < 4; ++s) {
        if (c->bc[s] != IDUGKS_BC_WALL) continue;
        host_equilibrium(b, c->K, 1.0, c->wall_u[s], c->wall_v[s], c->wall_T[s], &b.gw[(size_t)s * b.nvp], tmpH.data());
        b.wKRT[s] = c->K * 0.5 * c->wall_T[s];
    }
    b.ginf.assign(b.nvp, 0.0);
    b.hinf.assign(b.nvp, 0.0);
    host_equilibrium(b, c->K, c->far_rho, c->far_u, c->far_v, c->far_T, b.ginf.data(), b.hinf.data());
    b.eq0.assign((size_t)2 * b.nvp, 0.0);
    host_equilibrium(b, c->K, c->init_rho, c->init_u, c->init_v, c->init_T, b.eq0.data(), b.eq0.data() + b.nvp);
    // derivatives of the wall Maxwellians with respect to the wall's tangential speed (along
    // x) and its temperature, for the sensitivities
    b.dgw.assign((size_t)2 * 4 * b.nvp, 0.0);
    b.dwden.assign((size_t)2 * b.nf, 0.0);
    {
        std::vector<HD> gd(b.nv);
        for (int s = 0; s < 4; ++s) {
            if (c->bc[s] != IDUGKS_BC_WALL) continue;
            host_equilibrium_g<HD>(b, hd(1.0), hd(c->wall_u[s], 1.0, 0.0), hd(c->wall_v[s]),
                                   hd(c->wall_T[s], 0.0, 1.0), gd.data());
            for (int v = 0; v < b.nv; ++v) {
                b.dgw[(size_t)s * b.nvp + v] = gd[v].d[0];
                b.dgw[((size_t)4 + s) * b.nvp + v] = gd[v].d[1];
            }
        }
    }
    b.wden.assign(b.nf, 0.0);
    b.bhalf.assign((size_t)b.nf * NM_MAX, 0.0);
    b.nwall = 0;
    std::vector<char> use(b.nv);
    std::vector<double> gH(b.nv);
    for (int k = 0; k < b.nf; ++k) {
        const Face &F = b.faces[k];
        if (F.type != FT_WALL && F.type != FT_FAR) continue;
        for (int v = 0; v < b.nv; ++v) {
            const double un = normal_speed(b.xi[v], b.eta[v], F.nx, F.ny);
            use[v] = F.type == FT_WALL ? (un <= 0.0) : (un < 0.0);
        }
        if (F.type == FT_WALL) {
            b.wall_faces.push_back(k);
            ++b.nwall;
            const double *g = &b.gw[(size_t)F.wside * b.nvp];
            double den = 0.0;
            for (int v = 0; v < b.nv; ++v) {
                const double un = normal_speed(b.xi[v], b.eta[v], F.nx, F.ny);
                if (un < 0.0) den += b.w[v] * un * g[v];
                gH[v] = b.wKRT[F.wside] * g[v];
            }
            b.wden[k] = den;
            raw12(b, g, gH.data(), use, &b.bhalf[(size_t)k * NM_MAX]);
            for (int q = 0; q < 2; ++q) {
                const double *dg = &b.dgw[((size_t)q * 4 + F.wside) * b.nvp];
                double dd = 0.0;
                for (int v = 0; v < b.nv; ++v) {
                    const double un = normal_speed(b.xi[v], b.eta[v], F.nx, F.ny);
                    if (un < 0.0) dd += b.w[v] * un * dg[v];
                }
                b.dwden[(size_t)q * b.nf + k] = dd;
            }
        } else {
            raw12(b, b.ginf.data(), b.hinf.data(), use, &b.bhalf[(size_t)k * NM_MAX]);
        }
    }
    return IDUGKS_OK;
}

// Workspace regions.
enum Region {
    R_CS, R_FACES, R_WALLF, R_AREA, R_XI, R_ETA, R_W, R_X1, R_WX1, R_Y1, R_WY1, R_VIX, R_VIY,
    R_GW, R_WKRT, R_GINF, R_HINF, R_WDEN, R_BHALF, R_F, R_D1, R_TAB, R_TABS, R_TABF, R_REC,
    R_RECS, R_RECF, R_FIELDS, R_RAW, R_WC, R_MW, R_DW, R_DWD, R_DTIMP, R_RHOOLD, R_DRHO, R_SCAL,
    R_STAGE, R_HPOFF, R_HPPOS, R_SGEO, R_SREC, R_SDRHO, R_MH, R_FV, R_MWC, R_RECT, R_RECFT,
    // sensitivities (empty unless BGK, no limiter, FP64)
    R_LT, R_GJ, R_FBAR, R_YBUF, R_AGR, R_FADJ, R_CADJ, R_DGW, R_DWDEN, R_JACC, R_JACF, R_RED,
    R_ADJS, R_DWR, R_GROW, R_GROWT, R_COUNT
};
static_assert(R_COUNT <= Layout::N, "more workspace regions than the layout holds");

// Sensitivities are available for BGK without limiter in the FP64 form.
// (the transposed micro iteration runs the hyperplane sweep kernel)
bool adjoint_capable(const idugks_config *c) {
    return c->model == IDUGKS_BGK && c->limiter == 0 && c->precision == IDUGKS_FP64 && !c->cell_nodes &&
           c->sweep_order != IDUGKS_SWEEPS_LEVELS && sweep_plan(c).hyper_micro_fits;
}

// Wall faces the layout provides for: all boundary faces of a structured mesh, the built
// count on an unstructured one (idugks_workspace_size and init use the same bound).
int wall_bound(const idugks_config *c, const Built &b) {
    return c->cell_nodes ? b.nwall : 2 * (c->ni + c->nj);
}

constexpr int ADJS_N = 16;  // device scalars: [0..3] theta-bar, J of the last product;
                            // [4] mass dot; [5..6] update norms; [8..11] objective theta, J

Layout layout(const idugks_config *c, int nc, int nf, int nvp, int nvx, int nvy, int nwall) {
    Layout L;
    const size_t S = c->precision == IDUGKS_FP32_MIXED ? 4 : 8, TW = (size_t)nvx + nvy;
    // rows of the hyperplane-ordered sweep arrays: the staging waves read whole passes past
    // the last cell of a hyperplane, so these arrays carry min(ni, nj) + HP_SPARE spare rows
    const size_t ncs = (size_t)nc + (c->cell_nodes ? 1 : std::min(c->ni, c->nj)) + HP_SPARE;
    const int nv = c->nvx * c->nvy, nch = (nv + vel_chunk(nv) - 1) / vel_chunk(nv);
    const size_t adj = adjoint_capable(c) ? 1 : 0;
    const size_t sizes[R_COUNT] = {
        sizeof(CellSide) * 4 * (size_t)nc, sizeof(Face) * (size_t)nf, sizeof(int) * (size_t)std::max(nwall, 1),
        8 * (size_t)nc, 8 * (size_t)nvp, 8 * (size_t)nvp, 8 * (size_t)nvp, 8 * (size_t)nvx, 8 * (size_t)nvx,
        8 * (size_t)nvy, 8 * (size_t)nvy, 2 * (size_t)nvp, 2 * (size_t)nvp,
        8 * 4 * (size_t)nvp, 8 * 4, 8 * (size_t)nvp, 8 * (size_t)nvp, 8 * (size_t)nf, 8 * (size_t)nf * NM_MAX,
        S * 2 * (size_t)nc * nvp, S * 2 * (size_t)nc * nvp, S * (size_t)nc * TW, S * (size_t)nc * TW,
        S * (size_t)nf * TW, sizeof(Rec) * (size_t)nc, sizeof(Rec) * (size_t)nc, sizeof(Rec) * (size_t)nf,
        8 * (size_t)nc * 8, 8 * (size_t)nc * NM_MAX, 8 * 4 * (size_t)nc, 8 * 4 * (size_t)nc,
        8 * 4 * (size_t)nc, 8 * (size_t)nc, 8 * (size_t)nc, 8 * (size_t)nc, 8 * (size_t)nf, 8 * SC_NUM,
        8 * (size_t)std::max(nc, 2) * nvp, sizeof(int) * (size_t)(nc + 2), sizeof(int) * (size_t)nc,
        8 * (size_t)SG_N * ncs, 8 * (size_t)SR_N * ncs, 8 * 4 * (size_t)ncs, 8 * (size_t)MH_N * ncs,
        S * 2 * (size_t)nf * nvp, nch > 1 ? 8 * (size_t)nc * nch * 4 : 0,
        S * RT_N * (size_t)nc, S * RT_N * (size_t)nf,
        adj * 8 * 2 * (size_t)nc * nvp, adj * 8 * 2 * (size_t)nc * nvp, adj * 8 * 2 * (size_t)nc * nvp,
        adj * 8 * 2 * (size_t)nc * nvp, adj * 8 * 6 * (size_t)nc * nvp, adj * 8 * (size_t)FA_N * nf,
        adj * 8 * (size_t)CA_N * nc, adj * 8 * 8 * (size_t)nvp, adj * 8 * 2 * (size_t)nf,
        adj * 8 * 32 * (size_t)nc, adj * 8 * 32 * (size_t)nf, adj * 8 * (size_t)RED_N, adj * 8 * ADJS_N,
        8 * 4 * (size_t)nc, sizeof(int) * GR_N * (size_t)nc, S * GT_N * (size_t)nc};
    for (int r = 0; r < R_COUNT; ++r) L.add(sizes[r]);
    L.bytes = (L.bytes + 255) & ~size_t(255);
    return L;
}

// ---------------------------------------------------------------------------------------
// kernel sequence
// ---------------------------------------------------------------------------------------
template <class F>
idugks_status timed(idugks_ctx *x, int kid, F &&launch) {
    size_t slot = 0;
    const bool rec = x->prof && ((x->prof_mask >> kid) & 1u);
    if (rec) {
        slot = x->ev_used++;
        while (x->evs.size() < 2 * x->ev_used) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            x->evs.push_back(e);
        }
        if (x->ev_kid.size() < x->ev_used) x->ev_kid.resize(x->ev_used);
        x->ev_kid[slot] = kid;
        HIPCHK(hipEventRecord(x->evs[2 * slot], x->st));
    }
    hipError_t e = launch();
    if (e != hipSuccess)
        return fail(IDUGKS_E_DEVICE, std::string("kernel ") + kKernelNames[kid] + ": " + hipGetErrorString(e));
    if (rec) HIPCHK(hipEventRecord(x->evs[2 * slot + 1], x->st));
    return IDUGKS_OK;
}

#define RUN(kid, call)                                            \
    do {                                                          \
        idugks_status s_ = timed(x, kid, [&] { return (call); }); \
        if (s_ != IDUGKS_OK) return s_;                           \
    } while (0)

// cell and face records, reconstruction at the faces
idugks_status face_pipeline(idugks_ctx *x) {
    const Params &p = x->p;
    RUN(KID_RECORDS, launch_records(p, x->fp32, 0, x->st));
    RUN(KID_PARTIALS, launch_partials(p, x->fp32, x->st));
    RUN(KID_FACE_RECORDS, launch_face_records(p, x->fp32, x->st));
    return IDUGKS_OK;
}

idugks_status flux_pipeline(idugks_ctx *x) {
    idugks_status s = face_pipeline(x);
    if (s != IDUGKS_OK) return s;
    RUN(KID_FLUX, launch_flux(x->p, x->fp32, x->st));
    return IDUGKS_OK;
}

idugks_status finalize_state(idugks_ctx *x, int mode) {
    const Params &p = x->p;
    RUN(KID_RAW, launch_raw(p, x->fp32, p.nm, x->st));
    RUN(KID_FINALIZE, launch_finalize(p, x->fp32, mode, x->st));
    return IDUGKS_OK;
}

// The implicit CFL of the next implicit iteration: cfl_imp, or the start-up ramp
// min(cfl_imp, cfl_start cfl_growth^n) after n implicit iterations.
double implicit_cfl(const idugks_ctx *x) {
    if (!(x->cfl_start > 0)) return x->p.cfl_imp;
    const double c = x->cfl_start * pow(x->cfl_growth, (double)x->imp_iters);
    return c < x->p.cfl_imp ? c : x->p.cfl_imp;
}

idugks_status one_step(idugks_ctx *x, int mode) {
    const Params &p = x->p;
    idugks_status s = face_pipeline(x);
    if (s != IDUGKS_OK) return s;
    if (mode == IDUGKS_IMPLICIT) {
        Params q = p;  // the macro rows (implicit time step) take this iteration's CFL
        q.cfl_imp = implicit_cfl(x);
        if (p.nch == 1) {  // the flux blocks write the macro rows
            q.prep_in_flux = 1;
            RUN(KID_FLUX, launch_flux(q, x->fp32, x->st));
        } else {
            RUN(KID_FLUX, launch_flux(p, x->fp32, x->st));
            RUN(KID_MACRO_PREP, launch_macro_prep(q, x->st));
        }
        if (p.predictor == 1) RUN(KID_MACRO_RELAX, launch_macro_relax(p, x->st));
        else RUN(KID_MACRO, launch_macro(p, x->st));
        RUN(KID_RECORDS_PRED, launch_records(p, x->fp32, 1, x->st));
        RUN(KID_LOWER, launch_sweep(p, x->fp32, false, x->sweep, x->st));
        RUN(KID_WALL_GHOST, launch_wall_ghost(p, x->fp32, x->st));
        RUN(KID_UPPER, launch_sweep(p, x->fp32, true, x->sweep, x->st));
    } else {
        RUN(KID_FLUX, launch_flux(p, x->fp32, x->st));
        RUN(KID_EXPLICIT, launch_explicit(p, x->fp32, x->st));
    }
    return finalize_state(x, mode == IDUGKS_IMPLICIT ? 1 : 2);
}

idugks_status read_scalars(idugks_ctx *x, double *sc) {
    HIPCHK(hipMemcpyAsync(sc, x->p.scal, sizeof(double) * SC_NUM, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------
// Static scratch array: the workspace of contexts made by idugks_init_noalloc, for callers
// that cannot allocate device memory.  Each GPU the library runs on holds its own copy until
// the process ends.  In host code the array's name is only a stand-in for the symbol: its
// device address, per device, comes from hipGetSymbolAddress with that device current.  At
// most one such context may live per device (its contents are the context's state).
// ---------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[IDUGKS_NOALLOC_MAX_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device (null: not yet)
bool g_scratch_busy[kMaxDevices];   // a live context uses that device's array

idugks_status acquire_scratch(int *dev, void **ptr) {
    int d = -1;
    HIPCHK(hipGetDevice(&d));
    if (d < 0 || d >= kMaxDevices) return fail(IDUGKS_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_busy[d])
        return fail(IDUGKS_E_STATE, "the static scratch array of this device is in use by another context "
                                    "(destroy it first)");
    if (!g_scratch_ptr[d]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(IDUGKS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[d] = p;
    }
    g_scratch_busy[d] = true;
    *dev = d;
    *ptr = g_scratch_ptr[d];
    return IDUGKS_OK;
}

void release_scratch(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) g_scratch_busy[dev] = false;
}
}  // namespace

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------
extern "C" {

const char *idugks_last_error(void) { return g_err.c_str(); }

idugks_status idugks_workspace_size(const idugks_config *cfg, size_t *bytes) {
    if (!bytes) return fail(IDUGKS_E_INVALID, "null output");
    idugks_status s = validate(cfg);
    if (s != IDUGKS_OK) return s;
    if (cfg->cell_nodes) {  // face and wall counts come from the mesh
        Built b;
        s = build(cfg, b);
        if (s != IDUGKS_OK) return s;
        *bytes = layout(cfg, b.nc, b.nf, b.nvp, b.nvx, b.nvy, wall_bound(cfg, b)).bytes;
        return IDUGKS_OK;
    }
    const int nc = cfg->ni * cfg->nj, nf = (cfg->ni + 1) * cfg->nj + cfg->ni * (cfg->nj + 1);
    const int nv = cfg->nvx * cfg->nvy, nvp = (nv + VPAD - 1) / VPAD * VPAD;
    *bytes = layout(cfg, nc, nf, nvp, cfg->nvx, cfg->nvy, 2 * (cfg->ni + cfg->nj)).bytes;
    return IDUGKS_OK;
}

idugks_status idugks_describe(const idugks_config *cfg, double *xi, double *eta, double *w, double *dt,
                              double *area, int32_t *nb, double *nx, double *ny, double *S, double *ax,
                              double *ay) {
    idugks_status s = validate(cfg);
    if (s != IDUGKS_OK) return s;
    Built b;
    s = build(cfg, b);
    if (s != IDUGKS_OK) return s;
    for (int v = 0; v < b.nv; ++v) {
        if (xi) xi[v] = b.xi[v];
        if (eta) eta[v] = b.eta[v];
        if (w) w[v] = b.w[v];
    }
    if (dt) *dt = b.dt;
    for (int c = 0; c < b.nc; ++c) {
        if (area) area[c] = b.area[c];
        for (int k = 0; k < 4; ++k) {
            const CellSide &q = b.cs[(size_t)4 * c + k];
            const int m = 4 * c + k;
            if (nb) nb[m] = q.nb;
            if (nx) nx[m] = q.nx;
            if (ny) ny[m] = q.ny;
            if (S) S[m] = q.S;
            if (ax) ax[m] = q.ax;
            if (ay) ay[m] = q.ay;
        }
    }
    return IDUGKS_OK;
}

// Context on a validated configuration and a workspace of at least the required size.
static idugks_status init_ctx(const idugks_config *cfg, void *d_workspace, void *hip_stream, int scratch_dev,
                              idugks_ctx **out) {
    idugks_status s;
    Built b;
    s = build(cfg, b);
    if (s != IDUGKS_OK) return s;
    Layout L = layout(cfg, b.nc, b.nf, b.nvp, b.nvx, b.nvy, wall_bound(cfg, b));
    char *base = (char *)d_workspace;
    auto R = [&](int r) { return (void *)(base + L.off[r]); };

    idugks_ctx *x = new idugks_ctx();
    x->scratch_dev = -1;  // set by the caller once the context exists
    x->cfg = *cfg;
    x->cfg.xn = x->cfg.yn = nullptr;
    x->cfg.cell_nodes = x->cfg.side_tag = nullptr;
    x->fp32 = cfg->precision == IDUGKS_FP32_MIXED;
    x->cfl_start = cfg->cfl_start;
    x->cfl_growth = cfg->cfl_growth;
    x->imp_iters = 0;
    x->st = (hipStream_t)hip_stream;
    const SweepPlan plan = sweep_plan(cfg);
    // the hyperplane shape serves the micro sweeps and the adjoint's transposed sweeps
    x->sweep = plan.hyper_micro_fits ? sweep_shape(b.ni, b.nj, b.nv, x->fp32 ? 4 : 8) : SweepShape{};
    if (!plan.micro_levels && x->sweep.vb == 0) {
        delete x;
        return fail(IDUGKS_E_INVALID, "no sweep launch shape fits this mesh");
    }
    x->iters = 0;
    x->prof = false;
    x->ev_used = 0;
    x->area_h = b.area;
    x->xi_h.assign(b.xi.begin(), b.xi.begin() + b.nv);
    x->eta_h.assign(b.eta.begin(), b.eta.begin() + b.nv);
    x->w_h.assign(b.w.begin(), b.w.begin() + b.nv);
    Params &p = x->p;
    memset(&p, 0, sizeof p);
    p.ni = b.ni; p.nj = b.nj; p.nc = b.nc; p.nf = b.nf; p.nv = b.nv; p.nvp = b.nvp;
    p.vch = vel_chunk(b.nv); p.nch = (b.nv + p.vch - 1) / p.vch; p.prep_in_flux = 0;
    p.per_i = cfg->bc[0] == IDUGKS_BC_PERIODIC; p.per_j = cfg->bc[2] == IDUGKS_BC_PERIODIC;
    p.nvx = b.nvx; p.nvy = b.nvy; p.K = cfg->K; p.model = cfg->model; p.limiter = cfg->limiter;
    p.closed = b.closed; p.nm = cfg->model == IDUGKS_SHAKHOV ? NM_SHAKHOV : NM_BGK; p.nwall = b.nwall;
    p.dt = b.dt; p.h = 0.5 * b.dt; p.Pr = cfg->Pr; p.mu_ref = cfg->Kn / sqrt(M_PI);
    p.omega = cfg->omega; p.cfl_imp = cfg->cfl_imp; p.gam = (cfg->K + 4.0) / (cfg->K + 2.0);
    p.cs = (const CellSide *)R(R_CS); p.faces = (const Face *)R(R_FACES);
    p.wall_faces = (const int *)R(R_WALLF); p.area = (const double *)R(R_AREA);
    p.xi = (const double *)R(R_XI); p.eta = (const double *)R(R_ETA); p.w = (const double *)R(R_W);
    p.x1 = (const double *)R(R_X1); p.wx1 = (const double *)R(R_WX1);
    p.y1 = (const double *)R(R_Y1); p.wy1 = (const double *)R(R_WY1);
    p.vix = (const int16_t *)R(R_VIX); p.viy = (const int16_t *)R(R_VIY);
    p.gw = (const double *)R(R_GW); p.wKRT = (const double *)R(R_WKRT);
    p.ginf = (const double *)R(R_GINF); p.hinf = (const double *)R(R_HINF);
    p.wden = (const double *)R(R_WDEN); p.bhalf = (const double *)R(R_BHALF);
    p.f = R(R_F); p.d1 = R(R_D1); p.tab = R(R_TAB); p.tabs = R(R_TABS); p.tabf = R(R_TABF);
    p.rec = (Rec *)R(R_REC); p.recs = (Rec *)R(R_RECS); p.recf = (Rec *)R(R_RECF);
    p.fields = (double *)R(R_FIELDS); p.raw = (double *)R(R_RAW); p.Wc = (double *)R(R_WC);
    p.MW = (double *)R(R_MW); p.dW = (double *)R(R_DW); p.DWd = (double *)R(R_DWD);
    p.dWr = (double *)R(R_DWR);
    p.predictor = cfg->predictor; p.relax_sweeps = cfg->relax_sweeps;
    p.dtimp = (double *)R(R_DTIMP); p.rho_old = (double *)R(R_RHOOLD); p.drho = (double *)R(R_DRHO);
    p.scal = (double *)R(R_SCAL);
    p.hp_off = (const int *)R(R_HPOFF); p.hp_pos = (const int *)R(R_HPPOS);
    p.graph = plan.micro_levels; p.gmacro = plan.macro_levels; p.nlev = b.nlev; p.grow = (const int *)R(R_GROW);
    p.growT = R(R_GROWT);
    p.sgeo = (const double *)R(R_SGEO); p.srec = (double *)R(R_SREC); p.sdrho = (double *)R(R_SDRHO);
    p.mh = (double *)R(R_MH); p.fv = R(R_FV); p.recT = R(R_RECT); p.recfT = R(R_RECFT);
    p.MWc = (double *)R(R_MWC);
    x->stage = (double *)R(R_STAGE);
    p.Kn = cfg->Kn;
    for (int s4 = 0; s4 < 4; ++s4) { p.wall_u[s4] = cfg->wall_u[s4]; p.wall_v[s4] = cfg->wall_v[s4]; }
    x->adj = adjoint_capable(cfg);
    if (x->adj) {
        x->lt = (double *)R(R_LT); x->gJ = (double *)R(R_GJ); x->ybuf = (double *)R(R_YBUF);
        x->adjs = (double *)R(R_ADJS);
        p.fbar = (double *)R(R_FBAR); p.agr = (double *)R(R_AGR); p.fadj = (double *)R(R_FADJ);
        p.cadj = (double *)R(R_CADJ); p.dgw = (const double *)R(R_DGW); p.dwden = (const double *)R(R_DWDEN);
        p.jacc = (double *)R(R_JACC); p.jacf = (double *)R(R_JACF); p.red = (double *)R(R_RED);
    }

    auto up = [&](void *dst, const void *src, size_t n) {
        return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, x->st);
    };
    hipError_t e = hipSuccess;
#define UP(r, vec) if (e == hipSuccess && !(vec).empty()) e = up(R(r), (vec).data(), (vec).size() * sizeof((vec)[0]))
    UP(R_GROW, b.grow);
    // the level sweeps' rows in the state precision: the static side geometry, zeros for
    // the record and ghost increments (written each iteration; off the walls they stay 0)
    std::vector<unsigned char> growT(L.size(R_GROWT), 0);
    for (int pos = 0; pos < b.nc; ++pos)
        for (int e = 0; e < 8; ++e) {
            const double g = b.sgeo[(size_t)pos * SG_N + e];
            if (x->fp32) ((float *)growT.data())[(size_t)pos * GT_N + GT_GEO + e] = (float)g;
            else ((double *)growT.data())[(size_t)pos * GT_N + GT_GEO + e] = g;
        }
    UP(R_GROWT, growT);
    UP(R_CS, b.cs); UP(R_HPOFF, b.hp_off); UP(R_HPPOS, b.hp_pos); UP(R_SGEO, b.sgeo); UP(R_FACES, b.faces); UP(R_WALLF, b.wall_faces); UP(R_AREA, b.area);
    UP(R_XI, b.xi); UP(R_ETA, b.eta); UP(R_W, b.w); UP(R_X1, b.x1); UP(R_WX1, b.wx1);
    UP(R_Y1, b.y1); UP(R_WY1, b.wy1); UP(R_VIX, b.vix); UP(R_VIY, b.viy); UP(R_GW, b.gw);
    UP(R_WKRT, b.wKRT); UP(R_GINF, b.ginf); UP(R_HINF, b.hinf); UP(R_WDEN, b.wden); UP(R_BHALF, b.bhalf);
    UP(R_STAGE, b.eq0);
    if (x->adj) { UP(R_DGW, b.dgw); UP(R_DWDEN, b.dwden); }
#undef UP
    if (e == hipSuccess) e = hipMemsetAsync(p.drho, 0, sizeof(double) * b.nf, x->st);
    if (e == hipSuccess) e = hipMemsetAsync(p.sdrho, 0, sizeof(double) * 4 * b.nc, x->st);
    if (e == hipSuccess) e = hipMemsetAsync(p.rho_old, 0, sizeof(double) * b.nc, x->st);
    if (e == hipSuccess) e = hipMemsetAsync(p.scal, 0, sizeof(double) * SC_NUM, x->st);
    if (e == hipSuccess) e = hipMemsetAsync(p.dW, 0, sizeof(double) * 4 * b.nc, x->st);
    if (e == hipSuccess) e = launch_fill_uniform(p, x->fp32, x->stage, x->st);
    if (e == hipSuccess) e = hipStreamSynchronize(x->st);  // host vectors die with b
    if (e != hipSuccess) {
        delete x;
        return fail(IDUGKS_E_DEVICE, std::string("init upload: ") + hipGetErrorString(e));
    }
    s = finalize_state(x, 0);
    double sc[SC_NUM];
    if (s == IDUGKS_OK) s = read_scalars(x, sc);
    if (s != IDUGKS_OK) {
        idugks_destroy(x);
        return s;
    }
    p.M0 = sc[SC_MASS];
    x->scratch_dev = scratch_dev;
    *out = x;
    return IDUGKS_OK;
}

idugks_status idugks_init(const idugks_config *cfg, void *d_workspace, size_t bytes, void *hip_stream,
                          idugks_ctx **out) {
    if (!out) return fail(IDUGKS_E_INVALID, "null output");
    *out = nullptr;
    idugks_status s = validate(cfg);
    if (s != IDUGKS_OK) return s;
    if (!d_workspace) return fail(IDUGKS_E_INVALID, "null workspace");
    size_t need = 0;
    idugks_workspace_size(cfg, &need);
    if (bytes < need) return fail(IDUGKS_E_INVALID, "workspace too small");
    return init_ctx(cfg, d_workspace, hip_stream, -1, out);
}

idugks_status idugks_init_noalloc(const idugks_config *cfg, void *hip_stream, idugks_ctx **out) {
    if (!out) return fail(IDUGKS_E_INVALID, "null output");
    *out = nullptr;
    idugks_status s = validate(cfg);
    if (s != IDUGKS_OK) return s;
    size_t need = 0;
    idugks_workspace_size(cfg, &need);
    if (need > IDUGKS_NOALLOC_MAX_BYTES)
        return fail(IDUGKS_E_NOMEM, "configuration needs " + std::to_string(need) +
                                        " bytes of workspace, above the static scratch array's " +
                                        std::to_string((size_t)IDUGKS_NOALLOC_MAX_BYTES));
    int dev = -1;
    void *ptr = nullptr;
    s = acquire_scratch(&dev, &ptr);
    if (s != IDUGKS_OK) return s;
    // the array keeps the last context's contents: start from zeros, like a fresh buffer
    hipError_t e = launch_zero(ptr, need, (hipStream_t)hip_stream);
    if (e != hipSuccess) {
        release_scratch(dev);
        return fail(IDUGKS_E_DEVICE, std::string("scratch clear: ") + hipGetErrorString(e));
    }
    s = init_ctx(cfg, ptr, hip_stream, dev, out);
    if (s != IDUGKS_OK) release_scratch(dev);
    return s;
}

void idugks_destroy(idugks_ctx *ctx) {
    if (!ctx) return;
    for (hipEvent_t e : ctx->evs) (void)hipEventDestroy(e);
    if (ctx->scratch_dev >= 0) release_scratch(ctx->scratch_dev);
    delete ctx;
}

idugks_status idugks_get_info(idugks_ctx *x, idugks_info *out) {
    if (!x || !out) return fail(IDUGKS_E_INVALID, "null argument");
    out->nc = x->p.nc; out->nv = x->p.nv; out->nvp = x->p.nvp; out->nf = x->p.nf;
    out->nwall = x->p.nwall; out->nvx = x->p.nvx; out->nvy = x->p.nvy;
    out->precision = x->cfg.precision; out->dt = x->p.dt; out->M0 = x->p.M0;
    out->iterations = x->iters;
    return IDUGKS_OK;
}

idugks_status idugks_velocities(idugks_ctx *x, double *xi, double *eta, double *w) {
    if (!x || !xi || !eta || !w) return fail(IDUGKS_E_INVALID, "null argument");
    memcpy(xi, x->xi_h.data(), sizeof(double) * x->p.nv);
    memcpy(eta, x->eta_h.data(), sizeof(double) * x->p.nv);
    memcpy(w, x->w_h.data(), sizeof(double) * x->p.nv);
    return IDUGKS_OK;
}

idugks_status idugks_step(idugks_ctx *x, int32_t mode, int32_t nsteps, double *res_out) {
    if (!x) return fail(IDUGKS_E_INVALID, "null context");
    if (mode != IDUGKS_EXPLICIT && mode != IDUGKS_IMPLICIT) return fail(IDUGKS_E_INVALID, "unknown mode");
    if (nsteps < 0) return fail(IDUGKS_E_INVALID, "negative step count");
    for (int n = 0; n < nsteps; ++n) {
        idugks_status s = one_step(x, mode);
        if (s != IDUGKS_OK) return s;
        ++x->iters;
        if (mode == IDUGKS_IMPLICIT) ++x->imp_iters;
    }
    double sc[SC_NUM];
    idugks_status s = read_scalars(x, sc);
    if (s != IDUGKS_OK) return s;
    if (res_out) *res_out = sc[SC_RES];
    if (sc[SC_FLAG] != 0.0 || !std::isfinite(sc[SC_RES]))
        return fail(IDUGKS_E_DIVERGED, "non-physical state (rho <= 0, E <= 0 or NaN)");
    return IDUGKS_OK;
}

idugks_status idugks_solve(idugks_ctx *x, double tol, int32_t max_iter, int32_t *iters, double *res_out) {
    if (!x) return fail(IDUGKS_E_INVALID, "null context");
    if (!(tol > 0) || max_iter < 0) return fail(IDUGKS_E_INVALID, "bad tolerance or iteration limit");
    double r = INFINITY, prev = INFINITY;
    int n = 0, grown = 0;
    idugks_status s = IDUGKS_OK;
    while (n < max_iter) {
        s = idugks_step(x, IDUGKS_IMPLICIT, 1, &r);
        ++n;
        if (s != IDUGKS_OK || r < tol) break;
        // a residual that keeps growing: stop while the state is still physical
        grown = r > prev ? grown + 1 : 0;
        prev = r;
        if (x->cfg.diverge_iters > 0 && grown >= x->cfg.diverge_iters) {
            s = fail(IDUGKS_E_DIVERGED, "residual grew in " + std::to_string(grown) + " consecutive iterations");
            break;
        }
    }
    if (iters) *iters = n;
    if (res_out) *res_out = r;
    if (s != IDUGKS_OK) return s;
    return r < tol ? IDUGKS_OK : fail(IDUGKS_E_NOT_CONVERGED, "iteration limit reached");
}

static idugks_status copy_out(idugks_ctx *x, void *dst, const void *src, size_t n, int on_host) {
    HIPCHK(hipMemcpyAsync(dst, src, n, on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

idugks_status idugks_flux(idugks_ctx *x, double *M, int32_t on_host) {
    if (!x || !M) return fail(IDUGKS_E_INVALID, "null argument");
    idugks_status s = flux_pipeline(x);
    if (s != IDUGKS_OK) return s;
    const size_t n = (size_t)x->p.nc * x->p.nv;
    for (int sp = 0; sp < 2; ++sp) {
        double *dst = on_host ? x->stage : M + sp * n;
        HIPCHK(launch_pack(x->p, x->fp32, x->p.d1, dst, sp, 1, 0, x->st));
        if (on_host) {
            s = copy_out(x, M + sp * n, x->stage, n * sizeof(double), 1);
            if (s != IDUGKS_OK) return s;
        }
    }
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

idugks_status idugks_face_moments(idugks_ctx *x, double *Wf, double *rho_w, int32_t on_host) {
    if (!x) return fail(IDUGKS_E_INVALID, "null context");
    idugks_status s = flux_pipeline(x);
    if (s != IDUGKS_OK) return s;
    const int nf = x->p.nf;
    std::vector<Rec> r(nf);
    std::vector<Face> F(nf);
    HIPCHK(hipMemcpyAsync(r.data(), x->p.recf, sizeof(Rec) * nf, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipMemcpyAsync(F.data(), x->p.faces, sizeof(Face) * nf, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    std::vector<double> W(4 * (size_t)nf, 0.0), rw(nf, 0.0);
    for (int k = 0; k < nf; ++k) {
        if (F[k].type == FT_SELF) continue;
        const Rec &q = r[k];
        W[4 * k] = q.rho;
        W[4 * k + 1] = q.rho * q.U;
        W[4 * k + 2] = q.rho * q.V;
        W[4 * k + 3] = 0.5 * q.rho * (q.U * q.U + q.V * q.V + (x->p.K + 2) * q.RT);
        rw[k] = q.rw;
    }
    const hipMemcpyKind kind = on_host ? hipMemcpyHostToHost : hipMemcpyHostToDevice;
    if (Wf) HIPCHK(hipMemcpyAsync(Wf, W.data(), sizeof(double) * 4 * nf, kind, x->st));
    if (rho_w) HIPCHK(hipMemcpyAsync(rho_w, rw.data(), sizeof(double) * nf, kind, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

idugks_status idugks_macro_residual(idugks_ctx *x, double *MW, int32_t on_host) {
    if (!x || !MW) return fail(IDUGKS_E_INVALID, "null argument");
    idugks_status s = flux_pipeline(x);
    if (s != IDUGKS_OK) return s;
    return copy_out(x, MW, x->p.MW, sizeof(double) * 4 * x->p.nc, on_host);
}

idugks_status idugks_predict(idugks_ctx *x, double *Wstar, double *dt_imp, int32_t on_host) {
    if (!x) return fail(IDUGKS_E_INVALID, "null context");
    idugks_status s = flux_pipeline(x);
    if (s != IDUGKS_OK) return s;
    Params q = x->p;
    q.cfl_imp = implicit_cfl(x);
    RUN(KID_MACRO_PREP, launch_macro_prep(q, x->st));
    if (x->p.predictor == 1) RUN(KID_MACRO_RELAX, launch_macro_relax(x->p, x->st));
    else RUN(KID_MACRO, launch_macro(x->p, x->st));
    const int nc = x->p.nc;
    std::vector<double> W(4 * nc), dW(4 * nc);
    HIPCHK(hipMemcpyAsync(W.data(), x->p.Wc, sizeof(double) * 4 * nc, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipMemcpyAsync(dW.data(), x->p.dW, sizeof(double) * 4 * nc, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    for (int i = 0; i < 4 * nc; ++i) W[i] += dW[i];
    if (Wstar) {
        HIPCHK(hipMemcpyAsync(Wstar, W.data(), sizeof(double) * 4 * nc,
                              on_host ? hipMemcpyHostToHost : hipMemcpyHostToDevice, x->st));
    }
    if (dt_imp) {
        HIPCHK(hipMemcpyAsync(dt_imp, x->p.dtimp, sizeof(double) * nc,
                              on_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, x->st));
    }
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

// ---- sensitivities --------------------------------------------------------------------
static idugks_status adjoint_check(idugks_ctx *x) {
    if (!x) return fail(IDUGKS_E_INVALID, "null context");
    if (!x->adj) return fail(IDUGKS_E_INVALID, "sensitivities need the BGK model, no limiter, the FP64 form and a structured mesh whose hyperplane sweeps fit (sweep_order AUTO or HYPERPLANES)");
    return IDUGKS_OK;
}

// Forward values the reverse pass reads: records, face values and records, flux, record
// Jacobians.
static idugks_status adjoint_forward(idugks_ctx *x) {
    idugks_status s = flux_pipeline(x);
    if (s != IDUGKS_OK) return s;
    HIPCHK(launch_rec_jac(x->p, x->st));
    return IDUGKS_OK;
}

// f-bar = lam^T dR/df (+ seed of objective obj), theta-bar and J into out[0..3]
static idugks_status vjp_core(idugks_ctx *x, const double *lam, int obj, double *out) {
    Params q = x->p;
    q.lam = lam;
    HIPCHK(launch_adj_face(q, obj, x->st));
    HIPCHK(launch_adj_gather(q, obj, x->st));
    HIPCHK(launch_adj_cell(q, x->st));
    HIPCHK(launch_adj_theta(q, out, x->st));
    return IDUGKS_OK;
}

// canonical [2][nc][nv] (host or device) -> device layout [nc][2][nvp]
static idugks_status canonical_in(idugks_ctx *x, const double *src, int on_host, double *dst) {
    const size_t n = (size_t)2 * x->p.nc * x->p.nv;
    if (on_host) {
        HIPCHK(hipMemcpyAsync(x->ybuf, src, n * sizeof(double), hipMemcpyHostToDevice, x->st));
        src = x->ybuf;
    }
    HIPCHK(launch_to_dev(x->p, src, dst, x->st));
    return IDUGKS_OK;
}

static idugks_status canonical_out(idugks_ctx *x, const double *src, double scale, double *dst, int on_host) {
    const size_t n = (size_t)2 * x->p.nc * x->p.nv;
    double *d = on_host ? x->ybuf : dst;
    HIPCHK(launch_from_dev(x->p, src, d, scale, x->st));
    if (on_host) HIPCHK(hipMemcpyAsync(dst, x->ybuf, n * sizeof(double), hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

idugks_status idugks_vjp(idugks_ctx *x, const double *lam, double *f_bar, double theta_bar[3], int32_t on_host) {
    idugks_status s = adjoint_check(x);
    if (s != IDUGKS_OK) return s;
    if (!lam) return fail(IDUGKS_E_INVALID, "null lam");
    if ((s = adjoint_forward(x)) != IDUGKS_OK) return s;
    if ((s = canonical_in(x, lam, on_host, x->lt)) != IDUGKS_OK) return s;
    if ((s = vjp_core(x, x->lt, -1, x->adjs)) != IDUGKS_OK) return s;
    if (f_bar && (s = canonical_out(x, x->p.fbar, 1.0, f_bar, on_host)) != IDUGKS_OK) return s;
    double t[4];
    HIPCHK(hipMemcpyAsync(t, x->adjs, sizeof t, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    if (theta_bar)
        for (int a = 0; a < 3; ++a) theta_bar[a] = t[a];
    return IDUGKS_OK;
}

idugks_status idugks_objective(idugks_ctx *x, int32_t objective, double *J, double *dJ_df,
                               double dJ_dtheta[3], int32_t on_host) {
    idugks_status s = adjoint_check(x);
    if (s != IDUGKS_OK) return s;
    if (objective != 0 && objective != 1) return fail(IDUGKS_E_INVALID, "unknown objective");
    if ((s = adjoint_forward(x)) != IDUGKS_OK) return s;
    HIPCHK(hipMemsetAsync(x->lt, 0, sizeof(double) * 2 * x->p.nc * x->p.nvp, x->st));
    if ((s = vjp_core(x, x->lt, objective, x->adjs)) != IDUGKS_OK) return s;
    if (dJ_df && (s = canonical_out(x, x->p.fbar, 1.0, dJ_df, on_host)) != IDUGKS_OK) return s;
    double t[4];
    HIPCHK(hipMemcpyAsync(t, x->adjs, sizeof t, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    if (dJ_dtheta)
        for (int a = 0; a < 3; ++a) dJ_dtheta[a] = t[a];
    if (J) *J = t[3];
    return IDUGKS_OK;
}

idugks_status idugks_adjoint(idugks_ctx *x, int32_t objective, double tol, int32_t max_iter, double *J,
                             double grad[3], int32_t *iters, double *res_out, double *lam, int32_t on_host) {
    idugks_status s = adjoint_check(x);
    if (s != IDUGKS_OK) return s;
    if (objective != 0 && objective != 1) return fail(IDUGKS_E_INVALID, "unknown objective");
    if (!(tol > 0) || max_iter < 1) return fail(IDUGKS_E_INVALID, "bad tolerance or iteration limit");
    const Params &p = x->p;
    const size_t nd = (size_t)2 * p.nc * p.nvp;
    if ((s = adjoint_forward(x)) != IDUGKS_OK) return s;
    HIPCHK(launch_macro_prep(p, x->st));   // dt_imp of the current state
    HIPCHK(launch_adj_diag(p, x->st));      // diagonal of the preconditioner
    // g = dJ/df and dJ/dtheta at fixed f
    HIPCHK(hipMemsetAsync(x->lt, 0, nd * sizeof(double), x->st));
    if ((s = vjp_core(x, x->lt, objective, x->adjs + 8)) != IDUGKS_OK) return s;
    HIPCHK(hipMemcpyAsync(x->gJ, p.fbar, nd * sizeof(double), hipMemcpyDeviceToDevice, x->st));
    // Fixed-point iteration of the adjoint of one micro LU-SGS iteration with the mass
    // rescale (closed domains): with y = lt - l_M (f.lt)/M0 and z = P^-T y,
    //   lt <- y + (dR/df)^T z + g,
    // whose limit gives the Lagrange multipliers lam = -z of the steady problem and
    // dJ/dtheta = dJ/dtheta|_f + z^T dR/dtheta.  P is the micro operator of Eq. 26 (current
    // records, no predictor): its transpose is an ascending and a descending sweep along
    // the outflow couplings.
    double r = INFINITY, h[4];
    int it = 0;
    const double dotscale = p.closed ? 1.0 : 0.0;
    for (it = 1; it <= max_iter; ++it) {
        HIPCHK(launch_dot(p, (const double *)p.f, x->lt, dotscale, x->adjs + 4, x->st));
        HIPCHK(launch_adj_project(p, x->lt, x->ybuf, x->adjs + 4, x->st));
        HIPCHK(launch_adj_sweep(p, false, x->sweep, x->st));
        HIPCHK(launch_adj_sweep(p, true, x->sweep, x->st));
        if ((s = vjp_core(x, (const double *)p.d1, -1, x->adjs)) != IDUGKS_OK) return s;
        HIPCHK(launch_adj_update(p, x->lt, x->ybuf, x->gJ, x->adjs + 5, x->st));
        double nrm[2];
        HIPCHK(hipMemcpyAsync(nrm, x->adjs + 5, sizeof nrm, hipMemcpyDeviceToHost, x->st));
        HIPCHK(hipStreamSynchronize(x->st));
        r = nrm[1] > 0 ? sqrt(nrm[0] / nrm[1]) : 0.0;
        if (!std::isfinite(r)) return fail(IDUGKS_E_DIVERGED, "adjoint iteration diverged");
        if (r < tol) break;
    }
    double t[12];
    HIPCHK(hipMemcpyAsync(t, x->adjs, sizeof t, hipMemcpyDeviceToHost, x->st));
    HIPCHK(hipStreamSynchronize(x->st));
    for (int a = 0; a < 3; ++a) h[a] = t[8 + a] + t[a];
    if (grad)
        for (int a = 0; a < 3; ++a) grad[a] = h[a];
    if (J) *J = t[11];
    if (iters) *iters = it > max_iter ? max_iter : it;
    if (res_out) *res_out = r;
    if (lam && (s = canonical_out(x, (const double *)p.d1, -1.0, lam, on_host)) != IDUGKS_OK) return s;
    return r < tol ? IDUGKS_OK : fail(IDUGKS_E_NOT_CONVERGED, "adjoint iteration limit reached");
}

idugks_status idugks_residual(idugks_ctx *x, double out_l2[4]) {
    if (!x || !out_l2) return fail(IDUGKS_E_INVALID, "null argument");
    const int nc = x->p.nc;
    std::vector<double> MW(4 * nc);
    idugks_status s = idugks_macro_residual(x, MW.data(), 1);
    if (s != IDUGKS_OK) return s;
    for (int a = 0; a < 4; ++a) {
        double acc = 0.0;
        for (int c = 0; c < nc; ++c) {
            const double r = MW[4 * c + a] / x->area_h[c];
            acc += r * r;
        }
        out_l2[a] = sqrt(acc / nc);
    }
    return IDUGKS_OK;
}

idugks_status idugks_moments(idugks_ctx *x, double *out, int32_t out_on_host) {
    if (!x || !out) return fail(IDUGKS_E_INVALID, "null argument");
    HIPCHK(launch_raw(x->p, x->fp32, NM_MAX, x->st));
    HIPCHK(launch_fields(x->p, x->p.fields, x->st));
    return copy_out(x, out, x->p.fields, sizeof(double) * 8 * x->p.nc, out_on_host);
}

idugks_status idugks_get_state(idugks_ctx *x, double *f, int32_t on_host) {
    if (!x || !f) return fail(IDUGKS_E_INVALID, "null argument");
    const size_t n = (size_t)x->p.nc * x->p.nv;
    for (int sp = 0; sp < 2; ++sp) {
        double *dst = on_host ? x->stage : f + sp * n;
        HIPCHK(launch_pack(x->p, x->fp32, x->p.f, dst, sp, 1, 1, x->st));
        if (on_host) {
            idugks_status s = copy_out(x, f + sp * n, x->stage, n * sizeof(double), 1);
            if (s != IDUGKS_OK) return s;
        }
    }
    HIPCHK(hipStreamSynchronize(x->st));
    return IDUGKS_OK;
}

idugks_status idugks_set_state(idugks_ctx *x, const double *f, int32_t on_host) {
    if (!x || !f) return fail(IDUGKS_E_INVALID, "null argument");
    const size_t n = (size_t)x->p.nc * x->p.nv;
    for (int sp = 0; sp < 2; ++sp) {
        const double *src = f + sp * n;
        if (on_host) {
            HIPCHK(hipMemcpyAsync(x->stage, src, n * sizeof(double), hipMemcpyHostToDevice, x->st));
            src = x->stage;
        }
        HIPCHK(launch_unpack(x->p, x->fp32, src, sp, 1, x->st));
        HIPCHK(hipStreamSynchronize(x->st));
    }
    HIPCHK(hipMemsetAsync(x->p.rho_old, 0, sizeof(double) * x->p.nc, x->st));
    HIPCHK(hipMemsetAsync(x->p.drho, 0, sizeof(double) * x->p.nf, x->st));
    HIPCHK(hipMemsetAsync(x->p.sdrho, 0, sizeof(double) * 4 * x->p.nc, x->st));
    idugks_status s = finalize_state(x, 0);
    double sc[SC_NUM];
    if (s == IDUGKS_OK) s = read_scalars(x, sc);
    if (s != IDUGKS_OK) return s;
    x->p.M0 = sc[SC_MASS];
    x->iters = 0;
    x->imp_iters = 0;
    return IDUGKS_OK;
}

int32_t idugks_num_kernels(void) { return KID_COUNT; }

const char *idugks_kernel_name(int32_t k) { return (k >= 0 && k < KID_COUNT) ? kKernelNames[k] : ""; }

idugks_status idugks_profile_mask(idugks_ctx *x, int32_t mode, int32_t nsteps, uint32_t kernel_mask,
                                  double *ms, int64_t *counts) {
    if (!x || !ms) return fail(IDUGKS_E_INVALID, "null argument");
    for (int k = 0; k < KID_COUNT; ++k) { x->ms[k] = 0.0; x->cnt[k] = 0; }
    x->prof = true;
    x->prof_mask = kernel_mask;
    x->ev_used = 0;
    idugks_status s = idugks_step(x, mode, nsteps, nullptr);
    x->prof = false;
    HIPCHK(hipStreamSynchronize(x->st));
    for (size_t i = 0; i < x->ev_used; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, x->evs[2 * i], x->evs[2 * i + 1]));
        x->ms[x->ev_kid[i]] += ms;
        x->cnt[x->ev_kid[i]] += 1;
    }
    for (int k = 0; k < KID_COUNT; ++k) {
        ms[k] = x->ms[k];
        if (counts) counts[k] = x->cnt[k];
    }
    return s;
}

idugks_status idugks_profile(idugks_ctx *x, int32_t mode, int32_t nsteps, double *ms, int64_t *counts) {
    return idugks_profile_mask(x, mode, nsteps, 0xFFFFFFFFu, ms, counts);
}

}  // extern "C"
