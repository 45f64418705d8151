/*
 * idugks.h - C ABI of the MI355X (gfx950) implicit DUGKS solver.
 *
 * Method: Pan, Zhong & Zhuo, "An implicit discrete unified gas-kinetic scheme for
 * simulations of steady flow in all flow regimes", arXiv:1709.01819.
 *   Section 2.1 (Eq. 1-20)   explicit DUGKS: BGK/Shakhov collision, reduced distributions
 *                            G, H, interface flux by characteristic reconstruction;
 *   Section 2.2 (Eq. 21-32)  implicit DUGKS: predicted macroscopic LU-SGS step, micro
 *                            LU-SGS sweeps over (cell x discrete velocity), update;
 *   Section 2.3 (Eq. 33-35)  ghost-cell and diffuse-wall boundary conditions.
 *
 * Conventions
 *   - structured quadrilateral mesh of ni x nj cells; cell (i, j) has index i + j*ni;
 *     node (i, j) has index i + j*(ni+1); boundary sides are ordered i-, i+, j-, j+;
 *     or an unstructured mesh of quadrilaterals and triangles (idugks_config.cell_nodes),
 *     whose boundary sides name one of the same four boundary-condition slots;
 *   - tensor-product discrete velocities, index v = ix*nvy + iy;
 *   - units: gas constant R = 1/2 (so T = 2RT and the reference Maxwellian is
 *     exp(-|xi|^2)/pi), Knudsen number Kn as in Eq. 37 with rho = L = 2RT_ref = 1;
 *   - the canonical state is FP64 [2][nc][nv]: species 0 is G~, species 1 is H~ (the
 *     transformed distributions of Eq. 10).
 *
 * Memory and streams
 *   - the library never allocates device memory: the caller passes one device buffer
 *     of idugks_workspace_size() bytes (it must outlive the context) and a HIP stream;
 *     all device work is enqueued on that stream;
 *   - pointers marked "device" point into caller-owned device memory, pointers marked
 *     "host" into caller-owned host memory; functions with an on_host flag accept either;
 *   - the only calls that wait for the stream are those returning values on the host.
 *
 * Errors
 *   Every call returns an idugks_status and never aborts.  Invalid arguments or
 *   configurations are rejected before any device work with IDUGKS_E_INVALID; HIP
 *   failures give IDUGKS_E_DEVICE.  idugks_last_error() returns a thread-local
 *   message describing the last failure.
 */
#ifndef IDUGKS_H
#define IDUGKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct idugks_ctx idugks_ctx;

typedef enum {
    IDUGKS_OK = 0,
    IDUGKS_E_INVALID = 1,        /* bad argument or configuration; nothing was done */
    IDUGKS_E_NOMEM = 2,          /* workspace too small (host allocation failure) */
    IDUGKS_E_DEVICE = 3,         /* a HIP call failed */
    IDUGKS_E_DIVERGED = 4,       /* non-physical state (rho <= 0, T <= 0 or NaN), or in
                                    idugks_solve a residual that kept growing
                                    (idugks_config.diverge_iters) */
    IDUGKS_E_NOT_CONVERGED = 5,  /* iteration limit reached; the state stays valid */
    IDUGKS_E_STATE = 6           /* call not allowed in the current state */
} idugks_status;

enum { IDUGKS_BC_WALL = 0, IDUGKS_BC_FARFIELD = 1, IDUGKS_BC_PERIODIC = 2 };
enum { IDUGKS_GAUSS_HERMITE = 0, IDUGKS_NEWTON_COTES = 1 };
enum { IDUGKS_BGK = 0, IDUGKS_SHAKHOV = 1 };
enum { IDUGKS_FP64 = 0, IDUGKS_FP32_MIXED = 1 };
enum { IDUGKS_EXPLICIT = 0, IDUGKS_IMPLICIT = 1 };
enum { IDUGKS_SWEEPS_AUTO = 0, IDUGKS_SWEEPS_LEVELS = 1, IDUGKS_SWEEPS_HYPERPLANES = 2 };

/* Problem statement (Section 2 and Section 3 of the paper). */
typedef struct {
    uint32_t struct_size;        /* = sizeof(idugks_config) */
    int32_t ni, nj;              /* cells; periodic directions need 1 or >= 3 cells */
    const double *xn, *yn;       /* host, (ni+1)*(nj+1) node coordinates, read during init */
    int32_t bc[4];               /* IDUGKS_BC_* for sides i-, i+, j-, j+ (periodic in pairs) */
    double wall_u[4], wall_v[4]; /* wall velocity of each side (diffuse walls, Eq. 34) */
    double wall_T[4];            /* wall temperature of each side */
    double far_rho, far_u, far_v, far_T; /* far-field state (incoming half of the ghost) */
    int32_t quad, nvx, nvy;      /* velocity quadrature (Section 2.2, last paragraph) */
    double vmax;                 /* Newton-Cotes range [-vmax, vmax]; ignored by Gauss-Hermite */
    int32_t model;               /* IDUGKS_BGK (Eq. 1) or IDUGKS_SHAKHOV (Eq. 20, needs K = 1) */
    double Kn, Pr, omega;        /* Knudsen number (Eq. 36-37), Prandtl number, mu ~ T^omega */
    int32_t K;                   /* internal degrees of freedom (Eq. 2) */
    double cfl_phys;             /* physical time step: cfl_phys * min cell size / max |xi| */
    double cfl_imp;              /* implicit pseudo time step (Eq. 26, Eq. 30) */
    int32_t limiter;             /* 0 none, 1 Venkatakrishnan (Eq. 16-17) */
    int32_t precision;           /* IDUGKS_FP64 or IDUGKS_FP32_MIXED (FP32 distributions,
                                    FP64 moments, records, predictor and residuals) */
    double init_rho, init_u, init_v, init_T; /* initial uniform equilibrium */
    int32_t predictor;           /* macroscopic prediction step (Section 2.2; the conclusions
                                    name both): 0 LU-SGS sweeps of Eq. 29-31, 1 point
                                    relaxation of the same system (Jacobi) */
    int32_t relax_sweeps;        /* point relaxation: Jacobi sweeps after the point-implicit
                                    step dW = D^-1 M_W, 0..64 */
    double cfl_start;            /* start-up ramp of the implicit CFL (an addition; the paper
                                    starts at its final CFL): with cfl_start > 0, implicit
                                    iteration n, counted from init or the last set_state, uses
                                    min(cfl_imp, cfl_start * cfl_growth^n); 0 = no ramp.
                                    The adjoint iteration keeps cfl_imp. */
    double cfl_growth;           /* ramp factor per implicit iteration, 1 <= g < 1000 */
    /* Unstructured mesh of quadrilaterals and triangles (the finite-volume form of
       Section 2.1 sums over the faces of any cell; Section 3 runs hybrid meshes).  With
       cell_nodes != NULL the mesh is this one, ni and nj are ignored and xn, yn hold nnodes
       node coordinates.  cell_nodes [ncells][4] (host, read during init): the nodes of each
       cell counter-clockwise, -1 in the fourth slot of a triangle; side s of a cell is the
       edge from its node s to the next.  side_tag [ncells][4] (host): on a side that lies on
       the boundary, which of the four boundary conditions (bc[t], wall_*[t], far_*) applies,
       t = 0..3 (periodic ones are refused); ignored elsewhere.  An edge belongs to at most
       two cells.  The implicit sweeps take the cells in index order (Eq. 24-26, Eq. 29-31),
       level by level of that order's dependency graph.  Sensitivities (idugks_vjp,
       idugks_objective, idugks_adjoint) are not available on such meshes. */
    int32_t nnodes, ncells;
    const int32_t *cell_nodes, *side_tag;
    int32_t sweep_order;         /* how the implicit sweeps walk the cell order (the same
                                    order, hence the same result up to rounding):
                                    IDUGKS_SWEEPS_AUTO (0) the library's choice: on structured
                                    meshes the micro sweeps by levels for at least 8192
                                    velocities (or where the hyperplane shape does not fit),
                                    else by i+j hyperplanes, and the macro sweep by
                                    hyperplanes where it fits; IDUGKS_SWEEPS_LEVELS (1) both by
                                    levels of the order's dependency graph;
                                    IDUGKS_SWEEPS_HYPERPLANES (2) both by i+j hyperplanes
                                    (structured meshes that fit the LDS-resident fronts).
                                    Unstructured meshes take AUTO or LEVELS (both by levels). */
    int32_t diverge_iters;       /* idugks_solve stops with IDUGKS_E_DIVERGED once the
                                    residual has grown in this many consecutive iterations,
                                    before the state turns non-physical; 0 = never on growth
                                    alone (the non-physical-state check always applies).
                                    The state stays valid and can be read or replaced. */
} idugks_config;

typedef struct {
    int32_t nc, nv, nvp, nf, nwall, nvx, nvy, precision;
    double dt;                   /* physical time step */
    double M0;                   /* reference mass of a closed domain */
    int64_t iterations;          /* steps taken since init or set_state */
} idugks_info;

/* Host-only description of a configuration; no device work.  All outputs are host
   arrays (any may be NULL): the velocity set xi, eta, w [nv] (Section 2.2, last paragraph),
   the physical time step dt [1], cell areas [nc], and per cell and side [nc][4] the
   neighbour index (-1 at a boundary, the cell itself across a one-cell periodic
   direction), outward unit normal nx, ny, face length S and least-squares gradient
   weights ax, ay of that neighbour (Eq. 15). */
idugks_status idugks_describe(const idugks_config *cfg, double *xi, double *eta, double *w,
                              double *dt, double *area, int32_t *nb, double *nx, double *ny,
                              double *S, double *ax, double *ay);

/* Bytes of device workspace a configuration needs (Section 2 problem size).
   cfg: host; bytes: host output. */
idugks_status idugks_workspace_size(const idugks_config *cfg, size_t *bytes);

/* Builds the mesh geometry, velocity set (Gauss-Hermite or Newton-Cotes, Section 2.2),
   boundary distributions (Section 2.3) and the initial uniform equilibrium (Eq. 2) in
   the workspace.  d_workspace: device, >= idugks_workspace_size() bytes, caller-owned and
   alive until idugks_destroy; hip_stream: hipStream_t (NULL for the default stream). */
idugks_status idugks_init(const idugks_config *cfg, void *d_workspace, size_t bytes,
                          void *hip_stream, idugks_ctx **out);

/* Largest workspace idugks_init_noalloc can hold: the size of the library's static scratch
   array, which every GPU the library is loaded on holds until the process ends. */
#define IDUGKS_NOALLOC_MAX_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code that runs under HIP graph capture,
   tight serving loops, harnesses that forbid allocation): idugks_init with the workspace
   taken from the library's static scratch array on the current device instead of a caller
   buffer; no device memory is allocated or freed.  The array is cleared (by a kernel on
   hip_stream) before use, so nothing of an earlier context carries over.  One such context
   may live per device at a time: a second call before idugks_destroy of the first returns
   IDUGKS_E_STATE (contexts sharing the array would overwrite each other's state).
   Configurations whose idugks_workspace_size exceeds IDUGKS_NOALLOC_MAX_BYTES return
   IDUGKS_E_NOMEM before any device work.  All other calls work on the context as usual. */
idugks_status idugks_init_noalloc(const idugks_config *cfg, void *hip_stream, idugks_ctx **out);

/* Sizes and scalars of a context: cell, velocity (Section 2.2, last paragraph) and face
   counts, the physical time step of Eq. 21 and the reference mass that the closed-domain
   rescale holds (Section 2.3).  out: host. */
idugks_status idugks_get_info(idugks_ctx *ctx, idugks_info *out);

/* The discrete velocity set: xi, eta, weights (weight function included).  host, nv each. */
idugks_status idugks_velocities(idugks_ctx *ctx, double *xi, double *eta, double *w);

/* nsteps explicit DUGKS steps (Eq. 21) or implicit DUGKS iterations (Eq. 22-35).
   res_out (host, may be NULL): relative L2 change of the cell densities in the last step;
   reading it waits for the stream. */
idugks_status idugks_step(idugks_ctx *ctx, int32_t mode, int32_t nsteps, double *res_out);

/* Implicit iterations until res < tol or max_iter.  iters, res_out: host (may be NULL).
   Returns IDUGKS_E_NOT_CONVERGED at the iteration limit, IDUGKS_E_DIVERGED on a
   non-physical state or, with diverge_iters > 0, when the residual has grown in that many
   consecutive iterations (iters and res_out then give the iteration it stopped at). */
idugks_status idugks_solve(idugks_ctx *ctx, double tol, int32_t max_iter, int32_t *iters,
                           double *res_out);

/* RMS over cells of the macroscopic residual M_W / cell area (Eq. 27) of the current
   state, per conserved variable (rho, rho U, rho V, rho E).  out_l2: host [4]. */
idugks_status idugks_residual(idugks_ctx *ctx, double out_l2[4]);

/* Cell fields [nc][8]: rho, U, V, T, p, qx, qy, tau (Eq. 4; q is the physical heat flux). */
idugks_status idugks_moments(idugks_ctx *ctx, double *out, int32_t out_on_host);

/* Interface flux sum M_i(v) of the current state (Eq. 11-19, Eq. 23), FP64 [2][nc][nv]. */
idugks_status idugks_flux(idugks_ctx *ctx, double *M, int32_t on_host);

/* Moments (rho, rho U, rho V, rho E) of phi-bar at every face [nf][4] and the density of
   the reflected wall Maxwellian [nf] (0 off walls) for the current state (the interface
   equilibrium is built from these moments, Section 2.1).  Faces are numbered i-faces
   first, (i, j) -> j*(ni+1) + i, then j-faces, (i, j) -> (ni+1)*nj + j*ni + i; entries of
   faces that a periodic direction merges away are zero. */
idugks_status idugks_face_moments(idugks_ctx *ctx, double *Wf, double *rho_w, int32_t on_host);

/* Macroscopic residual M_W [nc][4] of the current state (Eq. 27). */
idugks_status idugks_macro_residual(idugks_ctx *ctx, double *MW, int32_t on_host);

/* Predicted macroscopic state W* [nc][4] and implicit time step [nc] (Eq. 28-31). */
idugks_status idugks_predict(idugks_ctx *ctx, double *Wstar, double *dt_imp, int32_t on_host);

/* Canonical FP64 state [2][nc][nv]: the transformed distributions G~, H~ of Eq. 10 (the
   solver's unknowns, Eq. 21-22) per cell and discrete velocity, G~ first; f: host if
   on_host, else device.  set_state makes the set state the closed-domain reference mass
   and restarts the iteration counter; the FP32-mixed form rounds it to FP32. */
idugks_status idugks_get_state(idugks_ctx *ctx, double *f, int32_t on_host);
idugks_status idugks_set_state(idugks_ctx *ctx, const double *f, int32_t on_host);

/* Sensitivities (BGK, no limiter, FP64 form; IDUGKS_E_INVALID otherwise).
   The steady residual is R(f; theta) = M(f) - (2 Omega/(2 tau + dt)) (phi~ - phi_eq) per cell
   and velocity (Eq. 11-23 in the implicit scheme's form; Eq. 21 and Eq. 22 share its zero),
   with theta = (tangential speed of the j+ wall, temperature of every wall (one common value),
   Kn).  Objectives, from the Eq. 18 wall-face distributions phi_k (n_k out of the gas):
     0: sum over j+ wall faces of S_k sum_v w xi_x (xi.n_k) G_k          (lid x-momentum flux)
     1: sum over wall faces of S_k sum_v w (xi.n_k) (|xi - U_w|^2 G_k + H_k)/2  (heat flux)
   Arrays lam, f_bar, dJ_df use the canonical FP64 layout [2][nc][nv], device memory unless
   on_host; theta-sized arrays are host memory. */

/* f_bar = lam^T dR/df, theta_bar = lam^T dR/dtheta at the current state. */
idugks_status idugks_vjp(idugks_ctx *ctx, const double *lam, double *f_bar, double theta_bar[3],
                         int32_t on_host);

/* Objective J, dJ/df and dJ/dtheta at fixed f, at the current state (any may be NULL). */
idugks_status idugks_objective(idugks_ctx *ctx, int32_t objective, double *J, double *dJ_df,
                               double dJ_dtheta[3], int32_t on_host);

/* Steady sensitivity of a closed domain at the current (converged) state: solves
   A^T lam + mu l_M = dJ/df (A = dR/df, l_M the total-mass functional) by the transposed
   micro LU-SGS iteration (Eq. 26, transposed) and returns grad = dJ/dtheta = dJ/dtheta|_f -
   lam^T dR/dtheta, J, the iteration count and the relative change of the last iteration.
   lam (may be NULL) receives the multipliers, defined up to multiples of w on G.  Returns
   IDUGKS_E_NOT_CONVERGED at the iteration limit (outputs hold the last iterate). */
idugks_status idugks_adjoint(idugks_ctx *ctx, int32_t objective, double tol, int32_t max_iter,
                             double *J, double grad[3], int32_t *iters, double *res, double *lam,
                             int32_t on_host);

/* Kernel timing: runs nsteps steps of `mode` recording a HIP event pair around every
   kernel launch on the context's stream (no waits between launches), then waits once;
   ms (host, [nk]) receives the summed milliseconds per kernel and counts (host, [nk], may
   be NULL) the launch counts, in the order of idugks_kernel_name(k), k < idugks_num_kernels(). */
int32_t idugks_num_kernels(void);
const char *idugks_kernel_name(int32_t k);
idugks_status idugks_profile(idugks_ctx *ctx, int32_t mode, int32_t nsteps, double *ms,
                             int64_t *counts);

/* As idugks_profile, but events bracket only the kernels k with bit k of kernel_mask set
   (each event pair adds a few microseconds to a step; the others run as in idugks_step). */
idugks_status idugks_profile_mask(idugks_ctx *ctx, int32_t mode, int32_t nsteps, uint32_t kernel_mask,
                                  double *ms, int64_t *counts);

/* Thread-local message of the last failure. */
const char *idugks_last_error(void);

/* Releases host resources (the workspace stays the caller's).  NULL-safe. */
void idugks_destroy(idugks_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif
