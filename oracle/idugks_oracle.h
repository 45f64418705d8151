/*
 * CPU FP64 reference ("oracle") for explicit DUGKS and the implicit DUGKS (IDUGKS)
 * of Pan, Zhong & Zhuo, "An implicit discrete unified gas-kinetic scheme for
 * simulations of steady flow in all flow regimes" (arXiv:1709.01819).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the GPU library and must never be used as a fallback for it.
 *
 * Conventions (shared with the GPU library as an interface, not as code):
 *   - structured quadrilateral mesh, ni x nj cells, cell (i,j) -> c = i + j*ni;
 *     node (i,j) -> i + j*(ni+1);
 *   - boundary sides ordered i-, i+, j-, j+;
 *   - tensor-product discrete velocities, v = ix*nvy + iy;
 *   - state arrays [2][nc][nv]: species 0 is G~, species 1 is H~ (Eq. 5, Eq. 10);
 *   - units: R = 1/2, so T = 2RT and the reference Maxwellian is exp(-|xi|^2)/pi.
 */
#ifndef IDUGKS_ORACLE_H
#define IDUGKS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t ni, nj;
    const double *xn, *yn;          /* (ni+1)*(nj+1) node coordinates, read during create only */
    int32_t bc[4];                  /* 0 wall, 1 far field, 2 periodic; sides i-, i+, j-, j+ */
    double wall_u[4], wall_v[4], wall_T[4];
    double far_rho, far_u, far_v, far_T;
    int32_t quad, nvx, nvy;         /* 0 Gauss-Hermite, 1 Newton-Cotes on [-vmax, vmax] */
    double vmax;
    int32_t model;                  /* 0 BGK, 1 Shakhov (Eq. 20) */
    double Kn, Pr, omega;           /* Eq. 37 Knudsen number, Prandtl number, mu ~ T^omega */
    int32_t K;                      /* internal degrees of freedom (Eq. 2) */
    double cfl_phys, cfl_imp;       /* physical (flux) and implicit (pseudo-time) CFL numbers */
    int32_t limiter;                /* 0 none, 1 Venkatakrishnan (Eq. 16-17) */
    double init_rho, init_u, init_v, init_T;
    int32_t predictor;              /* 0 LU-SGS, 1 point relaxation (both named in Section 4) */
    int32_t relax_sweeps;           /* point relaxation: Jacobi sweeps after the diagonal step */
    /* start-up ramp of the implicit CFL (not in the paper): with cfl_start > 0, implicit
       iteration n (counted from creation) uses min(cfl_imp, cfl_start cfl_growth^n);
       cfl_start = 0 keeps cfl_imp throughout */
    double cfl_start, cfl_growth;
} orc_config;

/* Unstructured mesh of quadrilaterals and triangles.  cell_nodes [ncells][4]: node indices
   counter-clockwise, -1 in the fourth slot of a triangle; side s of a cell is the edge from
   node s to the next.  side_tag [ncells][4]: for a side on the boundary, which of the four
   boundary conditions of the configuration (bc, wall_*, far_*) applies, 0..3; ignored
   elsewhere.  The sweeps take the cells in index order. */
typedef struct {
    int32_t nnodes;
    const double *xn, *yn;
    int32_t ncells;
    const int32_t *cell_nodes;
    const int32_t *side_tag;
} orc_mesh;

typedef struct orc_problem orc_problem;

/* Return codes. */
enum { ORC_OK = 0, ORC_INVALID = 1, ORC_NOMEM = 2, ORC_DIVERGED = 4, ORC_NOT_CONVERGED = 5 };

int orc_create(const orc_config *cfg, orc_problem **out);
/* as orc_create on an unstructured mesh (the structured fields ni, nj, xn, yn are ignored;
   no periodic sides) */
int orc_create_mesh(const orc_config *cfg, const orc_mesh *mesh, orc_problem **out);
void orc_destroy(orc_problem *p);
const char *orc_last_error(void);

/* nc, nv, nf, number of wall faces */
void orc_sizes(const orc_problem *p, int32_t out[4]);
double orc_dt(const orc_problem *p);
/* 1D rule used by the velocity set: nodes and total weights (weight function included) */
int orc_quadrature_1d(int32_t quad, int32_t n, double vmax, double *x, double *w);
void orc_velocities(const orc_problem *p, double *xi, double *eta, double *w);
/* per cell: area, centroid x, centroid y */
void orc_cells(const orc_problem *p, double *area, double *xc, double *yc);
/* per cell and side (4): neighbour index (-1 boundary), outward normal x/y, face length,
   face-midpoint offset x/y from the centroid, least-squares weights x/y */
void orc_cell_sides(const orc_problem *p, int32_t *nb, double *nx, double *ny, double *S,
                    double *dx, double *dy, double *ax, double *ay);

void orc_get_state(const orc_problem *p, double *f);
/* Sets the state; the closed-domain reference mass becomes that of f, the lagged wall
   increments are cleared and the iteration counter restarts. */
void orc_set_state(orc_problem *p, const double *f);

/* Equilibrium (G, H) whose discrete conserved moments equal W (rho, rhoU, rhoV, rhoE);
   q is the heat flux used by the Shakhov correction (ignored for BGK). */
void orc_equilibrium(const orc_problem *p, const double W[4], const double q[2], double *G,
                     double *H);
/* Conserved moments of a pair (G, H) on the velocity set. */
void orc_moments_of(const orc_problem *p, const double *G, const double *H, double W[4]);
/* Heat flux of a pair (G, H) about the bulk velocity of its own moments. */
void orc_heat_flux_of(const orc_problem *p, const double *G, const double *H, double q[2]);

/* [nc][8]: rho, U, V, T, p, qx, qy, tau of the current state (q: Shakhov physical heat flux) */
void orc_moments(const orc_problem *p, double *out);
/* phi-bar-plus of the current state, [2][nc][nv] */
void orc_barplus(orc_problem *p, double *out);
/* interface flux sum M_i(v) of the current state, [2][nc][nv] (Eq. 23) */
int orc_flux(orc_problem *p, double *M);
/* face moments [nf][4] and wall densities [nf] (0 elsewhere) of the current state */
int orc_face_moments(orc_problem *p, double *Wf, double *rho_w);
/* macroscopic residual M_W [nc][4] (Eq. 27) */
int orc_macro_residual(orc_problem *p, double *MW);
/* predicted macroscopic state W* [nc][4] and implicit time step [nc] (Eq. 28-31) */
int orc_predict(orc_problem *p, double *Wstar, double *dt_imp);
/* after orc_predict: for velocity v, the micro diagonal D [nc] and the couplings
   C [nc][4] (coefficient of the side-s neighbour, 0 if none) of Eq. 26 */
int orc_micro_operator(orc_problem *p, int32_t v, double *D, double *C);
/* after orc_predict: applies the LU-SGS lower+upper sweeps for velocity v to rhs [nc] */
int orc_micro_sweep(orc_problem *p, int32_t v, const double *rhs, double *out);

/* nsteps of explicit DUGKS (Eq. 21) or implicit DUGKS; res = density increment norm */
int orc_explicit_step(orc_problem *p, int32_t nsteps, double *res);
int orc_implicit_step(orc_problem *p, int32_t nsteps, double *res);
int orc_solve(orc_problem *p, double tol, int32_t max_iter, int32_t *iters, double *res);
/* RMS over cells of M_W / area for each conserved variable */
int orc_residual(orc_problem *p, double out[4]);

/* Intermediate quantities, for the pins of individual steps: */
/* limited least-squares gradient of phi-bar-plus of the current state, [2][nc][nv] each */
int orc_gradients(orc_problem *p, double *sx, double *sy);
/* least-squares gradient (Eq. 15) of an arbitrary cell field phi [nc], limited by Eq. 16-17
   when limiter != 0 */
int orc_lsq_gradient(const orc_problem *p, const double *phi, int32_t limiter, double *gx, double *gy);
/* faces [nf]: cells L, R (-1 at a boundary), type (0 interior, 1 self-periodic, 2 wall,
   3 far field), boundary side (-1 inside), unit normal from L to R (outward at a boundary),
   length, midpoint in L's frame */
void orc_faces(const orc_problem *p, int32_t *L, int32_t *R, int32_t *type, int32_t *side,
               double *nx, double *ny, double *S, double *mx, double *my);
/* face fluxes S (xi.n) phi_k [2][nf][nv] of the current state (Eq. 18-19) */
int orc_face_flux(orc_problem *p, double *F);
/* the macroscopic LU-SGS (Eq. 29-31) of the current state applied to the right-hand side
   rhs [nc][4] in place of M_W; dW [nc][4] */
int orc_macro_sweep_rhs(orc_problem *p, const double *rhs, double *dW);
/* one implicit iteration that also returns the forward-sweep increment [2][nc][nv] and the
   wall ghost density increments [nf] formed from it (Eq. 35) */
int orc_implicit_detail(orc_problem *p, double *delta_star, double *drho, double *res);

/* analysis switch: first_order != 0 drops the gradient from the reconstruction (the
   first-order upwind residual) */
void orc_set_first_order(orc_problem *p, int32_t first_order);

#ifdef __cplusplus
}
#endif

#endif
