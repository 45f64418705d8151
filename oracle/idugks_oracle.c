/*
 * CPU FP64 reference ("oracle") of explicit DUGKS and implicit DUGKS (IDUGKS).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline of the benchmark; never by the product path.  Plain loops in the
 * order the paper states the method; the only parallelism is OpenMP over
 * independent cells or velocities, so results do not depend on the thread count.
 *
 * Paper: Pan, Zhong & Zhuo, arXiv:1709.01819.  Section 2.1 (Eq. 1-20) is the
 * explicit DUGKS, Section 2.2 (Eq. 21-32) the implicit scheme, Section 2.3
 * (Eq. 33-35) the boundary conditions.  Where the paper is silent or garbled the
 * readings below are used (each one is listed in the design notes):
 *   - Q is scaled by the cell area: Q = -(2 Omega/(2 tau + dt)) (phi~ - phi_eq), the form
 *     that follows from Eq. 10 and Eq. 21 and is the diagonal of Eq. 26;
 *   - phi-bar-plus from phi~: ((2tau-h)/(2tau+dt)) phi~ + (3h/(2tau+dt)) phi_eq, h = dt/2
 *     (Eq. 10 and Eq. 12 combined);
 *   - the reconstruction of Eq. 13-14 is taken in the upwind cell of each face;
 *   - a global physical dt (cfl_phys) sets the flux; a local dt_imp (cfl_imp) only the
 *     pseudo-time diagonal of Eq. 26 and Eq. 30;
 *   - equilibria are Maxwellians corrected so their discrete conserved moments are
 *     exact (Gram system over the velocity set);
 *   - Shakhov (Eq. 20) in its monatomic reduced form (K = 1), heat flux of the
 *     transformed distributions rescaled by 2tau/(2tau + dt Pr) (cells) and
 *     2tau/(2tau + h Pr) (faces);
 *   - macro LU-SGS (Eq. 29-31): Rusanov split with lambda = |U.n| + sqrt(gamma RT), one
 *     half of the spectral sum on the diagonal, matrix-free flux differences; the
 *     macroscopic ghost increment is zero at far-field faces and the mirror image of the
 *     inner increment at walls (Eq. 33), which puts a wall face's whole lambda S on the
 *     diagonal;
 *   - micro LU-SGS: the forward sweep starts with zero ghost increments, the wall ghost
 *     density increment of Eq. 35 is then formed from the forward-sweep increments of
 *     the wall cell and enters the backward sweep;
 *   - closed domains are rescaled to their initial mass after each implicit step;
 *   - Res = ||rho^{n+1} - rho^n||_2 / ||rho^{n+1}||_2 over cells;
 *   - an optional start-up ramp of the implicit CFL, min(cfl_imp, cfl_start g^n) at
 *     implicit iteration n (the paper starts at its final CFL and gives no ramp).
 */
#include "idugks_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum { F_INTERIOR = 0, F_SELF = 1, F_WALL = 2, F_FAR = 3 };
enum { BC_WALL = 0, BC_FAR = 1, BC_PERIODIC = 2 };

/* Normal particle speed xi.n at a face.  The upwind side is undefined for velocities
   tangent to the face; a velocity whose normal speed is below 1e-12 of its speed counts as
   tangent (normal speed exactly 0), so that the tie rules below do not depend on the
   rounding of face normals. */
static double normal_speed(double x, double y, double nx, double ny)
{
    double un = x * nx + y * ny;
    return fabs(un) <= 1e-12 * (fabs(x) + fabs(y)) ? 0.0 : un;
}

static _Thread_local char g_err[512];

static int fail(int code, const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

const char *orc_last_error(void) { return g_err; }

struct orc_problem {
    int ni, nj, nc, nf, nv, nvx, nvy, nwall;
    /* velocity set, v = ix*nvy + iy */
    double *xi, *eta, *w;
    /* cells */
    double *area, *xc, *yc;
    int *cf;              /* [nc][4] face on side s */
    int *nb;              /* [nc][4] neighbour across side s, -1 at a boundary */
    double *nbdx, *nbdy;  /* [nc][4] neighbour image centroid minus own centroid */
    double *fdx, *fdy;    /* [nc][4] face midpoint (own frame) minus own centroid */
    double *onx, *ony;    /* [nc][4] outward unit normal of side s */
    double *sS;           /* [nc][4] face length of side s */
    double *ax, *ay;      /* [nc][4] least-squares weights (Eq. 15) */
    double *sgn;          /* [nc][4] +1 if the cell is the L end of the side's face, -1 if R */
    /* faces */
    int *fL, *fR, *ftype, *fside;
    double *fnx, *fny, *fS;      /* unit normal from L to R (outward for boundary faces) */
    double *fmx, *fmy;           /* midpoint in L's frame */
    double *fshx, *fshy;         /* periodic shift: R's frame = L's frame - shift */
    /* gas */
    int model, K, limiter, closed, predictor, relax_sweeps;
    double Kn, Pr, omega, mu_ref, dt, h, cfl_imp, cfl_start, cfl_growth;
    long imp_iters;              /* implicit iterations done (the CFL ramp's n) */
    double wall_u[4], wall_v[4], wall_RT[4];
    double *gw;                  /* [4][nv] G of the wall Maxwellian at unit density */
    double *ginf, *hinf;         /* [nv] free-stream equilibrium */
    double *wden;                /* [nf] sum over incoming v of w (xi.n) gw, wall faces */
    /* state */
    double *f;                   /* [2][nc][nv] */
    double M0;
    double *drho_g;              /* [nf] ghost density increment of wall faces (Eq. 35) */
    /* work */
    double *W, *RT, *tau, *q;    /* cell records */
    double *feq, *bp, *sx, *sy;  /* [2][nc][nv] */
    double *F;                   /* [2][nf][nv] face flux S (xi.n) phi_k */
    double *Wf, *rhow;           /* [nf][4], [nf] */
    double *M;                   /* [2][nc][nv] */
    double *MW, *dW, *Wst, *dtimp, *DW, *RTst, *taust;
    double *feqst;               /* [2][nc][nv] */
    double *delta;               /* [2][nc][nv] */
    int predicted;
    /* optional captures of one implicit iteration (tests): the forward-sweep increment
       [2][nc][nv] and the wall ghost density increments [nf] */
    double *cap_dstar, *cap_drho;
    int first_order;             /* analysis switch: no gradient in the reconstruction */
};

/* ------------------------------------------------------------------------- */
/* Small dense solve (Gaussian elimination with partial pivoting).            */
/* ------------------------------------------------------------------------- */
static int solve_dense(int n, double *A, double *b)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[r * n + k]) > fabs(A[piv * n + k])) piv = r;
        if (A[piv * n + k] == 0.0) return 1;
        if (piv != k) {
            for (int c = 0; c < n; ++c) {
                double t = A[k * n + c];
                A[k * n + c] = A[piv * n + c];
                A[piv * n + c] = t;
            }
            double t = b[k];
            b[k] = b[piv];
            b[piv] = t;
        }
        for (int r = k + 1; r < n; ++r) {
            double m = A[r * n + k] / A[k * n + k];
            for (int c = k; c < n; ++c) A[r * n + c] -= m * A[k * n + c];
            b[r] -= m * b[k];
        }
    }
    for (int k = n - 1; k >= 0; --k) {
        double s = b[k];
        for (int c = k + 1; c < n; ++c) s -= A[k * n + c] * b[c];
        b[k] = s / A[k * n + k];
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Velocity quadrature (Section 2.2, last paragraph: Gauss-Hermite or          */
/* Newton-Cotes in each velocity direction; the internal variable stays        */
/* continuous).  Weights returned here integrate g(x) dx directly, i.e. the    */
/* Gauss-Hermite weights already carry the factor exp(x^2).                    */
/* ------------------------------------------------------------------------- */

/* Orthonormal Hermite functions psi_k(x) = H_k(x) exp(-x^2/2) / sqrt(2^k k! sqrt(pi));
   returns psi_n(x) and sum_{k<n} psi_k(x)^2. */
static double hermite_function(int n, double x, double *sumsq)
{
    double pm = 0.0, pc = pow(M_PI, -0.25) * exp(-0.5 * x * x), s = 0.0;
    for (int k = 0; k < n; ++k) {
        s += pc * pc;
        double pn = x * sqrt(2.0 / (k + 1)) * pc - sqrt((double)k / (k + 1)) * pm;
        pm = pc;
        pc = pn;
    }
    if (sumsq) *sumsq = s;
    return pc;
}

static int gauss_hermite(int n, double *x, double *wt)
{
    /* all n roots of psi_n lie in (-sqrt(2n+1), sqrt(2n+1)); bracket every sign change
       on a fine grid and bisect to full precision */
    double lim = sqrt(2.0 * n + 1.0) + 0.5, step = 1e-3;
    int found = 0;
    double xa = -lim, fa = hermite_function(n, xa, NULL);
    while (xa < lim && found < n) {
        double xb = xa + step, fb = hermite_function(n, xb, NULL);
        if (fa == 0.0) {
            x[found++] = xa;
        } else if (fa * fb < 0.0) {
            double lo = xa, hi = xb, flo = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                double fm = hermite_function(n, mid, NULL);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0) == (flo < 0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            x[found++] = 0.5 * (lo + hi);
        }
        xa = xb;
        fa = fb;
    }
    if (found != n) return 1;
    /* symmetrise (the roots are symmetric about 0) */
    for (int i = 0; i < n / 2; ++i) {
        double a = 0.5 * (x[n - 1 - i] - x[i]);
        x[i] = -a;
        x[n - 1 - i] = a;
    }
    if (n % 2) x[n / 2] = 0.0;
    /* Christoffel numbers: w_i exp(x_i^2) = 1 / sum_{k<n} psi_k(x_i)^2 */
    for (int i = 0; i < n; ++i) {
        double s;
        hermite_function(n, x[i], &s);
        wt[i] = 1.0 / s;
    }
    return 0;
}

static int newton_cotes(int n, double vmax, double *x, double *wt)
{
    if (n < 2 || !(vmax > 0)) return 1;
    int m = n - 1;
    double dx = 2.0 * vmax / m;
    for (int i = 0; i < n; ++i) x[i] = -vmax + i * dx;
    for (int i = 0; i < n; ++i) wt[i] = 0.0;
    if (m % 4 == 0) {          /* composite Boole */
        static const double c[5] = {7, 32, 12, 32, 7};
        for (int p = 0; p < m; p += 4)
            for (int k = 0; k < 5; ++k) wt[p + k] += 2.0 * dx / 45.0 * c[k];
    } else if (m % 3 == 0) {   /* composite Simpson 3/8 */
        static const double c[4] = {1, 3, 3, 1};
        for (int p = 0; p < m; p += 3)
            for (int k = 0; k < 4; ++k) wt[p + k] += 3.0 * dx / 8.0 * c[k];
    } else if (m % 2 == 0) {   /* composite Simpson */
        static const double c[3] = {1, 4, 1};
        for (int p = 0; p < m; p += 2)
            for (int k = 0; k < 3; ++k) wt[p + k] += dx / 3.0 * c[k];
    } else {                   /* composite trapezoid */
        for (int p = 0; p < m; ++p) {
            wt[p] += 0.5 * dx;
            wt[p + 1] += 0.5 * dx;
        }
    }
    return 0;
}

int orc_quadrature_1d(int32_t quad, int32_t n, double vmax, double *x, double *w)
{
    if (n < 2) return fail(ORC_INVALID, "need at least 2 velocity points per direction");
    if (quad == 0) return gauss_hermite(n, x, w) ? fail(ORC_INVALID, "Gauss-Hermite failed") : 0;
    if (quad == 1) return newton_cotes(n, vmax, x, w) ? fail(ORC_INVALID, "bad Newton-Cotes") : 0;
    return fail(ORC_INVALID, "unknown quadrature");
}

/* ------------------------------------------------------------------------- */
/* Gas model: moments (Eq. 4 with Eq. 5), equilibrium (Eq. 2, Eq. 20), tau.    */
/* ------------------------------------------------------------------------- */
static void moments(const orc_problem *p, const double *G, const double *H, double W[4])
{
    double m0 = 0, m1 = 0, m2 = 0, m3 = 0;
    for (int v = 0; v < p->nv; ++v) {
        double wv = p->w[v], x = p->xi[v], y = p->eta[v];
        m0 += wv * G[v];
        m1 += wv * x * G[v];
        m2 += wv * y * G[v];
        m3 += wv * 0.5 * ((x * x + y * y) * G[v] + H[v]);
    }
    W[0] = m0;
    W[1] = m1;
    W[2] = m2;
    W[3] = m3;
}

/* RT from rho E = rho(|U|^2 + (K+2) RT)/2 (Eq. 4, with 1/(2 lambda) = RT) */
static double rt_of(const double W[4], int K)
{
    double U = W[1] / W[0], V = W[2] / W[0];
    return (2.0 * W[3] / W[0] - U * U - V * V) / (K + 2);
}

/* tau = mu/p, mu = mu_ref (T/T_ref)^omega with mu_ref from Eq. 37 (rho = L = 2RT_ref = 1) */
static double tau_of(const orc_problem *p, double rho, double RT)
{
    return p->mu_ref * pow(2.0 * RT, p->omega) / (rho * RT);
}

/* q = sum_v w c (|c|^2 G + H)/2, c = xi - U */
static void heat_flux(const orc_problem *p, const double *G, const double *H, const double W[4],
                      double q[2])
{
    double U = W[1] / W[0], V = W[2] / W[0], qx = 0, qy = 0;
    for (int v = 0; v < p->nv; ++v) {
        double cx = p->xi[v] - U, cy = p->eta[v] - V;
        double e = 0.5 * ((cx * cx + cy * cy) * G[v] + H[v]);
        qx += p->w[v] * cx * e;
        qy += p->w[v] * cy * e;
    }
    q[0] = qx;
    q[1] = qy;
}

/* Equilibrium with exact discrete conserved moments W.
 * G_M = rho (lambda/pi) exp(-lambda |xi - U|^2) (Eq. 2 integrated over the internal
 * variable, Eq. 5), H_M = K RT G_M.  With psi = (1, xi, eta, |xi|^2/2 + K RT/2) the
 * corrected pair is G = G_M (1 + beta.psi), H = K RT G, where A beta = W - sum w psi G_M
 * and A = sum w psi psi^T G_M.  Shakhov (Eq. 20, monatomic reduced form):
 * dG = k (c.q)(|c|^2/RT - 4) G_M, dH = k (c.q) K (|c|^2/RT - 2) RT G_M,
 * k = (1 - Pr)/(5 p RT), with its conserved moments projected out by the same A. */
static void equilibrium(const orc_problem *p, const double W[4], const double q[2], double *G,
                        double *H)
{
    const int nv = p->nv, K = p->K;
    double rho = W[0], U = W[1] / rho, V = W[2] / rho, RT = rt_of(W, K), lam = 0.5 / RT;
    double e0 = 0.5 * K * RT;
    double A[16] = {0}, r[4] = {W[0], W[1], W[2], W[3]};
    for (int v = 0; v < nv; ++v) {
        double x = p->xi[v], y = p->eta[v];
        double c2 = (x - U) * (x - U) + (y - V) * (y - V);
        double gm = rho * lam / M_PI * exp(-lam * c2);
        G[v] = gm;
        double ps[4] = {1.0, x, y, 0.5 * (x * x + y * y) + e0};
        for (int a = 0; a < 4; ++a) {
            r[a] -= p->w[v] * ps[a] * gm;
            for (int b = 0; b < 4; ++b) A[a * 4 + b] += p->w[v] * ps[a] * ps[b] * gm;
        }
    }
    double A2[16];
    memcpy(A2, A, sizeof A);
    solve_dense(4, A2, r); /* r <- beta */
    double gam[4] = {0, 0, 0, 0};
    int shakhov = (p->model == 1) && (q[0] != 0.0 || q[1] != 0.0);
    double kap = (1.0 - p->Pr) / (5.0 * rho * RT * RT);
    if (shakhov) {
        for (int v = 0; v < nv; ++v) {
            double x = p->xi[v], y = p->eta[v], cx = x - U, cy = y - V, c2 = cx * cx + cy * cy;
            double cq = cx * q[0] + cy * q[1];
            double dg = kap * cq * (c2 / RT - 4.0) * G[v];
            double dh = kap * cq * K * (c2 / RT - 2.0) * RT * G[v];
            gam[0] += p->w[v] * dg;
            gam[1] += p->w[v] * x * dg;
            gam[2] += p->w[v] * y * dg;
            gam[3] += p->w[v] * 0.5 * ((x * x + y * y) * dg + dh);
        }
        memcpy(A2, A, sizeof A);
        solve_dense(4, A2, gam);
    }
    for (int v = 0; v < nv; ++v) {
        double x = p->xi[v], y = p->eta[v], gm = G[v];
        double ps[4] = {1.0, x, y, 0.5 * (x * x + y * y) + e0};
        double corr = 1.0;
        for (int a = 0; a < 4; ++a) corr += (r[a] - gam[a]) * ps[a];
        double g = gm * corr, hh = K * RT * gm * corr;
        if (shakhov) {
            double cx = x - U, cy = y - V, c2 = cx * cx + cy * cy;
            double cq = cx * q[0] + cy * q[1];
            g += kap * cq * (c2 / RT - 4.0) * gm;
            hh += kap * cq * K * (c2 / RT - 2.0) * RT * gm;
        }
        G[v] = g;
        H[v] = hh;
    }
}

void orc_equilibrium(const orc_problem *p, const double W[4], const double q[2], double *G,
                     double *H)
{
    equilibrium(p, W, q, G, H);
}

void orc_moments_of(const orc_problem *p, const double *G, const double *H, double W[4])
{
    moments(p, G, H, W);
}

void orc_heat_flux_of(const orc_problem *p, const double *G, const double *H, double q[2])
{
    double W[4];
    moments(p, G, H, W);
    heat_flux(p, G, H, W, q);
}

/* ------------------------------------------------------------------------- */
/* Mesh (Fig. 1: cells adjacent through faces are the reconstruction stencil) */
/* ------------------------------------------------------------------------- */
#define NODE(i, j) ((i) + (j) * (ni + 1))
#define CELL(i, j) ((i) + (j) * ni)

static int build_mesh(orc_problem *p, const orc_config *cfg)
{
    const int ni = cfg->ni, nj = cfg->nj, nc = ni * nj;
    const double *xn = cfg->xn, *yn = cfg->yn;
    p->ni = ni;
    p->nj = nj;
    p->nc = nc;
    p->area = calloc(nc, sizeof(double));
    p->xc = calloc(nc, sizeof(double));
    p->yc = calloc(nc, sizeof(double));
    /* cells: shoelace area and area centroid of the quadrilateral */
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            int idx[4] = {NODE(i, j), NODE(i + 1, j), NODE(i + 1, j + 1), NODE(i, j + 1)};
            double a = 0, cx = 0, cy = 0;
            for (int k = 0; k < 4; ++k) {
                double x0 = xn[idx[k]], y0 = yn[idx[k]];
                double x1 = xn[idx[(k + 1) % 4]], y1 = yn[idx[(k + 1) % 4]];
                double cr = x0 * y1 - x1 * y0;
                a += cr;
                cx += (x0 + x1) * cr;
                cy += (y0 + y1) * cr;
            }
            a *= 0.5;
            if (!(a > 0)) return fail(ORC_INVALID, "non-positive cell area");
            p->area[CELL(i, j)] = a;
            p->xc[CELL(i, j)] = cx / (6.0 * a);
            p->yc[CELL(i, j)] = cy / (6.0 * a);
        }
    /* faces: i-faces (constant i) then j-faces (constant j) */
    int maxf = (ni + 1) * nj + ni * (nj + 1);
    p->fL = malloc(maxf * sizeof(int));
    p->fR = malloc(maxf * sizeof(int));
    p->ftype = malloc(maxf * sizeof(int));
    p->fside = malloc(maxf * sizeof(int));
    p->fnx = malloc(maxf * sizeof(double));
    p->fny = malloc(maxf * sizeof(double));
    p->fS = malloc(maxf * sizeof(double));
    p->fmx = malloc(maxf * sizeof(double));
    p->fmy = malloc(maxf * sizeof(double));
    p->fshx = calloc(maxf, sizeof(double));
    p->fshy = calloc(maxf, sizeof(double));
    p->cf = malloc(4 * nc * sizeof(int));
    for (int k = 0; k < 4 * nc; ++k) p->cf[k] = -1;
    int nf = 0, nwall = 0;
    const int per_i = cfg->bc[0] == BC_PERIODIC, per_j = cfg->bc[2] == BC_PERIODIC;
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i <= ni; ++i) {
            if (i == 0 && per_i) continue;
            double ax_ = xn[NODE(i, j)], ay_ = yn[NODE(i, j)];
            double bx_ = xn[NODE(i, j + 1)], by_ = yn[NODE(i, j + 1)];
            double tx = bx_ - ax_, ty = by_ - ay_, S = sqrt(tx * tx + ty * ty);
            double nx = ty / S, ny = -tx / S; /* +i direction */
            int k = nf++;
            p->fS[k] = S;
            p->fmx[k] = 0.5 * (ax_ + bx_);
            p->fmy[k] = 0.5 * (ay_ + by_);
            p->fnx[k] = nx;
            p->fny[k] = ny;
            p->fside[k] = -1;
            if (i > 0 && i < ni) {
                p->ftype[k] = F_INTERIOR;
                p->fL[k] = CELL(i - 1, j);
                p->fR[k] = CELL(i, j);
                p->cf[4 * CELL(i - 1, j) + 1] = k;
                p->cf[4 * CELL(i, j) + 0] = k;
            } else if (i == ni && per_i) {
                p->fL[k] = CELL(ni - 1, j);
                p->fR[k] = CELL(0, j);
                p->ftype[k] = (ni == 1) ? F_SELF : F_INTERIOR;
                p->fshx[k] = xn[NODE(ni, j)] - xn[NODE(0, j)];
                p->fshy[k] = yn[NODE(ni, j)] - yn[NODE(0, j)];
                p->cf[4 * CELL(ni - 1, j) + 1] = k;
                p->cf[4 * CELL(0, j) + 0] = k;
            } else {
                int side = (i == 0) ? 0 : 1;
                int c = (i == 0) ? CELL(0, j) : CELL(ni - 1, j);
                if (i == 0) {
                    p->fnx[k] = -nx;
                    p->fny[k] = -ny;
                }
                p->fL[k] = c;
                p->fR[k] = -1;
                p->fside[k] = side;
                p->ftype[k] = cfg->bc[side] == BC_WALL ? F_WALL : F_FAR;
                if (p->ftype[k] == F_WALL) ++nwall;
                p->cf[4 * c + side] = k;
            }
        }
    for (int j = 0; j <= nj; ++j)
        for (int i = 0; i < ni; ++i) {
            if (j == 0 && per_j) continue;
            double ax_ = xn[NODE(i, j)], ay_ = yn[NODE(i, j)];
            double bx_ = xn[NODE(i + 1, j)], by_ = yn[NODE(i + 1, j)];
            double tx = bx_ - ax_, ty = by_ - ay_, S = sqrt(tx * tx + ty * ty);
            double nx = -ty / S, ny = tx / S; /* +j direction */
            int k = nf++;
            p->fS[k] = S;
            p->fmx[k] = 0.5 * (ax_ + bx_);
            p->fmy[k] = 0.5 * (ay_ + by_);
            p->fnx[k] = nx;
            p->fny[k] = ny;
            p->fside[k] = -1;
            if (j > 0 && j < nj) {
                p->ftype[k] = F_INTERIOR;
                p->fL[k] = CELL(i, j - 1);
                p->fR[k] = CELL(i, j);
                p->cf[4 * CELL(i, j - 1) + 3] = k;
                p->cf[4 * CELL(i, j) + 2] = k;
            } else if (j == nj && per_j) {
                p->fL[k] = CELL(i, nj - 1);
                p->fR[k] = CELL(i, 0);
                p->ftype[k] = (nj == 1) ? F_SELF : F_INTERIOR;
                p->fshx[k] = xn[NODE(i, nj)] - xn[NODE(i, 0)];
                p->fshy[k] = yn[NODE(i, nj)] - yn[NODE(i, 0)];
                p->cf[4 * CELL(i, nj - 1) + 3] = k;
                p->cf[4 * CELL(i, 0) + 2] = k;
            } else {
                int side = (j == 0) ? 2 : 3;
                int c = (j == 0) ? CELL(i, 0) : CELL(i, nj - 1);
                if (j == 0) {
                    p->fnx[k] = -nx;
                    p->fny[k] = -ny;
                }
                p->fL[k] = c;
                p->fR[k] = -1;
                p->fside[k] = side;
                p->ftype[k] = cfg->bc[side] == BC_WALL ? F_WALL : F_FAR;
                if (p->ftype[k] == F_WALL) ++nwall;
                p->cf[4 * c + side] = k;
            }
        }
    p->nf = nf;
    p->nwall = nwall;
    /* per cell and side: neighbour, image offsets, outward normal, face offsets */
    p->nb = malloc(4 * nc * sizeof(int));
    p->nbdx = calloc(4 * nc, sizeof(double));
    p->nbdy = calloc(4 * nc, sizeof(double));
    p->fdx = calloc(4 * nc, sizeof(double));
    p->fdy = calloc(4 * nc, sizeof(double));
    p->onx = calloc(4 * nc, sizeof(double));
    p->ony = calloc(4 * nc, sizeof(double));
    p->sS = calloc(4 * nc, sizeof(double));
    p->ax = calloc(4 * nc, sizeof(double));
    p->ay = calloc(4 * nc, sizeof(double));
    p->sgn = calloc(4 * nc, sizeof(double));
    for (int c = 0; c < nc; ++c)
        for (int s = 0; s < 4; ++s) {
            int k = p->cf[4 * c + s], m = 4 * c + s;
            /* which end of the face is this cell?  Sides i+ / j+ are the L end of their
               face, sides i- / j- the R end (a boundary face's only cell is its L end). */
            int isL = (p->fR[k] < 0) || (s == 1 || s == 3);
            double sgn = isL ? 1.0 : -1.0;
            p->sgn[m] = sgn;
            p->onx[m] = sgn * p->fnx[k];
            p->ony[m] = sgn * p->fny[k];
            p->sS[m] = p->fS[k];
            double mx = p->fmx[k] - (isL ? 0.0 : p->fshx[k]);
            double my = p->fmy[k] - (isL ? 0.0 : p->fshy[k]);
            p->fdx[m] = mx - p->xc[c];
            p->fdy[m] = my - p->yc[c];
            if (p->fR[k] < 0) {
                p->nb[m] = -1;
            } else {
                int o = isL ? p->fR[k] : p->fL[k];
                p->nb[m] = o;
                double ox = p->xc[o] + (isL ? p->fshx[k] : -p->fshx[k]);
                double oy = p->yc[o] + (isL ? p->fshy[k] : -p->fshy[k]);
                p->nbdx[m] = ox - p->xc[c];
                p->nbdy[m] = oy - p->yc[c];
            }
        }
    /* least-squares gradient weights (Eq. 15): grad = A^{-1} sum_j d_j (phi_j - phi_0) */
    for (int c = 0; c < nc; ++c) {
        double a11 = 0, a12 = 0, a22 = 0;
        for (int s = 0; s < 4; ++s) {
            int m = 4 * c + s;
            if (p->nb[m] < 0) continue;
            a11 += p->nbdx[m] * p->nbdx[m];
            a12 += p->nbdx[m] * p->nbdy[m];
            a22 += p->nbdy[m] * p->nbdy[m];
        }
        double det = a11 * a22 - a12 * a12;
        if (!(det > 0)) return fail(ORC_INVALID, "degenerate least-squares stencil");
        for (int s = 0; s < 4; ++s) {
            int m = 4 * c + s;
            if (p->nb[m] < 0) continue;
            p->ax[m] = (a22 * p->nbdx[m] - a12 * p->nbdy[m]) / det;
            p->ay[m] = (-a12 * p->nbdx[m] + a11 * p->nbdy[m]) / det;
        }
    }
    return 0;
}

/* Unstructured mesh of quadrilaterals and triangles (nodes counter-clockwise; a triangle
   has -1 as its fourth node).  Side s of a cell is the edge from its node s to the next one;
   a triangle's fourth side is absent and points at one shared zero-length face of the
   self type, which every step skips.  Two cells sharing an edge share a face whose L end
   is the lower-indexed cell; a boundary edge carries the tag (0..3) that selects its
   boundary condition among the four of the configuration. */
typedef struct { int a, b, cell, side; } edge_rec;

static int edge_cmp(const void *x, const void *y)
{
    const edge_rec *e = x, *f = y;
    if (e->a != f->a) return e->a < f->a ? -1 : 1;
    if (e->b != f->b) return e->b < f->b ? -1 : 1;
    if (e->cell != f->cell) return e->cell < f->cell ? -1 : 1;
    return e->side - f->side;
}

static int build_mesh_unstructured(orc_problem *p, const orc_config *cfg, const orc_mesh *m)
{
    const int nc = m->ncells;
    const double *xn = m->xn, *yn = m->yn;
    p->ni = nc;
    p->nj = 1;
    p->nc = nc;
    p->area = calloc(nc, sizeof(double));
    p->xc = calloc(nc, sizeof(double));
    p->yc = calloc(nc, sizeof(double));
    for (int c = 0; c < nc; ++c) {
        const int32_t *cn = m->cell_nodes + 4 * c;
        int nn = cn[3] < 0 ? 3 : 4;
        double a = 0, cx = 0, cy = 0;
        for (int k = 0; k < nn; ++k) {
            int i0 = cn[k], i1 = cn[(k + 1) % nn];
            if (i0 < 0 || i0 >= m->nnodes || i1 < 0 || i1 >= m->nnodes) return fail(ORC_INVALID, "bad node index");
            double x0 = xn[i0], y0 = yn[i0], x1 = xn[i1], y1 = yn[i1], cr = x0 * y1 - x1 * y0;
            a += cr;
            cx += (x0 + x1) * cr;
            cy += (y0 + y1) * cr;
        }
        a *= 0.5;
        if (!(a > 0)) return fail(ORC_INVALID, "non-positive cell area (cells must be counter-clockwise)");
        p->area[c] = a;
        p->xc[c] = cx / (6.0 * a);
        p->yc[c] = cy / (6.0 * a);
    }
    /* pair up the edges */
    edge_rec *e = malloc(4 * (size_t)nc * sizeof(edge_rec));
    int ne = 0;
    for (int c = 0; c < nc; ++c) {
        const int32_t *cn = m->cell_nodes + 4 * c;
        int nn = cn[3] < 0 ? 3 : 4;
        for (int k = 0; k < nn; ++k) {
            int i0 = cn[k], i1 = cn[(k + 1) % nn];
            e[ne].a = i0 < i1 ? i0 : i1;
            e[ne].b = i0 < i1 ? i1 : i0;
            e[ne].cell = c;
            e[ne].side = k;
            ++ne;
        }
    }
    qsort(e, ne, sizeof(edge_rec), edge_cmp);
    int maxf = ne + 1;
    p->fL = malloc(maxf * sizeof(int));
    p->fR = malloc(maxf * sizeof(int));
    p->ftype = malloc(maxf * sizeof(int));
    p->fside = malloc(maxf * sizeof(int));
    p->fnx = malloc(maxf * sizeof(double));
    p->fny = malloc(maxf * sizeof(double));
    p->fS = malloc(maxf * sizeof(double));
    p->fmx = malloc(maxf * sizeof(double));
    p->fmy = malloc(maxf * sizeof(double));
    p->fshx = calloc(maxf, sizeof(double));
    p->fshy = calloc(maxf, sizeof(double));
    p->cf = malloc(4 * nc * sizeof(int));
    p->nb = malloc(4 * nc * sizeof(int));
    p->nbdx = calloc(4 * nc, sizeof(double));
    p->nbdy = calloc(4 * nc, sizeof(double));
    p->fdx = calloc(4 * nc, sizeof(double));
    p->fdy = calloc(4 * nc, sizeof(double));
    p->onx = calloc(4 * nc, sizeof(double));
    p->ony = calloc(4 * nc, sizeof(double));
    p->sS = calloc(4 * nc, sizeof(double));
    p->ax = calloc(4 * nc, sizeof(double));
    p->ay = calloc(4 * nc, sizeof(double));
    p->sgn = calloc(4 * nc, sizeof(double));
    for (int k = 0; k < 4 * nc; ++k) { p->cf[k] = -1; p->nb[k] = -1; }
    int nf = 0, nwall = 0;
    for (int i = 0; i < ne;) {
        int j = i + 1;
        while (j < ne && e[j].a == e[i].a && e[j].b == e[i].b) ++j;
        if (j - i > 2) { free(e); return fail(ORC_INVALID, "an edge shared by more than two cells"); }
        const edge_rec *L = &e[i];  /* lower cell index first (sorted) */
        const int32_t *cn = m->cell_nodes + 4 * L->cell;
        int nn = cn[3] < 0 ? 3 : 4;
        int i0 = cn[L->side], i1 = cn[(L->side + 1) % nn];
        double tx = xn[i1] - xn[i0], ty = yn[i1] - yn[i0], S = sqrt(tx * tx + ty * ty);
        int k = nf++;
        p->fS[k] = S;
        p->fnx[k] = ty / S;  /* outward of the counter-clockwise L cell */
        p->fny[k] = -tx / S;
        p->fmx[k] = 0.5 * (xn[i0] + xn[i1]);
        p->fmy[k] = 0.5 * (yn[i0] + yn[i1]);
        p->fL[k] = L->cell;
        p->cf[4 * L->cell + L->side] = k;
        p->sgn[4 * L->cell + L->side] = 1.0;
        if (j - i == 2) {
            const edge_rec *R = &e[i + 1];
            p->fR[k] = R->cell;
            p->ftype[k] = F_INTERIOR;
            p->fside[k] = -1;
            p->cf[4 * R->cell + R->side] = k;
            p->sgn[4 * R->cell + R->side] = -1.0;
            p->nb[4 * L->cell + L->side] = R->cell;
            p->nb[4 * R->cell + R->side] = L->cell;
        } else {
            int tag = m->side_tag[4 * L->cell + L->side];
            if (tag < 0 || tag > 3) { free(e); return fail(ORC_INVALID, "boundary edge without a tag 0..3"); }
            p->fR[k] = -1;
            p->fside[k] = tag;
            p->ftype[k] = cfg->bc[tag] == BC_WALL ? F_WALL : F_FAR;
            if (p->ftype[k] == F_WALL) ++nwall;
        }
        i = j;
    }
    free(e);
    /* the shared absent side of the triangles */
    int kabs = nf++;
    p->fL[kabs] = p->fR[kabs] = -1;
    p->ftype[kabs] = F_SELF;
    p->fside[kabs] = -1;
    p->fnx[kabs] = p->fny[kabs] = p->fS[kabs] = p->fmx[kabs] = p->fmy[kabs] = 0.0;
    for (int c = 0; c < nc; ++c)
        if (m->cell_nodes[4 * c + 3] < 0) p->cf[4 * c + 3] = kabs;
    p->nf = nf;
    p->nwall = nwall;
    for (int c = 0; c < nc; ++c)
        for (int s = 0; s < 4; ++s) {
            int m4 = 4 * c + s, k = p->cf[m4];
            if (p->ftype[k] == F_SELF) continue;  /* absent side: zero geometry */
            double sg = p->sgn[m4];
            p->onx[m4] = sg * p->fnx[k];
            p->ony[m4] = sg * p->fny[k];
            p->sS[m4] = p->fS[k];
            p->fdx[m4] = p->fmx[k] - p->xc[c];
            p->fdy[m4] = p->fmy[k] - p->yc[c];
            int o = p->nb[m4];
            if (o >= 0) {
                p->nbdx[m4] = p->xc[o] - p->xc[c];
                p->nbdy[m4] = p->yc[o] - p->yc[c];
            }
        }
    for (int c = 0; c < nc; ++c) {
        double a11 = 0, a12 = 0, a22 = 0;
        for (int s = 0; s < 4; ++s) {
            int m4 = 4 * c + s;
            if (p->nb[m4] < 0) continue;
            a11 += p->nbdx[m4] * p->nbdx[m4];
            a12 += p->nbdx[m4] * p->nbdy[m4];
            a22 += p->nbdy[m4] * p->nbdy[m4];
        }
        double det = a11 * a22 - a12 * a12;
        if (!(det > 0)) return fail(ORC_INVALID, "degenerate least-squares stencil");
        for (int s = 0; s < 4; ++s) {
            int m4 = 4 * c + s;
            if (p->nb[m4] < 0) continue;
            p->ax[m4] = (a22 * p->nbdx[m4] - a12 * p->nbdy[m4]) / det;
            p->ay[m4] = (-a12 * p->nbdx[m4] + a11 * p->nbdy[m4]) / det;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Creation                                                                   */
/* ------------------------------------------------------------------------- */
static int validate(const orc_config *c, const orc_mesh *mesh)
{
    if (!c) return fail(ORC_INVALID, "null config");
    if (mesh) {
        if (mesh->nnodes < 3 || mesh->ncells < 1 || !mesh->xn || !mesh->yn || !mesh->cell_nodes ||
            !mesh->side_tag)
            return fail(ORC_INVALID, "incomplete unstructured mesh");
        for (int s = 0; s < 4; ++s)
            if (c->bc[s] == BC_PERIODIC) return fail(ORC_INVALID, "no periodic sides on unstructured meshes");
    } else {
        if (c->ni < 1 || c->nj < 1) return fail(ORC_INVALID, "mesh needs ni, nj >= 1");
        if (!c->xn || !c->yn) return fail(ORC_INVALID, "missing node coordinates");
    }
    if (c->predictor < 0 || c->predictor > 1) return fail(ORC_INVALID, "unknown predictor");
    if (c->relax_sweeps < 0 || c->relax_sweeps > 64) return fail(ORC_INVALID, "relax_sweeps must be 0..64");
    if (c->nvx < 2 || c->nvy < 2) return fail(ORC_INVALID, "need nv >= 2");
    if (!(c->Kn > 0)) return fail(ORC_INVALID, "Kn must be positive");
    if (!(c->Pr > 0)) return fail(ORC_INVALID, "Pr must be positive");
    if (c->K < 0) return fail(ORC_INVALID, "K must be >= 0");
    if (c->model != 0 && c->model != 1) return fail(ORC_INVALID, "unknown collision model");
    if (c->model == 1 && c->K != 1) return fail(ORC_INVALID, "Shakhov model requires K = 1");
    if (c->quad != 0 && c->quad != 1) return fail(ORC_INVALID, "unknown quadrature");
    if (c->quad == 1 && !(c->vmax > 0)) return fail(ORC_INVALID, "Newton-Cotes needs vmax > 0");
    if (!(c->cfl_phys > 0) || !(c->cfl_imp > 0)) return fail(ORC_INVALID, "CFL must be positive");
    if (!(c->cfl_start >= 0) || (c->cfl_start > 0 && !(c->cfl_growth >= 1 && c->cfl_growth < 1e3)))
        return fail(ORC_INVALID, "CFL ramp needs cfl_start >= 0 and 1 <= cfl_growth < 1000");
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] < 0 || c->bc[s] > 2) return fail(ORC_INVALID, "unknown boundary type");
    if ((c->bc[0] == BC_PERIODIC) != (c->bc[1] == BC_PERIODIC) ||
        (c->bc[2] == BC_PERIODIC) != (c->bc[3] == BC_PERIODIC))
        return fail(ORC_INVALID, "periodic sides must come in pairs");
    if (c->bc[0] == BC_PERIODIC && c->ni == 2) return fail(ORC_INVALID, "periodic ni must be 1 or >= 3");
    if (c->bc[2] == BC_PERIODIC && c->nj == 2) return fail(ORC_INVALID, "periodic nj must be 1 or >= 3");
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] == BC_WALL && !(c->wall_T[s] > 0)) return fail(ORC_INVALID, "wall T must be positive");
    if (!(c->init_rho > 0) || !(c->init_T > 0)) return fail(ORC_INVALID, "initial state must be positive");
    for (int s = 0; s < 4; ++s)
        if (c->bc[s] == BC_FAR && (!(c->far_rho > 0) || !(c->far_T > 0)))
            return fail(ORC_INVALID, "far-field state must be positive");
    return 0;
}

static void free_problem(orc_problem *p)
{
    if (!p) return;
    void *ptrs[] = {p->xi, p->eta, p->w, p->area, p->xc, p->yc, p->cf, p->nb, p->nbdx, p->nbdy,
                    p->fdx, p->fdy, p->onx, p->ony, p->sS, p->ax, p->ay, p->sgn, p->fL, p->fR, p->ftype,
                    p->fside, p->fnx, p->fny, p->fS, p->fmx, p->fmy, p->fshx, p->fshy, p->gw,
                    p->ginf, p->hinf, p->wden, p->f, p->drho_g, p->W, p->RT, p->tau, p->q,
                    p->feq, p->bp, p->sx, p->sy, p->F, p->Wf, p->rhow, p->M, p->MW, p->dW,
                    p->Wst, p->dtimp, p->DW, p->RTst, p->taust, p->feqst, p->delta};
    for (size_t i = 0; i < sizeof ptrs / sizeof ptrs[0]; ++i) free(ptrs[i]);
    free(p);
}

void orc_destroy(orc_problem *p) { free_problem(p); }

static void state_W(const orc_problem *p, double rho, double u, double v, double T, double W[4])
{
    double RT = 0.5 * T;
    W[0] = rho;
    W[1] = rho * u;
    W[2] = rho * v;
    W[3] = 0.5 * rho * (u * u + v * v + (p->K + 2) * RT);
}

static double total_mass(const orc_problem *p, const double *f)
{
    double m = 0.0;
    for (int c = 0; c < p->nc; ++c) {
        double r = 0.0;
        for (int v = 0; v < p->nv; ++v) r += p->w[v] * f[(size_t)c * p->nv + v];
        m += p->area[c] * r;
    }
    return m;
}

static int create(const orc_config *cfg, const orc_mesh *mesh, orc_problem **out)
{
    if (!out) return fail(ORC_INVALID, "null output pointer");
    *out = NULL;
    int rc = validate(cfg, mesh);
    if (rc) return rc;
    orc_problem *p = calloc(1, sizeof *p);
    if (!p) return fail(ORC_NOMEM, "out of memory");
    p->model = cfg->model;
    p->K = cfg->K;
    p->limiter = cfg->limiter;
    p->predictor = cfg->predictor;
    p->relax_sweeps = cfg->relax_sweeps;
    p->Kn = cfg->Kn;
    p->Pr = cfg->Pr;
    p->omega = cfg->omega;
    p->cfl_imp = cfg->cfl_imp;
    p->cfl_start = cfg->cfl_start;
    p->cfl_growth = cfg->cfl_growth;
    p->imp_iters = 0;
    p->mu_ref = cfg->Kn / sqrt(M_PI); /* Eq. 37 with rho = L = 2RT = 1 */
    if ((rc = mesh ? build_mesh_unstructured(p, cfg, mesh) : build_mesh(p, cfg))) {
        free_problem(p);
        return rc;
    }
    const int nc = p->nc, nf = p->nf;
    /* velocity set */
    p->nvx = cfg->nvx;
    p->nvy = cfg->nvy;
    p->nv = cfg->nvx * cfg->nvy;
    const int nv = p->nv;
    double *x1 = malloc(cfg->nvx * sizeof(double)), *w1 = malloc(cfg->nvx * sizeof(double));
    double *y1 = malloc(cfg->nvy * sizeof(double)), *w2 = malloc(cfg->nvy * sizeof(double));
    rc = orc_quadrature_1d(cfg->quad, cfg->nvx, cfg->vmax, x1, w1);
    if (!rc) rc = orc_quadrature_1d(cfg->quad, cfg->nvy, cfg->vmax, y1, w2);
    if (rc) {
        free(x1), free(w1), free(y1), free(w2);
        free_problem(p);
        return rc;
    }
    p->xi = malloc(nv * sizeof(double));
    p->eta = malloc(nv * sizeof(double));
    p->w = malloc(nv * sizeof(double));
    for (int ix = 0; ix < cfg->nvx; ++ix)
        for (int iy = 0; iy < cfg->nvy; ++iy) {
            int v = ix * cfg->nvy + iy;
            p->xi[v] = x1[ix];
            p->eta[v] = y1[iy];
            p->w[v] = w1[ix] * w2[iy];
        }
    free(x1), free(w1), free(y1), free(w2);
    /* physical time step: cfl_phys * min cell size / max particle speed */
    double hmin = INFINITY, smax = 0.0;
    for (int c = 0; c < nc; ++c) {
        double d = INFINITY;
        for (int s = 0; s < 4; ++s) {
            int m = 4 * c + s;
            if (p->sS[m] == 0.0) continue; /* absent side of a triangle */
            double e = fabs(p->fdx[m] * p->onx[m] + p->fdy[m] * p->ony[m]);
            if (e < d) d = e;
        }
        if (2.0 * d < hmin) hmin = 2.0 * d;
    }
    for (int v = 0; v < nv; ++v) {
        double s = sqrt(p->xi[v] * p->xi[v] + p->eta[v] * p->eta[v]);
        if (s > smax) smax = s;
    }
    p->dt = cfg->cfl_phys * hmin / smax;
    p->h = 0.5 * p->dt;
    /* arrays */
    size_t big = (size_t)2 * nc * nv;
    p->f = calloc(big, sizeof(double));
    p->feq = calloc(big, sizeof(double));
    p->bp = calloc(big, sizeof(double));
    p->sx = calloc(big, sizeof(double));
    p->sy = calloc(big, sizeof(double));
    p->M = calloc(big, sizeof(double));
    p->feqst = calloc(big, sizeof(double));
    p->delta = calloc(big, sizeof(double));
    p->F = calloc((size_t)2 * nf * nv, sizeof(double));
    p->W = calloc(4 * nc, sizeof(double));
    p->RT = calloc(nc, sizeof(double));
    p->tau = calloc(nc, sizeof(double));
    p->q = calloc(2 * nc, sizeof(double));
    p->Wf = calloc(4 * nf, sizeof(double));
    p->rhow = calloc(nf, sizeof(double));
    p->MW = calloc(4 * nc, sizeof(double));
    p->dW = calloc(4 * nc, sizeof(double));
    p->Wst = calloc(4 * nc, sizeof(double));
    p->dtimp = calloc(nc, sizeof(double));
    p->DW = calloc(nc, sizeof(double));
    p->RTst = calloc(nc, sizeof(double));
    p->taust = calloc(nc, sizeof(double));
    p->drho_g = calloc(nf, sizeof(double));
    p->wden = calloc(nf, sizeof(double));
    p->gw = calloc(4 * (size_t)nv, sizeof(double));
    p->ginf = calloc(nv, sizeof(double));
    p->hinf = calloc(nv, sizeof(double));
    double *scratch = calloc(nv, sizeof(double));
    if (!p->f || !p->feq || !p->bp || !p->sx || !p->sy || !p->M || !p->feqst || !p->delta ||
        !p->F || !scratch) {
        free(scratch);
        free_problem(p);
        return fail(ORC_NOMEM, "out of memory");
    }
    /* boundary distributions */
    double qz[2] = {0.0, 0.0};
    p->closed = 1;
    for (int s = 0; s < 4; ++s) {
        if (cfg->bc[s] == BC_FAR) p->closed = 0;
        p->wall_u[s] = cfg->wall_u[s];
        p->wall_v[s] = cfg->wall_v[s];
        p->wall_RT[s] = 0.5 * cfg->wall_T[s];
        if (cfg->bc[s] == BC_WALL) {
            double Ww[4];
            state_W(p, 1.0, cfg->wall_u[s], cfg->wall_v[s], cfg->wall_T[s], Ww);
            equilibrium(p, Ww, qz, p->gw + (size_t)s * nv, scratch);
        }
    }
    {
        double Wi[4];
        state_W(p, cfg->far_rho, cfg->far_u, cfg->far_v, cfg->far_T, Wi);
        equilibrium(p, Wi, qz, p->ginf, p->hinf);
    }
    for (int k = 0; k < nf; ++k) {
        if (p->ftype[k] != F_WALL) continue;
        const double *g = p->gw + (size_t)p->fside[k] * nv;
        double den = 0.0;
        for (int v = 0; v < nv; ++v) {
            double un = normal_speed(p->xi[v], p->eta[v], p->fnx[k], p->fny[k]);
            if (un < 0) den += p->w[v] * un * g[v];
        }
        p->wden[k] = den;
    }
    free(scratch);
    /* initial state: uniform equilibrium, for which phi~ = phi = phi_eq */
    {
        double W0[4];
        state_W(p, cfg->init_rho, cfg->init_u, cfg->init_v, cfg->init_T, W0);
        equilibrium(p, W0, qz, p->f, p->f + (size_t)nc * nv);
        for (int c = 1; c < nc; ++c) {
            memcpy(p->f + (size_t)c * nv, p->f, nv * sizeof(double));
            memcpy(p->f + (size_t)(nc + c) * nv, p->f + (size_t)nc * nv, nv * sizeof(double));
        }
    }
    p->M0 = total_mass(p, p->f);
    *out = p;
    return ORC_OK;
}

int orc_create(const orc_config *cfg, orc_problem **out) { return create(cfg, NULL, out); }

int orc_create_mesh(const orc_config *cfg, const orc_mesh *mesh, orc_problem **out)
{
    return create(cfg, mesh, out);
}

void orc_sizes(const orc_problem *p, int32_t out[4])
{
    out[0] = p->nc;
    out[1] = p->nv;
    out[2] = p->nf;
    out[3] = p->nwall;
}

double orc_dt(const orc_problem *p) { return p->dt; }

void orc_velocities(const orc_problem *p, double *xi, double *eta, double *w)
{
    memcpy(xi, p->xi, p->nv * sizeof(double));
    memcpy(eta, p->eta, p->nv * sizeof(double));
    memcpy(w, p->w, p->nv * sizeof(double));
}

void orc_cells(const orc_problem *p, double *area, double *xc, double *yc)
{
    memcpy(area, p->area, p->nc * sizeof(double));
    memcpy(xc, p->xc, p->nc * sizeof(double));
    memcpy(yc, p->yc, p->nc * sizeof(double));
}

void orc_cell_sides(const orc_problem *p, int32_t *nb, double *nx, double *ny, double *S,
                    double *dx, double *dy, double *ax, double *ay)
{
    for (int m = 0; m < 4 * p->nc; ++m) {
        nb[m] = p->nb[m];
        nx[m] = p->onx[m];
        ny[m] = p->ony[m];
        S[m] = p->sS[m];
        dx[m] = p->fdx[m];
        dy[m] = p->fdy[m];
        ax[m] = p->ax[m];
        ay[m] = p->ay[m];
    }
}

void orc_get_state(const orc_problem *p, double *f)
{
    memcpy(f, p->f, (size_t)2 * p->nc * p->nv * sizeof(double));
}

void orc_set_state(orc_problem *p, const double *f)
{
    memcpy(p->f, f, (size_t)2 * p->nc * p->nv * sizeof(double));
    p->M0 = total_mass(p, p->f);
    p->predicted = 0;
    p->imp_iters = 0;
}

/* ------------------------------------------------------------------------- */
/* Explicit DUGKS residual (Section 2.1)                                      */
/* ------------------------------------------------------------------------- */

/* Cell records: conserved moments of phi~ (they equal those of phi), RT, tau, the
   Shakhov heat flux q = 2 tau q~ / (2 tau + dt Pr), and the cell equilibrium. */
static void cell_records(orc_problem *p)
{
    const int nc = p->nc, nv = p->nv;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c) {
        const double *G = p->f + (size_t)c * nv, *H = p->f + (size_t)(nc + c) * nv;
        double *W = p->W + 4 * c;
        moments(p, G, H, W);
        p->RT[c] = rt_of(W, p->K);
        p->tau[c] = tau_of(p, W[0], p->RT[c]);
        double q[2] = {0.0, 0.0};
        if (p->model == 1) {
            double qt[2];
            heat_flux(p, G, H, W, qt);
            double t2 = 2.0 * p->tau[c];
            q[0] = t2 * qt[0] / (t2 + p->dt * p->Pr);
            q[1] = t2 * qt[1] / (t2 + p->dt * p->Pr);
        }
        p->q[2 * c] = q[0];
        p->q[2 * c + 1] = q[1];
        equilibrium(p, W, q, p->feq + (size_t)c * nv, p->feq + (size_t)(nc + c) * nv);
    }
}

/* Theta of the Venkatakrishnan limiter (Eq. 17) */
static double venkat_theta(double x) { return (x * x + 2.0 * x) / (x * x + x + 2.0); }

/* Least-squares gradient (Eq. 15) of a cell field val[j * stride] at cell c, optionally
   limited by Venkatakrishnan's function (Eq. 16-17): phi = min over the cell's faces of
   theta(r_k), r_k the room to the largest (Delta_k > 0) or smallest (Delta_k < 0) value over
   the cell and its neighbours divided by the unlimited increment Delta_k from the centroid
   to the face midpoint; theta = 1 where Delta_k = 0, and phi <= 1. */
static void cell_gradient(const orc_problem *p, int c, const double *val, size_t stride, int limiter,
                          double *gx_out, double *gy_out)
{
    double b0 = val[(size_t)c * stride], gx = 0.0, gy = 0.0, bmax = b0, bmin = b0;
    for (int side = 0; side < 4; ++side) {
        int m = 4 * c + side, j = p->nb[m];
        if (j < 0) continue;
        double bj = val[(size_t)j * stride];
        gx += p->ax[m] * (bj - b0);
        gy += p->ay[m] * (bj - b0);
        if (bj > bmax) bmax = bj;
        if (bj < bmin) bmin = bj;
    }
    if (limiter) {
        double phi = 1.0;
        for (int side = 0; side < 4; ++side) {
            int m = 4 * c + side;
            double d = gx * p->fdx[m] + gy * p->fdy[m], th = 1.0;
            if (d > 0) th = venkat_theta((bmax - b0) / d);
            else if (d < 0) th = venkat_theta((bmin - b0) / d);
            if (th < phi) phi = th;
        }
        gx *= phi;
        gy *= phi;
    }
    *gx_out = gx;
    *gy_out = gy;
}

/* phi-bar-plus at cell centres and its least-squares gradient (Eq. 12-17). */
static void barplus_gradients(orc_problem *p)
{
    const int nc = p->nc, nv = p->nv;
    const double dt = p->dt, h = p->h;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c) {
        double t2 = 2.0 * p->tau[c];
        double a = (t2 - h) / (t2 + dt), b = 3.0 * h / (t2 + dt);
        for (int s = 0; s < 2; ++s) {
            size_t o = (size_t)(s * nc + c) * nv;
            for (int v = 0; v < nv; ++v) p->bp[o + v] = a * p->f[o + v] + b * p->feq[o + v];
        }
    }
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c)
        for (int s = 0; s < 2; ++s)
            for (int v = 0; v < nv; ++v) {
                size_t o = (size_t)(s * nc + c) * nv + v;
                if (p->first_order) p->sx[o] = p->sy[o] = 0.0;
                else cell_gradient(p, c, p->bp + (size_t)s * nc * nv + v, nv, p->limiter, p->sx + o, p->sy + o);
            }
}

/* Interface distributions, their equilibria and the fluxes S (xi.n) phi_k
   (Eq. 11, 13, 14, 18, 19; boundary ghost values per Section 2.3). */
static void face_fluxes(orc_problem *p)
{
    const int nc = p->nc, nv = p->nv, nf = p->nf, K = p->K;
    const double h = p->h;
#pragma omp parallel
    {
        double *fb = malloc((size_t)2 * nv * sizeof(double));
        double *fe = malloc((size_t)2 * nv * sizeof(double));
#pragma omp for schedule(dynamic, 16)
        for (int k = 0; k < nf; ++k) {
            double *FG = p->F + (size_t)k * nv, *FH = p->F + (size_t)(nf + k) * nv;
            if (p->ftype[k] == F_SELF) {
                memset(FG, 0, nv * sizeof(double));
                memset(FH, 0, nv * sizeof(double));
                continue;
            }
            const int L = p->fL[k], R = p->fR[k], type = p->ftype[k];
            const double nx = p->fnx[k], ny = p->fny[k];
            double *bG = fb, *bH = fb + nv;
            double num = 0.0;
            for (int v = 0; v < nv; ++v) {
                double x = p->xi[v], y = p->eta[v], un = normal_speed(x, y, nx, ny);
                int u;
                double dx, dy;
                if (un > 0 || type != F_INTERIOR) {
                    u = L;
                    dx = p->fmx[k] - p->xc[L];
                    dy = p->fmy[k] - p->yc[L];
                } else {
                    u = R;
                    dx = p->fmx[k] - p->fshx[k] - p->xc[R];
                    dy = p->fmy[k] - p->fshy[k] - p->yc[R];
                }
                double rx = dx - h * x, ry = dy - h * y;
                size_t oG = (size_t)u * nv + v, oH = (size_t)(nc + u) * nv + v;
                bG[v] = p->bp[oG] + p->sx[oG] * rx + p->sy[oG] * ry;
                bH[v] = p->bp[oH] + p->sx[oH] * rx + p->sy[oH] * ry;
                if (type == F_WALL && un > 0) num += p->w[v] * un * bG[v];
            }
            double rho_w = 0.0;
            if (type == F_WALL) {
                int side = p->fside[k];
                const double *g = p->gw + (size_t)side * nv;
                rho_w = -num / p->wden[k];
                for (int v = 0; v < nv; ++v) {
                    double un = normal_speed(p->xi[v], p->eta[v], nx, ny);
                    if (un <= 0) {
                        bG[v] = rho_w * g[v];
                        bH[v] = rho_w * K * p->wall_RT[side] * g[v];
                    }
                }
            } else if (type == F_FAR) {
                for (int v = 0; v < nv; ++v) {
                    double un = normal_speed(p->xi[v], p->eta[v], nx, ny);
                    if (un < 0) {
                        bG[v] = p->ginf[v];
                        bH[v] = p->hinf[v];
                    }
                }
            }
            double Wk[4], qk[2] = {0.0, 0.0};
            moments(p, bG, bH, Wk);
            double RTk = rt_of(Wk, K), tk = tau_of(p, Wk[0], RTk), t2 = 2.0 * tk;
            if (p->model == 1) {
                double qb[2];
                heat_flux(p, bG, bH, Wk, qb);
                qk[0] = t2 * qb[0] / (t2 + h * p->Pr);
                qk[1] = t2 * qb[1] / (t2 + h * p->Pr);
            }
            equilibrium(p, Wk, qk, fe, fe + nv);
            for (int v = 0; v < nv; ++v) {
                double un = normal_speed(p->xi[v], p->eta[v], nx, ny);
                double pg = (t2 * bG[v] + h * fe[v]) / (t2 + h);
                double ph = (t2 * bH[v] + h * fe[nv + v]) / (t2 + h);
                FG[v] = p->fS[k] * un * pg;
                FH[v] = p->fS[k] * un * ph;
            }
            for (int a = 0; a < 4; ++a) p->Wf[4 * k + a] = Wk[a];
            p->rhow[k] = rho_w;
        }
        free(fb);
        free(fe);
    }
}

/* M_i(v) = - sum over faces of S (xi.n_out) phi_k (Eq. 23); faces joining a cell to
   itself (one-cell periodic direction) cancel exactly and are skipped. */
static void flux_sum(orc_problem *p)
{
    const int nc = p->nc, nv = p->nv, nf = p->nf;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c)
        for (int s = 0; s < 2; ++s) {
            double *Mc = p->M + (size_t)(s * nc + c) * nv;
            for (int v = 0; v < nv; ++v) Mc[v] = 0.0;
            for (int side = 0; side < 4; ++side) {
                int k = p->cf[4 * c + side];
                if (p->ftype[k] == F_SELF) continue;
                const double *Fk = p->F + (size_t)(s * nf + k) * nv;
                if (p->sgn[4 * c + side] > 0)
                    for (int v = 0; v < nv; ++v) Mc[v] -= Fk[v];
                else
                    for (int v = 0; v < nv; ++v) Mc[v] += Fk[v];
            }
        }
}

static void explicit_residual(orc_problem *p)
{
    cell_records(p);
    barplus_gradients(p);
    face_fluxes(p);
    flux_sum(p);
}

/* M_W = sum_v w psi M (Eq. 27) */
static void macro_residual(orc_problem *p)
{
    const int nc = p->nc, nv = p->nv;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c)
        moments(p, p->M + (size_t)c * nv, p->M + (size_t)(nc + c) * nv, p->MW + 4 * c);
}

static int check_state(const orc_problem *p)
{
    for (int c = 0; c < p->nc; ++c)
        if (!(p->W[4 * c] > 0) || !(p->RT[c] > 0) || !isfinite(p->tau[c]))
            return fail(ORC_DIVERGED, "non-physical state (rho <= 0, T <= 0 or NaN)");
    return 0;
}

int orc_flux(orc_problem *p, double *M)
{
    explicit_residual(p);
    if (M) memcpy(M, p->M, (size_t)2 * p->nc * p->nv * sizeof(double));
    return check_state(p);
}

int orc_face_moments(orc_problem *p, double *Wf, double *rho_w)
{
    explicit_residual(p);
    if (Wf) memcpy(Wf, p->Wf, 4 * (size_t)p->nf * sizeof(double));
    if (rho_w) memcpy(rho_w, p->rhow, (size_t)p->nf * sizeof(double));
    return check_state(p);
}

void orc_barplus(orc_problem *p, double *out)
{
    cell_records(p);
    barplus_gradients(p);
    memcpy(out, p->bp, (size_t)2 * p->nc * p->nv * sizeof(double));
}

int orc_macro_residual(orc_problem *p, double *MW)
{
    explicit_residual(p);
    macro_residual(p);
    if (MW) memcpy(MW, p->MW, 4 * (size_t)p->nc * sizeof(double));
    return check_state(p);
}

int orc_residual(orc_problem *p, double out[4])
{
    int rc = orc_macro_residual(p, NULL);
    for (int a = 0; a < 4; ++a) {
        double s = 0.0;
        for (int c = 0; c < p->nc; ++c) {
            double r = p->MW[4 * c + a] / p->area[c];
            s += r * r;
        }
        out[a] = sqrt(s / p->nc);
    }
    return rc;
}

void orc_moments(const orc_problem *p, double *out)
{
    const int nc = p->nc, nv = p->nv;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c) {
        const double *G = p->f + (size_t)c * nv, *H = p->f + (size_t)(nc + c) * nv;
        double W[4], qt[2];
        moments(p, G, H, W);
        double RT = rt_of(W, p->K), tau = tau_of(p, W[0], RT);
        heat_flux(p, G, H, W, qt);
        double Pr = p->model == 1 ? p->Pr : 1.0, t2 = 2.0 * tau;
        double *o = out + 8 * c;
        o[0] = W[0];
        o[1] = W[1] / W[0];
        o[2] = W[2] / W[0];
        o[3] = 2.0 * RT;
        o[4] = W[0] * RT;
        o[5] = t2 * qt[0] / (t2 + p->dt * Pr);
        o[6] = t2 * qt[1] / (t2 + p->dt * Pr);
        o[7] = tau;
    }
}

/* Relative L2 change of the cell densities. */
static double density_change(const orc_problem *p, const double *rho_old)
{
    double num = 0.0, den = 0.0;
    for (int c = 0; c < p->nc; ++c) {
        double r = 0.0;
        for (int v = 0; v < p->nv; ++v) r += p->w[v] * p->f[(size_t)c * p->nv + v];
        num += (r - rho_old[c]) * (r - rho_old[c]);
        den += r * r;
    }
    return sqrt(num / den);
}

int orc_explicit_step(orc_problem *p, int32_t nsteps, double *res)
{
    const int nc = p->nc, nv = p->nv;
    double *rho0 = malloc(nc * sizeof(double));
    double r = 0.0;
    for (int n = 0; n < nsteps; ++n) {
        explicit_residual(p);
        int rc = check_state(p);
        if (rc) {
            free(rho0);
            return rc;
        }
        for (int c = 0; c < nc; ++c) rho0[c] = p->W[4 * c];
        /* Eq. 21 with phi~+ - phi~ = -(2 dt/(2 tau + dt))(phi~ - phi_eq) */
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc; ++c) {
            double coef = 2.0 * p->area[c] / (2.0 * p->tau[c] + p->dt), g = p->dt / p->area[c];
            for (int s = 0; s < 2; ++s) {
                size_t o = (size_t)(s * nc + c) * nv;
                for (int v = 0; v < nv; ++v)
                    p->f[o + v] += g * (p->M[o + v] - coef * (p->f[o + v] - p->feq[o + v]));
            }
        }
        r = density_change(p, rho0);
    }
    free(rho0);
    if (res) *res = r;
    p->predicted = 0;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Implicit DUGKS (Section 2.2)                                               */
/* ------------------------------------------------------------------------- */

/* Euler flux along n (used in the matrix-free macro LU-SGS); p = rho RT */
static void euler_flux(const double W[4], double nx, double ny, int K, double F[4])
{
    double rho = W[0], U = W[1] / rho, V = W[2] / rho;
    double pr = (2.0 * W[3] - rho * (U * U + V * V)) / (K + 2);
    double un = U * nx + V * ny;
    F[0] = rho * un;
    F[1] = W[1] * un + pr * nx;
    F[2] = W[2] * un + pr * ny;
    F[3] = (W[3] + pr) * un;
}

/* 1/2 S (F_n(W_j + dW_j) - F_n(W_j) - lambda_j dW_j) of one cell side m with neighbour j:
   the matrix-free off-diagonal term of Eq. 30 (Rusanov split, lambda of Eq. 31) */
static void offdiag(const orc_problem *p, const double *C, int m, int j, const double *dWj,
                    double out[4])
{
    double nx = p->onx[m], ny = p->ony[m], S = p->sS[m];
    const double *Wj = p->W + 4 * j;
    double lam = fabs((Wj[1] * nx + Wj[2] * ny) / Wj[0]) + C[j];
    double Wn[4] = {Wj[0] + dWj[0], Wj[1] + dWj[1], Wj[2] + dWj[2], Wj[3] + dWj[3]};
    double F1[4], F0[4];
    euler_flux(Wn, nx, ny, p->K, F1);
    euler_flux(Wj, nx, ny, p->K, F0);
    for (int a = 0; a < 4; ++a) out[a] = 0.5 * S * (F1[a] - F0[a] - lam * dWj[a]);
}

/* Point relaxation of (L + D + U) dW = M_W (the paper's second predictor, Section 4; it
   gives no formula): the point-implicit step dW = D^-1 M_W, then Jacobi sweeps
   dW <- D^-1 (M_W - (L + U) dW) with every neighbour's dW of the previous sweep. */
static void macro_point_relax(orc_problem *p, const double *C)
{
    const int nc = p->nc;
    double *old = malloc(4 * (size_t)nc * sizeof(double));
    for (int c = 0; c < nc; ++c)
        for (int a = 0; a < 4; ++a) p->dW[4 * c + a] = p->MW[4 * c + a] / p->DW[c];
    for (int k = 0; k < p->relax_sweeps; ++k) {
        memcpy(old, p->dW, 4 * (size_t)nc * sizeof(double));
        for (int c = 0; c < nc; ++c) {
            double r[4];
            for (int a = 0; a < 4; ++a) r[a] = p->MW[4 * c + a];
            for (int side = 0; side < 4; ++side) {
                int m = 4 * c + side, kf = p->cf[m], j = p->nb[m];
                if (p->ftype[kf] == F_SELF || j < 0) continue;
                double o[4];
                offdiag(p, C, m, j, old + 4 * j, o);
                for (int a = 0; a < 4; ++a) r[a] -= o[a];
            }
            for (int a = 0; a < 4; ++a) p->dW[4 * c + a] = r[a] / p->DW[c];
        }
    }
    free(old);
}

/* Predicted macroscopic step (Eq. 27-31): LU-SGS on (L + D + U) dW = M_W, or point
   relaxation of the same system. */
/* The implicit CFL of the current iteration: cfl_imp, or the start-up ramp
   min(cfl_imp, cfl_start cfl_growth^n) after n implicit iterations. */
static double implicit_cfl(const orc_problem *p)
{
    if (!(p->cfl_start > 0)) return p->cfl_imp;
    const double c = p->cfl_start * pow(p->cfl_growth, (double)p->imp_iters);
    return c < p->cfl_imp ? c : p->cfl_imp;
}

static void macro_lusgs(orc_problem *p)
{
    const int nc = p->nc, K = p->K;
    const double gam = (K + 4.0) / (K + 2.0);
    const double cfl = implicit_cfl(p);
    double *C = malloc(nc * sizeof(double));
    for (int c = 0; c < nc; ++c) C[c] = sqrt(gam * p->RT[c]);
    for (int c = 0; c < nc; ++c) {
        double U = p->W[4 * c + 1] / p->W[4 * c], V = p->W[4 * c + 2] / p->W[4 * c], ls = 0.0;
        for (int side = 0; side < 4; ++side) {
            int m = 4 * c + side, k = p->cf[m];
            if (p->ftype[k] == F_SELF) continue;
            ls += (fabs(U * p->onx[m] + V * p->ony[m]) + C[c]) * p->sS[m];
        }
        /* mirrored wall ghost: the wall face's dissipation acts on 2 dW_c */
        double lw = 0.0;
        for (int side = 0; side < 4; ++side) {
            int m = 4 * c + side, k = p->cf[m];
            if (p->ftype[k] == F_WALL) lw += (fabs(U * p->onx[m] + V * p->ony[m]) + C[c]) * p->sS[m];
        }
        p->dtimp[c] = cfl * p->area[c] / ls;
        p->DW[c] = p->area[c] / p->dtimp[c] + 0.5 * ls + 0.5 * lw;
    }
    if (p->predictor == 1) {
        macro_point_relax(p, C);
    } else {
        /* lower sweep (ascending cell index) */
        for (int c = 0; c < nc; ++c) {
            double r[4];
            for (int a = 0; a < 4; ++a) r[a] = p->MW[4 * c + a];
            for (int side = 0; side < 4; ++side) {
                int m = 4 * c + side, k = p->cf[m], j = p->nb[m];
                if (p->ftype[k] == F_SELF || j < 0 || j > c) continue;
                double nx = p->onx[m], ny = p->ony[m], S = p->sS[m];
                const double *Wj = p->W + 4 * j, *dWj = p->dW + 4 * j;
                double lam = fabs((Wj[1] * nx + Wj[2] * ny) / Wj[0]) + C[j];
                double Wn[4] = {Wj[0] + dWj[0], Wj[1] + dWj[1], Wj[2] + dWj[2], Wj[3] + dWj[3]};
                double F1[4], F0[4];
                euler_flux(Wn, nx, ny, K, F1);
                euler_flux(Wj, nx, ny, K, F0);
                for (int a = 0; a < 4; ++a) r[a] -= 0.5 * S * (F1[a] - F0[a] - lam * dWj[a]);
            }
            for (int a = 0; a < 4; ++a) p->dW[4 * c + a] = r[a] / p->DW[c];
        }
        /* upper sweep (descending cell index) */
        for (int c = nc - 1; c >= 0; --c) {
            double r[4] = {0, 0, 0, 0};
            for (int side = 0; side < 4; ++side) {
                int m = 4 * c + side, k = p->cf[m], j = p->nb[m];
                if (p->ftype[k] == F_SELF || j < 0 || j < c) continue;
                double nx = p->onx[m], ny = p->ony[m], S = p->sS[m];
                const double *Wj = p->W + 4 * j, *dWj = p->dW + 4 * j;
                double lam = fabs((Wj[1] * nx + Wj[2] * ny) / Wj[0]) + C[j];
                double Wn[4] = {Wj[0] + dWj[0], Wj[1] + dWj[1], Wj[2] + dWj[2], Wj[3] + dWj[3]};
                double F1[4], F0[4];
                euler_flux(Wn, nx, ny, K, F1);
                euler_flux(Wj, nx, ny, K, F0);
                for (int a = 0; a < 4; ++a) r[a] += 0.5 * S * (F1[a] - F0[a] - lam * dWj[a]);
            }
            for (int a = 0; a < 4; ++a) p->dW[4 * c + a] -= r[a] / p->DW[c];
        }
    }
    free(C);
    /* W* = W^n + dW; tau* and the predicted equilibrium (heat flux of step n) */
    const int nv = p->nv;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < nc; ++c) {
        double *Ws = p->Wst + 4 * c;
        for (int a = 0; a < 4; ++a) Ws[a] = p->W[4 * c + a] + p->dW[4 * c + a];
        p->RTst[c] = rt_of(Ws, K);
        p->taust[c] = tau_of(p, Ws[0], p->RTst[c]);
        equilibrium(p, Ws, p->q + 2 * c, p->feqst + (size_t)c * nv,
                    p->feqst + (size_t)(nc + c) * nv);
    }
    p->predicted = 1;
}

int orc_predict(orc_problem *p, double *Wstar, double *dt_imp)
{
    explicit_residual(p);
    int rc = check_state(p);
    if (rc) return rc;
    macro_residual(p);
    macro_lusgs(p);
    if (Wstar) memcpy(Wstar, p->Wst, 4 * (size_t)p->nc * sizeof(double));
    if (dt_imp) memcpy(dt_imp, p->dtimp, (size_t)p->nc * sizeof(double));
    return 0;
}

/* Diagonal of Eq. 26 for cell c and velocity v: Omega/dt_imp - dM/dphi_i - dQ/dphi_i */
static double micro_diag(const orc_problem *p, int c, int v)
{
    double x = p->xi[v], y = p->eta[v], D = p->area[c] / p->dtimp[c];
    for (int side = 0; side < 4; ++side) {
        int m = 4 * c + side, k = p->cf[m];
        if (p->ftype[k] == F_SELF) continue;
        double un = normal_speed(x, y, p->onx[m], p->ony[m]);
        if (un > 0) D += un * p->sS[m];
    }
    return D + 2.0 * p->area[c] / (2.0 * p->taust[c] + p->dt);
}

/* Coupling to the neighbour across side s (first-order upwind implicit flux, Eq. 24-25):
   incoming velocities (xi.n_out < 0) bring -(xi.n_out) S delta_j into cell c. */
static double micro_coupling(const orc_problem *p, int c, int side, int v)
{
    int m = 4 * c + side, k = p->cf[m];
    if (p->ftype[k] == F_SELF || p->nb[m] < 0) return 0.0;
    double un = normal_speed(p->xi[v], p->eta[v], p->onx[m], p->ony[m]);
    return un < 0 ? -un * p->sS[m] : 0.0;
}

/* Forward (lower) sweep for one velocity: (D + L) d* = r, ascending cell index. */
static void sweep_lower(const orc_problem *p, int v, double *d, int stride)
{
    for (int c = 0; c < p->nc; ++c) {
        double s = d[(size_t)c * stride];
        for (int side = 0; side < 4; ++side) {
            int j = p->nb[4 * c + side];
            if (j < 0 || j >= c) continue;
            s += micro_coupling(p, c, side, v) * d[(size_t)j * stride];
        }
        d[(size_t)c * stride] = s / micro_diag(p, c, v);
    }
}

/* Backward (upper) sweep: d = d* + D^{-1}(couplings to higher cells + wall ghost inflow),
   descending cell index.  drho (may be NULL) holds the ghost density increment of each
   wall face; species 1 (H) carries the factor K RT_wall (Eq. 34 integrated over zeta). */
static void sweep_upper(const orc_problem *p, int v, double *d, int stride, const double *drho,
                        int species)
{
    for (int c = p->nc - 1; c >= 0; --c) {
        double s = 0.0;
        for (int side = 0; side < 4; ++side) {
            int j = p->nb[4 * c + side];
            if (j < 0 || j <= c) continue;
            s += micro_coupling(p, c, side, v) * d[(size_t)j * stride];
        }
        if (drho)
            for (int side = 0; side < 4; ++side) {
                int m = 4 * c + side, k = p->cf[m];
                if (p->ftype[k] != F_WALL) continue;
                double un = normal_speed(p->xi[v], p->eta[v], p->onx[m], p->ony[m]);
                if (un < 0) {
                    int ws = p->fside[k];
                    double in = -un * p->sS[m] * drho[k] * p->gw[(size_t)ws * p->nv + v];
                    s += species == 0 ? in : in * p->K * p->wall_RT[ws];
                }
            }
        d[(size_t)c * stride] += s / micro_diag(p, c, v);
    }
}

/* Ghost density increment of each wall face from the wall cell's G increment (Eq. 35). */
static void wall_ghost(orc_problem *p)
{
    const int nv = p->nv;
    for (int k = 0; k < p->nf; ++k) {
        p->drho_g[k] = 0.0;
        if (p->ftype[k] != F_WALL) continue;
        int c = p->fL[k];
        double num = 0.0;
        for (int v = 0; v < nv; ++v) {
            double un = normal_speed(p->xi[v], p->eta[v], p->fnx[k], p->fny[k]);
            if (un > 0) num += p->w[v] * un * p->delta[(size_t)c * nv + v];
        }
        p->drho_g[k] = -num / p->wden[k];
    }
}

int orc_micro_operator(orc_problem *p, int32_t v, double *D, double *C)
{
    if (!p->predicted) return fail(ORC_INVALID, "call orc_predict first");
    if (v < 0 || v >= p->nv) return fail(ORC_INVALID, "velocity index out of range");
    for (int c = 0; c < p->nc; ++c) {
        D[c] = micro_diag(p, c, v);
        for (int side = 0; side < 4; ++side) C[4 * c + side] = micro_coupling(p, c, side, v);
    }
    return 0;
}

int orc_micro_sweep(orc_problem *p, int32_t v, const double *rhs, double *out)
{
    if (!p->predicted) return fail(ORC_INVALID, "call orc_predict first");
    if (v < 0 || v >= p->nv) return fail(ORC_INVALID, "velocity index out of range");
    for (int c = 0; c < p->nc; ++c) out[c] = rhs[c];
    sweep_lower(p, v, out, 1);
    sweep_upper(p, v, out, 1, NULL, 0);
    return 0;
}

int orc_implicit_step(orc_problem *p, int32_t nsteps, double *res)
{
    const int nc = p->nc, nv = p->nv;
    double *rho0 = malloc(nc * sizeof(double));
    double r = 0.0;
    for (int n = 0; n < nsteps; ++n) {
        int rc = orc_predict(p, NULL, NULL);
        if (rc) {
            free(rho0);
            return rc;
        }
        for (int c = 0; c < nc; ++c) rho0[c] = p->W[4 * c];
        /* right-hand side R* = M + Q(W*) (Eq. 22-23, 26) */
#pragma omp parallel for schedule(static)
        for (int c = 0; c < nc; ++c) {
            double cst = 2.0 * p->area[c] / (2.0 * p->taust[c] + p->dt);
            for (int s = 0; s < 2; ++s) {
                size_t o = (size_t)(s * nc + c) * nv;
                for (int v = 0; v < nv; ++v)
                    p->delta[o + v] = p->M[o + v] - cst * (p->f[o + v] - p->feqst[o + v]);
            }
        }
        /* forward sweeps (zero ghost increments), every velocity and species independently */
#pragma omp parallel for schedule(dynamic, 4)
        for (int sv = 0; sv < 2 * nv; ++sv)
            sweep_lower(p, sv % nv, p->delta + (size_t)(sv / nv) * nc * nv + sv % nv, nv);
        /* wall ghost increments from the forward-sweep result (Eq. 34-35) */
        wall_ghost(p);
        if (p->cap_dstar) memcpy(p->cap_dstar, p->delta, (size_t)2 * nc * nv * sizeof(double));
        if (p->cap_drho) memcpy(p->cap_drho, p->drho_g, (size_t)p->nf * sizeof(double));
        /* backward sweeps */
#pragma omp parallel for schedule(dynamic, 4)
        for (int sv = 0; sv < 2 * nv; ++sv)
            sweep_upper(p, sv % nv, p->delta + (size_t)(sv / nv) * nc * nv + sv % nv, nv,
                        p->drho_g, sv / nv);
        /* update (Eq. 32) */
        for (size_t i = 0; i < (size_t)2 * nc * nv; ++i) p->f[i] += p->delta[i];
        /* closed domain: restore the reference mass */
        if (p->closed) {
            double s = p->M0 / total_mass(p, p->f);
            for (size_t i = 0; i < (size_t)2 * nc * nv; ++i) p->f[i] *= s;
        }
        r = density_change(p, rho0);
        ++p->imp_iters;
        if (!isfinite(r)) {
            free(rho0);
            return fail(ORC_DIVERGED, "non-finite residual");
        }
    }
    free(rho0);
    if (res) *res = r;
    p->predicted = 0;
    return 0;
}

int orc_solve(orc_problem *p, double tol, int32_t max_iter, int32_t *iters, double *res)
{
    double r = INFINITY;
    int n = 0;
    while (n < max_iter) {
        int rc = orc_implicit_step(p, 1, &r);
        ++n;
        if (rc) {
            if (iters) *iters = n;
            if (res) *res = r;
            return rc;
        }
        if (r < tol) break;
    }
    if (iters) *iters = n;
    if (res) *res = r;
    return r < tol ? 0 : fail(ORC_NOT_CONVERGED, "iteration limit reached");
}

/* ------------------------------------------------------------------------- */
/* Accessors of intermediate quantities (pins of the individual steps)        */
/* ------------------------------------------------------------------------- */
int orc_gradients(orc_problem *p, double *sx, double *sy)
{
    cell_records(p);
    barplus_gradients(p);
    size_t n = (size_t)2 * p->nc * p->nv;
    if (sx) memcpy(sx, p->sx, n * sizeof(double));
    if (sy) memcpy(sy, p->sy, n * sizeof(double));
    return check_state(p);
}

int orc_lsq_gradient(const orc_problem *p, const double *phi, int32_t limiter, double *gx, double *gy)
{
    for (int c = 0; c < p->nc; ++c) cell_gradient(p, c, phi, 1, limiter, gx + c, gy + c);
    return 0;
}

void orc_faces(const orc_problem *p, int32_t *L, int32_t *R, int32_t *type, int32_t *side,
               double *nx, double *ny, double *S, double *mx, double *my)
{
    for (int k = 0; k < p->nf; ++k) {
        L[k] = p->fL[k];
        R[k] = p->fR[k];
        type[k] = p->ftype[k];
        side[k] = p->fside[k];
        nx[k] = p->fnx[k];
        ny[k] = p->fny[k];
        S[k] = p->fS[k];
        mx[k] = p->fmx[k];
        my[k] = p->fmy[k];
    }
}

int orc_face_flux(orc_problem *p, double *F)
{
    explicit_residual(p);
    if (F) memcpy(F, p->F, (size_t)2 * p->nf * p->nv * sizeof(double));
    return check_state(p);
}

int orc_macro_sweep_rhs(orc_problem *p, const double *rhs, double *dW)
{
    cell_records(p);
    int rc = check_state(p);
    if (rc) return rc;
    memcpy(p->MW, rhs, 4 * (size_t)p->nc * sizeof(double));
    macro_lusgs(p);
    memcpy(dW, p->dW, 4 * (size_t)p->nc * sizeof(double));
    return 0;
}

int orc_implicit_detail(orc_problem *p, double *delta_star, double *drho, double *res)
{
    p->cap_dstar = delta_star;
    p->cap_drho = drho;
    int rc = orc_implicit_step(p, 1, res);
    p->cap_dstar = NULL;
    p->cap_drho = NULL;
    return rc;
}

/* Analysis switch: with first_order != 0 the reconstruction drops the gradient (the
   first-order upwind residual, whose Jacobian is the one the micro LU-SGS factorises). */
void orc_set_first_order(orc_problem *p, int32_t first_order) { p->first_order = first_order != 0; }
