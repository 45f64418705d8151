// HIP kernels (gfx950) of the implicit DUGKS hot path.
//
// Paper: Pan, Zhong & Zhuo, arXiv:1709.01819.  One implicit iteration is
//   records    cell equilibrium records from the conserved moments (Eq. 2, 4, 20)
//   partials   phi-bar-plus (Eq. 10, 12), least-squares gradient and limiter (Eq. 14-17),
//              upwind reconstruction at the faces (Eq. 11, 13), stored per face and velocity
//   face rec   face moments of the stored values, wall density, face equilibrium (Eq. 18)
//   flux       interface distribution (Eq. 18), flux (Eq. 19), M_i(v) (Eq. 23), M_W (Eq. 27)
//   macro      predicted macroscopic LU-SGS (Eq. 28-31) on i+j hyperplanes (or levels)
//   records*   predicted equilibrium
//   lower      forward micro sweep of Eq. 26 over hyperplanes (or the levels of the sweep
//              order's dependency graph on an unstructured mesh), all velocities in parallel
//   ghost      wall ghost density increment from the forward sweep (Eq. 34-35)
//   upper      backward sweep and update (Eq. 32)
//   raw        raw moments of the new state
//   finalize   closed-domain mass scale, density-change residual, divergence flag
// Nothing here is a dense contraction: every kernel streams [cell][species][v] rows and
// reduces over v with wave shuffles and an LDS tree in fixed order (no atomics).
#include <hip/hip_runtime.h>
#include <math.h>

#include "idugks_internal.hpp"
#include "idugks_kernels.hpp"

namespace idugks {

#define DEV __device__ __forceinline__

// ---------------------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------------------

// The velocity index v = ix nvy + iy split into its 1-D indices without a table: the FP32
// quotient v (1/nvy) is within 1 of v / nvy for every velocity set the library accepts
// (v < 2^24: a relative error of a few 2^-24 on a quotient below 4096), and one step on the
// integer remainder makes it exact.
DEV void split_velocity(int v, int nvy, float rnvy, int &ix, int &iy) {
    ix = (int)((float)v * rnvy);
    iy = v - ix * nvy;
    if (iy < 0) { --ix; iy += nvy; }
    else if (iy >= nvy) { ++ix; iy -= nvy; }
}

// element of a row at a 32-bit byte offset: a wave-uniform row base plus a per-lane
// offset that fits the load's 32-bit offset field
template <class S>
DEV S &at(S *row, unsigned byte_off) {
    return *(S *)((char *)row + byte_off);
}

// Block b of n is dispatched to XCD b % 8; give each XCD a contiguous range of cells so
// that neighbouring cells share an L2.
DEV int xcd_remap(int b, int n) {
    const int x = b & 7, local = b >> 3, per = n >> 3, rem = n & 7;
    return x * per + (x < rem ? x : rem) + local;
}

template <int N>
DEV void wave_sum(double (&a)[N]) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
        double x = a[m];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        a[m] = __shfl(x, 0, 64);  // every lane takes lane 0's (deterministic) sum
    }
}

// x of another lane by a DPP control (quad permutations 0xB1 = lane^1, 0x4E = lane^2; row
// mirror 0x140 = lane 15-i and half-row mirror 0x141 = lane 7-i within 16 lanes), two
// 32-bit moves; every lane of the wave must be active
template <int CTRL>
DEV double dpp_d(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

DEV double readlane_d(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave by DPP (the same value in every lane, fixed order): quad sums, then
// the sums of 8 and of 16 lanes by the mirrors (both partners add the same two values,
// so every lane of a row holds its row's sum), then the four row sums in order.  For
// waves with every lane active; a few register moves instead of six LDS permutes.
template <int N>
DEV void wave_sum_dpp(double (&a)[N]) {
#pragma unroll
    for (int m = 0; m < N; ++m) {
        double x = a[m];
        x += dpp_d<0xB1>(x);
        x += dpp_d<0x4E>(x);
        x += dpp_d<0x141>(x);
        x += dpp_d<0x140>(x);
        a[m] = (readlane_d(x, 0) + readlane_d(x, 16)) + (readlane_d(x, 32) + readlane_d(x, 48));
    }
}

// Sum over the whole block; sh must hold (blockDim/64)*N doubles.  Fixed order.  DPP: the
// wave sums by DPP (every lane of the block active at the call).
template <int N, bool DPP = false>
DEV void block_sum(double (&a)[N], double *sh) {
    if (DPP) wave_sum_dpp<N>(a);
    else wave_sum<N>(a);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < N; ++m) sh[wid * N + m] = a[m];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < N; ++m) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[w * N + m];
        a[m] = s;
    }
    __syncthreads();
}

// Sum over the whole block written to out[0..N) by lanes 0..N-1 (fixed order; no dynamic
// indexing of the register array).  sh must hold (blockDim/64)*N doubles.
template <int N, bool DPP = false>
DEV void block_sum_store(double (&a)[N], double *sh, double *out) {
    if (DPP) wave_sum_dpp<N>(a);
    else wave_sum<N>(a);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int m = 0; m < N; ++m) sh[wid * N + m] = a[m];
    __syncthreads();
    for (int m = threadIdx.x; m < N; m += blockDim.x) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sh[w * N + m];
        out[m] = s;
    }
}

// Block of a velocity-chunked per-cell kernel: ncp = nc rounded up to a multiple of 8
// blocks per chunk of vch velocities, chunk by chunk, so that XCD x takes a contiguous
// range of cells of every chunk.  False for the padding blocks.
DEV bool chunk_block(const Params &p, int vch, int &c, int &v0, int &v1) {
    const int ncp = (p.nc + 7) & ~7, ch = blockIdx.x / ncp;
    c = xcd_remap(blockIdx.x - ch * ncp, ncp);
    v0 = ch * vch;
    v1 = min(p.nv, v0 + vch);
    return c < p.nc;
}

// dst[c][m] = sum over the chunks k (in order) of src[c][k][m], m < n
__global__ __launch_bounds__(256) void k_combine(const double *src, double *dst, int nc, int nch, int n) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nc * n) return;
    const int c = e / n, m = e - c * n;
    double s = 0.0;
    for (int k = 0; k < nch; ++k) s += src[((size_t)c * nch + k) * n + m];
    dst[e] = s;
}

template <class T>
struct RecT {
    T U, V, c0, c1, c2c, c3, kqx, kqy, iRT, KRT, ab, bb;
};

template <class T>
DEV RecT<T> load_rec(const Rec &r) {
    RecT<T> o;
    o.U = (T)r.U; o.V = (T)r.V; o.c0 = (T)r.c0; o.c1 = (T)r.c1; o.c2c = (T)r.c2c;
    o.c3 = (T)r.c3; o.kqx = (T)r.kqx; o.kqy = (T)r.kqy; o.iRT = (T)r.iRT; o.KRT = (T)r.KRT;
    o.ab = (T)r.ab; o.bb = (T)r.bb;
    return o;
}

// Equilibrium pair at velocity (x, y) from a record and the factored Maxwellian E.
template <class T, bool SHAK>
DEV void eq_eval(const RecT<T> &r, T x, T y, T E, T &G, T &H) {
    const T cx = x - r.U, cy = y - r.V, c2 = cx * cx + cy * cy;
    const T base = r.c0 + r.c1 * cx + r.c2c * cy + r.c3 * c2;
    if (SHAK) {
        const T P = r.kqx * cx + r.kqy * cy;
        G = E * (base + P * (c2 * r.iRT - T(4)));
        H = r.KRT * E * (base + P * (c2 * r.iRT - T(2)));
    } else {
        G = E * base;
        H = r.KRT * G;
    }
}

template <class S>
DEV const S *rowp(const Params &p, const void *a, int c, int s) {
    return (const S *)a + ((size_t)c * 2 + s) * p.nvp;
}

// Raw moments of a pair at one velocity, accumulated in double.
template <int NM>
DEV void acc_moments(double *a, double w, double x, double y, double G, double H) {
    const double wG = w * G, wH = w * H, q2 = x * x + y * y;
    a[0] += wG;
    a[1] += wG * x;
    a[2] += wG * y;
    a[3] += 0.5 * (wG * q2 + wH);
    if (NM > 4) {
        a[4] += wG * x * x;
        a[5] += wG * x * y;
        a[6] += wG * y * y;
        a[7] += wG * x * q2;
        a[8 % NM] += wG * y * q2;
        a[9 % NM] += wH;
        a[10 % NM] += wH * x;
        a[11 % NM] += wH * y;
    }
}

// Heat flux about (U, V) from raw moments (q = sum w c (|c|^2 G + H)/2).
DEV void heat_from_raw(const double *m, double U, double V, double &qx, double &qy) {
    const double UU = U * U + V * V;
    const double sx = m[7] - 2.0 * (U * m[4] + V * m[5]) + UU * m[1] - U * (m[4] + m[6]) +
                      2.0 * U * (U * m[1] + V * m[2]) - U * UU * m[0];
    const double sy = m[8] - 2.0 * (U * m[5] + V * m[6]) + UU * m[2] - V * (m[4] + m[6]) +
                      2.0 * V * (U * m[1] + V * m[2]) - V * UU * m[0];
    qx = 0.5 * (sx + m[10] - U * m[9]);
    qy = 0.5 * (sy + m[11] - V * m[9]);
}

// Normal particle speed at a face; velocities tangent to the face within 1e-12 of their
// speed have normal speed exactly 0, so the upwind/tie classification does not depend on
// the rounding (or FMA contraction) of xi.n.  Always evaluated in FP64.
DEV double normal_speed(double x, double y, double nx, double ny) {
    const double un = x * nx + y * ny;
    return fabs(un) <= 1e-12 * (fabs(x) + fabs(y)) ? 0.0 : un;
}

DEV double tau_of(const Params &p, double rho, double RT) {
    return p.mu_ref * pow(2.0 * RT, p.omega) / (rho * RT);
}

// A x = b for a symmetric positive definite A (the moment matrix of the conserved-moment
// basis under a positive weight): elimination without pivoting is stable for it and
// unrolls to straight-line code (no dynamic register indexing)
DEV void solve_spd4(double A[4][4], double b[4]) {
    double ik[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        ik[k] = 1.0 / A[k][k];
#pragma unroll
        for (int r = k + 1; r < 4; ++r) {
            const double m = A[r][k] * ik[k];
#pragma unroll
            for (int c = k + 1; c < 4; ++c) A[r][c] -= m * A[k][c];
            b[r] -= m * b[k];
        }
    }
#pragma unroll
    for (int k = 3; k >= 0; --k) {
        double s = b[k];
#pragma unroll
        for (int c = k + 1; c < 4; ++c) s -= A[k][c] * b[c];
        b[k] = s * ik[k];
    }
}

// Equilibrium record with exact discrete conserved moments, built by one wave.
// G_M = A0 ex(cx) ey(cy) with A0 = rho lambda/pi; the correction lives in the span of
// psi = (1, cx, cy, |c|^2/2) (the same span as the conserved-moment weights) and solves
// A beta = (rho, 0, 0, rho RT) - sum w psi G_M, with A assembled from 1D central moments
// X_p = sum_ix w_ix cx^p ex, Y_p likewise.  Shakhov (monatomic reduced form of Eq. 20):
// dG = k P (|c|^2/RT - 4) G_M, dH = k P K (|c|^2/RT - 2) RT G_M, k = (1-Pr)/(5 p RT),
// P = c.q, projected out of the conserved moments with the same A.
template <class S, bool SHAK>
DEV void build_eq(const Params &p, double rho, double U, double V, double RT, double tau,
                  double qx, double qy, Rec *out, S *tab, int lane, S *outT = nullptr) {
    constexpr int NP = SHAK ? 6 : 5;
    const double lam = 0.5 / RT, A0 = rho * lam / M_PI;
    double X[NP], Y[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) X[k] = Y[k] = 0.0;
    for (int ix = lane; ix < p.nvx; ix += 64) {
        const double cx = p.x1[ix] - U, e = exp(-lam * cx * cx);
        tab[ix] = (S)(A0 * e);
        double t = p.wx1[ix] * e;
#pragma unroll
        for (int k = 0; k < NP; ++k) { X[k] += t; t *= cx; }
    }
    for (int iy = lane; iy < p.nvy; iy += 64) {
        const double cy = p.y1[iy] - V, e = exp(-lam * cy * cy);
        tab[p.nvx + iy] = (S)e;
        double t = p.wy1[iy] * e;
#pragma unroll
        for (int k = 0; k < NP; ++k) { Y[k] += t; t *= cy; }
    }
    wave_sum_dpp<NP>(X);
    wave_sum_dpp<NP>(Y);
    auto m = [&](int a, int b) { return A0 * X[a] * Y[b]; };
    double A[4][4], Ac[4][4], r[4];
    A[0][0] = m(0, 0); A[0][1] = m(1, 0); A[0][2] = m(0, 1); A[0][3] = 0.5 * (m(2, 0) + m(0, 2));
    A[1][1] = m(2, 0); A[1][2] = m(1, 1); A[1][3] = 0.5 * (m(3, 0) + m(1, 2));
    A[2][2] = m(0, 2); A[2][3] = 0.5 * (m(2, 1) + m(0, 3));
    A[3][3] = 0.25 * (m(4, 0) + 2.0 * m(2, 2) + m(0, 4));
    for (int a = 1; a < 4; ++a)
        for (int b = 0; b < a; ++b) A[a][b] = A[b][a];
    r[0] = rho - A[0][0];
    r[1] = -A[0][1];
    r[2] = -A[0][2];
    r[3] = rho * RT - A[0][3];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) Ac[a][b] = A[a][b];
    solve_spd4(Ac, r);
    double kap = 0.0;
    if (SHAK && (qx != 0.0 || qy != 0.0)) {
        kap = (1.0 - p.Pr) / (5.0 * rho * RT * RT);
        const double iRT = 1.0 / RT, e0 = 0.5 * p.K * RT;
        // sum w g P (|c|^2/RT - a) G_M for g = 1, cx, cy, |c|^2/2
        const double g1x = (m(3, 0) + m(1, 2)) * iRT, g1y = (m(2, 1) + m(0, 3)) * iRT;
        double d[4];
        d[0] = qx * (g1x - 4.0 * m(1, 0)) + qy * (g1y - 4.0 * m(0, 1));
        d[1] = qx * ((m(4, 0) + m(2, 2)) * iRT - 4.0 * m(2, 0)) +
               qy * ((m(3, 1) + m(1, 3)) * iRT - 4.0 * m(1, 1));
        d[2] = qx * ((m(3, 1) + m(1, 3)) * iRT - 4.0 * m(1, 1)) +
               qy * ((m(2, 2) + m(0, 4)) * iRT - 4.0 * m(0, 2));
        const double eG = 0.5 * (qx * ((m(5, 0) + 2.0 * m(3, 2) + m(1, 4)) * iRT -
                                       4.0 * (m(3, 0) + m(1, 2))) +
                                 qy * ((m(4, 1) + 2.0 * m(2, 3) + m(0, 5)) * iRT -
                                       4.0 * (m(2, 1) + m(0, 3))));
        const double eH = 0.5 * p.K * RT *
                          (qx * (g1x - 2.0 * m(1, 0)) + qy * (g1y - 2.0 * m(0, 1)));
        d[3] = eG + eH - e0 * d[0];
        for (int a = 0; a < 4; ++a) {
            d[a] *= kap;
            for (int b = 0; b < 4; ++b) Ac[a][b] = A[a][b];
        }
        solve_spd4(Ac, d);
        for (int a = 0; a < 4; ++a) r[a] -= d[a];
    }
    if (lane == 0) {
        Rec o;
        o.rho = rho; o.U = U; o.V = V; o.RT = RT; o.tau = tau; o.qx = qx; o.qy = qy;
        o.c0 = 1.0 + r[0]; o.c1 = r[1]; o.c2c = r[2]; o.c3 = 0.5 * r[3];
        o.kqx = kap * qx; o.kqy = kap * qy; o.iRT = 1.0 / RT; o.KRT = p.K * RT;
        o.ab = (2.0 * tau - p.h) / (2.0 * tau + p.dt);
        o.bb = 3.0 * p.h / (2.0 * tau + p.dt);
        o.alpha = 2.0 * tau / (2.0 * tau + p.h);
        o.rw = 0.0;
        *out = o;
        if (outT) {
            const double v[14] = {o.U, o.V, o.c0, o.c1, o.c2c, o.c3, o.kqx, o.kqy,
                                  o.iRT, o.KRT, o.ab, o.bb, o.alpha, o.rw};
            for (int i = 0; i < 14; ++i) outT[i] = (S)v[i];
        }
    }
}

// A record in the state precision; i is uniform over the wave (scalar loads)
template <class S>
DEV RecT<S> load_recT(const void *base, int i) {
    const S *r = (const S *)base + (size_t)__builtin_amdgcn_readfirstlane(i) * RT_N;
    RecT<S> o;
    o.U = r[0]; o.V = r[1]; o.c0 = r[2]; o.c1 = r[3]; o.c2c = r[4]; o.c3 = r[5];
    o.kqx = r[6]; o.kqy = r[7]; o.iRT = r[8]; o.KRT = r[9]; o.ab = r[10]; o.bb = r[11];
    return o;
}

// ---------------------------------------------------------------------------------------
// raw moments of the stored state, one wave per cell: the block's RW_W cells share the
// velocity set (xi, eta, w), staged into LDS a chunk at a time, so that the vector memory
// path carries only the state; a lane takes the velocities lane, lane + 64, ... in order
constexpr int RW_W = 8, RW_CH = 64 * RW_W;

template <class S, int NM>
__global__ __launch_bounds__(64 * RW_W) void k_raw(Params p) {
    constexpr int PER = RW_CH / 64;  // velocities per lane and chunk
    __shared__ double vx[RW_CH], vy[RW_CH], vw[RW_CH];
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * RW_W + (threadIdx.x >> 6);
    const bool live = c < p.nc;
    const S *G = rowp<S>(p, p.f, live ? c : 0, 0), *H = rowp<S>(p, p.f, live ? c : 0, 1);
    double a[NM];
#pragma unroll
    for (int m = 0; m < NM; ++m) a[m] = 0.0;
    for (int c0 = 0; c0 < p.nv; c0 += RW_CH) {
        const int vt = c0 + threadIdx.x;
        if (vt < p.nv) {
            vx[threadIdx.x] = p.xi[vt];
            vy[threadIdx.x] = p.eta[vt];
            vw[threadIdx.x] = p.w[vt];
        }
        __syncthreads();
        if (live) {
            S gs[PER], hs[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int v = c0 + 64 * u + lane, vc = v < p.nv ? v : 0;
                gs[u] = G[vc];
                hs[u] = H[vc];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int j = 64 * u + lane;
                if (c0 + j < p.nv) acc_moments<NM>(a, vw[j], vx[j], vy[j], (double)gs[u], (double)hs[u]);
            }
        }
        __syncthreads();
    }
    if (!live) return;
    wave_sum_dpp<NM>(a);
    if (lane == 0) {
#pragma unroll
        for (int m = 0; m < NM; ++m) p.raw[(size_t)c * NM_MAX + m] = a[m];
    }
}

// ---------------------------------------------------------------------------------------
// finalize: closed-domain mass scale, residual, divergence flag (one block)
// mode 0: after init/set_state (scale 1, no residual); 1: implicit; 2: explicit.
// The scale is applied lazily: every reader of the stored state multiplies by it.  With an
// FP32 state (round32) those readers multiply in FP32, so the scale is rounded to FP32 here
// and the records, the residual and the moments use that same value; an unrounded FP64 scale
// would leave a collision term (float(s) - s) phi that never vanishes at steady state.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_finalize(Params p, int mode, int round32) {
    __shared__ double sh[16 * 3];
    const int NM = NM_MAX;
    // each thread takes the cells tid, tid + B, ... (B = blockDim), four per pass so that
    // four passes of loads are in flight, and sums them in that order
    const int B = blockDim.x, tid = threadIdx.x;
    double a[1] = {0.0};
    for (int c0 = tid; c0 < p.nc; c0 += 4 * B) {
        double ar[4], rr[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * B, cc = c < p.nc ? c : 0;
            ar[u] = c < p.nc ? p.area[cc] : 0.0;
            rr[u] = p.raw[(size_t)cc * NM];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (c0 + u * B < p.nc) a[0] += ar[u] * rr[u];
    }
    block_sum<1, true>(a, sh);
    const double mass = a[0];
    double s = (mode == 1 && p.closed) ? p.M0 / mass : 1.0;
    if (round32) s = (double)(float)s;
    double b[3] = {0.0, 0.0, 0.0};
    for (int c0 = tid; c0 < p.nc; c0 += 4 * B) {
        double r0[4], r3[4], ro[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int c = c0 + u * B, cc = c < p.nc ? c : 0;
            r0[u] = p.raw[(size_t)cc * NM];
            r3[u] = p.raw[(size_t)cc * NM + 3];
            ro[u] = p.rho_old[cc];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (c0 + u * B >= p.nc) continue;
            const double r = s * r0[u], d = r - ro[u];
            b[0] += d * d;
            b[1] += r * r;
            const double e = s * r3[u];
            if (!(r > 0.0) || !(e > 0.0) || !isfinite(r) || !isfinite(e)) b[2] += 1.0;
            p.rho_old[c0 + u * B] = r;
        }
    }
    block_sum<3, true>(b, sh);
    if (threadIdx.x == 0) {
        p.scal[SC_SCALE] = s;
        p.scal[SC_MASS] = s * mass;
        p.scal[SC_RES] = mode == 0 ? 0.0 : sqrt(b[0] / b[1]);
        p.scal[SC_FLAG] = b[2];
    }
}

// ---------------------------------------------------------------------------------------
// equilibrium records.  which 0: cell records from the scaled raw moments (W^n, q^n);
// which 1: predicted records from W* = W^n + dW with the heat flux of step n.
// One wave per cell, four cells per block.
// ---------------------------------------------------------------------------------------
template <class S, bool SHAK>
__global__ __launch_bounds__(256) void k_records(Params p, int which) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= p.nc) return;
    const int NM = NM_MAX;
    const int TW = p.nvx + p.nvy;
    double W[4], qx = 0.0, qy = 0.0;
    if (which == 0) {
        const double s = p.scal[SC_SCALE];
        const double *m = p.raw + (size_t)c * NM;
        for (int a = 0; a < 4; ++a) W[a] = s * m[a];
        for (int a = 0; a < 4; ++a) p.Wc[(size_t)c * 4 + a] = W[a];
    } else {
        for (int a = 0; a < 4; ++a) W[a] = p.Wc[(size_t)c * 4 + a] + p.dW[(size_t)c * 4 + a];
    }
    const double rho = W[0], U = W[1] / rho, V = W[2] / rho;
    const double RT = (2.0 * W[3] / rho - U * U - V * V) / (p.K + 2);
    const double tau = tau_of(p, rho, RT);
    if (SHAK) {
        if (which == 0) {
            double mm[12];
            const double s = p.scal[SC_SCALE];
            for (int a = 0; a < 12; ++a) mm[a] = s * p.raw[(size_t)c * NM + a];
            double qtx, qty;
            heat_from_raw(mm, U, V, qtx, qty);
            const double t2 = 2.0 * tau;
            qx = t2 * qtx / (t2 + p.dt * p.Pr);
            qy = t2 * qty / (t2 + p.dt * p.Pr);
        } else {
            qx = p.rec[c].qx;
            qy = p.rec[c].qy;
        }
    }
    Rec *out = which == 0 ? p.rec + c : p.recs + c;
    S *tab = (S *)(which == 0 ? p.tab : p.tabs) + (size_t)c * TW;
    build_eq<S, SHAK>(p, rho, U, V, RT, tau, qx, qy, out, tab, lane,
                      which == 0 ? (S *)p.recT + (size_t)c * RT_N : nullptr);
    if (which == 1 && lane == 0) {
        const Rec r = *out;  // written by this lane
        double *o = p.srec + (size_t)p.hp_pos[c] * SR_N;
        o[0] = r.U; o[1] = r.V; o[2] = r.c0; o[3] = r.c1; o[4] = r.c2c; o[5] = r.c3;
        o[6] = r.kqx; o[7] = r.kqy; o[8] = r.iRT; o[9] = r.KRT;
        o[10] = 2.0 * p.area[c] / (2.0 * tau + p.dt);    // collision coefficient (Eq. 26)
        o[11] = p.area[c] / p.dtimp[c] + o[10];           // cell part of the diagonal
        if (p.graph) {  // the level sweeps read it in the state precision
            S *g = (S *)p.growT + (size_t)p.hp_pos[c] * GT_N + GT_REC;
            for (int a = 0; a < SR_N; ++a) g[a] = (S)o[a];
        }
    }
}

// ---------------------------------------------------------------------------------------
// phi-bar-plus (Eq. 10 and Eq. 12 combined) and the limited least-squares gradient
// ---------------------------------------------------------------------------------------
// Loop-invariant data of a face-partial block, staged into LDS once: the records of the
// cell (slot 0) and of its neighbours (slot 1 + side; zeros for a missing neighbour) and
// the cell's side data.  The per-velocity loop then reads only the state and the velocity
// set from memory.
template <class S>
struct PartStage {
    S rec[5][RT_N];
    S ax[4], ay[4], dx[4], dy[4];
    double nx[4], ny[4];
    int nb[4], face[4], type[4], tie[4];
};

// phi-bar-plus = ab phi~ + bb phi_eq of one cell at one velocity (Eq. 10, 12), from its
// record r, factored Maxwellian tb and state row f (a block-uniform base; G at byte
// offset ov, H at oh)
template <class S, class T, bool SHAK>
DEV void barplus(const S *r, const S *tb, int nvx, const S *f, unsigned ov, unsigned oh, int ix, int iy,
                 T x, T y, T sc, T &bG, T &bH) {
    RecT<T> q;
    q.U = r[0]; q.V = r[1]; q.c0 = r[2]; q.c1 = r[3]; q.c2c = r[4]; q.c3 = r[5];
    q.kqx = r[6]; q.kqy = r[7]; q.iRT = r[8]; q.KRT = r[9]; q.ab = r[10]; q.bb = r[11];
    const T E = (T)tb[ix] * (T)tb[nvx + iy];
    T eG, eH;
    eq_eval<T, SHAK>(q, x, y, E, eG, eH);
    const T XG = sc * (T)at(f, ov), XH = sc * (T)at(f, oh);
    bG = q.ab * XG + q.bb * eG;
    bH = q.ab * XH + q.bb * eH;
}

template <class T>
DEV T venkat(T x) { return (x * x + T(2) * x) / (x * x + x + T(2)); }

template <class T>
DEV T limiter_phi(const T *dx, const T *dy, T b0, T bmax, T bmin, T gx, T gy) {
    T phi = T(1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const T d = gx * dx[s] + gy * dy[s];
        T th = T(1);
        if (d > T(0)) th = venkat<T>((bmax - b0) / d);
        else if (d < T(0)) th = venkat<T>((bmin - b0) / d);
        phi = th < phi ? th : phi;
    }
    return phi;
}

// ---------------------------------------------------------------------------------------
// face values: per (cell, velocity) the reconstruction of phi-bar-plus (value, limited
// least-squares gradient, Eq. 13-16), then at each face the cell is upwind of, the
// reconstructed phi-bar stored for the face-record and flux kernels.  TL: the five cells'
// factored Maxwellians are staged into LDS as well (when they fit).
// ---------------------------------------------------------------------------------------
template <class S, bool SHAK, bool LIM, bool TL>
__global__ __launch_bounds__(256) void k_partials(Params p) {
    using T = S;
    extern __shared__ double pdyn[];
    __shared__ PartStage<S> ps;
    int c, v0, v1;
    if (!chunk_block(p, p.nv, c, v0, v1)) return;
    const CellSide *cs = p.cs + 4 * c;
    const int TW = p.nvx + p.nvy, nvx = p.nvx, nvp = p.nvp, tid = threadIdx.x;
    if (tid < 4) {
        const CellSide &q = cs[tid];
        ps.nb[tid] = q.nb; ps.face[tid] = q.face; ps.type[tid] = q.type; ps.tie[tid] = q.tie;
        ps.ax[tid] = (S)q.ax; ps.ay[tid] = (S)q.ay; ps.dx[tid] = (S)q.dx; ps.dy[tid] = (S)q.dy;
        ps.nx[tid] = q.nx; ps.ny[tid] = q.ny;
    }
    if (tid < 5 * RT_N) {
        const int q = tid / RT_N, e = tid - q * RT_N, j = q == 0 ? c : cs[q - 1].nb;
        ps.rec[q][e] = j >= 0 ? ((const S *)p.recT)[(size_t)j * RT_N + e] : S(0);
    }
    // the 1-D velocity abscissae (x then y; xi = x1[ix], eta = y1[iy] exactly) and, when
    // they fit, the five cells' factored Maxwellians
    double *xy = pdyn;
    S *lt = (S *)(xy + TW);
    for (int e = tid; e < TW; e += blockDim.x) xy[e] = e < nvx ? p.x1[e] : p.y1[e - nvx];
    if (TL)
        for (int e = tid; e < 5 * TW; e += blockDim.x) {
            const int q = e / TW, i = e - q * TW, j = q == 0 ? c : cs[q - 1].nb;
            lt[e] = j >= 0 ? ((const S *)p.tab)[(size_t)j * TW + i] : S(0);
        }
    __syncthreads();
    auto tab_of = [&](int q, int j) {
        return TL ? (const S *)lt + q * TW : (const S *)p.tab + (size_t)j * TW;
    };
    const T sc = (T)p.scal[SC_SCALE], h = (T)p.h;
    // the block-uniform side data in scalar registers: neighbours, face types, tie flags
    // and the rows of the neighbours' states and of the faces' values
    int nbs[4], tys[4], tis[4];
    const S *frow[4];
    S *fvrow[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        nbs[s] = __builtin_amdgcn_readfirstlane(ps.nb[s]);
        tys[s] = __builtin_amdgcn_readfirstlane(ps.type[s]);
        tis[s] = __builtin_amdgcn_readfirstlane(ps.tie[s]);
        frow[s] = (const S *)p.f + (size_t)(nbs[s] < 0 ? c : nbs[s]) * 2 * nvp;
        fvrow[s] = (S *)p.fv + (size_t)__builtin_amdgcn_readfirstlane(ps.face[s]) * 2 * nvp;
    }
    const S *frow0 = (const S *)p.f + (size_t)c * 2 * nvp;
    const int nvy = p.nvy;
    const float rnvy = 1.0f / (float)nvy;
    for (int v = v0 + tid; v < v1; v += blockDim.x) {
        // keep the staged records in LDS, read per iteration (hoisted, the five records
        // would hold about 120 registers and halve the occupancy); emits no code
        asm volatile("" ::: "memory");
        int ix, iy;
        split_velocity(v, nvy, rnvy, ix, iy);
        const double xd = xy[ix], yd = xy[nvx + iy];
        const T x = (T)xd, y = (T)yd;
        // rows are a block-uniform base plus the lane's 32-bit byte offset
        const unsigned ov = (unsigned)v * sizeof(S), oh = (unsigned)(nvp + v) * sizeof(S);
        T bG, bH;
        barplus<S, T, SHAK>(ps.rec[0], tab_of(0, c), nvx, frow0, ov, oh, ix, iy, x, y, sc, bG, bH);
        T gxG = T(0), gyG = T(0), gxH = T(0), gyH = T(0);
        T mxG = bG, mnG = bG, mxH = bH, mnH = bH;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int n = nbs[s];
            if (n < 0) continue;
            T nG, nH;
            barplus<S, T, SHAK>(ps.rec[1 + s], tab_of(1 + s, n), nvx, frow[s], ov, oh, ix, iy, x, y, sc, nG, nH);
            const T ax = ps.ax[s], ay = ps.ay[s], dG = nG - bG, dH = nH - bH;
            gxG += ax * dG; gyG += ay * dG; gxH += ax * dH; gyH += ay * dH;
            if (LIM) {
                mxG = nG > mxG ? nG : mxG; mnG = nG < mnG ? nG : mnG;
                mxH = nH > mxH ? nH : mxH; mnH = nH < mnH ? nH : mnH;
            }
        }
        if (LIM) {
            const T pG = limiter_phi<T>(ps.dx, ps.dy, bG, mxG, mnG, gxG, gyG);
            const T pH = limiter_phi<T>(ps.dx, ps.dy, bH, mxH, mnH, gxH, gyH);
            gxG *= pG; gyG *= pG; gxH *= pH; gyH *= pH;
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (tys[s] == FT_SELF) continue;
            const double un = normal_speed(xd, yd, ps.nx[s], ps.ny[s]);
            if (!(un > 0.0 || (un == 0.0 && tis[s]))) continue;
            const T rx = ps.dx[s] - h * x, ry = ps.dy[s] - h * y;
            at(fvrow[s], ov) = (S)(bG + gxG * rx + gyG * ry);
            at(fvrow[s], oh) = (S)(bH + gxH * rx + gyH * ry);
        }
    }
}

// ---------------------------------------------------------------------------------------
// face records: moments of phi-bar at every face, wall density (zero normal mass flux),
// face equilibrium (heat flux 2 tau qbar / (2 tau + h Pr)).  One wave per face.
// ---------------------------------------------------------------------------------------
// The velocity set (xi, eta, w) is staged into LDS a chunk at a time and shared by the
// block's FR_W faces, so that the vector memory path carries only the face values.
constexpr int FR_W = 8, FR_CH = 64 * FR_W;

template <class S, bool SHAK>
__global__ __launch_bounds__(64 * FR_W) void k_face_records(Params p) {
    constexpr int NM = SHAK ? NM_SHAKHOV : NM_BGK;
    constexpr int PER = FR_CH / 64;  // velocities per lane and chunk
    __shared__ double vx[FR_CH], vy[FR_CH], vw[FR_CH];
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * FR_W + (threadIdx.x >> 6);
    Face F{};
    CellSide cL{};
    bool live = false;
    if (k < p.nf) {
        F = p.faces[k];
        live = F.type != FT_SELF;
        // (a face without flux may have no cell: L = -1 on an unused periodic face)
        if (live) cL = p.cs[4 * F.L + F.sL];
    }
    // moments of the stored face values: every velocity at an interior face, the outflow
    // half (the interior cell upwind) at a boundary face; a lane takes the velocities
    // lane, lane + 64, ... in order
    const S *fvG = (const S *)p.fv + (size_t)(live ? k : 0) * 2 * p.nvp, *fvH = fvG + p.nvp;
    double m[NM];
    for (int i = 0; i < NM; ++i) m[i] = 0.0;
    for (int c0 = 0; c0 < p.nv; c0 += FR_CH) {
        const int vt = c0 + threadIdx.x;
        if (vt < p.nv) {
            vx[threadIdx.x] = p.xi[vt];
            vy[threadIdx.x] = p.eta[vt];
            vw[threadIdx.x] = p.w[vt];
        }
        __syncthreads();
        if (live) {
            S gs[PER], hs[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int v = c0 + 64 * u + lane, vc = v < p.nv ? v : 0;
                gs[u] = fvG[vc];
                hs[u] = fvH[vc];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int j = 64 * u + lane;
                bool use = c0 + j < p.nv;
                const double xs = vx[j], ys = vy[j];
                if (F.type != FT_INTERIOR) {
                    const double un = normal_speed(xs, ys, cL.nx, cL.ny);
                    use = use && (un > 0.0 || (un == 0.0 && cL.tie));
                }
                // (the inflow half of a boundary face is never written: skip it, do not weight it)
                if (use) acc_moments<NM>(m, vw[j], xs, ys, (double)gs[u], (double)hs[u]);
            }
        }
        __syncthreads();
    }
    if (!live) return;
    wave_sum_dpp<NM>(m);
    double rw = 0.0;
    if (F.type != FT_INTERIOR) {
        const double *b = p.bhalf + (size_t)k * NM_MAX;
        if (F.type == FT_WALL) rw = -(F.nx * m[1] + F.ny * m[2]) / p.wden[k];
        const double sc = F.type == FT_WALL ? rw : 1.0;
        for (int i = 0; i < NM; ++i) m[i] += sc * b[i];
    }
    const double rho = m[0], U = m[1] / rho, V = m[2] / rho;
    const double RT = (2.0 * m[3] / rho - U * U - V * V) / (p.K + 2);
    const double tau = tau_of(p, rho, RT);
    double qx = 0.0, qy = 0.0;
    if (SHAK) {
        double qbx, qby;
        heat_from_raw(m, U, V, qbx, qby);
        const double t2 = 2.0 * tau;
        qx = t2 * qbx / (t2 + p.h * p.Pr);
        qy = t2 * qby / (t2 + p.h * p.Pr);
    }
    S *tab = (S *)p.tabf + (size_t)k * (p.nvx + p.nvy);
    build_eq<S, SHAK>(p, rho, U, V, RT, tau, qx, qy, p.recf + k, tab, lane, (S *)p.recfT + (size_t)k * RT_N);
    if (lane == 0) {
        p.recf[k].rw = rw;
        ((S *)p.recfT)[(size_t)k * RT_N + 13] = (S)rw;
    }
}

// ---------------------------------------------------------------------------------------
// Everything of Eq. 30-31 that does not depend on the increments, per cell: implicit time
// step and inverse diagonal (a wall face carries its whole lambda S: mirrored ghost), stored
// as the cell's macro row in i+j hyperplane order: M_W, 1/D, packed side codes, the cell's
// W and sound speed, per side nx, ny, S.  The sweep takes a neighbour's W and sound speed
// from the neighbour's own row (through LDS) and forms lambda_j there.
// ---------------------------------------------------------------------------------------
DEV void macro_row(const Params &p, int c, const double mw[4]) {
    const CellSide *cs = p.cs + 4 * c;
    double *m = p.mh + (size_t)p.hp_pos[c] * MH_N;
    const double U = p.rec[c].U, V = p.rec[c].V, C = sqrt(p.gam * p.rec[c].RT);
    double ls = 0.0, lw = 0.0;
    int codes = 0;
    for (int s = 0; s < 4; ++s) {
        if (cs[s].type != FT_SELF && cs[s].nb >= 0)
            codes |= (cs[s].nb < c ? SG_LOWER : SG_UPPER) << (MH_CODE_BITS * s);
        double *ms = m + MH_SIDE + MH_SN * s;
        ms[0] = cs[s].nx; ms[1] = cs[s].ny; ms[2] = cs[s].S;
        if (cs[s].type == FT_SELF) continue;
        const double l = (fabs(U * cs[s].nx + V * cs[s].ny) + C) * cs[s].S;
        ls += l;
        if (cs[s].type == FT_WALL) lw += l;
    }
    const double dti = p.cfl_imp * p.area[c] / ls;
    p.dtimp[c] = dti;
    for (int a = 0; a < 4; ++a) {
        m[a] = mw[a];
        m[6 + a] = p.Wc[(size_t)c * 4 + a];
    }
    m[4] = 1.0 / (p.area[c] / dti + 0.5 * ls + 0.5 * lw);
    m[5] = (double)codes;
    m[10] = C;
}

// ---------------------------------------------------------------------------------------
// flux: M_i(v) = -sum_k S (xi.n_out) phi_k (Eq. 18, 19, 23) and M_W = sum w psi M (Eq. 27);
// with a single velocity chunk the block holds its cell's whole M_W and, in an implicit
// step, writes the cell's macro row as well (no separate launch)
// ---------------------------------------------------------------------------------------
// Loop-invariant data of a flux block, staged into LDS once: per side the face record
// (with alpha and the wall density) and the side data.
template <class S>
struct FluxStage {
    S rec[4][RT_N];
    S nxT[4], nyT[4], ST[4];
    double nx[4], ny[4];
    int face[4], type[4], tie[4], wside[4];
};

template <class S, bool SHAK, bool TL, bool PREP>
__global__ __launch_bounds__(256) void k_flux(Params p) {
    using T = S;
    extern __shared__ double fdyn[];
    __shared__ FluxStage<S> fs;
    __shared__ double sh[4 * 4];
    int c, v0, v1;
    if (!chunk_block(p, p.vch, c, v0, v1)) return;
    const CellSide *cs = p.cs + 4 * c;
    const int TW = p.nvx + p.nvy, nvx = p.nvx, nvp = p.nvp, tid = threadIdx.x;
    if (tid < 4) {
        const CellSide &q = cs[tid];
        fs.face[tid] = q.face; fs.type[tid] = q.type; fs.tie[tid] = q.tie; fs.wside[tid] = q.wside;
        fs.nx[tid] = q.nx; fs.ny[tid] = q.ny;
        fs.nxT[tid] = (S)q.nx; fs.nyT[tid] = (S)q.ny; fs.ST[tid] = (S)q.S;
    }
    if (tid < 4 * RT_N) {
        const int q = tid / RT_N, e = tid - q * RT_N;
        fs.rec[q][e] = cs[q].type == FT_SELF ? S(0) : ((const S *)p.recfT)[(size_t)cs[q].face * RT_N + e];
    }
    // the 1-D velocity abscissae and weights (x then y; xi = x1[ix], eta = y1[iy] and
    // w = wx1[ix] wy1[iy] exactly) and, when they fit, the four faces' factored Maxwellians
    double *xy = fdyn, *wxy = fdyn + TW;
    S *lt = (S *)(fdyn + 2 * TW);
    for (int e = tid; e < TW; e += blockDim.x) {
        xy[e] = e < nvx ? p.x1[e] : p.y1[e - nvx];
        wxy[e] = e < nvx ? p.wx1[e] : p.wy1[e - nvx];
    }
    if (TL)
        for (int e = tid; e < 4 * TW; e += blockDim.x) {
            const int q = e / TW, i = e - q * TW;
            lt[e] = cs[q].type == FT_SELF ? S(0) : ((const S *)p.tabf)[(size_t)cs[q].face * TW + i];
        }
    __syncthreads();
    S *MG = (S *)p.d1 + ((size_t)c * 2) * nvp, *MH = MG + nvp;
    double mw[4] = {0.0, 0.0, 0.0, 0.0};
    // the block-uniform side data in scalar registers: face types, tie flags, the rows of
    // the faces' values and of the wall Maxwellians, the wall K RT
    int tys[4], tis[4];
    const S *fvrow[4];
    const double *gwrow[4];
    T wkrt[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        tys[s] = __builtin_amdgcn_readfirstlane(fs.type[s]);
        tis[s] = __builtin_amdgcn_readfirstlane(fs.tie[s]);
        fvrow[s] = (const S *)p.fv + (size_t)__builtin_amdgcn_readfirstlane(fs.face[s]) * 2 * nvp;
        const int ws = tys[s] == FT_WALL ? __builtin_amdgcn_readfirstlane(fs.wside[s]) : 0;
        gwrow[s] = p.gw + (size_t)ws * nvp;
        wkrt[s] = (T)p.wKRT[ws];
    }
    const int nvy = p.nvy;
    const float rnvy = 1.0f / (float)nvy;
    // two velocities per lane and iteration (v and v + blockDim), which share each side's
    // record read from LDS
    constexpr int VU = 2;
    const int B = blockDim.x;
    for (int v00 = v0 + tid; v00 < v1; v00 += VU * B) {
        // keep the staged records in LDS, read per iteration (emits no code)
        asm volatile("" ::: "memory");
        int vv[VU], ix[VU], iy[VU];
        bool ok[VU];
        double xd[VU], yd[VU];
        T x[VU], y[VU];
        unsigned ov[VU], oh[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) {
            ok[u] = v00 + u * B < v1;
            vv[u] = ok[u] ? v00 + u * B : v00;
            split_velocity(vv[u], nvy, rnvy, ix[u], iy[u]);
            xd[u] = xy[ix[u]];
            yd[u] = xy[nvx + iy[u]];
            x[u] = (T)xd[u];
            y[u] = (T)yd[u];
            ov[u] = (unsigned)vv[u] * sizeof(S);
            oh[u] = (unsigned)(nvp + vv[u]) * sizeof(S);
        }
        // every side's stored face values first (they depend only on the velocity; a
        // boundary face's value is read whichever way the velocity points and used only
        // where this cell is upwind), then the classification and the arithmetic
        T fG[VU][4], fH[VU][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (tys[s] == FT_SELF) continue;
#pragma unroll
            for (int u = 0; u < VU; ++u) {
                fG[u][s] = at(fvrow[s], ov[u]);
                fH[u][s] = at(fvrow[s], oh[u]);
            }
        }
        T un[VU][4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int type = tys[s];
            if (type == FT_SELF) continue;
#pragma unroll
            for (int u = 0; u < VU; ++u) {
                // an interior face's value is the stored reconstruction whichever cell is
                // upwind, so only boundary faces classify the velocity (with the tie rule,
                // in FP64); tangent velocities carry no flux either way
                if (type == FT_INTERIOR) {
                    un[u][s] = x[u] * fs.nxT[s] + y[u] * fs.nyT[s];
                    continue;
                }
                const double und = normal_speed(xd[u], yd[u], fs.nx[s], fs.ny[s]);
                un[u][s] = (T)und;
                if (und > 0.0 || (und == 0.0 && tis[s])) continue;  // reconstructed by this cell
                if (type == FT_WALL) {
                    const T rw = fs.rec[s][13];
                    const T g = (T)gwrow[s][vv[u]];
                    fG[u][s] = rw * g;
                    fH[u][s] = rw * wkrt[s] * g;
                } else {
                    fG[u][s] = (T)p.ginf[vv[u]];
                    fH[u][s] = (T)p.hinf[vv[u]];
                }
            }
        }
        T accG[VU], accH[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) accG[u] = accH[u] = T(0);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            if (tys[s] == FT_SELF) continue;
            const S *r = fs.rec[s];
            RecT<T> rf;
            rf.U = r[0]; rf.V = r[1]; rf.c0 = r[2]; rf.c1 = r[3]; rf.c2c = r[4]; rf.c3 = r[5];
            rf.kqx = r[6]; rf.kqy = r[7]; rf.iRT = r[8]; rf.KRT = r[9]; rf.ab = r[10]; rf.bb = r[11];
            const T al = r[12], ST = fs.ST[s];
            const S *tf = TL ? (const S *)lt + s * TW : (const S *)p.tabf + (size_t)__builtin_amdgcn_readfirstlane(fs.face[s]) * TW;
#pragma unroll
            for (int u = 0; u < VU; ++u) {
                T eG, eH;
                eq_eval<T, SHAK>(rf, x[u], y[u], (T)tf[ix[u]] * (T)tf[nvx + iy[u]], eG, eH);
                const T pG = al * fG[u][s] + (T(1) - al) * eG, pH = al * fH[u][s] + (T(1) - al) * eH;
                const T fl = ST * un[u][s];
                accG[u] -= fl * pG;
                accH[u] -= fl * pH;
            }
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
            if (!ok[u]) continue;
            MG[vv[u]] = (S)accG[u];
            MH[vv[u]] = (S)accH[u];
            const double wv = wxy[ix[u]] * wxy[nvx + iy[u]], dG = (double)accG[u];
            mw[0] += wv * dG;
            mw[1] += wv * xd[u] * dG;
            mw[2] += wv * yd[u] * dG;
            mw[3] += 0.5 * wv * ((xd[u] * xd[u] + yd[u] * yd[u]) * dG + (double)accH[u]);
        }
    }
    if (PREP) {
        block_sum<4, true>(mw, sh);
        if (tid == 0) {
#pragma unroll
            for (int a = 0; a < 4; ++a) p.MW[(size_t)c * 4 + a] = mw[a];
            macro_row(p, c, mw);
        }
    } else {
        block_sum_store<4, true>(mw, sh, p.nch > 1 ? p.MWc + ((size_t)c * p.nch + v0 / p.vch) * 4 : p.MW + (size_t)c * 4);
    }
}

// ---------------------------------------------------------------------------------------
// predicted macroscopic step: LU-SGS of Eq. 29-31 (Rusanov split, matrix-free flux
// differences, mirrored wall ghost) over i+j hyperplanes in one block
// ---------------------------------------------------------------------------------------
// 1/x within about an ulp for a positive normal x (a density, a diagonal): the hardware
// estimate refined by Newton steps, a shorter dependency chain than a correctly rounded
// division
DEV float rcp_nr(float x) {
    const float r = __builtin_amdgcn_rcpf(x);
    return fmaf(r, fmaf(-x, r, 1.0f), r);
}

DEV double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Euler flux through a face of unit normal n of the state W = (rho, rho U, rho V, rho E);
// ik2 = 1/(K+2), so that p = (2 rho E - rho |U|^2)/(K+2)
DEV double euler_flux_n(const double W[4], double nx, double ny, double ik2, double F[4]) {
    const double ir = rcp_nr(W[0]);
    const double U = W[1] * ir, V = W[2] * ir;
    const double pr = (2.0 * W[3] - W[0] * (U * U + V * V)) * ik2;
    const double un = U * nx + V * ny;
    F[0] = W[0] * un;
    F[1] = W[1] * un + pr * nx;
    F[2] = W[2] * un + pr * ny;
    F[3] = (W[3] + pr) * un;
    return un;
}

// The macro row of cell c from its M_W (the rest of Eq. 30-31 that does not depend on the
// increments is computed here).
__global__ __launch_bounds__(256) void k_macro_prep(Params p) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.nc) return;
    double mw[4];
    for (int a = 0; a < 4; ++a) mw[a] = p.MW[(size_t)c * 4 + a];
    macro_row(p, c, mw);
}

// All data exchanged inside the sweep kernels goes through LDS, so their barrier orders
// LDS only: global loads issued for later hyperplanes stay in flight across it.
DEV void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

DEV void hp_bounds(int s, int ni, int nj, int &lo, int &hi) {
    lo = s - nj + 1 > 0 ? s - nj + 1 : 0;
    hi = s < ni - 1 ? s : ni - 1;
}

// Both sweep kernels split their block into compute waves and staging waves.  The
// staging waves copy the per-cell rows of hyperplane t+1 (contiguous in hyperplane order)
// from HBM into one of two LDS buffers during step t, having issued the loads a fixed
// number of steps earlier (SDEPTH in the micro sweeps, MD in the macro sweep); the compute
// waves read only LDS for per-cell data.  A wave's loads complete in order, so keeping
// these copies out of the compute waves lets the compute waves' own prefetches run ahead
// without waiting for them.
constexpr int SDEPTH = 4;  // hyperplanes of staging loads in flight (micro sweeps)
static_assert(SG_UPPER < 1 << MH_CODE_BITS, "side codes must fit their field of the macro row");
// a staging wave reads up to 64 x 16 values past the first row of a hyperplane, the last of
// which starts at row nc - 1: the min(ni, nj) + HP_SPARE spare rows of the staged arrays cover it
static_assert((HP_SPARE + 1) * MH_N >= 64 * 16, "macro staging reads past the spare rows");

// x of the lane (lane ^ 1) or (lane ^ 2) of the same quad: a DPP quad permutation
// (CTRL 0xB1 = [1,0,3,2], 0x4E = [2,3,0,1]), two 32-bit moves in registers
template <int CTRL>
DEV double quad_swap(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int N>
DEV void stage_store(const double (&reg)[N], double *dst, int n, int sl, int nsl) {
#pragma unroll
    for (int q = 0; q < N; ++q) {
        const int e = sl + q * nsl;
        if (e < n) dst[e] = reg[q];
    }
}

// Macro LU-SGS sweeps (Eq. 29-31) over i+j hyperplanes in one block.  Waves below nct
// compute, LPC lanes per cell of a hyperplane, lane q taking the sides q NS .. q NS + NS - 1
// (NS = 4 / LPC: with two lanes, one has the i sides and the other the j sides, so each
// has one coupled side per direction in the interior):
//   r -= 1/2 S (F_n(W_j + dW_j) - F_n(W_j) - lambda_j dW_j),  lambda_j = |U_j.n| + c_j
// over the lower (forward) or upper (backward) neighbours; the lanes of a cell sum their
// parts by quad permutations, each keeping the components it finishes (q, q + LPC, ...).
// LDS holds, per cell of the previous hyperplane, its increment, W and sound speed (fronts
// of MF values, with a padding cell at each end), the same for the cells next to a periodic
// seam (wI: column i = 0 / ni-1, wJ: row j = 0 / nj-1, the only non-adjacent neighbours;
// allocated and written for periodic directions only),
// the staged rows of the current and the next hyperplane and the increments of the last
// two hyperplanes on their way to HBM.  The forward sweep's dW* go into the first four
// values of each cell's row, which the backward sweep stages back.  The staging waves keep
// MD hyperplanes of SPWM values per lane in flight and write the increments out one step
// later (the compute waves only touch LDS); one CU's load latency, not its bandwidth,
// bounds the staging, so the depth matters more than the lane count.
constexpr int MF = 9;  // front entry: dW [4], W [4], c

template <int LPC, int SPWM, int MD>
__global__ __launch_bounds__(1024) void k_macro_sweep(Params p, int nct) {
    extern __shared__ double lds[];
    const int ni = p.ni, nj = p.nj, nh = ni + nj - 1, L = ni < nj ? ni : nj;
    // LDS offsets (in doubles): the two fronts, the seam copies, the staged rows, the
    // out-buffers; the front of the previous hyperplane is A after an even number of steps
    const int oA = MF, oB = oA + MF * (ni + 1), oI = oB + MF * (ni + 1);
    const int oJ = oI + (p.per_i ? MF * nj : 0), oE = oJ + (p.per_j ? MF * ni : 0);
    double *st0 = lds + oE, *st1 = st0 + (size_t)L * MH_N;
    double *ob0 = st1 + (size_t)L * MH_N, *ob1 = ob0 + 4 * L;  // out-buffers by step parity
    int *hpo = (int *)(ob1 + 4 * L);
    for (int h = threadIdx.x; h <= nh; h += blockDim.x) hpo[h] = p.hp_off[h];
    for (int e = threadIdx.x; e < oE; e += blockDim.x) lds[e] = 0.0;
    __syncthreads();
    const double ik2 = 1.0 / (p.K + 2);
    // Both roles run the same number of barriers: one after the prologue and one per
    // hyperplane in each direction, plus the block-wide one between the directions.
    if ((int)threadIdx.x >= nct) {
        const int sl = (int)threadIdx.x - nct, nsl = (int)blockDim.x - nct;
        // register set k holds the row values of a hyperplane t with t % MD == k; the
        // loads of hyperplane t+1 are issued MD steps before it is staged
        double reg[MD][SPWM];
        // rows past the hyperplane are read (spare rows at the end of mh) but never staged
        auto issue = [&](double (&rg)[SPWM], int h) {
            const double *src = p.mh + (size_t)hpo[h] * MH_N + sl;
#pragma unroll
            for (int q = 0; q < SPWM; ++q) rg[q] = src[q * nsl];
        };
        for (int dir = 0; dir < 2; ++dir) {
            const bool upper = dir == 1;
            auto hp = [&](int t) { return upper ? nh - 1 - t : t; };
            auto hcl = [&](int t) { return hp(t < nh ? t : nh - 1); };  // repeated rows are not staged
            auto cells = [&](int t) { return hpo[hp(t) + 1] - hpo[hp(t)]; };
            // the increments of hyperplane t, left in the out-buffer of its parity by the
            // compute waves during step t, go to HBM during step t+1: dW* into the first
            // four values of the rows (forward), dW (backward)
            auto flush = [&](int t) {
                const int h = hp(t), n = 4 * cells(t);
                const double *ob = t & 1 ? ob1 : ob0;
                int lo, hi;
                hp_bounds(h, ni, nj, lo, hi);
                for (int e = sl; e < n; e += nsl) {
                    const int kk = e >> 2, a = e & 3;
                    if (upper) p.dW[(size_t)(lo + kk + (h - lo - kk) * ni) * 4 + a] = ob[e];
                    else p.mh[(size_t)(hpo[h] + kk) * MH_N + a] = ob[e];
                }
            };
            issue(reg[0], hcl(0));
            stage_store(reg[0], st0, cells(0) * MH_N, sl, nsl);
#pragma unroll
            for (int d = 1; d <= MD; ++d) issue(reg[d % MD], hcl(d));
            lds_barrier();
            int t0 = 0;
            for (; t0 + MD <= nh; t0 += MD) {
#pragma unroll
                for (int d = 0; d < MD; ++d) {
                    const int t = t0 + d;
                    if (t + 1 < nh) stage_store(reg[(d + 1) % MD], (t + 1) & 1 ? st1 : st0, cells(t + 1) * MH_N, sl, nsl);
                    issue(reg[(d + 1) % MD], hcl(t + 1 + MD));
                    if (t > 0) flush(t - 1);
                    lds_barrier();
                }
            }
#pragma unroll
            for (int d = 0; d < MD - 1; ++d) {
                const int t = t0 + d;
                if (t < nh) {
                    if (t + 1 < nh) stage_store(reg[(d + 1) % MD], (t + 1) & 1 ? st1 : st0, cells(t + 1) * MH_N, sl, nsl);
                    if (t > 0) flush(t - 1);
                    lds_barrier();
                }
            }
            flush(nh - 1);
            __syncthreads();
        }
        return;
    }
    constexpr int NS = 4 / LPC;  // sides (and components) per lane
    const int k = (int)threadIdx.x / LPC, q = (int)threadIdx.x % LPC;
    int T = 0;  // steps so far
    for (int dir = 0; dir < 2; ++dir) {
        const bool upper = dir == 1;
        const int need = upper ? SG_UPPER : SG_LOWER;
        // The one neighbour each side of this lane can couple to in this direction (sides
        // i-, i+, j-, j+): forward front[i-1], wI[j], front[i], wJ[i]; backward wI[j],
        // front[i+1], wJ[i], front[i].  Per side: whether it is a front entry, the offset of
        // its index, and the seam copy (indexed by j for wI, i for wJ).  A seam side of a
        // direction that is not periodic has no coupling; it reads entry 0 of front A.
        bool isf[NS], usej[NS], idx[NS];
        int dl[NS], sb[NS];
#pragma unroll
        for (int u = 0; u < NS; ++u) {
            const int sd = q * NS + u;
            isf[u] = (sd & 1) == (upper ? 1 : 0);
            usej[u] = !isf[u] && sd < 2;
            dl[u] = isf[u] && sd < 2 ? (upper ? 1 : -1) : 0;
            const bool per = sd < 2 ? p.per_i : p.per_j;
            idx[u] = isf[u] || per;
            sb[u] = per ? (sd < 2 ? oI : oJ) : oA;
        }
        lds_barrier();
        for (int t = 0; t < nh; ++t, ++T) {
            const int s = upper ? nh - 1 - t : t;
            int lo, hi;
            hp_bounds(s, ni, nj, lo, hi);
            const int cur = T & 1 ? oB : oA, nxt = T & 1 ? oA : oB;
            // idle lanes (past the hyperplane's end) read the data of its first cell
            const bool live = lo + k <= hi;
            const int i = live ? lo + k : lo, j = s - i;
            const double *m = (t & 1 ? st1 : st0) + (size_t)(live ? k : 0) * MH_N;
            // this lane's row values and its neighbours' front entries: one batch of LDS reads
            const int codes = (int)m[5];
            double ms[NS][MH_SN], mr[NS], wo[NS], nb[NS][MF];
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int o = (isf[u] ? cur : sb[u]) + (idx[u] ? MF * (usej[u] ? j : i + dl[u]) : 0);
#pragma unroll
                for (int e = 0; e < MF; ++e) nb[u][e] = lds[o + e];
                mr[u] = m[q + u * LPC];      // component q + u LPC of M_W, which this lane finishes
                wo[u] = m[6 + q + u * LPC];  // and of the cell's own W
#pragma unroll
                for (int e = 0; e < MH_SN; ++e) ms[u][e] = m[MH_SIDE + MH_SN * (q * NS + u) + e];
            }
            const double iD = m[4], co = m[10];
            double r[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int u = 0; u < NS; ++u) {
                const int sd = q * NS + u;
                if (!(live && ((codes >> (MH_CODE_BITS * sd)) & need))) continue;
                const double *dW = nb[u], *Wj = nb[u] + 4;
                double Wn[4], F0[4], F1[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) Wn[a] = Wj[a] + dW[a];
                const double lam = fabs(euler_flux_n(Wj, ms[u][0], ms[u][1], ik2, F0)) + nb[u][8];
                euler_flux_n(Wn, ms[u][0], ms[u][1], ik2, F1);
                const double hS = 0.5 * ms[u][2];
#pragma unroll
                for (int a = 0; a < 4; ++a) r[a] += hS * (F1[a] - F0[a] - lam * dW[a]);
            }
            // Sum over the cell's lanes, each lane keeping only the components it finishes
            // (q + u LPC): exchange with lane q^1 the two components of the other parity,
            // then (four lanes) with lane q^2 the one of the other half.
            const bool p1 = q & 1;
            const double c0 = (p1 ? r[1] : r[0]) + quad_swap<0xB1>(p1 ? r[0] : r[1]);
            const double c1 = (p1 ? r[3] : r[2]) + quad_swap<0xB1>(p1 ? r[2] : r[3]);
            double ra[NS];
            if (LPC == 4) {
                const bool h1 = q & 2;
                ra[0] = (h1 ? c1 : c0) + quad_swap<0x4E>(h1 ? c0 : c1);
            } else {
                ra[0] = c0;
                ra[NS - 1] = c1;
            }
            if (live) {
                const bool sI = p.per_i && i == (upper ? ni - 1 : 0), sJ = p.per_j && j == (upper ? nj - 1 : 0);
#pragma unroll
                for (int u = 0; u < NS; ++u) {
                    const int a = q + u * LPC;
                    // forward dW* = (M_W - r)/D, backward dW = dW* - r/D
                    const double d = upper ? mr[u] - ra[u] * iD : (mr[u] - ra[u]) * iD;
                    (t & 1 ? ob1 : ob0)[4 * k + a] = d;  // to HBM by the staging waves
                    lds[nxt + MF * i + a] = d;
                    lds[nxt + MF * i + 4 + a] = wo[u];
                    if (sI) { lds[oI + MF * j + a] = d; lds[oI + MF * j + 4 + a] = wo[u]; }
                    if (sJ) { lds[oJ + MF * i + a] = d; lds[oJ + MF * i + 4 + a] = wo[u]; }
                }
                if (q == 0) {
                    lds[nxt + MF * i + 8] = co;
                    if (sI) lds[oI + MF * j + 8] = co;
                    if (sJ) lds[oJ + MF * i + 8] = co;
                }
            }
            lds_barrier();
        }
        // the forward sweep's row writes must be visible to the backward staging loads
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------------------
// point relaxation of the macroscopic system (L + D + U) dW = M_W (the paper's second
// prediction scheme, named in its conclusions without a formula): sweep 0 is the
// point-implicit step dW = D^-1 M_W, every later sweep a Jacobi sweep
//   dW_i <- D_i^-1 (M_W,i - sum_j 1/2 S (F_n(W_j + dW_j) - F_n(W_j) - lambda_j dW_j))
// over all neighbours j with the previous sweep's dW.  One thread per cell; the cell's
// M_W, 1/D and side geometry and the neighbours' W and sound speed come from the macro
// rows (hyperplane order), the increments in and out in cell order.
// ---------------------------------------------------------------------------------------
template <bool FIRST>
__global__ __launch_bounds__(256) void k_macro_relax(Params p, const double *dWin, double *dWout) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.nc) return;
    const double *m = p.mh + (size_t)p.hp_pos[c] * MH_N;
    double r[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) r[a] = m[a];
    if (!FIRST) {
        const CellSide *cs = p.cs + 4 * c;
        const double ik2 = 1.0 / (p.K + 2);
        for (int sd = 0; sd < 4; ++sd) {
            const int j = cs[sd].nb;
            if (cs[sd].type == FT_SELF || j < 0) continue;
            const double *mj = p.mh + (size_t)p.hp_pos[j] * MH_N, *dWj = dWin + (size_t)j * 4;
            const double nx = m[MH_SIDE + MH_SN * sd], ny = m[MH_SIDE + MH_SN * sd + 1];
            const double hS = 0.5 * m[MH_SIDE + MH_SN * sd + 2];
            double Wj[4], Wn[4], F0[4], F1[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                Wj[a] = mj[6 + a];
                Wn[a] = Wj[a] + dWj[a];
            }
            const double lam = fabs(euler_flux_n(Wj, nx, ny, ik2, F0)) + mj[10];
            euler_flux_n(Wn, nx, ny, ik2, F1);
#pragma unroll
            for (int a = 0; a < 4; ++a) r[a] -= hS * (F1[a] - F0[a] - lam * dWj[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) dWout[(size_t)c * 4 + a] = r[a] * m[4];
}

// ---------------------------------------------------------------------------------------
// micro LU-SGS sweeps (Eq. 24-26) over i+j hyperplanes.  One block per slice of vb
// velocities (slices of one XCD are contiguous, so neighbouring slices share cache lines
// in its L2); compute lane = (cell of the hyperplane, velocity of the slice), handling
// both species (they share the diagonal and the couplings).  LDS holds the increments of
// the previous hyperplane and of the cells next to a periodic seam, and the staged
// per-cell data (record, geometry, coupling weights) of the current and next hyperplane.
// Each compute lane keeps the HBM loads of its next RING items (one per hyperplane) in
// flight in fixed registers.
// ---------------------------------------------------------------------------------------
constexpr int STG = 24;  // staged values per cell: record (12), nx S (4), ny S (4), weights (4)
constexpr int RING = 3;

template <class S, int VPL>
struct SweepItem {
    S aG[VPL], aH[VPL], bG[VPL], bH[VPL];  // forward: M, phi~ (G, H); backward: increment, phi~
    S e1[VPL], e2[VPL];                    // forward: factored Maxwellian
};

// Staging of the micro sweeps: staging lane sl copies column r = sl % STG of the staged
// rows of cells k = sl / STG + q * KP (KP = cells per pass, q < SPW_MICRO) of a
// hyperplane.  Columns of the forward sweep: record (12), nx S (4), ny S (4), forward
// coupling weights (4).  The backward sweep stages the wall ghost density increments of
// the 4 sides (0 on every side that is not a wall) in place of the equilibrium part of the
// record, and its own coupling weights.  Each lane reads one source column with a fixed
// stride: one load per value and no divergence between the lanes of a wave.
constexpr int SPW_MICRO = 8;

template <bool UPPER>
struct StageCol {
    const double *base;
    int stride, r, k0;
    bool zero;  // the column is constant 0 (or the lane is idle)
    DEV StageCol(const Params &p, int sl, int nsl) {
        const int kp = nsl / STG;
        r = sl % STG;
        k0 = sl / STG;
        base = p.srec;  // zero columns and idle lanes read this value and discard it
        stride = 0;
        zero = true;
        if (k0 >= kp) return;  // idle lane
        zero = false;
        stride = SG_N;
        if (r >= SR_N + 8) base = p.sgeo + (UPPER ? 12 : 8) + (r - SR_N - 8);  // coupling weights
        else if (r >= SR_N) base = p.sgeo + (r - SR_N);                      // nx S, ny S
        else if (!UPPER || r >= 10) { base = p.srec + r; stride = SR_N; }
        else if (r < 4) { base = p.sdrho + r; stride = 4; }
        else { base = p.srec; stride = 0; zero = true; }
    }
};

// rows past the hyperplane's last cell are read but never staged (the arrays have spare
// rows at their end)
template <class T, bool UPPER>
DEV void sweep_issue(const StageCol<UPPER> &col, T (&reg)[SPW_MICRO], const int *hpo, int h, int kp) {
    const double *src = col.base + (size_t)(hpo[h] + col.k0) * col.stride;
    const size_t step = (size_t)kp * col.stride;
#pragma unroll
    for (int q = 0; q < SPW_MICRO; ++q) reg[q] = (T)src[q * step];
}

template <class T, bool UPPER>
DEV void sweep_stage(const StageCol<UPPER> &col, const T (&reg)[SPW_MICRO], T *dst, const int *hpo,
                     int h, int kp, int nsl) {
    const int cells = hpo[h + 1] - hpo[h];
    if (col.k0 >= nsl / STG) return;
    T *d = dst + col.k0 * STG + col.r;
#pragma unroll
    for (int q = 0; q < SPW_MICRO; ++q)
        if (col.k0 + q * kp < cells) d[q * kp * STG] = col.zero ? T(0) : reg[q];
}

// ADJ: the transposed operator of the adjoint iteration (FP64): the couplings run along
// the outflow side (xi.n > 0) of the lower / upper neighbours, the right-hand side of the
// ascending sweep is d1 itself and the descending sweep writes its result to d1.
// VPL: velocities per compute lane (the block's slice has W = vb VPL velocities; lane
// (slot, vl) takes the columns vl, vl + vb, ...): the staged row, the coupling weights
// and all per-hyperplane arithmetic are shared by them, and their chains are independent.
template <class S, bool SHAK, bool UPPER, bool ADJ, int VPL>
__global__ __launch_bounds__(1024) void k_sweep(Params p, int vb, int nct) {
    using T = S;
    extern __shared__ unsigned char lds_raw[];
    const int ni = p.ni, nj = p.nj, nh = ni + nj - 1, L = ni < nj ? ni : nj;
    const int W = vb * VPL;
    // one species' fronts: [pad][f0][pad][f1][pad][wI][wJ], the pads (W values) taking the
    // reads of the columns -1 and ni of lanes on the hyperplane's first and last cell
    const int FR = (3 * ni + nj + 3) * W;
    T *f0 = (T *)lds_raw + W, *f1 = f0 + (ni + 1) * W, *wI = f1 + (ni + 1) * W, *wJ = wI + nj * W;
    T *st0 = (T *)lds_raw + 2 * FR, *st1 = st0 + L * STG;
    int *hpo = (int *)(st1 + L * STG);
    for (int h = threadIdx.x; h <= nh; h += blockDim.x) hpo[h] = p.hp_off[h];
    // every front value is finite from the start: uncoupled sides multiply theirs by 0
    for (int e = threadIdx.x; e < 2 * FR; e += blockDim.x) ((T *)lds_raw)[e] = T(0);
    __syncthreads();
    auto hp = [&](int t) { return UPPER ? nh - 1 - t : t; };
    // Both roles run one barrier after the prologue and one per hyperplane.
    if ((int)threadIdx.x >= nct) {
        const int sl = (int)threadIdx.x - nct, nsl = (int)blockDim.x - nct, kp = nsl / STG;
        const StageCol<UPPER> col(p, sl, nsl);
        // register set k holds a hyperplane t with t % SDEPTH == k; the loads of hyperplane
        // t+1 are issued SDEPTH steps before it is staged
        T reg[SDEPTH][SPW_MICRO];
        auto hcl = [&](int t) { return hp(t < nh ? t : nh - 1); };  // repeated rows are not staged
        sweep_issue<T, UPPER>(col, reg[0], hpo, hcl(0), kp);
        sweep_stage<T, UPPER>(col, reg[0], st0, hpo, hp(0), kp, nsl);
#pragma unroll
        for (int d = 1; d <= SDEPTH; ++d) sweep_issue<T, UPPER>(col, reg[d % SDEPTH], hpo, hcl(d), kp);
        lds_barrier();
        int t0 = 0;
        for (; t0 + SDEPTH <= nh; t0 += SDEPTH) {
#pragma unroll
            for (int d = 0; d < SDEPTH; ++d) {
                const int t = t0 + d;
                if (t + 1 < nh) sweep_stage<T, UPPER>(col, reg[(d + 1) % SDEPTH], (t + 1) & 1 ? st1 : st0, hpo, hp(t + 1), kp, nsl);
                sweep_issue<T, UPPER>(col, reg[(d + 1) % SDEPTH], hpo, hcl(t + 1 + SDEPTH), kp);
                lds_barrier();
            }
        }
#pragma unroll
        for (int d = 0; d < SDEPTH - 1; ++d) {
            const int t = t0 + d;
            if (t < nh) {
                if (t + 1 < nh) sweep_stage<T, UPPER>(col, reg[(d + 1) % SDEPTH], (t + 1) & 1 ? st1 : st0, hpo, hp(t + 1), kp, nsl);
                lds_barrier();
            }
        }
        return;
    }
    // Compute lanes.  On hyperplane h (cells i = lo..hi, j = h - i) the lane of slot k has the
    // cell i = lo + k if k <= hi - lo.  Its ring loads take i = lo + min(k, hi - lo) (lanes
    // past the hyperplane's end load its last cell and discard it, so every load stays in
    // bounds): the cell index is the one of (hi, h - hi) plus max(hi - lo - k, 0) (ni - 1),
    // a per-hyperplane scalar plus a lane constant under a max, and so are its offsets in
    // the state and the tables.  (Velocities past nv lie in the padding of the velocity
    // arrays; those lanes compute but store nothing.)
    const int vl = threadIdx.x % vb, slot = threadIdx.x / vb;
    const int v = xcd_remap(blockIdx.x, gridDim.x) * W + vl;  // velocity u: v + u vb
    const int kk = slot < L ? slot : L - 1;
    const int nv2 = 2 * p.nvp, ntb = p.nvx + p.nvy;
    const int kc = kk * (ni - 1) * nv2, kt = kk * (ni - 1) * ntb, ks = slot * W;
    bool vok[VPL];
    T x[VPL], y[VPL];
    int ix[VPL], iy[VPL];
#pragma unroll
    for (int u = 0; u < VPL; ++u) {
        const int vu = v + u * vb;
        vok[u] = slot < L && vu < p.nv;
        x[u] = (T)p.xi[vu];
        y[u] = (T)p.eta[vu];
        ix[u] = p.vix[vu];
        iy[u] = p.viy[vu];
    }
    const T sc = (T)p.scal[SC_SCALE];
    T gwv[VPL][4] = {}, kw[4] = {T(0), T(0), T(0), T(0)};
    if (UPPER && !ADJ) {
#pragma unroll
        for (int sd = 0; sd < 4; ++sd) {
            kw[sd] = (T)p.wKRT[sd];
#pragma unroll
            for (int u = 0; u < VPL; ++u) gwv[u][sd] = (T)p.gw[(size_t)sd * p.nvp + v + u * vb];
        }
    }
    auto state_off = [&](int h, int lo, int hi) {
        return (hi + (h - hi) * ni) * nv2 + max((hi - lo) * (ni - 1) * nv2 - kc, 0) + v;
    };
    auto load = [&](SweepItem<S, VPL> &it, int t) {
        const int h = hp(t < nh ? t : nh - 1);
        int lo, hi;
        hp_bounds(h, ni, nj, lo, hi);
        const unsigned o = state_off(h, lo, hi);
        const S *a = (const S *)p.d1 + o, *b = (const S *)p.f + o;
#pragma unroll
        for (int u = 0; u < VPL; ++u) {
            it.aG[u] = a[u * vb];
            it.aH[u] = a[p.nvp + u * vb];
            if (!ADJ) {
                it.bG[u] = b[u * vb];
                it.bH[u] = b[p.nvp + u * vb];
            }
        }
        if (!UPPER && !ADJ) {
            const unsigned ot = (hi + (h - hi) * ni) * ntb + max((hi - lo) * (ni - 1) * ntb - kt, 0);
            const S *tb = (const S *)p.tabs + ot;
#pragma unroll
            for (int u = 0; u < VPL; ++u) {
                it.e1[u] = tb[ix[u]];
                it.e2[u] = tb[p.nvx + iy[u]];
            }
        }
    };
    SweepItem<S, VPL> ring[RING];
#pragma unroll
    for (int d = 0; d < RING; ++d) load(ring[d], d);
    lds_barrier();
    // One step: the hyperplane t with ring slot d.  Full groups of RING steps are unrolled
    // without guards, so that the waits for a slot's loads are exact; the tail is guarded.
    auto step = [&](const int t, SweepItem<S, VPL> &cur) {
        const int h = hp(t);
        int lo, hi;
        hp_bounds(h, ni, nj, lo, hi);
        if (slot <= hi - lo) {
            const int fi = lo * W + ks + vl, fj = (h - lo) * W - ks + vl;  // i W + vl, j W + vl
            const T *m = ((t & 1) ? st1 : st0) + slot * STG;
            // The staged row, then the one neighbour increment each side can couple to in
            // this direction (sides i-, i+, j-, j+): forward f0[i-1], wI[j], f0[i], wJ[i];
            // backward wI[j], f0[i+1], wJ[i], f0[i] (the neighbours across a periodic seam
            // sit in wI / wJ), all read in one batch.
            const T *sp[4];
            if (UPPER) { sp[0] = wI + fj; sp[1] = f0 + fi + W; sp[2] = wJ + fi; sp[3] = f0 + fi; }
            else { sp[0] = f0 + fi - W; sp[1] = wI + fj; sp[2] = f0 + fi; sp[3] = wJ + fi; }
            T fg[VPL][4], fh[VPL][4];
#pragma unroll
            for (int u = 0; u < VPL; ++u)
#pragma unroll
                for (int sd = 0; sd < 4; ++sd) {
                    fg[u][sd] = sp[sd][u * vb];
                    fh[u][sd] = sp[sd][FR + u * vb];
                }
            T mr[STG];
#pragma unroll
            for (int e = 0; e < STG; ++e) mr[e] = m[e];
            RecT<T> r;
            if (!UPPER && !ADJ) {
                r.U = mr[0]; r.V = mr[1]; r.c0 = mr[2]; r.c1 = mr[3]; r.c2c = mr[4]; r.c3 = mr[5];
                r.kqx = mr[6]; r.kqy = mr[7]; r.iRT = mr[8]; r.KRT = mr[9];
            }
            T dG[VPL], dH[VPL];
#pragma unroll
            for (int u = 0; u < VPL; ++u) {
                T D = mr[11], sG, sH;
                if (!UPPER && ADJ) {
                    sG = cur.aG[u];
                    sH = cur.aH[u];
                } else if (!UPPER) {
                    T eG, eH;
                    eq_eval<T, SHAK>(r, x[u], y[u], cur.e1[u] * cur.e2[u], eG, eH);
                    sG = cur.aG[u] - mr[10] * (sc * cur.bG[u] - eG);
                    sH = cur.aH[u] - mr[10] * (sc * cur.bH[u] - eH);
                } else {
                    sG = sH = T(0);
                }
                // per side, by weights instead of branches: outflow (xi.n > 0) adds to the
                // diagonal; inflow from a coupled neighbour adds its increment, inflow
                // through a wall (backward sweep) the ghost's; the transposed operator
                // couples along the outflow instead.  A weight of 0 adds an exact 0 (all
                // fronts are finite).
#pragma unroll
                for (int sd = 0; sd < 4; ++sd) {
                    const T unS = x[u] * mr[SR_N + sd] + y[u] * mr[SR_N + 4 + sd];  // (xi.n) S
                    const T uo = fmax(unS, T(0)), ui = fmin(unS, T(0));
                    D += uo;
                    const T uc = (ADJ ? uo : ui) * mr[SR_N + 8 + sd];
                    if (ADJ) {
                        sG += uc * fg[u][sd];
                        sH += uc * fh[u][sd];
                    } else {
                        sG -= uc * fg[u][sd];
                        sH -= uc * fh[u][sd];
                    }
                    if (UPPER && !ADJ) {  // the ghost density increment is 0 off the walls
                        const T gw = -gwv[u][sd] * mr[sd] * ui;
                        sG += gw;
                        sH += gw * kw[sd];
                    }
                }
                const T iD = rcp_nr(D);
                dG[u] = UPPER ? cur.aG[u] + sG * iD : sG * iD;
                dH[u] = UPPER ? cur.aH[u] + sH * iD : sH * iD;
            }
            const unsigned o = state_off(h, lo, hi);
            const int i = lo + slot, j = h - i;
#pragma unroll
            for (int u = 0; u < VPL; ++u) {
                if (!vok[u]) continue;
                if (UPPER && !ADJ) {
                    ((S *)p.f)[o + u * vb] = (S)(sc * cur.bG[u] + dG[u]);
                    ((S *)p.f)[o + p.nvp + u * vb] = (S)(sc * cur.bH[u] + dH[u]);
                } else {
                    ((S *)p.d1)[o + u * vb] = (S)dG[u];
                    ((S *)p.d1)[o + p.nvp + u * vb] = (S)dH[u];
                }
                const int fu = fi + u * vb;
                f1[fu] = dG[u];
                f1[FR + fu] = dH[u];
                // the seam copies: a cell off the seam column / row writes its f1 value again
                T *qI = i == (UPPER ? ni - 1 : 0) ? wI + fj + u * vb : f1 + fu;
                T *qJ = j == (UPPER ? nj - 1 : 0) ? wJ + fu : f1 + fu;
                qI[0] = dG[u];
                qI[FR] = dH[u];
                qJ[0] = dG[u];
                qJ[FR] = dH[u];
            }
        }
        // the slot's loads were issued RING steps ago; it is refilled only after use, so
        // the new loads land in the same registers (no copies that would wait on them)
        load(cur, t + RING);
    };
    int t0 = 0;
    for (; t0 + RING <= nh; t0 += RING) {
#pragma unroll
        for (int d = 0; d < RING; ++d) {
            step(t0 + d, ring[d]);
            lds_barrier();
            T *tp = f0; f0 = f1; f1 = tp;
        }
    }
#pragma unroll
    for (int d = 0; d < RING - 1; ++d) {
        if (t0 + d < nh) {
            step(t0 + d, ring[d]);
            lds_barrier();
            T *tp = f0; f0 = f1; f1 = tp;
        }
    }
}

// ---------------------------------------------------------------------------------------
// micro LU-SGS sweeps (Eq. 24-26) level by level: the sweep order is the cell index order
// and a level holds cells whose lower-indexed neighbours all lie on earlier levels, so the
// cells of a level are independent in the forward sweep and, taken in reverse, in the
// backward one.  This serves any mesh (unstructured ones; structured ones on request,
// where the levels are the i+j hyperplanes).  One block of GS_NW waves per slice of 64
// velocities; wave w takes the cells w, w + GS_NW, ... of a level, in batches of up to CB
// cells: all loads of a batch are issued before any arithmetic (the stores of one cell
// would otherwise hold back the loads of the next); each cell stores as it finishes.  A cell's rows (index row; side
// geometry, record and ghost increments in the state precision) are scalar loads.  The
// neighbours' increments, written by this block on an earlier level (a block barrier
// separates the levels), come from an LDS ring of the recent positions, or from d1 for a
// neighbour older than the ring holds (the backward sweep leaves an increment in d1 only
// where a later cell reads it from there).  Per cell and velocity the arithmetic is the
// hyperplane kernel's, in the same order.
// ---------------------------------------------------------------------------------------
constexpr int GS_NW = 16, GS_THREADS = 64 * GS_NW;

// a position's rows as wave-uniform vector loads (16-byte rows, so they become wide
// scalar loads): the first eight values of the index row, and the value row
DEV void grow8(const int *gr, int (&g)[8]) {
    const int4 a = ((const int4 *)gr)[0], b = ((const int4 *)gr)[1];
    g[0] = a.x; g[1] = a.y; g[2] = a.z; g[3] = a.w; g[4] = b.x; g[5] = b.y; g[6] = b.z; g[7] = b.w;
}
DEV void growt(const float *gt, float (&r)[GT_N]) {
#pragma unroll
    for (int e = 0; e < GT_N; e += 4) {
        const float4 a = ((const float4 *)gt)[e / 4];
        r[e] = a.x; r[e + 1] = a.y; r[e + 2] = a.z; r[e + 3] = a.w;
    }
}
DEV void growt(const double *gt, double (&r)[GT_N]) {
#pragma unroll
    for (int e = 0; e < GT_N; e += 2) {
        const double2 a = ((const double2 *)gt)[e / 2];
        r[e] = a.x; r[e + 1] = a.y;
    }
}

// The slice's recent increments in LDS: a ring of N positions (slot = position mod N),
// per slot and lane the G and H increments side by side.  With every level at most N
// cells, the slot of a neighbour on an earlier level (forward sweep) or a later one
// (backward sweep) still holds it while fewer than N positions lie between it and the far
// end of the current level (forward q + N >= off + n, backward q < off + N, for the
// neighbour's position q and the current level's first position off and size n).  The
// host marks such sides in the index row; the others are read from d1.
template <class S>
struct GsRing {
    static constexpr int N = gs_ring_positions(sizeof(S) == 4);
    using V = typename std::conditional<sizeof(S) == 4, float2, double2>::type;
};

// the loads of one cell of a batch
template <class S>
struct GItem {
    S aG, aH, bG, bH, e1, e2;
    S nG[4], nH[4];
};

// The per-position rows come in as separate read-only, unaliased kernel arguments: their
// wave-uniform reads then become scalar loads, and the record, geometry and ghost values
// (in the state precision, growT) are used as scalar operands of the arithmetic.
template <class S, bool SHAK, bool UPPER, int CB>
__global__ __launch_bounds__(GS_THREADS) void k_gsweep(Params p, const int *__restrict__ grow,
                                                       const S *__restrict__ growT) {
    using T = S;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    // 32-bit byte offsets of the lane's velocity in a row: a load is a wave-uniform row
    // base plus that offset
    const int v = xcd_remap(blockIdx.x, gridDim.x) * 64 + lane;  // < nvp (padding reads zeros)
    const bool vok = v < p.nv;
    const int nvp = p.nvp, nv2 = 2 * p.nvp, ntb = p.nvx + p.nvy;
    const unsigned ov = (unsigned)v * sizeof(S), oh = (unsigned)(nvp + v) * sizeof(S);
    const T x = (T)p.xi[v], y = (T)p.eta[v];
    const unsigned ox = (unsigned)p.vix[v] * sizeof(S), oy = (unsigned)(p.nvx + p.viy[v]) * sizeof(S);
    const T sc = (T)p.scal[SC_SCALE];
    S *d1 = (S *)p.d1, *f = (S *)p.f;
    const int nlev = p.nlev;
    constexpr int RN = GsRing<S>::N;
    using V2 = typename GsRing<S>::V;
    __shared__ V2 ring[RN * 64];
    for (int t = 0; t < nlev; ++t) {
        const int l = UPPER ? nlev - 1 - t : t;
        const int off = p.hp_off[l], n = p.hp_off[l + 1] - off;
        for (int base = 0; base < n; base += GS_NW * CB) {
            GItem<S> it[CB];
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int k = base + wave + GS_NW * b;
                if (k >= n) continue;  // wave-uniform
                int g[8];
                grow8(grow + (size_t)(off + k) * GR_N, g);
                const int c = g[GR_CELL], mask = g[GR_MASK];
                const S *dr = d1 + (size_t)c * nv2, *fr = f + (size_t)c * nv2;  // wave-uniform
                it[b].aG = at(dr, ov);
                it[b].aH = at(dr, oh);
                it[b].bG = at(fr, ov);
                it[b].bH = at(fr, oh);
                if (!UPPER) {
                    const S *tb = (const S *)p.tabs + (size_t)c * ntb;
                    it[b].e1 = at(tb, ox);
                    it[b].e2 = at(tb, oy);
                }
#pragma unroll
                for (int sd = 0; sd < 4; ++sd) {
                    if ((mask >> (UPPER ? 4 + sd : sd)) & 1) {
                        const int q = g[GR_SRC + sd];
                        if ((mask >> (12 + sd)) & 1) {  // in the ring: q is the position
                            const V2 e = ring[(q & (RN - 1)) * 64 + lane];
                            it[b].nG[sd] = e.x;
                            it[b].nH[sd] = e.y;
                        } else {
                            const S *nr = d1 + (size_t)q * nv2;
                            it[b].nG[sd] = at(nr, ov);
                            it[b].nH[sd] = at(nr, oh);
                        }
                    }
                }
            }
            // the rows of cell b + 1 are loaded (unconditionally, a valid position) before
            // cell b's arithmetic, so that their scalar loads overlap it
            int gn[8];
            T gtn[GT_N];
            {
                const int k = base + wave < n ? base + wave : 0;
                grow8(grow + (size_t)(off + k) * GR_N, gn);
                growt(growT + (size_t)(off + k) * GT_N, gtn);
            }
#pragma unroll
            for (int b = 0; b < CB; ++b) {
                const int k = base + wave + GS_NW * b;
                int g[8];
                T gt[GT_N];
#pragma unroll
                for (int e = 0; e < 8; ++e) g[e] = gn[e];
#pragma unroll
                for (int e = 0; e < GT_N; ++e) gt[e] = gtn[e];
                if (b + 1 < CB) {
                    const int kn = k + GS_NW < n ? k + GS_NW : 0;
                    grow8(grow + (size_t)(off + kn) * GR_N, gn);
                    growt(growT + (size_t)(off + kn) * GT_N, gtn);
                }
                if (k >= n) continue;
                const GItem<S> &q = it[b];
                const int c = g[GR_CELL], mask = g[GR_MASK];
                T D = gt[GT_REC + 11], sG, sH;
                if (!UPPER) {
                    RecT<T> rc;
                    rc.U = gt[GT_REC]; rc.V = gt[GT_REC + 1]; rc.c0 = gt[GT_REC + 2]; rc.c1 = gt[GT_REC + 3];
                    rc.c2c = gt[GT_REC + 4]; rc.c3 = gt[GT_REC + 5]; rc.kqx = gt[GT_REC + 6];
                    rc.kqy = gt[GT_REC + 7]; rc.iRT = gt[GT_REC + 8]; rc.KRT = gt[GT_REC + 9];
                    T eG, eH;
                    eq_eval<T, SHAK>(rc, x, y, q.e1 * q.e2, eG, eH);
                    const T cst = gt[GT_REC + 10];
                    sG = q.aG - cst * (sc * q.bG - eG);
                    sH = q.aH - cst * (sc * q.bH - eH);
                } else {
                    sG = sH = T(0);
                }
#pragma unroll
                for (int sd = 0; sd < 4; ++sd) {
                    const T unS = x * gt[GT_GEO + sd] + y * gt[GT_GEO + 4 + sd];  // (xi.n) S
                    const T uo = fmax(unS, T(0)), ui = fmin(unS, T(0));
                    D += uo;
                    if ((mask >> (UPPER ? 4 + sd : sd)) & 1) {  // inflow from a coupled neighbour
                        sG -= ui * q.nG[sd];
                        sH -= ui * q.nH[sd];
                    }
                    if (UPPER && ((mask >> (8 + sd)) & 1)) {
                        const int j = g[GR_SRC + sd];
                        {  // inflow through a wall: the ghost's increment
                            // (a cache-resident table, read here to keep the batch's registers)
                            const T gwv = (T)p.gw[(size_t)(-1 - j) * nvp + v];
                            const T g = -gwv * gt[GT_DRHO + sd] * ui;
                            sG += g;
                            sH += g * (T)p.wKRT[-1 - j];
                        }
                    }
                }
                const T iD = rcp_nr(D);
                const T dG = UPPER ? q.aG + sG * iD : sG * iD;
                const T dH = UPPER ? q.aH + sH * iD : sH * iD;
                if (UPPER) {
                    ring[((off + k) & (RN - 1)) * 64 + lane] = V2{(S)dG, (S)dH};
                    if (vok) {
                        S *dr = d1 + (size_t)c * nv2, *fr = f + (size_t)c * nv2;
                        if (!((mask >> 16) & 1)) {  // a later cell reads it from d1
                            at(dr, ov) = dG;
                            at(dr, oh) = dH;
                        }
                        at(fr, ov) = (S)(sc * q.bG + dG);
                        at(fr, oh) = (S)(sc * q.bH + dH);
                    }
                } else {
                    ring[((off + k) & (RN - 1)) * 64 + lane] = V2{(S)dG, (S)dH};
                    if (vok) {
                        S *dr = d1 + (size_t)c * nv2;
                        at(dr, ov) = dG;
                        at(dr, oh) = dH;
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Macro LU-SGS sweeps (Eq. 29-31) level by level in one block, the work split across
// waves so that none of them waits for its own stores: the compute waves take a phase of
// at most G2_PH cells of a level, four lanes per cell (one side each, the parts summed by
// DPP quad swaps), and touch only LDS; the loader waves stage the next phase's rows (own
// data, and per position the W and sound speed its neighbours need) into LDS; the writer
// wave copies the increments of the previous phase from LDS to HBM (dW* into the macro
// rows, where the backward sweep's loader finds them in position order; dW by cell).  Per
// position an LDS ring of G2_RS slots (slot = position mod G2_RS) holds W, c, the
// increment and the cell; a neighbour older than the ring's window is read from HBM (its
// macro row and dW, flushed long before).  Positions are staged and computed in increasing
// order in the forward sweep and in decreasing order in the backward one, a phase being at
// most G2_PH consecutive positions, so a slot holds the position last written to it.
constexpr int G2_PH = 128;                     // cells per phase
constexpr int G2_CW = 4 * G2_PH / 64;          // compute waves: four lanes per cell
constexpr int G2_LW = G2_PH / 64;              // loader waves: one position per lane
constexpr int G2_THREADS = 64 * (G2_CW + G2_LW + 1);
constexpr int G2_RS = 1024;
static_assert(3 * G2_PH <= G2_RS && (G2_RS & (G2_RS - 1)) == 0, "ring too small");

struct G2Row {  // a cell's own data in its phase
    double mw[4], iD, geo[12];
    int codes, c, nb[4], np[4];
};

struct G2Ring {  // per position, for its neighbours
    double W[4], C, dW[4];
    int cell;
};

// the phases of one sweep: round r of level t (levels in sweep order); s, cnt its positions
struct G2Phase {
    int t, r, s, cnt;
};

DEV bool g2_set(const Params &p, bool upper, G2Phase &ph) {
    if (ph.t >= p.nlev) return false;
    const int l = upper ? p.nlev - 1 - ph.t : ph.t;
    const int off = p.hp_off[l], n = p.hp_off[l + 1] - off;
    if (upper) {  // a level's rounds from its far end
        const int e = off + n - ph.r * G2_PH;
        ph.s = e - G2_PH > off ? e - G2_PH : off;
        ph.cnt = e - ph.s;
    } else {
        ph.s = off + ph.r * G2_PH;
        ph.cnt = n - ph.r * G2_PH < G2_PH ? n - ph.r * G2_PH : G2_PH;
    }
    return true;
}

DEV void g2_next(const Params &p, bool upper, G2Phase &ph) {
    const int l = upper ? p.nlev - 1 - ph.t : ph.t;
    const int n = p.hp_off[l + 1] - p.hp_off[l];
    if ((ph.r + 1) * G2_PH < n) {
        ++ph.r;
    } else {
        ++ph.t;
        ph.r = 0;
    }
}

__global__ __launch_bounds__(G2_THREADS) void k_gmacro(Params p) {
    __shared__ G2Row stage[2][G2_PH];
    __shared__ G2Ring ring[G2_RS];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int role = wave < G2_CW ? 0 : wave < G2_CW + G2_LW ? 1 : 2;  // compute, loader, writer
    const double ik2 = 1.0 / (p.K + 2);
    // loader: the rows of phase ph into stage buffer b and the ring (the macro row holds
    // M_W in the forward sweep and, written there by the forward sweep, dW* in the backward one)
    auto stage_phase = [&](const G2Phase &ph, int b) {
        const int k = tid - 64 * G2_CW;
        if (k >= ph.cnt) return;
        const int pos = ph.s + k;
        const double *m = p.mh + (size_t)pos * MH_N;
        const int *g = p.grow + (size_t)pos * GR_N;
        G2Row &o = stage[b][k];
        const int c = g[GR_CELL];
        o.c = c;
#pragma unroll
        for (int a = 0; a < 4; ++a) o.mw[a] = m[a];
        o.iD = m[4];
        o.codes = (int)m[5];
#pragma unroll
        for (int e = 0; e < 12; ++e) o.geo[e] = m[MH_SIDE + e];
#pragma unroll
        for (int sd = 0; sd < 4; ++sd) {
            o.nb[sd] = g[GR_NB + sd];
            o.np[sd] = g[GR_NPOS + sd];
        }
        G2Ring &q = ring[pos & (G2_RS - 1)];
#pragma unroll
        for (int a = 0; a < 4; ++a) q.W[a] = m[6 + a];
        q.C = m[10];
        q.cell = c;
    };
    // writer: the increments of phase ph: dW* into the macro rows (position order) in the
    // forward sweep, dW (cell order) in the backward one
    auto flush = [&](const G2Phase &ph, bool upper) {
        for (int k = lane; k < ph.cnt; k += 64) {
            const int pos = ph.s + k;
            const G2Ring &q = ring[pos & (G2_RS - 1)];
            double *dst = upper ? p.dW + (size_t)q.cell * 4 : p.mh + (size_t)pos * MH_N;
#pragma unroll
            for (int a = 0; a < 4; ++a) dst[a] = q.dW[a];
        }
    };
    for (int dir = 0; dir < 2; ++dir) {
        const bool upper = dir == 1;
        const int need = upper ? SG_UPPER : SG_LOWER;
        G2Phase cur{0, 0, 0, 0}, prev{0, 0, 0, 0};
        g2_set(p, upper, cur);
        if (role == 1) stage_phase(cur, 0);
        __syncthreads();
        bool has_prev = false;
        for (int i = 0;; ++i) {
            G2Phase nxt = cur;
            g2_next(p, upper, nxt);
            const bool has_next = g2_set(p, upper, nxt);
            if (role == 0) {
                // lane 4k + sd: side sd of cell k (the quad's lanes stay together for the sums)
                const int k = tid >> 2, sd = tid & 3;
                const bool live = k < cur.cnt;
                const G2Row &o = stage[i & 1][live ? k : 0];
                double r[4] = {0.0, 0.0, 0.0, 0.0};
                if (live && ((o.codes >> (MH_CODE_BITS * sd)) & need)) {
                    const int pj = o.np[sd];
                    // in the ring unless its slot has been (or is being) reused by a later
                    // position: the staging of the next phase reaches at most G2_PH
                    // positions past this one
                    const bool in = upper ? pj < cur.s - G2_PH + G2_RS : pj >= cur.s + 2 * G2_PH - G2_RS;
                    double Wj[4], dWj[4], Cj;
                    const double *mj = p.mh + (size_t)pj * MH_N;
                    if (in) {
                        const G2Ring &q = ring[pj & (G2_RS - 1)];
#pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            Wj[a] = q.W[a];
                            dWj[a] = q.dW[a];
                        }
                        Cj = q.C;
                    } else {  // flushed long before: dW* in the row, dW by cell
                        const double *dj = upper ? p.dW + (size_t)o.nb[sd] * 4 : mj;
#pragma unroll
                        for (int a = 0; a < 4; ++a) {
                            Wj[a] = mj[6 + a];
                            dWj[a] = dj[a];
                        }
                        Cj = mj[10];
                    }
                    const double nx = o.geo[MH_SN * sd], ny = o.geo[MH_SN * sd + 1];
                    const double hS = 0.5 * o.geo[MH_SN * sd + 2];
                    double Wn[4], F0[4], F1[4];
#pragma unroll
                    for (int a = 0; a < 4; ++a) Wn[a] = Wj[a] + dWj[a];
                    const double lam = fabs(euler_flux_n(Wj, nx, ny, ik2, F0)) + Cj;
                    euler_flux_n(Wn, nx, ny, ik2, F1);
#pragma unroll
                    for (int a = 0; a < 4; ++a) r[a] = hS * (F1[a] - F0[a] - lam * dWj[a]);
                }
                // the four sides' parts: (side 0 + side 1) + (side 2 + side 3) in every lane
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    r[a] += quad_swap<0xB1>(r[a]);
                    r[a] += quad_swap<0x4E>(r[a]);
                }
                if (live) {  // lane sd finishes component sd
                    const double ra = sd == 0 ? r[0] : sd == 1 ? r[1] : sd == 2 ? r[2] : r[3];
                    const double ma = sd == 0 ? o.mw[0] : sd == 1 ? o.mw[1] : sd == 2 ? o.mw[2] : o.mw[3];
                    // forward dW* = (M_W - r)/D, backward dW = dW* - r/D
                    ring[(cur.s + k) & (G2_RS - 1)].dW[sd] = upper ? ma - ra * o.iD : (ma - ra) * o.iD;
                }
            } else if (role == 1) {
                if (has_next) stage_phase(nxt, (i + 1) & 1);
            } else if (has_prev) {
                flush(prev, upper);
            }
            __syncthreads();
            if (!has_next) break;
            prev = cur;
            has_prev = true;
            cur = nxt;
        }
        // the last phase's increments (the forward sweep's before the backward sweep stages
        // its rows)
        if (role == 2) flush(cur, upper);
        __syncthreads();
    }
}

// wall ghost density increment of each wall face from the forward-sweep G increment: one
// wave per wall face, the block's FR_W faces sharing the velocity set staged into LDS a
// chunk at a time (as in the face records); a lane takes the velocities lane, lane + 64, ...
template <class S>
__global__ __launch_bounds__(64 * FR_W) void k_wall_ghost(Params p) {
    constexpr int PER = FR_CH / 64;
    __shared__ double vx[FR_CH], vy[FR_CH], vw[FR_CH];
    const int lane = threadIdx.x & 63;
    const int wi = blockIdx.x * FR_W + (threadIdx.x >> 6);
    const bool live = wi < p.nwall;
    Face F{};
    int k = 0;
    if (live) {
        k = p.wall_faces[wi];
        F = p.faces[k];
    }
    const S *d = (const S *)p.d1 + ((size_t)(live ? F.L : 0) * 2) * p.nvp;
    double a[1] = {0.0};
    for (int c0 = 0; c0 < p.nv; c0 += FR_CH) {
        const int vt = c0 + threadIdx.x;
        if (vt < p.nv) {
            vx[threadIdx.x] = p.xi[vt];
            vy[threadIdx.x] = p.eta[vt];
            vw[threadIdx.x] = p.w[vt];
        }
        __syncthreads();
        if (live) {
            S ds[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int v = c0 + 64 * u + lane;
                ds[u] = d[v < p.nv ? v : 0];
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int j = 64 * u + lane;
                if (c0 + j >= p.nv) continue;
                const double un = vx[j] * F.nx + vy[j] * F.ny;
                if (un > 0.0) a[0] += vw[j] * un * (double)ds[u];
            }
        }
        __syncthreads();
    }
    if (!live) return;
    wave_sum_dpp<1>(a);
    if (lane == 0) {
        const double dr = -a[0] / p.wden[k];
        p.drho[k] = dr;
        p.sdrho[(size_t)p.hp_pos[F.L] * 4 + F.sL] = dr;
        if (p.graph) ((S *)p.growT)[(size_t)p.hp_pos[F.L] * GT_N + GT_DRHO + F.sL] = (S)dr;
    }
}

// explicit DUGKS update (Eq. 21)
template <class S, bool SHAK>
__global__ __launch_bounds__(256) void k_explicit(Params p) {
    using T = S;
    const int c = xcd_remap(blockIdx.x, p.nc);
    const RecT<T> r = load_rec<T>(p.rec[c]);
    const S *tb = (const S *)p.tab + (size_t)c * (p.nvx + p.nvy);
    const T area = (T)p.area[c], dt = (T)p.dt, sc = (T)p.scal[SC_SCALE];
    const T cst = T(2) * area / (T(2) * (T)p.rec[c].tau + dt), g = dt / area;
    for (int v = threadIdx.x; v < p.nv; v += blockDim.x) {
        T eG, eH;
        eq_eval<T, SHAK>(r, (T)p.xi[v], (T)p.eta[v], (T)tb[p.vix[v]] * (T)tb[p.nvx + p.viy[v]], eG, eH);
        for (int sp = 0; sp < 2; ++sp) {
            const size_t o = ((size_t)c * 2 + sp) * p.nvp + v;
            const T X = sc * (T)((const S *)p.f)[o];
            const T M = (T)((const S *)p.d1)[o];
            ((S *)p.f)[o] = (S)(X + g * (M - cst * (X - (sp == 0 ? eG : eH))));
        }
    }
}

// ---------------------------------------------------------------------------------------
// state conversion between the device layout and the canonical FP64 [2][nc][nv] layout
// ---------------------------------------------------------------------------------------
template <class S>
__global__ void k_pack(Params p, const void *src_dev_layout, double *dst, int sp, int nsp,
                       int scaled) {
    const size_t n = (size_t)p.nc * p.nv;
    const double sc = scaled ? p.scal[SC_SCALE] : 1.0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n * nsp;
         t += (size_t)gridDim.x * blockDim.x) {
        const int s = sp + (int)(t / n);
        const size_t r = t % n;
        const int c = (int)(r / p.nv), v = (int)(r % p.nv);
        dst[t] = sc * (double)((const S *)src_dev_layout)[((size_t)c * 2 + s) * p.nvp + v];
    }
}

template <class S>
__global__ void k_unpack(Params p, const double *src, int sp, int nsp) {
    const size_t n = (size_t)p.nc * p.nv;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n * nsp;
         t += (size_t)gridDim.x * blockDim.x) {
        const int s = sp + (int)(t / n);
        const size_t r = t % n;
        const int c = (int)(r / p.nv), v = (int)(r % p.nv);
        ((S *)p.f)[((size_t)c * 2 + s) * p.nvp + v] = (S)src[t];
    }
}

// zeros over n16 16-byte words (a fill kernel rather than a memset node)
__global__ void k_zero(uint4 *p, size_t n16) {
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n16; t += (size_t)gridDim.x * blockDim.x)
        p[t] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
    hipLaunchKernelGGL(k_zero, dim3(1024), dim3(256), 0, st, (uint4 *)p, bytes / 16);
    return hipGetLastError();
}

// uniform initial state: f[c][s][v] = eq[s][v] (eq staged as FP64 [2][nvp] in d1)
template <class S>
__global__ void k_fill_uniform(Params p, const double *eq) {
    const size_t n = (size_t)p.nc * 2 * p.nvp;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n;
         t += (size_t)gridDim.x * blockDim.x) {
        const size_t r = t % ((size_t)2 * p.nvp);
        const int s = (int)(r / p.nvp), v = (int)(r % p.nvp);
        ((S *)p.f)[t] = (S)(v < p.nv ? eq[(size_t)s * p.nvp + v] : 0.0);
    }
}

// cell output fields [nc][8] from 12 raw moments
__global__ void k_fields(Params p, double *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.nc) return;
    const double s = p.scal[SC_SCALE];
    double m[12];
    for (int a = 0; a < 12; ++a) m[a] = s * p.raw[(size_t)c * NM_MAX + a];
    const double rho = m[0], U = m[1] / rho, V = m[2] / rho;
    const double RT = (2.0 * m[3] / rho - U * U - V * V) / (p.K + 2);
    const double tau = tau_of(p, rho, RT);
    double qx, qy;
    heat_from_raw(m, U, V, qx, qy);
    const double Pr = p.model == 1 ? p.Pr : 1.0, t2 = 2.0 * tau;
    double *o = out + (size_t)c * 8;
    o[0] = rho; o[1] = U; o[2] = V; o[3] = 2.0 * RT; o[4] = rho * RT;
    o[5] = t2 * qx / (t2 + p.dt * Pr);
    o[6] = t2 * qy / (t2 + p.dt * Pr);
    o[7] = tau;
}

// ---------------------------------------------------------------------------------------
// Sensitivities: vector-Jacobian product of the steady residual
//   R_i(v) = M_i(v) - c_i (phi~_i(v) - phi_eq,i(v)),  c_i = 2 Omega_i / (2 tau_i + dt)
// (Eq. 11-23, BGK, no limiter, FP64 state), with theta = (lid speed, wall T, Kn).  The
// reverse pass runs the forward chain backwards: Eq. 18 blend and flux of each face,
// face equilibrium and tau (records), face moments, diffuse-wall density (Eq. 34), upwind
// reconstruction (Eq. 13-14), least-squares gradient (Eq. 15), phi-bar-plus (Eq. 10, 12),
// cell equilibrium and tau, cell moments.  The forward values (records, tables, face
// values) are those of the last flux evaluation at the same state.
// ---------------------------------------------------------------------------------------

// Forward-mode number with four tangents (derivatives with respect to W).
struct D4 {
    double v, d[4];
};
DEV D4 dconst(double a) { D4 r; r.v = a; r.d[0] = r.d[1] = r.d[2] = r.d[3] = 0.0; return r; }
DEV D4 operator+(const D4 &a, const D4 &b) { D4 r; r.v = a.v + b.v; for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
DEV D4 operator-(const D4 &a, const D4 &b) { D4 r; r.v = a.v - b.v; for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
DEV D4 operator-(const D4 &a) { D4 r; r.v = -a.v; for (int i = 0; i < 4; ++i) r.d[i] = -a.d[i]; return r; }
DEV D4 operator*(const D4 &a, const D4 &b) { D4 r; r.v = a.v * b.v; for (int i = 0; i < 4; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
DEV D4 operator*(double a, const D4 &b) { D4 r; r.v = a * b.v; for (int i = 0; i < 4; ++i) r.d[i] = a * b.d[i]; return r; }
DEV D4 operator/(const D4 &a, const D4 &b) {
    D4 r; r.v = a.v / b.v;
    for (int i = 0; i < 4; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
    return r;
}
DEV D4 dexp(const D4 &a) { D4 r; r.v = exp(a.v); for (int i = 0; i < 4; ++i) r.d[i] = r.v * a.d[i]; return r; }

DEV void solve4_d(D4 A[4][4], D4 b[4]) {
    for (int k = 0; k < 4; ++k) {
        int piv = k;
        for (int r = k + 1; r < 4; ++r)
            if (fabs(A[r][k].v) > fabs(A[piv][k].v)) piv = r;
        if (piv != k) {
            for (int c = 0; c < 4; ++c) { D4 t = A[k][c]; A[k][c] = A[piv][c]; A[piv][c] = t; }
            D4 t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < 4; ++r) {
            const D4 m = A[r][k] / A[k][k];
            for (int c = k; c < 4; ++c) A[r][c] = A[r][c] - m * A[k][c];
            b[r] = b[r] - m * b[k];
        }
    }
    for (int k = 3; k >= 0; --k) {
        D4 s = b[k];
        for (int c = k + 1; c < 4; ++c) s = s - A[k][c] * b[c];
        b[k] = s / A[k][k];
    }
}

// Jacobian J[m][a] = d p_m / d W_a of the BGK equilibrium record
// p = (rho, U, V, RT, c0, c1, c2c, c3) from the conserved moments W, by the same steps as
// build_eq (central basis, factored 1-D moments) in forward-mode arithmetic.  One wave;
// every lane returns J.
DEV void record_jacobian(const Params &p, const double W[4], double J[8][4], int lane) {
    D4 w[4];
    for (int a = 0; a < 4; ++a) { w[a] = dconst(W[a]); w[a].d[a] = 1.0; }
    const D4 rho = w[0], U = w[1] / rho, V = w[2] / rho;
    const D4 RT = (2.0 * (w[3] / rho) - U * U - V * V) / dconst((double)(p.K + 2));
    const D4 lam = dconst(0.5) / RT, A0 = rho * lam / dconst(M_PI);
    constexpr int NP = 5;
    double X[NP * 5], Y[NP * 5];
    for (int i = 0; i < NP * 5; ++i) X[i] = Y[i] = 0.0;
    for (int ix = lane; ix < p.nvx; ix += 64) {
        const D4 cx = dconst(p.x1[ix]) - U;
        const D4 e = dexp(-(lam * cx * cx));
        D4 t = p.wx1[ix] * e;
        for (int k = 0; k < NP; ++k) {
            X[5 * k] += t.v;
            for (int i = 0; i < 4; ++i) X[5 * k + 1 + i] += t.d[i];
            t = t * cx;
        }
    }
    for (int iy = lane; iy < p.nvy; iy += 64) {
        const D4 cy = dconst(p.y1[iy]) - V;
        const D4 e = dexp(-(lam * cy * cy));
        D4 t = p.wy1[iy] * e;
        for (int k = 0; k < NP; ++k) {
            Y[5 * k] += t.v;
            for (int i = 0; i < 4; ++i) Y[5 * k + 1 + i] += t.d[i];
            t = t * cy;
        }
    }
    wave_sum<NP * 5>(X);
    wave_sum<NP * 5>(Y);
    auto get = [&](const double *Z, int k) { D4 r; r.v = Z[5 * k]; for (int i = 0; i < 4; ++i) r.d[i] = Z[5 * k + 1 + i]; return r; };
    auto m = [&](int a, int b) { return A0 * get(X, a) * get(Y, b); };
    D4 A[4][4], r[4];
    A[0][0] = m(0, 0); A[0][1] = m(1, 0); A[0][2] = m(0, 1); A[0][3] = 0.5 * (m(2, 0) + m(0, 2));
    A[1][1] = m(2, 0); A[1][2] = m(1, 1); A[1][3] = 0.5 * (m(3, 0) + m(1, 2));
    A[2][2] = m(0, 2); A[2][3] = 0.5 * (m(2, 1) + m(0, 3));
    A[3][3] = 0.25 * (m(4, 0) + 2.0 * m(2, 2) + m(0, 4));
    for (int a = 1; a < 4; ++a)
        for (int b = 0; b < a; ++b) A[a][b] = A[b][a];
    r[0] = rho - A[0][0];
    r[1] = -A[0][1];
    r[2] = -A[0][2];
    r[3] = rho * RT - A[0][3];
    solve4_d(A, r);
    const D4 out[8] = {rho, U, V, RT, dconst(1.0) + r[0], r[1], r[2], 0.5 * r[3]};
    for (int mm = 0; mm < 8; ++mm)
        for (int a = 0; a < 4; ++a) J[mm][a] = out[mm].d[a];
}

// Per velocity: accumulate, for the equilibrium adjoint (eG, eH) of a record r with
// Maxwellian factor M (= tab[ix] tab[nvx+iy]), the sums S_m = sum_v d(E)/d(p_m) . e-bar
// (p = rho, U, V, RT, c0, c1, c2c, c3).
DEV void eq_adjoint_acc(const Rec &r, double x, double y, double M, double eG, double eH, double *S) {
    const double cx = x - r.U, cy = y - r.V, c2 = cx * cx + cy * cy;
    const double poly = r.c0 + r.c1 * cx + r.c2c * cy + r.c3 * c2;
    const double G = M * poly;
    const double e = eG + r.KRT * eH;       // H = K RT G
    const double Me = M * e;
    S[0] += e * G / r.rho;
    S[1] += Me * (r.iRT * cx * poly - r.c1 - 2.0 * r.c3 * cx);
    S[2] += Me * (r.iRT * cy * poly - r.c2c - 2.0 * r.c3 * cy);
    S[3] += Me * poly * (0.5 * c2 * r.iRT - 1.0) * r.iRT + (r.KRT * r.iRT) * eH * G;  // K G = KRT G / RT
    S[4] += Me;
    S[5] += Me * cx;
    S[6] += Me * cy;
    S[7] += Me * c2;
}

// W-bar = J^T p-bar with p-bar = S + tau-bar d(tau)/d(rho, RT); W from the record.
DEV void record_wbar(const Params &p, const Rec &r, const double S[8], double taubar,
                     double J[8][4], double Wb[4]) {
    double pb[8];
    for (int m = 0; m < 8; ++m) pb[m] = S[m];
    pb[0] += taubar * (-r.tau / r.rho);
    pb[3] += taubar * r.tau * (p.omega - 1.0) / r.RT;
    for (int a = 0; a < 4; ++a) {
        double s = 0.0;
        for (int m = 0; m < 8; ++m) s += J[m][a] * pb[m];
        Wb[a] = s;
    }
}

DEV void rec_W(const Params &p, const Rec &r, double W[4]) {
    W[0] = r.rho;
    W[1] = r.rho * r.U;
    W[2] = r.rho * r.V;
    W[3] = 0.5 * r.rho * (r.U * r.U + r.V * r.V + (p.K + 2) * r.RT);
}

// objective seeds: d J / d phi_k(v) at a wall face seen from its gas side (un = xi.n_out)
template <int OBJ>
DEV void objective_seed(const Params &p, const Face &F, double S, double x, double y, double wv,
                        double un, double &sG, double &sH) {
    sG = sH = 0.0;
    if (OBJ == 0 && F.type == FT_WALL && F.wside == 3) {
        sG = S * wv * x * un;
    } else if (OBJ == 1 && F.type == FT_WALL) {
        const double cx = x - p.wall_u[F.wside], cy = y - p.wall_v[F.wside];
        sG = S * wv * un * 0.5 * (cx * cx + cy * cy);
        sH = S * wv * un * 0.5;
    }
}

// One wave per face: the adjoint of phi_k = alpha phi-bar_k + (1 - alpha) E_k, of the face
// record (W-bar_k), of the wall density and of theta through the wall Maxwellian.
template <int OBJ>
__global__ __launch_bounds__(256) void k_adj_face(Params p) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= p.nf) return;
    const Face F = p.faces[k];
    double *fa = p.fadj + (size_t)k * FA_N;
    if (F.type == FT_SELF) {
        if (lane < FA_N) fa[lane] = 0.0;
        return;
    }
    const CellSide cL = p.cs[4 * F.L + F.sL];
    const Rec r = p.recf[k];
    const double *tf = (const double *)p.tabf + (size_t)k * (p.nvx + p.nvy);
    const double h = p.h, al = r.alpha, S = cL.S, sc = p.scal[SC_SCALE];
    (void)sc;
    const double *fvG = (const double *)p.fv + (size_t)k * 2 * p.nvp, *fvH = fvG + p.nvp;
    const double *lL = p.lam + (size_t)F.L * 2 * p.nvp;
    const double *lR = F.type == FT_INTERIOR ? p.lam + (size_t)F.R * 2 * p.nvp : nullptr;
    const int ws = F.type == FT_WALL ? F.wside : 0;
    const double *gw = p.gw + (size_t)ws * p.nvp;
    const double KRTw = p.wKRT[ws];
    // pass 1: alpha-bar, the equilibrium sums and the objective value
    double acc[10];
    for (int i = 0; i < 10; ++i) acc[i] = 0.0;
    for (int v = lane; v < p.nv; v += 64) {
        const double x = p.xi[v], y = p.eta[v], wv = p.w[v];
        const double un = normal_speed(x, y, cL.nx, cL.ny);
        const bool mineL = un > 0.0 || (un == 0.0 && cL.tie);
        double fG, fH;
        if (mineL || F.type == FT_INTERIOR) {  // reconstructed by the upwind cell
            fG = fvG[v];
            fH = fvH[v];
        } else if (F.type == FT_WALL) {
            fG = r.rw * gw[v];
            fH = r.rw * KRTw * gw[v];
        } else {
            fG = p.ginf[v];
            fH = p.hinf[v];
        }
        const double M = tf[p.vix[v]] * tf[p.nvx + p.viy[v]];
        const RecT<double> rr = load_rec<double>(r);
        double eG, eH;
        eq_eval<double, false>(rr, x, y, M, eG, eH);
        double sG, sH;
        objective_seed<OBJ>(p, F, S, x, y, wv, un, sG, sH);
        const double dlG = lL[v] - (lR ? lR[v] : 0.0), dlH = lL[p.nvp + v] - (lR ? lR[p.nvp + v] : 0.0);
        const double pbG = -S * un * dlG + sG, pbH = -S * un * dlH + sH;
        acc[0] += pbG * (fG - eG) + pbH * (fH - eH);
        eq_adjoint_acc(r, x, y, M, (1.0 - al) * pbG, (1.0 - al) * pbH, acc + 1);
        acc[9] += sG * (al * fG + (1.0 - al) * eG) + sH * (al * fH + (1.0 - al) * eH);
    }
    wave_sum<10>(acc);
    double J[8][4];
    for (int mm = 0; mm < 8; ++mm)
        for (int a = 0; a < 4; ++a) J[mm][a] = p.jacf[(size_t)k * 32 + 4 * mm + a];
    const double t2h = 2.0 * r.tau + h;
    const double taubar = acc[0] * 2.0 * h / (t2h * t2h);
    double Wb[4];
    record_wbar(p, r, acc + 1, taubar, J, Wb);
    double th[3] = {0.0, 0.0, taubar * r.tau / p.Kn}, rwb = 0.0;
    if (OBJ == 1 && F.type == FT_WALL && F.wside == 3) {
        // J2 depends on the lid speed explicitly through |xi - U_w|^2
        double a[1] = {0.0};
        for (int v = lane; v < p.nv; v += 64) {
            const double x = p.xi[v], y = p.eta[v];
            const double un = normal_speed(x, y, cL.nx, cL.ny);
            const bool mineL = un > 0.0;
            const double fG = mineL ? fvG[v] : r.rw * gw[v];
            const double M = tf[p.vix[v]] * tf[p.nvx + p.viy[v]];
            const RecT<double> rr = load_rec<double>(r);
            double eG, eH;
            eq_eval<double, false>(rr, x, y, M, eG, eH);
            a[0] += S * p.w[v] * un * (-(x - p.wall_u[3])) * (al * fG + (1.0 - al) * eG);
        }
        wave_sum<1>(a);
        th[0] += a[0];
    }
    if (F.type == FT_WALL) {
        // incoming half: phi-bar = rho_w g_w(theta), rho_w = -sum_out w un phi-bar / wden(theta)
        const double *dgU = p.dgw + (size_t)ws * p.nvp, *dgT = p.dgw + (size_t)(4 + ws) * p.nvp;
        const double dKT = 0.5 * p.K;  // d(K RT_w)/dT_w
        double a[3] = {0.0, 0.0, 0.0};
        for (int v = lane; v < p.nv; v += 64) {
            const double x = p.xi[v], y = p.eta[v], wv = p.w[v];
            const double un = normal_speed(x, y, cL.nx, cL.ny);
            if (un > 0.0) continue;
            double sG, sH;
            objective_seed<OBJ>(p, F, S, x, y, wv, un, sG, sH);
            const double dlG = lL[v], dlH = lL[p.nvp + v];
            const double pbG = -S * un * dlG + sG, pbH = -S * un * dlH + sH;
            const double q2 = x * x + y * y;
            const double bbG = al * pbG + wv * (Wb[0] + x * Wb[1] + y * Wb[2] + 0.5 * q2 * Wb[3]);
            const double bbH = al * pbH + wv * 0.5 * Wb[3];
            a[0] += (bbG + bbH * KRTw) * gw[v];
            a[1] += r.rw * (bbG + bbH * KRTw) * dgU[v];
            a[2] += r.rw * (bbG * dgT[v] + bbH * (dKT * gw[v] + KRTw * dgT[v]));
        }
        wave_sum<3>(a);
        rwb = a[0];
        const double drw = -r.rw / p.wden[k];  // d(rho_w)/d(wden)
        if (ws == 3) th[0] += a[1] + rwb * drw * p.dwden[k];
        th[1] += a[2] + rwb * drw * p.dwden[p.nf + k];
    }
    if (lane == 0) {
        for (int a = 0; a < 4; ++a) fa[FA_WB + a] = Wb[a];
        fa[FA_RHOW] = rwb;
        for (int a = 0; a < 3; ++a) fa[FA_TH + a] = th[a];
        fa[FA_J] = acc[9];
    }
}

// Per cell and velocity: gather, from each face at which the cell is upwind, the adjoint of
// the reconstructed phi-bar_k into phi-bar-plus-bar (direct part) and sigma-bar.
template <int OBJ>
__global__ __launch_bounds__(256) void k_adj_gather(Params p) {
    const int c = xcd_remap(blockIdx.x, p.nc);
    const CellSide *cs = p.cs + 4 * c;
    const double h = p.h;
    const double *lc = p.lam + (size_t)c * 2 * p.nvp;
    double *out = p.agr + (size_t)c * 6 * p.nvp;
    for (int v = threadIdx.x; v < p.nv; v += blockDim.x) {
        const double x = p.xi[v], y = p.eta[v], wv = p.w[v], q2 = x * x + y * y;
        double dG = 0.0, dH = 0.0, sxG = 0.0, syG = 0.0, sxH = 0.0, syH = 0.0;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int type = cs[s].type;
            if (type == FT_SELF) continue;
            const double un = normal_speed(x, y, cs[s].nx, cs[s].ny);
            if (!(un > 0.0 || (un == 0.0 && cs[s].tie))) continue;
            const int k = cs[s].face;
            const double *fa = p.fadj + (size_t)k * FA_N;
            const double al = p.recf[k].alpha;
            double lnG = 0.0, lnH = 0.0;
            if (type == FT_INTERIOR) {
                const double *ln = p.lam + (size_t)cs[s].nb * 2 * p.nvp;
                lnG = ln[v];
                lnH = ln[p.nvp + v];
            }
            double sG = 0.0, sH = 0.0;
            if (type == FT_WALL) objective_seed<OBJ>(p, p.faces[k], cs[s].S, x, y, wv, un, sG, sH);
            const double pbG = -cs[s].S * un * (lc[v] - lnG) + sG;
            const double pbH = -cs[s].S * un * (lc[p.nvp + v] - lnH) + sH;
            double bbG = al * pbG + wv * (fa[0] + x * fa[1] + y * fa[2] + 0.5 * q2 * fa[3]);
            const double bbH = al * pbH + wv * 0.5 * fa[3];
            if (type == FT_WALL) bbG += -fa[FA_RHOW] * wv * un / p.wden[k];
            const double rx = cs[s].dx - h * x, ry = cs[s].dy - h * y;
            dG += bbG; dH += bbH;
            sxG += bbG * rx; syG += bbG * ry; sxH += bbH * rx; syH += bbH * ry;
        }
        out[v] = dG;
        out[p.nvp + v] = dH;
        out[2 * p.nvp + v] = sxG;
        out[3 * p.nvp + v] = syG;
        out[4 * p.nvp + v] = sxH;
        out[5 * p.nvp + v] = syH;
    }
}

// Per cell: phi-bar-plus-bar = direct + sum_j a_ji sigma-bar_j - (sum_j a_ij) sigma-bar_i,
// then the collision term, phi-bar-plus and the cell record in reverse, and the moments.
__global__ __launch_bounds__(256) void k_adj_cell(Params p) {
    __shared__ double sh[4 * 11];
    __shared__ double wb[5];
    const int c = xcd_remap(blockIdx.x, p.nc);
    const CellSide *cs = p.cs + 4 * c;
    const Rec r = p.rec[c];
    const double *tb = (const double *)p.tab + (size_t)c * (p.nvx + p.nvy);
    const double sc = p.scal[SC_SCALE];
    const double t2d = 2.0 * r.tau + p.dt, cc = 2.0 * p.area[c] / t2d;
    double Ax = 0.0, Ay = 0.0;
    for (int s = 0; s < 4; ++s)
        if (cs[s].nb >= 0 && cs[s].nb != c) { Ax += cs[s].ax; Ay += cs[s].ay; }
    const double *own = p.agr + (size_t)c * 6 * p.nvp;
    const double *lc = p.lam + (size_t)c * 2 * p.nvp;
    const double *fc = (const double *)p.f + (size_t)c * 2 * p.nvp;
    double *fb = p.fbar + (size_t)c * 2 * p.nvp;
    double acc[11];
    for (int i = 0; i < 11; ++i) acc[i] = 0.0;
    const RecT<double> rr = load_rec<double>(r);
    for (int v = threadIdx.x; v < p.nv; v += blockDim.x) {
        const double x = p.xi[v], y = p.eta[v];
        double pG = own[v] - (Ax * own[2 * p.nvp + v] + Ay * own[3 * p.nvp + v]);
        double pH = own[p.nvp + v] - (Ax * own[4 * p.nvp + v] + Ay * own[5 * p.nvp + v]);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = cs[s].nb;
            if (j < 0 || j == c) continue;
            const CellSide &cj = p.cs[4 * j + (s ^ 1)];
            const double *oj = p.agr + (size_t)j * 6 * p.nvp;
            pG += cj.ax * oj[2 * p.nvp + v] + cj.ay * oj[3 * p.nvp + v];
            pH += cj.ax * oj[4 * p.nvp + v] + cj.ay * oj[5 * p.nvp + v];
        }
        const double M = tb[p.vix[v]] * tb[p.nvx + p.viy[v]];
        double eG, eH;
        eq_eval<double, false>(rr, x, y, M, eG, eH);
        const double lG = lc[v], lH = lc[p.nvp + v];
        const double XG = sc * fc[v], XH = sc * fc[p.nvp + v];
        fb[v] = -cc * lG + r.ab * pG;
        fb[p.nvp + v] = -cc * lH + r.ab * pH;
        acc[0] += -(lG * (XG - eG) + lH * (XH - eH));   // c-bar
        acc[1] += pG * XG + pH * XH;                     // a-bar
        acc[2] += pG * eG + pH * eH;                     // b-bar
        eq_adjoint_acc(r, x, y, M, cc * lG + r.bb * pG, cc * lH + r.bb * pH, acc + 3);
    }
    block_sum<11>(acc, sh);
    {
        double J[8][4];
        for (int mm = 0; mm < 8; ++mm)
            for (int a = 0; a < 4; ++a) J[mm][a] = p.jacc[(size_t)c * 32 + 4 * mm + a];
        if (threadIdx.x == 0) {
            const double taubar = acc[0] * (-2.0 * cc / t2d) + acc[1] * 2.0 * (p.dt + p.h) / (t2d * t2d) +
                                  acc[2] * (-6.0 * p.h) / (t2d * t2d);
            double Wb[4];
            record_wbar(p, r, acc + 3, taubar, J, Wb);
            for (int a = 0; a < 4; ++a) wb[a] = Wb[a];
            wb[4] = taubar * r.tau / p.Kn;
        }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < p.nv; v += blockDim.x) {
        const double x = p.xi[v], y = p.eta[v], wv = p.w[v];
        fb[v] += wv * (wb[0] + x * wb[1] + y * wb[2] + 0.5 * (x * x + y * y) * wb[3]);
        fb[p.nvp + v] += wv * 0.5 * wb[3];
    }
    if (threadIdx.x < CA_N) p.cadj[(size_t)c * CA_N + threadIdx.x] = threadIdx.x < 4 ? wb[threadIdx.x] : wb[4];
}

// Record Jacobians d p / d W of all cells (which = 0) or faces (1), one wave each; they
// depend on the state only, so one evaluation serves every product at that state.
__global__ __launch_bounds__(256) void k_rec_jac(Params p, int which) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int n = which ? p.nf : p.nc;
    if (k >= n) return;
    double *out = (which ? p.jacf : p.jacc) + (size_t)k * 32;
    if (which && p.faces[k].type == FT_SELF) {
        if (lane < 32) out[lane] = 0.0;
        return;
    }
    const Rec r = which ? p.recf[k] : p.rec[k];
    double W[4], J[8][4];
    rec_W(p, r, W);
    record_jacobian(p, W, J, lane);
    if (lane == 0)
        for (int mm = 0; mm < 8; ++mm)
            for (int a = 0; a < 4; ++a) out[4 * mm + a] = J[mm][a];
}

// theta-bar and J: fixed-order sums of the face and cell parts (one block); out[0..2]
// theta-bar, out[3] J
__global__ __launch_bounds__(1024) void k_adj_theta(Params p, double *out) {
    __shared__ double sh[16 * 4];
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < p.nf; k += blockDim.x) {
        const double *fa = p.fadj + (size_t)k * FA_N;
        a[0] += fa[FA_TH];
        a[1] += fa[FA_TH + 1];
        a[2] += fa[FA_TH + 2];
        a[3] += fa[FA_J];
    }
    for (int c = threadIdx.x; c < p.nc; c += blockDim.x) a[2] += p.cadj[(size_t)c * CA_N + CA_TH];
    block_sum_store<4>(a, sh, out);
}

// ---- vectors of the adjoint iteration (FP64, device layout [nc][2][nvp], pad lanes 0) ----
// partial sums of a.b over blocks (fixed order within a block)
__global__ __launch_bounds__(256) void k_dot(Params p, const double *a, const double *b, double scale_a, int nblk) {
    __shared__ double sh[4];
    double s[1] = {0.0};
    const size_t n = (size_t)p.nc * 2 * p.nvp;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)nblk * blockDim.x)
        s[0] += scale_a * a[t] * b[t];
    block_sum_store<1>(s, sh, p.red + blockIdx.x);
}

// out[0] = sum of the nblk partials (fixed order)
__global__ void k_dot_final(Params p, int nblk, double *out) {
    __shared__ double sh[4];
    double s[1] = {0.0};
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s[0] += p.red[i];
    block_sum_store<1>(s, sh, out);
}

// y = lt - l_M (f*.lt) / M0 (l_M = area w on G; f* = scale f, the stored state times its
// pending mass scale; dot = f.lt), written to y and to the sweep input d1
__global__ __launch_bounds__(256) void k_adj_project(Params p, const double *lt, double *y, const double *dot) {
    const size_t n = (size_t)p.nc * 2 * p.nvp;
    const double k = dot[0] * p.scal[SC_SCALE] / p.M0;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / (2 * (size_t)p.nvp)), r = (int)(t % (2 * (size_t)p.nvp));
        const int sp = r / p.nvp, v = r % p.nvp;
        double val = v < p.nv ? lt[t] : 0.0;
        if (sp == 0 && v < p.nv) val -= p.area[c] * p.w[v] * k;
        y[t] = val;
        ((double *)p.d1)[t] = val;
    }
}

// lt_new = y + fbar + g; partial sums of |lt_new - lt|^2 and |lt_new|^2 per block
__global__ __launch_bounds__(256) void k_adj_update(Params p, double *lt, const double *y, const double *g, int nblk) {
    __shared__ double sh[8];
    double s[2] = {0.0, 0.0};
    const size_t n = (size_t)p.nc * 2 * p.nvp;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)nblk * blockDim.x) {
        const double nw = y[t] + p.fbar[t] + g[t];
        const double d = nw - lt[t];
        s[0] += d * d;
        s[1] += nw * nw;
        lt[t] = nw;
    }
    block_sum_store<2>(s, sh, p.red + 2 * blockIdx.x);
}

__global__ void k_adj_update_final(Params p, int nblk, double *out) {
    __shared__ double sh[8];
    double s[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) { s[0] += p.red[2 * i]; s[1] += p.red[2 * i + 1]; }
    block_sum_store<2>(s, sh, out);
}

// srec base of the adjoint sweeps: Omega/dt_imp + c of the current record (no predictor)
__global__ __launch_bounds__(256) void k_adj_diag(Params p) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.nc) return;
    const double cc = 2.0 * p.area[c] / (2.0 * p.rec[c].tau + p.dt);
    double *row = p.srec + (size_t)p.hp_pos[c] * SR_N;
    row[10] = cc;
    row[11] = p.area[c] / p.dtimp[c] + cc;
}

// copy between the canonical [2][nc][nv] layout and the device layout
__global__ void k_to_dev(Params p, const double *src, double *dst) {
    const size_t n = (size_t)p.nc * 2 * p.nvp;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int c = (int)(t / (2 * (size_t)p.nvp)), r = (int)(t % (2 * (size_t)p.nvp));
        const int s = r / p.nvp, v = r % p.nvp;
        dst[t] = v < p.nv ? src[((size_t)s * p.nc + c) * p.nv + v] : 0.0;
    }
}

__global__ void k_from_dev(Params p, const double *src, double *dst, double scale) {
    const size_t n = (size_t)p.nc * p.nv;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < 2 * n; t += (size_t)gridDim.x * blockDim.x) {
        const int s = (int)(t / n);
        const size_t r = t % n;
        const int c = (int)(r / p.nv), v = (int)(r % p.nv);
        dst[t] = scale * src[((size_t)c * 2 + s) * p.nvp + v];
    }
}

// ---------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------
#define DISPATCH_S(fp32, ...) \
    do { if (fp32) { using S = float; __VA_ARGS__; } else { using S = double; __VA_ARGS__; } } while (0)

hipError_t launch_raw(const Params &p, bool fp32, int nm, hipStream_t st) {
    DISPATCH_S(fp32, {
        const dim3 g((p.nc + RW_W - 1) / RW_W);
        if (nm == 12) hipLaunchKernelGGL((k_raw<S, 12>), g, dim3(64 * RW_W), 0, st, p);
        else hipLaunchKernelGGL((k_raw<S, 4>), g, dim3(64 * RW_W), 0, st, p);
    });
    return hipGetLastError();
}

hipError_t launch_finalize(const Params &p, bool fp32, int mode, hipStream_t st) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, st, p, mode, fp32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_records(const Params &p, bool fp32, int which, hipStream_t st) {
    const dim3 g((p.nc + 3) / 4);
    DISPATCH_S(fp32, {
        if (p.model == 1) hipLaunchKernelGGL((k_records<S, true>), g, dim3(256), 0, st, p, which);
        else hipLaunchKernelGGL((k_records<S, false>), g, dim3(256), 0, st, p, which);
    });
    return hipGetLastError();
}

static dim3 chunk_grid(const Params &p, int nch) { return dim3(((p.nc + 7) & ~7) * nch); }

static hipError_t combine(const double *src, double *dst, const Params &p, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_combine, dim3((p.nc * n + 255) / 256), dim3(256), 0, st, src, dst, p.nc, p.nch, n);
    return hipGetLastError();
}

// the factored Maxwellians of the five cells go to LDS when they take at most 16 KiB
template <class S, bool SHAK, bool LIM>
static void launch_partials_t(const Params &p, hipStream_t st) {
    const dim3 g = chunk_grid(p, 1);
    const size_t xy = (size_t)(p.nvx + p.nvy) * sizeof(double), tl = (size_t)5 * (p.nvx + p.nvy) * sizeof(S);
    if (tl <= 16384) hipLaunchKernelGGL((k_partials<S, SHAK, LIM, true>), g, dim3(256), xy + tl, st, p);
    else hipLaunchKernelGGL((k_partials<S, SHAK, LIM, false>), g, dim3(256), xy, st, p);
}

hipError_t launch_partials(const Params &p, bool fp32, hipStream_t st) {
    DISPATCH_S(fp32, {
        if (p.model == 1) {
            if (p.limiter) launch_partials_t<S, true, true>(p, st);
            else launch_partials_t<S, true, false>(p, st);
        } else {
            if (p.limiter) launch_partials_t<S, false, true>(p, st);
            else launch_partials_t<S, false, false>(p, st);
        }
    });
    return hipGetLastError();
}

hipError_t launch_face_records(const Params &p, bool fp32, hipStream_t st) {
    const dim3 g((p.nf + FR_W - 1) / FR_W);
    DISPATCH_S(fp32, {
        if (p.model == 1) hipLaunchKernelGGL((k_face_records<S, true>), g, dim3(64 * FR_W), 0, st, p);
        else hipLaunchKernelGGL((k_face_records<S, false>), g, dim3(64 * FR_W), 0, st, p);
    });
    return hipGetLastError();
}

// the factored Maxwellians of the four faces go to LDS when they take at most 16 KiB
template <class S, bool SHAK>
static void launch_flux_t(const Params &p, hipStream_t st) {
    const dim3 g = chunk_grid(p, p.nch);
    const size_t xy = (size_t)2 * (p.nvx + p.nvy) * sizeof(double), tl = (size_t)4 * (p.nvx + p.nvy) * sizeof(S);
    if (p.prep_in_flux) {  // one chunk per cell (checked by the caller)
        if (tl <= 16384) hipLaunchKernelGGL((k_flux<S, SHAK, true, true>), g, dim3(256), xy + tl, st, p);
        else hipLaunchKernelGGL((k_flux<S, SHAK, false, true>), g, dim3(256), xy, st, p);
    } else {
        if (tl <= 16384) hipLaunchKernelGGL((k_flux<S, SHAK, true, false>), g, dim3(256), xy + tl, st, p);
        else hipLaunchKernelGGL((k_flux<S, SHAK, false, false>), g, dim3(256), xy, st, p);
    }
}

hipError_t launch_flux(const Params &p, bool fp32, hipStream_t st) {
    DISPATCH_S(fp32, {
        if (p.model == 1) launch_flux_t<S, true>(p, st);
        else launch_flux_t<S, false>(p, st);
    });
    if (p.nch > 1) return combine(p.MWc, p.MW, p, 4, st);
    return hipGetLastError();
}

static int round64(int n) { return (n + 63) / 64 * 64; }

// The deepest staging prefetch first (fewest values per staging lane: 32 registers hold
// MD x SPWM values), then the most lanes per cell (4 or 2), that fit 1024 lanes.  Meshes
// too wide for that are rejected at init (their LDS would not fit either).
MacroShape macro_shape(int ni, int nj, bool per_i, bool per_j) {
    const int L = ni < nj ? ni : nj, nh = ni + nj - 1;
    auto waves = [&](int spw) { return (L * MH_N + 64 * spw - 1) / (64 * spw); };
    MacroShape m{};
    for (int spw = 4; spw <= 16; spw *= 2) {
        for (int lpc = 4; lpc >= 2; lpc /= 2) {
            m.lpc = lpc;
            m.spw = spw;
            m.nct = round64(lpc * L);
            m.threads = m.nct + 64 * waves(spw);
            if (m.threads <= 1024) break;
        }
        if (m.threads <= 1024) break;
    }
    const int seams = (per_i ? nj : 0) + (per_j ? ni : 0);
    m.lds = (size_t)(MF * (2 * ni + 3 + seams) + 2 * L * MH_N + 8 * L) * sizeof(double) + (size_t)(nh + 1) * sizeof(int);
    return m;
}

template <int LPC, int SPWM>
static hipError_t launch_macro_t(const Params &p, const MacroShape &m, hipStream_t st) {
    constexpr int MD = 32 / SPWM;
    const void *fn = (const void *)k_macro_sweep<LPC, SPWM, MD>;
    if (m.lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)m.lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_macro_sweep<LPC, SPWM, MD>), dim3(1), dim3(m.threads), m.lds, st, p, m.nct);
    return hipGetLastError();
}

template <int LPC>
static hipError_t launch_macro_l(const Params &p, const MacroShape &m, hipStream_t st) {
    switch (m.spw) {
    case 4: return launch_macro_t<LPC, 4>(p, m, st);
    case 8: return launch_macro_t<LPC, 8>(p, m, st);
    default: return launch_macro_t<LPC, 16>(p, m, st);
    }
}

hipError_t launch_macro_prep(const Params &p, hipStream_t st) {
    hipLaunchKernelGGL(k_macro_prep, dim3((p.nc + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

// sweeps 0 .. relax_sweeps alternate between dWr and dW so that the last one writes dW
hipError_t launch_macro_relax(const Params &p, hipStream_t st) {
    const dim3 g((p.nc + 255) / 256);
    double *buf[2] = {p.dW, p.dWr};
    int o = p.relax_sweeps % 2 == 0 ? 0 : 1;
    hipLaunchKernelGGL(k_macro_relax<true>, g, dim3(256), 0, st, p, (const double *)nullptr, buf[o]);
    for (int k = 1; k <= p.relax_sweeps; ++k) {
        hipLaunchKernelGGL(k_macro_relax<false>, g, dim3(256), 0, st, p, (const double *)buf[o], buf[1 - o]);
        o = 1 - o;
    }
    return hipGetLastError();
}

hipError_t launch_macro(const Params &p, hipStream_t st) {
    if (p.gmacro) {
        hipLaunchKernelGGL(k_gmacro, dim3(1), dim3(G2_THREADS), 0, st, p);
        return hipGetLastError();
    }
    const MacroShape m = macro_shape(p.ni, p.nj, p.per_i, p.per_j);
    return m.lpc == 4 ? launch_macro_l<4>(p, m, st) : launch_macro_l<2>(p, m, st);
}

// Velocities per sweep block: the largest slice (at most 16) that fits one block of at
// most 1024 lanes with the staging waves and 150 KiB of LDS and still gives at least 192
// blocks; else the smallest slice that fits.
SweepShape sweep_shape(int ni, int nj, int nv, size_t s_bytes) {
    const int L = ni < nj ? ni : nj, nh = ni + nj - 1;
    // staging waves: KP = 64 nsw / STG cells per pass, SPW_MICRO passes must cover L cells
    int nsw = 1;
    while ((64 * nsw / STG) * SPW_MICRO < L) ++nsw;
    auto lds_of = [&](int w) {
        return ((size_t)2 * (3 * ni + nj + 3) * w + (size_t)2 * L * STG) * s_bytes + (size_t)(nh + 1) * sizeof(int);
    };
    SweepShape best{0, 0, 0, 0, 0};
    for (int vb = 16; vb >= 1; vb /= 2) {
        SweepShape c;
        c.vb = vb;
        c.vpl = 1;
        c.nct = round64(vb * L);
        c.threads = c.nct + 64 * nsw;
        c.lds = lds_of(vb);
        if (c.threads > 1024 || c.lds > 150 * 1024) continue;
        best = c;
        if ((nv + vb - 1) / vb >= 192) break;
    }
    // FP32 with slices to spare: two velocities per lane halve the slices, and each staged
    // row serves twice the velocities
    if (best.vb && s_bytes == 4) {
        SweepShape c = best;
        c.vpl = 2;
        c.lds = lds_of(2 * c.vb);
        if (c.lds <= 150 * 1024 && (nv + 2 * c.vb - 1) / (2 * c.vb) >= 1024) best = c;
    }
    return best;
}

template <class S, bool SHAK, bool UPPER, bool ADJ, int VPL>
static hipError_t sweep_launch(const Params &p, const SweepShape &sh, hipStream_t st) {
    const void *fn = (const void *)k_sweep<S, SHAK, UPPER, ADJ, VPL>;
    if (sh.lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh.lds);
        if (e != hipSuccess) return e;
    }
    const dim3 g((p.nv + sh.vb * VPL - 1) / (sh.vb * VPL));
    hipLaunchKernelGGL((k_sweep<S, SHAK, UPPER, ADJ, VPL>), g, dim3(sh.threads), sh.lds, st, p, sh.vb, sh.nct);
    return hipGetLastError();
}

// two velocities per lane exist for the FP32 state only
template <class S, bool SHAK, bool UPPER>
static hipError_t sweep_launch_v(const Params &p, const SweepShape &sh, hipStream_t st) {
    if constexpr (sizeof(S) == 4) {
        if (sh.vpl == 2) return sweep_launch<S, SHAK, UPPER, false, 2>(p, sh, st);
    }
    return sweep_launch<S, SHAK, UPPER, false, 1>(p, sh, st);
}

// cells per wave and batch within the 128 registers of a 16-wave block: FP32 eight in the
// backward sweep (a level of up to 128 cells in one batch) and six in the forward one
// (whose cells also load the two Maxwellian factors; seven fill the registers, eight are
// slower), FP64 three
template <class S, bool SHAK, bool UPPER>
static hipError_t gsweep_launch(const Params &p, hipStream_t st) {
    constexpr int CB = sizeof(S) == 4 ? (UPPER ? 8 : 6) : 3;
    hipLaunchKernelGGL((k_gsweep<S, SHAK, UPPER, CB>), dim3(p.nvp / 64), dim3(GS_THREADS), 0, st, p,
                       p.grow, (const S *)p.growT);
    return hipGetLastError();
}

hipError_t launch_sweep(const Params &p, bool fp32, bool upper, const SweepShape &sh, hipStream_t st) {
    if (p.graph) {
        DISPATCH_S(fp32, {
            if (p.model == 1) return upper ? gsweep_launch<S, true, true>(p, st) : gsweep_launch<S, true, false>(p, st);
            return upper ? gsweep_launch<S, false, true>(p, st) : gsweep_launch<S, false, false>(p, st);
        });
        return hipSuccess;
    }
    if (!fp32 && sh.vpl != 1) return hipErrorInvalidValue;
    DISPATCH_S(fp32, {
        if (p.model == 1) return upper ? sweep_launch_v<S, true, true>(p, sh, st) : sweep_launch_v<S, true, false>(p, sh, st);
        return upper ? sweep_launch_v<S, false, true>(p, sh, st) : sweep_launch_v<S, false, false>(p, sh, st);
    });
    return hipSuccess;
}

hipError_t launch_wall_ghost(const Params &p, bool fp32, hipStream_t st) {
    if (p.nwall == 0) return hipSuccess;
    const dim3 g((p.nwall + FR_W - 1) / FR_W);
    DISPATCH_S(fp32, hipLaunchKernelGGL((k_wall_ghost<S>), g, dim3(64 * FR_W), 0, st, p));
    return hipGetLastError();
}

hipError_t launch_explicit(const Params &p, bool fp32, hipStream_t st) {
    DISPATCH_S(fp32, {
        if (p.model == 1) hipLaunchKernelGGL((k_explicit<S, true>), dim3(p.nc), dim3(256), 0, st, p);
        else hipLaunchKernelGGL((k_explicit<S, false>), dim3(p.nc), dim3(256), 0, st, p);
    });
    return hipGetLastError();
}

hipError_t launch_pack(const Params &p, bool fp32, const void *src, double *dst, int sp, int nsp,
                       int scaled, hipStream_t st) {
    DISPATCH_S(fp32, hipLaunchKernelGGL((k_pack<S>), dim3(2048), dim3(256), 0, st, p, src, dst, sp,
                                        nsp, scaled));
    return hipGetLastError();
}

hipError_t launch_unpack(const Params &p, bool fp32, const double *src, int sp, int nsp,
                         hipStream_t st) {
    DISPATCH_S(fp32, hipLaunchKernelGGL((k_unpack<S>), dim3(2048), dim3(256), 0, st, p, src, sp, nsp));
    return hipGetLastError();
}

hipError_t launch_fill_uniform(const Params &p, bool fp32, const double *eq, hipStream_t st) {
    DISPATCH_S(fp32, hipLaunchKernelGGL((k_fill_uniform<S>), dim3(2048), dim3(256), 0, st, p, eq));
    return hipGetLastError();
}

hipError_t launch_fields(const Params &p, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_fields, dim3((p.nc + 255) / 256), dim3(256), 0, st, p, out);
    return hipGetLastError();
}

// ---- sensitivities ---------------------------------------------------------------------
hipError_t launch_adj_face(const Params &p, int obj, hipStream_t st) {
    const dim3 g((p.nf + 3) / 4);
    if (obj == 0) hipLaunchKernelGGL((k_adj_face<0>), g, dim3(256), 0, st, p);
    else if (obj == 1) hipLaunchKernelGGL((k_adj_face<1>), g, dim3(256), 0, st, p);
    else hipLaunchKernelGGL((k_adj_face<-1>), g, dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_adj_gather(const Params &p, int obj, hipStream_t st) {
    if (obj == 0) hipLaunchKernelGGL((k_adj_gather<0>), dim3(p.nc), dim3(256), 0, st, p);
    else if (obj == 1) hipLaunchKernelGGL((k_adj_gather<1>), dim3(p.nc), dim3(256), 0, st, p);
    else hipLaunchKernelGGL((k_adj_gather<-1>), dim3(p.nc), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_rec_jac(const Params &p, hipStream_t st) {
    hipLaunchKernelGGL(k_rec_jac, dim3((p.nc + 3) / 4), dim3(256), 0, st, p, 0);
    hipLaunchKernelGGL(k_rec_jac, dim3((p.nf + 3) / 4), dim3(256), 0, st, p, 1);
    return hipGetLastError();
}

hipError_t launch_adj_cell(const Params &p, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_cell, dim3(p.nc), dim3(256), 0, st, p);
    return hipGetLastError();
}

hipError_t launch_adj_theta(const Params &p, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_theta, dim3(1), dim3(1024), 0, st, p, out);
    return hipGetLastError();
}

hipError_t launch_adj_sweep(const Params &p, bool upper, const SweepShape &sh, hipStream_t st) {
    if (sh.vpl != 1) return hipErrorInvalidValue;  // the sensitivities run on the FP64 state
    return upper ? sweep_launch<double, false, true, true, 1>(p, sh, st)
                 : sweep_launch<double, false, false, true, 1>(p, sh, st);
}

hipError_t launch_adj_diag(const Params &p, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_diag, dim3((p.nc + 255) / 256), dim3(256), 0, st, p);
    return hipGetLastError();
}

static int red_blocks(const Params &p) {
    const size_t n = (size_t)p.nc * 2 * p.nvp;
    size_t b = (n + 255) / 256;
    return (int)(b < RED_N / 2 ? b : RED_N / 2);
}

hipError_t launch_dot(const Params &p, const double *a, const double *b, double scale_a, double *out, hipStream_t st) {
    const int nb = red_blocks(p);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(256), 0, st, p, a, b, scale_a, nb);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(256), 0, st, p, nb, out);
    return hipGetLastError();
}

hipError_t launch_adj_project(const Params &p, const double *lt, double *y, const double *dot, hipStream_t st) {
    hipLaunchKernelGGL(k_adj_project, dim3(2048), dim3(256), 0, st, p, lt, y, dot);
    return hipGetLastError();
}

hipError_t launch_adj_update(const Params &p, double *lt, const double *y, const double *g, double *out, hipStream_t st) {
    const int nb = red_blocks(p);
    hipLaunchKernelGGL(k_adj_update, dim3(nb), dim3(256), 0, st, p, lt, y, g, nb);
    hipLaunchKernelGGL(k_adj_update_final, dim3(1), dim3(256), 0, st, p, nb, out);
    return hipGetLastError();
}

hipError_t launch_to_dev(const Params &p, const double *src, double *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_to_dev, dim3(2048), dim3(256), 0, st, p, src, dst);
    return hipGetLastError();
}

hipError_t launch_from_dev(const Params &p, const double *src, double *dst, double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_from_dev, dim3(2048), dim3(256), 0, st, p, src, dst, scale);
    return hipGetLastError();
}

}  // namespace idugks
