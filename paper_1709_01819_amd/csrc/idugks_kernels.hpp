// Launchers of the HIP kernels (defined in idugks_kernels.hip).  Every launcher enqueues
// on the given stream and returns hipGetLastError().
#pragma once

#include <hip/hip_runtime.h>

#include "idugks_internal.hpp"

namespace idugks {

hipError_t launch_raw(const Params &p, bool fp32, int nm, hipStream_t st);
hipError_t launch_finalize(const Params &p, bool fp32, int mode, hipStream_t st);
hipError_t launch_records(const Params &p, bool fp32, int which, hipStream_t st);
hipError_t launch_partials(const Params &p, bool fp32, hipStream_t st);
hipError_t launch_face_records(const Params &p, bool fp32, hipStream_t st);
hipError_t launch_flux(const Params &p, bool fp32, hipStream_t st);
// Launch shapes of the hyperplane sweeps: block = nct compute lanes + staging waves.
struct MacroShape {
    int lpc, spw;  // compute lanes per cell, staged values per staging lane
    int nct, threads;
    size_t lds;
};
struct SweepShape {
    int vb, vpl, nct, threads;  // velocity columns per slot and velocities per lane;
    size_t lds;                 // vb = 0: no shape fits
};
MacroShape macro_shape(int ni, int nj, bool per_i, bool per_j);
hipError_t launch_macro_relax(const Params &p, hipStream_t st);
SweepShape sweep_shape(int ni, int nj, int nv, size_t s_bytes);
hipError_t launch_macro_prep(const Params &p, hipStream_t st);  // k_macro_prep
hipError_t launch_macro(const Params &p, hipStream_t st);       // k_macro_sweep (after the prep)
hipError_t launch_sweep(const Params &p, bool fp32, bool upper, const SweepShape &sh, hipStream_t st);
hipError_t launch_wall_ghost(const Params &p, bool fp32, hipStream_t st);
hipError_t launch_explicit(const Params &p, bool fp32, hipStream_t st);
hipError_t launch_pack(const Params &p, bool fp32, const void *src, double *dst, int sp, int nsp,
                       int scaled, hipStream_t st);
hipError_t launch_unpack(const Params &p, bool fp32, const double *src, int sp, int nsp,
                         hipStream_t st);
hipError_t launch_fill_uniform(const Params &p, bool fp32, const double *eq, hipStream_t st);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);  // bytes: a multiple of 16
hipError_t launch_fields(const Params &p, double *out, hipStream_t st);

// sensitivities (FP64 state, BGK, no limiter); obj: -1 none, 0 lid x-momentum flux,
// 1 wall heat flux
hipError_t launch_rec_jac(const Params &p, hipStream_t st);
hipError_t launch_adj_face(const Params &p, int obj, hipStream_t st);
hipError_t launch_adj_gather(const Params &p, int obj, hipStream_t st);
hipError_t launch_adj_cell(const Params &p, hipStream_t st);
hipError_t launch_adj_theta(const Params &p, double *out, hipStream_t st);
hipError_t launch_adj_sweep(const Params &p, bool upper, const SweepShape &sh, hipStream_t st);
hipError_t launch_adj_diag(const Params &p, hipStream_t st);
hipError_t launch_dot(const Params &p, const double *a, const double *b, double scale_a, double *out, hipStream_t st);
hipError_t launch_adj_project(const Params &p, const double *lt, double *y, const double *dot, hipStream_t st);
hipError_t launch_adj_update(const Params &p, double *lt, const double *y, const double *g, double *out, hipStream_t st);
hipError_t launch_to_dev(const Params &p, const double *src, double *dst, hipStream_t st);
hipError_t launch_from_dev(const Params &p, const double *src, double *dst, double scale, hipStream_t st);

}  // namespace idugks
