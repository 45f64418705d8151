// Launchers of the HIP kernels (defined in idugks_kernels.hip).  Every launcher enqueues
// on the given stream and returns hipGetLastError().
#pragma once

#include <hip/hip_runtime.h>

#include "idugks_internal.hpp"

namespace idugks {

hipError_t launch_raw(const Params &p, bool fp32, int nm, hipStream_t st);
hipError_t launch_finalize(const Params &p, int mode, hipStream_t st);
hipError_t launch_records(const Params &p, bool fp32, int which, hipStream_t st);
hipError_t launch_partials(const Params &p, bool fp32, hipStream_t st);
hipError_t launch_face_records(const Params &p, bool fp32, hipStream_t st);
hipError_t launch_flux(const Params &p, bool fp32, hipStream_t st);
// Launch shapes of the hyperplane sweeps: block = nct compute lanes + staging waves.
struct MacroShape {
    int nct, threads;
    size_t lds;
};
struct SweepShape {
    int vb, nct, threads;  // vb = 0: no shape fits
    size_t lds;
};
MacroShape macro_shape(int ni, int nj);
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
hipError_t launch_fields(const Params &p, double *out, hipStream_t st);

}  // namespace idugks
