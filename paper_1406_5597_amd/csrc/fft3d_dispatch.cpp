// fft3d_dispatch.cpp -- host-side selection of the per-dtype kernel entry
// points, and the device set-up of the cooperative plane step.
#include "fft3d_batch.hpp"
#include "fft3d_internal.hpp"

namespace fft3d {

// The entry point of the plan's dtype, from the kernels compiled with radix-5/7 stages
// when the plan has them.
#define FFT3D_PICK(p, name, ...)                                                                   \
    ((p).dtype ? ((p).odd ? name##_f64_odd(__VA_ARGS__) : name##_f64(__VA_ARGS__))                 \
               : ((p).odd ? name##_f32_odd(__VA_ARGS__) : name##_f32(__VA_ARGS__)))

hipError_t coop_setup(Plan& p)
{
    if (!p.coop) return hipSuccess;
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = p.dtype ? coop_occupancy_f64(p, &per_cu) : coop_occupancy_f32(p, &per_cu);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    p.coop_grid = cus * per_cu;
    const int tasks = p.coop_rt + p.coop_ct;
    // slots per queue: every plane, the first empty slot, the lag, and one
    // slot per workgroup that may still take tickets beyond them before it
    // reaches a second-phase ticket of an empty plane and leaves
    (void)tasks;
    p.coop_nslots = (int)p.n0 + p.coop_lag + p.coop_grid + 2;
    p.coop_ctr_count = 2 + kCoopQueues + (int64_t)kCoopQueues * 2 * p.coop_nslots;
    e = hipMalloc(&p.d_ctr, (size_t)p.coop_ctr_count * sizeof(int));
    if (e != hipSuccess) return e;
    return hipMemset(p.d_ctr, 0, (size_t)p.coop_ctr_count * sizeof(int));
}

// Raising the dynamic-LDS limit is advisory: a launch that still exceeds what
// the device allows fails with a launch error, which the callers report.
hipError_t kernels_init()
{
    (void)init_plain_f32();
    (void)init_plain_f64();
    (void)init_coop_f32();
    (void)init_coop_f64();
    (void)init_pruned_f32();
    (void)init_pruned_f64();
    (void)init_plain_f32_odd();
    (void)init_plain_f64_odd();
    (void)init_pruned_f32_odd();
    (void)init_pruned_f64_odd();
    (void)init_batch();
    (void)init_level();
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t launch_plane_coop(const Plan& p, const void* in, void* out, bool inverse, hipStream_t st)
{
    return p.dtype ? launch_plane_coop_f64(p, in, out, inverse, st) : launch_plane_coop_f32(p, in, out, inverse, st);
}
hipError_t launch_swap01(const Plan& p, const void* in, void* out, int64_t na, int64_t nb, hipStream_t st)
{
    return FFT3D_PICK(p, launch_swap01, p, in, out, na, nb, st);
}
hipError_t launch_pruned_r2c(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t st)
{
    return FFT3D_PICK(p, launch_pruned_r2c, p, x, X, b, st);
}
hipError_t launch_pruned_c2r(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b,
                             hipStream_t st)
{
    return FFT3D_PICK(p, launch_pruned_c2r, p, X, y, work, b, st);
}
hipError_t launch_plane_r2c(const Plan& p, const void* x, void* X, hipStream_t st, bool padded)
{
    return FFT3D_PICK(p, launch_plane_r2c, p, x, X, st, padded);
}
hipError_t launch_plane_c2r(const Plan& p, const void* X, void* y, hipStream_t st, bool padded)
{
    return FFT3D_PICK(p, launch_plane_c2r, p, X, y, st, padded);
}
hipError_t launch_rows_r2c(const Plan& p, const void* x, void* X, int64_t nrows, int rev, hipStream_t st,
                           bool padded)
{
    return FFT3D_PICK(p, launch_rows_r2c, p, x, X, nrows, rev, st, padded);
}
hipError_t launch_rows_c2r(const Plan& p, const void* X, void* y, int64_t nrows, int rev, hipStream_t st,
                           bool padded)
{
    return FFT3D_PICK(p, launch_rows_c2r, p, X, y, nrows, rev, st, padded);
}
hipError_t launch_cols(const Plan& p, const ColPass& cp, int axis, int64_t tw_off, const void* in, void* out,
                       bool inverse, int rev, hipStream_t st)
{
    return FFT3D_PICK(p, launch_cols, p, cp, axis, tw_off, in, out, inverse, rev, st);
}

}  // namespace fft3d
