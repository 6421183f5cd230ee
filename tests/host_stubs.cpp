// host_stubs.cpp -- the device half of libfft3d replaced by functions that
// report "not supported", so that the library's host code (plans, tunings,
// the tuning table, the server in its no-device mode, the C interface) can be
// built with g++ and the host sanitizers (test infrastructure; built by
// tests/test_sanitizers.py).  None of these is reached by the host-only
// paths the sanitizer driver runs.
#include <hip/hip_runtime_api.h>

#include "../paper_1406_5597_amd/csrc/fft3d_batch.hpp"
#include "../paper_1406_5597_amd/csrc/fft3d_internal.hpp"

namespace fft3d {

#define FFT3D_STUB_DTYPE(sfx)                                                                                   \
    hipError_t init_plain_##sfx() { return hipErrorNotSupported; }                                             \
    hipError_t init_coop_##sfx() { return hipErrorNotSupported; }                                              \
    hipError_t coop_occupancy_##sfx(const Plan&, int*) { return hipErrorNotSupported; }                        \
    hipError_t launch_plane_coop_##sfx(const Plan&, const void*, void*, bool, hipStream_t)                     \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_plane_r2c_##sfx(const Plan&, const void*, void*, hipStream_t, bool)                      \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_plane_c2r_##sfx(const Plan&, const void*, void*, hipStream_t, bool)                      \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_rows_r2c_##sfx(const Plan&, const void*, void*, int64_t, int, hipStream_t, bool)         \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_rows_c2r_##sfx(const Plan&, const void*, void*, int64_t, int, hipStream_t, bool)         \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_cols_##sfx(const Plan&, const ColPass&, int, int64_t, const void*, void*, bool, int,     \
                                 hipStream_t)                                                                   \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_swap01_##sfx(const Plan&, const void*, void*, int64_t, int64_t, hipStream_t)             \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t init_pruned_##sfx() { return hipErrorNotSupported; }                                            \
    hipError_t launch_pruned_r2c_##sfx(const Plan&, const void*, void*, const PrunedBox&, hipStream_t)         \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }                                                                                                           \
    hipError_t launch_pruned_c2r_##sfx(const Plan&, const void*, void*, void*, const PrunedBox&, hipStream_t)  \
    {                                                                                                           \
        return hipErrorNotSupported;                                                                            \
    }
FFT3D_STUB_DTYPE(f32)
FFT3D_STUB_DTYPE(f64)
FFT3D_STUB_DTYPE(f32_odd)
FFT3D_STUB_DTYPE(f64_odd)
#undef FFT3D_STUB_DTYPE

hipError_t init_batch() { return hipErrorNotSupported; }
const void* batch_kernel() { return nullptr; }
hipError_t batch_occupancy(size_t, int*) { return hipErrorNotSupported; }
hipError_t launch_batch(unsigned, size_t, const void*, int*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t init_level() { return hipErrorNotSupported; }
const void* level_kernel(int, int, int) { return nullptr; }
hipError_t launch_level(int, int, int, unsigned, size_t, const BatchTask*, const int*, int, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t probe_xcc_ids(int, int*) { return hipErrorNotSupported; }
hipError_t static_scratch_setup(int) { return hipErrorNotSupported; }
void* static_scratch(int) { return nullptr; }
hipError_t stage_static_image(int, const void*, size_t, const void**, hipStream_t) { return hipErrorNotSupported; }

}  // namespace fft3d
