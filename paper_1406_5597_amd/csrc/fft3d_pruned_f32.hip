// fft3d_pruned_f32.hip -- float instantiations of the pruned transforms;
// see fft3d_pruned.hpp.
#include "fft3d_pruned.hpp"

// entry points defined here: name_f32, or name_f32_odd when the radix-5/7 stages are compiled in
#if FFT3D_ODD_RADICES
#define FFT3D_ENTRY(name) name##_f32_odd
#else
#define FFT3D_ENTRY(name) name##_f32
#endif

namespace fft3d {

hipError_t FFT3D_ENTRY(init_pruned)() { return init_pruned<float>(); }
hipError_t FFT3D_ENTRY(launch_pruned_r2c)(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t s)
{
    return pruned_r2c_t<float>(p, x, X, b, s);
}
hipError_t FFT3D_ENTRY(launch_pruned_c2r)(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b,
                                   hipStream_t s)
{
    return pruned_c2r_t<float>(p, X, y, work, b, s);
}

}  // namespace fft3d
