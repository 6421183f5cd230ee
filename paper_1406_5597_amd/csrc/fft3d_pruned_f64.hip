// fft3d_pruned_f64.hip -- double instantiations of the pruned transforms;
// see fft3d_pruned.hpp.
#include "fft3d_pruned.hpp"

// entry points defined here: name_f64, or name_f64_odd when the radix-5/7 stages are compiled in
#if FFT3D_ODD_RADICES
#define FFT3D_ENTRY(name) name##_f64_odd
#else
#define FFT3D_ENTRY(name) name##_f64
#endif

namespace fft3d {

hipError_t FFT3D_ENTRY(init_pruned)() { return init_pruned<double>(); }
hipError_t FFT3D_ENTRY(launch_pruned_r2c)(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t s)
{
    return pruned_r2c_t<double>(p, x, X, b, s);
}
hipError_t FFT3D_ENTRY(launch_pruned_c2r)(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b,
                                   hipStream_t s)
{
    return pruned_c2r_t<double>(p, X, y, work, b, s);
}

}  // namespace fft3d
