// fft3d_pruned_f64.hip -- double instantiations of the pruned transforms;
// see fft3d_pruned.hpp.
#include "fft3d_pruned.hpp"

namespace fft3d {

hipError_t init_pruned_f64() { return init_pruned<double>(); }
hipError_t launch_pruned_r2c_f64(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t s)
{
    return pruned_r2c_t<double>(p, x, X, b, s);
}
hipError_t launch_pruned_c2r_f64(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b,
                                   hipStream_t s)
{
    return pruned_c2r_t<double>(p, X, y, work, b, s);
}

}  // namespace fft3d
