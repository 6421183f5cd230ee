// fft3d_coop_f64.hip -- double instantiation of the cooperative plane
// kernel; see fft3d_kernels.hpp.
#include "fft3d_kernels.hpp"

namespace fft3d {

hipError_t init_coop_f64() { return init_coop<double>(); }
hipError_t coop_occupancy_f64(const Plan& p, int* per_cu) { return coop_occupancy<double>(p, per_cu); }
hipError_t launch_plane_coop_f64(const Plan& p, const void* in, void* out, bool inverse, hipStream_t s)
{
    return coop_t<double>(p, in, out, inverse, s);
}

}  // namespace fft3d
