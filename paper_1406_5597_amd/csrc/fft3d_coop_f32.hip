// fft3d_coop_f32.hip -- float instantiation of the cooperative plane
// kernel; see fft3d_kernels.hpp.
#include "fft3d_kernels.hpp"

namespace fft3d {

hipError_t init_coop_f32() { return init_coop<float>(); }
hipError_t coop_occupancy_f32(const Plan& p, int* per_cu) { return coop_occupancy<float>(p, per_cu); }
hipError_t launch_plane_coop_f32(const Plan& p, const void* in, void* out, bool inverse, hipStream_t s)
{
    return coop_t<float>(p, in, out, inverse, s);
}

}  // namespace fft3d
