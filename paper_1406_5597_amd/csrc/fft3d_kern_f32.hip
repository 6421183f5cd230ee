// fft3d_kern_f32.hip -- float instantiations of the standalone kernels
// (plane, rows, strided columns); see fft3d_kernels.hpp.
#include "fft3d_kernels.hpp"

namespace fft3d {

hipError_t init_plain_f32() { return init_plain<float>(); }
hipError_t launch_plane_r2c_f32(const Plan& p, const void* x, void* X, hipStream_t s)
{
    return plane_r2c_t<float>(p, x, X, s);
}
hipError_t launch_plane_c2r_f32(const Plan& p, const void* X, void* y, hipStream_t s)
{
    return plane_c2r_t<float>(p, X, y, s);
}
hipError_t launch_rows_r2c_f32(const Plan& p, const void* x, void* X, int64_t nrows, int rev, hipStream_t s)
{
    return rows_r2c_t<float>(p, x, X, nrows, rev, s);
}
hipError_t launch_rows_c2r_f32(const Plan& p, const void* X, void* y, int64_t nrows, int rev, hipStream_t s)
{
    return rows_c2r_t<float>(p, X, y, nrows, rev, s);
}
hipError_t launch_cols_f32(const Plan& p, const ColPass& cp, int axis, int64_t tw_off, const void* in,
                           void* out, bool inverse, int rev, hipStream_t s)
{
    return inverse ? cols_t<float, true>(p, cp, axis, tw_off, in, out, rev, s)
                   : cols_t<float, false>(p, cp, axis, tw_off, in, out, rev, s);
}

hipError_t launch_swap01_f32(const Plan& p, const void* in, void* out, int64_t na, int64_t nb, hipStream_t s)
{
    return swap01_t<float>(p, in, out, na, nb, s);
}

}  // namespace fft3d
