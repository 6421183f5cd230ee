// fft3d_kern_f32.hip -- float instantiations of the standalone kernels
// (plane, rows, strided columns); see fft3d_kernels.hpp.
#include "fft3d_kernels.hpp"

// entry points defined here: name_f32, or name_f32_odd when the radix-5/7 stages are compiled in
#if FFT3D_ODD_RADICES
#define FFT3D_ENTRY(name) name##_f32_odd
#else
#define FFT3D_ENTRY(name) name##_f32
#endif

namespace fft3d {

hipError_t FFT3D_ENTRY(init_plain)() { return init_plain<float>(); }
hipError_t FFT3D_ENTRY(launch_plane_r2c)(const Plan& p, const void* x, void* X, hipStream_t s, bool padded)
{
    return plane_r2c_t<float>(p, x, X, s, padded);
}
hipError_t FFT3D_ENTRY(launch_plane_c2r)(const Plan& p, const void* X, void* y, hipStream_t s, bool padded)
{
    return plane_c2r_t<float>(p, X, y, s, padded);
}
hipError_t FFT3D_ENTRY(launch_rows_r2c)(const Plan& p, const void* x, void* X, int64_t nrows, int rev, hipStream_t s,
                                        bool padded)
{
    return rows_r2c_t<float>(p, x, X, nrows, rev, s, padded);
}
hipError_t FFT3D_ENTRY(launch_rows_c2r)(const Plan& p, const void* X, void* y, int64_t nrows, int rev, hipStream_t s,
                                        bool padded)
{
    return rows_c2r_t<float>(p, X, y, nrows, rev, s, padded);
}
hipError_t FFT3D_ENTRY(launch_cols)(const Plan& p, const ColPass& cp, int axis, int64_t tw_off, const void* in,
                           void* out, bool inverse, int rev, hipStream_t s)
{
    return inverse ? cols_t<float, true>(p, cp, axis, tw_off, in, out, rev, s)
                   : cols_t<float, false>(p, cp, axis, tw_off, in, out, rev, s);
}

hipError_t FFT3D_ENTRY(launch_swap01)(const Plan& p, const void* in, void* out, int64_t na, int64_t nb, hipStream_t s)
{
    return swap01_t<float>(p, in, out, na, nb, s);
}

}  // namespace fft3d
