// fft3d_kernels.hip -- HIP kernels of the 3D r2c/c2r path for gfx950.
//
// The forward transform runs the paper's two steps (Sec. 2.1 items 1 and 3,
// without the transpose of item 2, Sec. 2.2):
//   step 1, plane r2c: every n1 x n2 real plane -> n1 x H complex (H = n2/2+1),
//           n2 rows (half-length complex FFT + split) then n1 columns;
//   step 3, strided column c2c: a length-n0 DFT down every flattened column
//           c = k1*H + k2 of the natural-order spectrum, element stride n1*H,
//           read and written in place -- the data stay in natural order.
// The inverse runs the same steps in reverse order (Sec. 2.1, last sentence).
//
// All kernels stage one tile through LDS: a coalesced global->LDS copy, the
// Stockham stages of fft3d_device.hpp on lines in LDS, a coalesced LDS->global
// copy.  Plane tiles hold whole planes when they fit in LDS (fused plane
// kernels); larger planes take a rows kernel and a strided n1 column pass.
// Column tiles are W consecutive columns by all rows, so each row of a tile is
// one contiguous W-element segment of memory.
#include "fft3d_device.hpp"
#include "fft3d_internal.hpp"

namespace fft3d {

// ------------------------------------------------------------- kernels --

template <typename T, int NT, int EPT, bool INV>
__global__ __launch_bounds__(NT) void k_cols(const cx<T>* in, cx<T>* out, AxisSched ax,
                                             const cx<T>* __restrict__ tw, int64_t S, int64_t ncols,
                                             int64_t bstride, int W, int wshift,
                                             int64_t tiles_per_batch)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int64_t t = blockIdx.x;
    const int64_t b = t / tiles_per_batch;
    const int64_t c0 = (t - b * tiles_per_batch) * W;
    const int n = ax.n;
    const int E = n << wshift;
    const int64_t rem = ncols - c0;
    const int width = rem < (int64_t)W ? (int)rem : W;
    const cx<T>* src = in + b * bstride + c0;
    cx<T>* dst = out + b * bstride + c0;
    const cx<T> zero = mk<T>((T)0, (T)0);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = (int)threadIdx.x + k * NT;
        if (e < E) {
            const int i = e >> wshift;
            const int w = e & (W - 1);
            buf[e] = (w < width) ? src[(int64_t)i * S + w] : zero;
        }
    }
    __syncthreads();
    LdsLines L;
    L.nlines = W;
    L.lpp = W;
    L.sp = 0;
    L.sw = 1;
    L.si = W;
    lds_fft<INV, true, NT, EPT, T>(buf, L, ax, tw);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int e = (int)threadIdx.x + k * NT;
        if (e < E) {
            const int i = e >> wshift;
            const int w = e & (W - 1);
            if (w < width) dst[(int64_t)i * S + w] = buf[e];
        }
    }
}

// Real rows -> LDS rows of H slots holding z[m] = x[2m] + i x[2m+1].
template <typename T, int NT>
__device__ __forceinline__ void load_real_rows(cx<T>* buf, const cx<T>* src, int rows, int h, int H)
{
    const int total = rows * h;
    for (int e = (int)threadIdx.x; e < total; e += NT) {
        const int q = e / h;
        const int m = e - q * h;
        buf[q * H + m] = src[e];
    }
}

// LDS rows of H slots holding z[m] -> real rows x[2m] = Re z, x[2m+1] = Im z.
template <typename T, int NT>
__device__ __forceinline__ void store_real_rows(cx<T>* dst, const cx<T>* buf, int rows, int h, int H)
{
    const int total = rows * h;
    for (int e = (int)threadIdx.x; e < total; e += NT) {
        const int q = e / h;
        const int m = e - q * h;
        dst[e] = buf[q * H + m];
    }
}

template <typename T, int NT>
__device__ __forceinline__ void copy_block(cx<T>* dst, const cx<T>* src, int count)
{
    for (int e = (int)threadIdx.x; e < count; e += NT) dst[e] = src[e];
}

// Split-plane forward: rpw real rows of length n2 -> rpw rows of H bins.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_rows_r2c(const T* x, cx<T>* X, AxisSched axh,
                                                 const cx<T>* __restrict__ tw,
                                                 const cx<T>* __restrict__ post, int64_t nrows,
                                                 int rpw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int h = axh.n, H = h + 1;
    const int64_t row0 = (int64_t)blockIdx.x * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    load_real_rows<T, NT>(buf, reinterpret_cast<const cx<T>*>(x) + row0 * h, rows, h, H);
    __syncthreads();
    LdsLines L;
    L.nlines = rows;
    L.lpp = rows;
    L.sp = 0;
    L.sw = H;
    L.si = 1;
    lds_fft<false, false, NT, EPT, T>(buf, L, axh, tw);
    split_rows<NT, T>(buf, rows, H, h, post);
    copy_block<T, NT>(X + row0 * H, buf, rows * H);
}

// Split-plane inverse: rpw rows of H bins -> rpw real rows of length n2.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_rows_c2r(const cx<T>* X, T* y, AxisSched axh,
                                                 const cx<T>* __restrict__ tw,
                                                 const cx<T>* __restrict__ post, int64_t nrows,
                                                 int rpw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int h = axh.n, H = h + 1;
    const int64_t row0 = (int64_t)blockIdx.x * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    copy_block<T, NT>(buf, X + row0 * H, rows * H);
    __syncthreads();
    merge_rows<NT, T>(buf, rows, H, h, post);
    LdsLines L;
    L.nlines = rows;
    L.lpp = rows;
    L.sp = 0;
    L.sw = H;
    L.si = 1;
    lds_fft<true, false, NT, EPT, T>(buf, L, axh, tw);
    store_real_rows<T, NT>(reinterpret_cast<cx<T>*>(y) + row0 * h, buf, rows, h, H);
}

// Fused plane forward: ppw whole planes per workgroup, held in LDS as
// [plane][n1][H]; rows, split, then the n1 columns, one HBM read and write.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_plane_r2c(const T* x, cx<T>* X, AxisSched axh, AxisSched ax1,
                                                  const cx<T>* __restrict__ tw2,
                                                  const cx<T>* __restrict__ post,
                                                  const cx<T>* __restrict__ tw1, int64_t nplanes,
                                                  int ppw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int h = axh.n, H = h + 1, n1 = ax1.n;
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int64_t left = nplanes - p0;
    const int np = left < ppw ? (int)left : ppw;
    const int rows = np * n1;
    load_real_rows<T, NT>(buf, reinterpret_cast<const cx<T>*>(x) + p0 * n1 * h, rows, h, H);
    __syncthreads();
    LdsLines Lr;
    Lr.nlines = rows;
    Lr.lpp = rows;
    Lr.sp = 0;
    Lr.sw = H;
    Lr.si = 1;
    lds_fft<false, false, NT, EPT, T>(buf, Lr, axh, tw2);
    split_rows<NT, T>(buf, rows, H, h, post);
    LdsLines Lc;
    Lc.nlines = np * H;
    Lc.lpp = H;
    Lc.sp = n1 * H;
    Lc.sw = 1;
    Lc.si = H;
    lds_fft<false, true, NT, EPT, T>(buf, Lc, ax1, tw1);
    copy_block<T, NT>(X + p0 * n1 * H, buf, rows * H);
}

// Fused plane inverse: n1 columns, merge, rows; one HBM read and write.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_plane_c2r(const cx<T>* X, T* y, AxisSched axh, AxisSched ax1,
                                                  const cx<T>* __restrict__ tw2,
                                                  const cx<T>* __restrict__ post,
                                                  const cx<T>* __restrict__ tw1, int64_t nplanes,
                                                  int ppw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int h = axh.n, H = h + 1, n1 = ax1.n;
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int64_t left = nplanes - p0;
    const int np = left < ppw ? (int)left : ppw;
    const int rows = np * n1;
    copy_block<T, NT>(buf, X + p0 * n1 * H, rows * H);
    __syncthreads();
    LdsLines Lc;
    Lc.nlines = np * H;
    Lc.lpp = H;
    Lc.sp = n1 * H;
    Lc.sw = 1;
    Lc.si = H;
    lds_fft<true, true, NT, EPT, T>(buf, Lc, ax1, tw1);
    merge_rows<NT, T>(buf, rows, H, h, post);
    LdsLines Lr;
    Lr.nlines = rows;
    Lr.lpp = rows;
    Lr.sp = 0;
    Lr.sw = H;
    Lr.si = 1;
    lds_fft<true, false, NT, EPT, T>(buf, Lr, axh, tw2);
    store_real_rows<T, NT>(reinterpret_cast<cx<T>*>(y) + p0 * n1 * h, buf, rows, h, H);
}

// ----------------------------------------------------------- launchers --

namespace {

template <typename T> const cx<T>* table(const Plan& p, int64_t off)
{
    return reinterpret_cast<const cx<T>*>(p.d_tw) + off;
}

template <typename K> hipError_t allow_lds(K kernel)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
}

template <typename T> hipError_t init_dtype()
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    hipError_t e = hipSuccess;
#define FFT3D_ALLOW(k)                       \
    do {                                     \
        hipError_t r_ = allow_lds(k);        \
        if (r_ != hipSuccess) e = r_;        \
    } while (0)
    FFT3D_ALLOW((k_cols<T, kNtSmall, ES, false>));
    FFT3D_ALLOW((k_cols<T, kNtSmall, ES, true>));
    FFT3D_ALLOW((k_cols<T, kNtBig, EB, false>));
    FFT3D_ALLOW((k_cols<T, kNtBig, EB, true>));
    FFT3D_ALLOW((k_rows_r2c<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_r2c<T, kNtBig, EB>));
    FFT3D_ALLOW((k_rows_c2r<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_c2r<T, kNtBig, EB>));
    FFT3D_ALLOW((k_plane_r2c<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_plane_r2c<T, kNtBig, EB>));
    FFT3D_ALLOW((k_plane_c2r<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_plane_c2r<T, kNtBig, EB>));
#undef FFT3D_ALLOW
    return e;
}

template <typename T>
hipError_t plane_r2c_t(const Plan& p, const void* x, void* X, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const unsigned grid = (unsigned)((p.n0 + p.ppw - 1) / p.ppw);
    const T* xi = static_cast<const T*>(x);
    cx<T>* Xo = static_cast<cx<T>*>(X);
    if (p.plane_big)
        hipLaunchKernelGGL((k_plane_r2c<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.plane_lds, st, xi,
                           Xo, p.ax2h, p.ax1, table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw);
    else
        hipLaunchKernelGGL((k_plane_r2c<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.plane_lds, st,
                           xi, Xo, p.ax2h, p.ax1, table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw);
    return hipGetLastError();
}

template <typename T>
hipError_t plane_c2r_t(const Plan& p, const void* X, void* y, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const unsigned grid = (unsigned)((p.n0 + p.ppw - 1) / p.ppw);
    const cx<T>* Xi = static_cast<const cx<T>*>(X);
    T* yo = static_cast<T*>(y);
    if (p.plane_big)
        hipLaunchKernelGGL((k_plane_c2r<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.plane_lds, st, Xi,
                           yo, p.ax2h, p.ax1, table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw);
    else
        hipLaunchKernelGGL((k_plane_c2r<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.plane_lds, st,
                           Xi, yo, p.ax2h, p.ax1, table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw);
    return hipGetLastError();
}

template <typename T>
hipError_t rows_r2c_t(const Plan& p, const void* x, void* X, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const int64_t nrows = p.n0 * p.n1;
    const unsigned grid = (unsigned)((nrows + p.rpw - 1) / p.rpw);
    const T* xi = static_cast<const T*>(x);
    cx<T>* Xo = static_cast<cx<T>*>(X);
    if (p.rows_big)
        hipLaunchKernelGGL((k_rows_r2c<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds, st, xi, Xo,
                           p.ax2h, table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw);
    else
        hipLaunchKernelGGL((k_rows_r2c<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds, st, xi,
                           Xo, p.ax2h, table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw);
    return hipGetLastError();
}

template <typename T>
hipError_t rows_c2r_t(const Plan& p, const void* X, void* y, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const int64_t nrows = p.n0 * p.n1;
    const unsigned grid = (unsigned)((nrows + p.rpw - 1) / p.rpw);
    const cx<T>* Xi = static_cast<const cx<T>*>(X);
    T* yo = static_cast<T*>(y);
    if (p.rows_big)
        hipLaunchKernelGGL((k_rows_c2r<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds, st, Xi, yo,
                           p.ax2h, table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw);
    else
        hipLaunchKernelGGL((k_rows_c2r<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds, st, Xi,
                           yo, p.ax2h, table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw);
    return hipGetLastError();
}

template <typename T, bool INV>
hipError_t cols_t(const Plan& p, const ColPass& cp, const AxisSched& ax, int64_t tw_off, const void* in,
                  void* out, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const unsigned grid = (unsigned)(cp.nbatch * cp.tiles_per_batch);
    const cx<T>* ci = static_cast<const cx<T>*>(in);
    cx<T>* co = static_cast<cx<T>*>(out);
    if (cp.big)
        hipLaunchKernelGGL((k_cols<T, kNtBig, EB, INV>), dim3(grid), dim3(kNtBig), cp.lds, st, ci, co, ax,
                           table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W, cp.wshift,
                           cp.tiles_per_batch);
    else
        hipLaunchKernelGGL((k_cols<T, kNtSmall, ES, INV>), dim3(grid), dim3(kNtSmall), cp.lds, st, ci, co,
                           ax, table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W, cp.wshift,
                           cp.tiles_per_batch);
    return hipGetLastError();
}

}  // namespace

// Raising the dynamic-LDS limit is advisory: a launch that still exceeds what
// the device allows fails with a launch error, which the callers report.
hipError_t kernels_init()
{
    (void)init_dtype<float>();
    (void)init_dtype<double>();
    (void)hipGetLastError();
    return hipSuccess;
}

hipError_t launch_plane_r2c(const Plan& p, const void* x, void* X, hipStream_t st)
{
    return p.dtype ? plane_r2c_t<double>(p, x, X, st) : plane_r2c_t<float>(p, x, X, st);
}
hipError_t launch_plane_c2r(const Plan& p, const void* X, void* y, hipStream_t st)
{
    return p.dtype ? plane_c2r_t<double>(p, X, y, st) : plane_c2r_t<float>(p, X, y, st);
}
hipError_t launch_rows_r2c(const Plan& p, const void* x, void* X, hipStream_t st)
{
    return p.dtype ? rows_r2c_t<double>(p, x, X, st) : rows_r2c_t<float>(p, x, X, st);
}
hipError_t launch_rows_c2r(const Plan& p, const void* X, void* y, hipStream_t st)
{
    return p.dtype ? rows_c2r_t<double>(p, X, y, st) : rows_c2r_t<float>(p, X, y, st);
}
hipError_t launch_cols(const Plan& p, const ColPass& cp, const AxisSched& ax, int64_t tw_off, const void* in,
                       void* out, bool inverse, hipStream_t st)
{
    if (p.dtype)
        return inverse ? cols_t<double, true>(p, cp, ax, tw_off, in, out, st)
                       : cols_t<double, false>(p, cp, ax, tw_off, in, out, st);
    return inverse ? cols_t<float, true>(p, cp, ax, tw_off, in, out, st)
                   : cols_t<float, false>(p, cp, ax, tw_off, in, out, st);
}

}  // namespace fft3d
