// fft3d_pruned.hpp -- kernels of the pruned (dealiased) transforms.
//
// A pseudo-spectral solver keeps only the modes of a truncated box -- with
// the two-thirds rule |k0| <= n0/3, |k1| <= n1/3, k2 <= n2/3 -- and zeroes
// the rest.  The forward transform then needs only the kept modes of its
// output, and the inverse reads only the kept modes of its input; every pass
// of the path can skip the rows and columns that are outside the box:
//   forward:  rows pass writes bins k2 <= K2 only; the n1 pass runs on those
//             columns and writes rows |k1| <= K1 only; the n0 pass runs on the
//             kept (k1, k2) columns and writes rows |k0| <= K0 only;
//   inverse:  the same in reverse, each pass reading only what is kept.
// Masked loads return zero and masked stores are skipped, and every line is
// transformed with the same schedule as in the full path, so each kept value
// is bit-identical to the full transform's (forward) and the inverse of a
// spectrum that is zero outside the box is bit-identical to the full inverse.
#pragma once

#include "fft3d_kernels.hpp"

namespace fft3d {
inline namespace FFT3D_KNS {

// Kept index along an axis of length n with cut K: |signed index| <= K.
// K < 0 keeps everything.
__device__ __forceinline__ bool kept(int i, int n, int K) { return K < 0 || i <= K || i >= n - K; }

// ColTileIO with a row mask on loads (kin) and on stores (kout): rows outside
// are neither read (they load as zero) nor written.
template <typename T> struct ColTileMaskIO {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    struct Pos {
        int64_t off;
        int row;
        bool ok;
    };
    const cx<T>* src;
    cx<T>* dst;
    int64_t S;
    int width;
    int n, kin, kout;
    __device__ __forceinline__ Pos at(int w, int i) const
    {
        Pos p;
        p.ok = w < width;
        p.off = (int64_t)i * S + (p.ok ? w : width - 1);
        p.row = i;
        return p;
    }
    __device__ __forceinline__ Pos adv(Pos p, int d) const
    {
        p.off += (int64_t)d * S;
        p.row += d;
        return p;
    }
    // Every lane loads (a masked row from the tile's first element, which is
    // cached) so that the loads of a stage stay in flight together; masked
    // rows then read as zero.
    __device__ __forceinline__ cx<T> get(Pos p) const
    {
        const bool keep = p.ok && kept(p.row, n, kin);
        const cx<T> v = src[keep ? p.off : 0];
        return keep ? v : mk<T>((T)0, (T)0);
    }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const
    {
        if (p.ok && kept(p.row, n, kout)) dst[p.off] = v;
    }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

// PlaneColsIO with the box: column c = k2 kept if c <= K2, row k1 kept if
// |k1| <= K1 (masked loads read zero, masked stores are skipped).
template <typename T> struct PlaneColsMaskIO {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    struct Pos {
        int off;
        int row;
        bool ok;  // the column is kept
    };
    const cx<T>* src;
    cx<T>* dst;
    int H, plane, n1, K1, K2;
    uint32_t mgH;
    __device__ __forceinline__ Pos at(int w, int i) const
    {
        const int p = fdiv(w, mgH);
        const int c = w - p * H;
        Pos q;
        q.off = p * plane + c + i * H;
        q.row = i;
        q.ok = c <= K2;
        return q;
    }
    __device__ __forceinline__ Pos adv(Pos p, int d) const
    {
        p.off += d * H;
        p.row += d;
        return p;
    }
    __device__ __forceinline__ cx<T> get(Pos p) const
    {
        const bool keep = p.ok && kept(p.row, n1, K1);
        const cx<T> v = src[keep ? p.off : 0];
        return keep ? v : mk<T>((T)0, (T)0);
    }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const
    {
        if (p.ok && kept(p.row, n1, K1)) dst[p.off] = v;
    }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

// Column pass over the kept columns: block b of the pass starts at
// (b < nb_lo ? b : b + nskip) * bstride (the two kept ranges of k1 for the
// n0 pass; nskip = 0 for the n1 pass), ncols = K2 + 1 columns per block.
// reverse: as in k_cols (each XCD walks its groups from the last).
template <typename T, int NT, int EPT, bool INV>
__global__ __launch_bounds__(NT) void k_cols_pr(const cx<T>* in, cx<T>* out, const AxisSched* __restrict__ axp,
                                                const cx<T>* __restrict__ tw, int64_t S, int64_t ncols,
                                                int64_t bstride, int W, uint32_t mg_w, int64_t tiles_per_batch,
                                                int64_t ntiles, int64_t ngroups, int gsize, int64_t nb_lo,
                                                int64_t nskip, int kin, int kout, int reverse)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int64_t t = group_tile(blockIdx.x, ngroups, gsize, reverse);
    if (t >= ntiles) return;  // padding workgroup
    const int64_t b = t / tiles_per_batch;
    const int64_t c0 = (t - b * tiles_per_batch) * W;
    const int64_t rem = ncols - c0;
    const int width = rem < (int64_t)W ? (int)rem : W;
    const int64_t off = (b < nb_lo ? b : b + nskip) * bstride + c0;
    const AxisSched& ax = *axp;
    ColTileMaskIO<T> g;
    g.src = in + off;
    g.dst = out + off;
    g.S = S;
    g.width = width;
    g.n = ax.n;
    g.kin = kin;
    g.kout = kout;
    LdsIO<T> l;
    l.buf = buf;
    l.L.nlines = W;
    l.L.lpp = W;
    l.L.sp = 0;
    l.L.sw = 1;
    l.L.si = W;
    l.L.mg_lines = mg_w;
    l.L.mg_lpp = mg_w;
    fft_lines<INV, true, NT, EPT, T>(g, l, g, W, mg_w, ax, tw);
}

// Rows pass, forward: as k_rows_r2c, writing bins 0 .. Hw-1 of each row only.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT, (rows_waves<T, EPT, false>())) void k_rows_r2c_pr(const T* x, cx<T>* X, const AxisSched* __restrict__ axp,
                                                    const cx<T>* __restrict__ tw, const cx<T>* __restrict__ post,
                                                    int64_t nrows, int rpw, int Hs, int Hw, uint32_t mgHw)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& axh = *axp;
    const int h = axh.n, H = h + 1;
    const int64_t row0 = (int64_t)blockIdx.x * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    RowsIO<T> g;
    g.src = reinterpret_cast<const cx<T>*>(x) + row0 * h;
    g.dst = nullptr;
    g.len = h;
    const LdsRowsIO<T> l = lds_rows<T>(buf, Hs);
    fft_lines<false, false, NT, EPT, T>(g, l, l, rows, 0u, axh, tw);
    split_rows<NT, T>(buf, rows, Hs, h, axh.mg_pairs, post);
    cx<T>* dst = X + row0 * H;
    const int count = rows * Hw;
    for (int e = (int)threadIdx.x; e < count; e += NT) {
        const int q = fdiv(e, mgHw);
        const int c = e - q * Hw;
        dst[(int64_t)q * H + c] = buf[q * Hs + pad16(c)];
    }
}

// Rows pass, inverse: as k_rows_c2r, reading bins 0 .. Hw-1 of each row only
// (the others are zero).  mgHw = div_magic(Hw), mgZ = div_magic(H - Hw).
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT, (rows_waves<T, EPT, true>())) void k_rows_c2r_pr(const cx<T>* X, T* y, const AxisSched* __restrict__ axp,
                                                    const cx<T>* __restrict__ tw, const cx<T>* __restrict__ post,
                                                    int64_t nrows, int rpw, int Hs, int Hw, uint32_t mgHw,
                                                    uint32_t mgZ)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& axh = *axp;
    const int h = axh.n, H = h + 1;
    const int64_t row0 = (int64_t)blockIdx.x * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    const cx<T>* src = X + row0 * H;
    // kept bins: 8 loads in flight per thread before the LDS stores.  Lanes
    // past the end repeat the last bin (same value to the same slot), so
    // loads and stores are unconditional and the loads are not serialised.
    constexpr int U = 8;
    const int count = rows * Hw;
    for (int base = 0; base < count; base += U * NT) {
        cx<T> v[U];
        int slot[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + (int)threadIdx.x + u * NT;
            const int ec = e < count ? e : count - 1;
            const int q = fdiv(ec, mgHw), c = ec - q * Hw;
            v[u] = src[(int64_t)q * H + c];
            slot[u] = q * Hs + pad16(c);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) buf[slot[u]] = v[u];
    }
    // the other bins are zero
    const int nz = H - Hw, zcount = rows * nz;
    for (int e = (int)threadIdx.x; e < zcount; e += NT) {
        const int q = fdiv(e, mgZ);
        buf[q * Hs + pad16(Hw + e - q * nz)] = mk<T>((T)0, (T)0);
    }
    __syncthreads();
    merge_rows<NT, T>(buf, rows, Hs, h, axh.mg_pairs, post);
    RowsIO<T> g;
    g.src = nullptr;
    g.dst = reinterpret_cast<cx<T>*>(y) + row0 * h;
    g.len = h;
    const LdsRowsIO<T> l = lds_rows<T>(buf, Hs);
    fft_lines<true, false, NT, EPT, T>(l, l, g, rows, 0u, axh, tw);
}

// Fused plane step, forward: the n1 columns write the kept box only.  (No
// restrict on the pointer arguments, as for the full fused plane kernels:
// fewer registers, no spills in the big tier.)
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_plane_r2c_pr(const T* x, cx<T>* X, const AxisSched* axhp,
                                                     const AxisSched* ax1p,
                                                     const cx<T>* tw2, const cx<T>* post,
                                                     const cx<T>* tw1, int64_t nplanes, int ppw, int Hs,
                                                     uint32_t mg_lines, uint32_t mgH, int K1, int K2)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& axh = *axhp;
    const AxisSched& ax1 = *ax1p;
    const int h = axh.n, H = h + 1, n1 = ax1.n;
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int64_t left = nplanes - p0;
    const int np = left < ppw ? (int)left : ppw;
    const uint32_t mg = np == ppw ? mg_lines : div_magic_dev(np * H);
    RowsIO<T> gi;
    gi.src = reinterpret_cast<const cx<T>*>(x) + p0 * n1 * h;
    gi.dst = nullptr;
    gi.len = h;
    const LdsRowsIO<T> lr = lds_rows<T>(buf, Hs);
    fft_lines<false, false, NT, EPT, T>(gi, lr, lr, np * n1, 0u, axh, tw2);
    split_rows<NT, T>(buf, np * n1, Hs, h, axh.mg_pairs, post);
    PlaneColsMaskIO<T> go;
    go.src = nullptr;
    go.dst = X + p0 * n1 * H;
    go.H = H;
    go.plane = n1 * H;
    go.n1 = n1;
    go.K1 = K1;
    go.K2 = K2;
    go.mgH = mgH;
    const LdsPlaneColsIO<T> lc = lds_plane_cols<T>(buf, n1, H, Hs, mgH);
    fft_lines<false, true, NT, EPT, T>(lc, lc, go, np * H, mg, ax1, tw1);
}

// Fused plane step, inverse: the n1 columns read the kept box only.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_plane_c2r_pr(const cx<T>* X, T* y, const AxisSched* axhp,
                                                     const AxisSched* ax1p,
                                                     const cx<T>* tw2, const cx<T>* post,
                                                     const cx<T>* tw1, int64_t nplanes, int ppw, int Hs,
                                                     uint32_t mg_lines, uint32_t mgH, int K1, int K2)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& axh = *axhp;
    const AxisSched& ax1 = *ax1p;
    const int h = axh.n, H = h + 1, n1 = ax1.n;
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int64_t left = nplanes - p0;
    const int np = left < ppw ? (int)left : ppw;
    const uint32_t mg = np == ppw ? mg_lines : div_magic_dev(np * H);
    PlaneColsMaskIO<T> gi;
    gi.src = X + p0 * n1 * H;
    gi.dst = nullptr;
    gi.H = H;
    gi.plane = n1 * H;
    gi.n1 = n1;
    gi.K1 = K1;
    gi.K2 = K2;
    gi.mgH = mgH;
    const LdsPlaneColsIO<T> lc = lds_plane_cols<T>(buf, n1, H, Hs, mgH);
    fft_lines<true, true, NT, EPT, T>(gi, lc, lc, np * H, mg, ax1, tw1);
    merge_rows<NT, T>(buf, np * n1, Hs, h, axh.mg_pairs, post);
    RowsIO<T> go;
    go.src = nullptr;
    go.dst = reinterpret_cast<cx<T>*>(y) + p0 * n1 * h;
    go.len = h;
    const LdsRowsIO<T> lr = lds_rows<T>(buf, Hs);
    fft_lines<true, false, NT, EPT, T>(lr, lr, go, np * n1, 0u, axh, tw2);
}

// ----------------------------------------------------------- launchers --

template <typename T> hipError_t init_pruned()
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    hipError_t e = hipSuccess;
#define FFT3D_ALLOW(k)                \
    do {                              \
        hipError_t r_ = allow_lds(k); \
        if (r_ != hipSuccess) e = r_; \
    } while (0)
    FFT3D_ALLOW((k_cols_pr<T, kNtSmall, ES, false>));
    FFT3D_ALLOW((k_cols_pr<T, kNtSmall, ES, true>));
    FFT3D_ALLOW((k_cols_pr<T, kNtWide, ES, false>));
    FFT3D_ALLOW((k_cols_pr<T, kNtWide, ES, true>));
    FFT3D_ALLOW((k_cols_pr<T, kNtBig, EB, false>));
    FFT3D_ALLOW((k_cols_pr<T, kNtBig, EB, true>));
    FFT3D_ALLOW((k_rows_r2c_pr<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_r2c_pr<T, kNtBig, EB>));
    FFT3D_ALLOW((k_rows_c2r_pr<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_c2r_pr<T, kNtBig, EB>));
    FFT3D_ALLOW((k_plane_r2c_pr<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_plane_r2c_pr<T, kNtBig, EB>));
    FFT3D_ALLOW((k_plane_c2r_pr<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_plane_c2r_pr<T, kNtBig, EB>));
#undef FFT3D_ALLOW
    return e;
}

// Column pass restricted to the kept columns.  axis 0: the n0 pass over the
// kept (k1, k2) columns (two k1 ranges); axis 1: the n1 pass over k2 <= K2
// of every plane.  kin / kout: row masks of the loads / stores.
template <typename T, bool INV>
hipError_t cols_pr_t(const Plan& p, const ColPass& cp0, int axis, int64_t tw_off, const void* in, void* out,
                     const PrunedBox& b, int kin, int kout, int rev, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    ColPass cp = cp0;
    int64_t nb_lo, nskip;
    const int64_t ncols = b.K2 + 1;
    if (axis == 0) {
        const int64_t nk1 = (b.K1 < 0 || 2 * (int64_t)b.K1 + 1 >= p.n1) ? p.n1 : 2 * (int64_t)b.K1 + 1;
        cp.nbatch = nk1;
        cp.bstride = p.H;
        nb_lo = nk1 == p.n1 ? nk1 : b.K1 + 1;
        nskip = p.n1 - nk1;
    } else {
        cp.nbatch = p.n0;
        cp.bstride = p.n1 * p.H;
        nb_lo = p.n0;
        nskip = 0;
    }
    cp.ncols = ncols;
    cp.tiles_per_batch = (ncols + cp.W - 1) / cp.W;
    const int64_t ntiles = cp.nbatch * cp.tiles_per_batch;
    const int gsize = (int)cp.tiles_per_batch;
    const int64_t ngroups = cp.nbatch;
    const unsigned grid = (unsigned)group_grid(ngroups, gsize);
    const AxisSched* ax = dsched(p, axis);
    const cx<T>* ci = static_cast<const cx<T>*>(in);
    cx<T>* co = static_cast<cx<T>*>(out);
    const uint32_t mgw = div_magic((uint32_t)cp.W);
#define FFT3D_COLS_PR(NT_, EPT_)                                                                               \
    hipLaunchKernelGGL((k_cols_pr<T, NT_, EPT_, INV>), dim3(grid), dim3(NT_), cp.lds, st, ci, co, ax,            \
                       table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W, mgw, cp.tiles_per_batch, ntiles, \
                       ngroups, gsize, nb_lo, nskip, kin, kout, rev)
    if (cp.big) FFT3D_COLS_PR(kNtBig, EB);
    else if (cp.wide) FFT3D_COLS_PR(kNtWide, ES);
    else FFT3D_COLS_PR(kNtSmall, ES);
#undef FFT3D_COLS_PR
    return hipGetLastError();
}

template <typename T>
hipError_t rows_pr_t(const Plan& p, const void* in, void* out, bool inverse, const PrunedBox& b, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const int64_t nrows = p.n0 * p.n1;
    const int rpw = inverse ? p.rpw_inv : p.rpw;
    const unsigned grid = (unsigned)((nrows + rpw - 1) / rpw);
    const int Hw = b.K2 + 1;
    if (!inverse) {
        const T* xi = static_cast<const T*>(in);
        cx<T>* Xo = static_cast<cx<T>*>(out);
        const uint32_t mg = div_magic((uint32_t)Hw);
        if (p.rows_big)
            hipLaunchKernelGGL((k_rows_r2c_pr<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds, st, xi, Xo,
                               dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw, p.Hs,
                               Hw, mg);
        else
            hipLaunchKernelGGL((k_rows_r2c_pr<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds, st, xi,
                               Xo, dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw,
                               p.Hs, Hw, mg);
    } else {
        const cx<T>* Xi = static_cast<const cx<T>*>(in);
        T* yo = static_cast<T*>(out);
        const uint32_t mg = div_magic((uint32_t)Hw), mgz = div_magic((uint32_t)(p.H - Hw));
        if (p.rows_big)
            hipLaunchKernelGGL((k_rows_c2r_pr<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds_inv, st, Xi, yo,
                               dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw_inv, p.Hs,
                               Hw, mg, mgz);
        else
            hipLaunchKernelGGL((k_rows_c2r_pr<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds_inv, st, Xi,
                               yo, dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw_inv,
                               p.Hs, Hw, mg, mgz);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t plane_pr_t(const Plan& p, const void* in, void* out, bool inverse, const PrunedBox& b, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const unsigned grid = (unsigned)((p.n0 + p.ppw - 1) / p.ppw);
    const uint32_t mgl = div_magic((uint32_t)(p.ppw * p.H)), mgH = div_magic((uint32_t)p.H);
#define FFT3D_PLANE_PR(K_, NT_, EPT_, IN_T, OUT_T)                                                                \
    hipLaunchKernelGGL((K_<T, NT_, EPT_>), dim3(grid), dim3(NT_), p.plane_lds, st, static_cast<IN_T>(in),         \
                       static_cast<OUT_T>(out), dsched(p, 2), dsched(p, 1), table<T>(p, p.off_ax2h),              \
                       table<T>(p, p.off_post), table<T>(p, p.off_ax1), p.n0, p.ppw, p.plane_Hs, mgl, mgH, b.K1, \
                       b.K2)
    if (!inverse) {
        if (p.plane_big) FFT3D_PLANE_PR(k_plane_r2c_pr, kNtBig, EB, const T*, cx<T>*);
        else FFT3D_PLANE_PR(k_plane_r2c_pr, kNtSmall, ES, const T*, cx<T>*);
    } else {
        if (p.plane_big) FFT3D_PLANE_PR(k_plane_c2r_pr, kNtBig, EB, const cx<T>*, T*);
        else FFT3D_PLANE_PR(k_plane_c2r_pr, kNtSmall, ES, const cx<T>*, T*);
    }
#undef FFT3D_PLANE_PR
    return hipGetLastError();
}

// Forward: plane step writing the kept (k1, k2) of every plane, then the n0
// pass over the kept columns writing the kept k0 rows.
template <typename T> hipError_t pruned_r2c_t(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t st)
{
    hipError_t e;
    if (p.fused_plane) {
        e = plane_pr_t<T>(p, x, X, false, b, st);
    } else {
        e = rows_pr_t<T>(p, x, X, false, b, st);
        if (e == hipSuccess && p.n1 > 1) e = cols_pr_t<T, false>(p, p.pass1, 1, p.off_ax1, X, X, b, -1, b.K1, (p.rev >> 1) & 1, st);
    }
    if (e == hipSuccess && p.n0 > 1) e = cols_pr_t<T, false>(p, p.pass0, 0, p.off_ax0, X, X, b, -1, b.K0, (p.rev >> 2) & 1, st);
    return e;
}

// Inverse: the n0 pass over the kept columns reading the kept k0 rows (into
// work, or in place), then the plane step reading the kept (k1, k2).
template <typename T>
hipError_t pruned_c2r_t(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b, hipStream_t st)
{
    hipError_t e = hipSuccess;
    void* scratch = work ? work : const_cast<void*>(X);
    const void* cur = X;
    if (p.n0 > 1) {
        e = cols_pr_t<T, true>(p, p.pass0, 0, p.off_ax0, cur, scratch, b, b.K0, -1, (p.rev >> 3) & 1, st);
        cur = scratch;
    }
    if (e != hipSuccess) return e;
    if (p.fused_plane) return plane_pr_t<T>(p, cur, y, true, b, st);
    if (p.n1 > 1) {
        e = cols_pr_t<T, true>(p, p.pass1, 1, p.off_ax1, cur, scratch, b, b.K1, -1, (p.rev >> 4) & 1, st);
        cur = scratch;
    }
    if (e == hipSuccess) e = rows_pr_t<T>(p, cur, y, true, b, st);
    return e;
}

}  // inline namespace FFT3D_KNS
}  // namespace fft3d
