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
#pragma once

#include <algorithm>

#include "fft3d_device.hpp"
#include "fft3d_internal.hpp"

namespace fft3d {
inline namespace FFT3D_KNS {

// ------------------------------------------------------------- kernels --

// div_magic on the device, for a partial last group of planes (uniform, rare).
__device__ __forceinline__ uint32_t div_magic_dev(uint32_t d)
{
    return d <= 1 ? 0u : (uint32_t)((1ull << 32) / d + 1);
}

// Contiguous copy of `count` elements by the workgroup, 8 loads in flight per
// thread before the matching stores.  LP / SP: cache policies.
template <typename T, int NT, int LP = LD_PLAIN, int SP = ST_PLAIN>
__device__ __forceinline__ void copy_block(cx<T>* dst, const cx<T>* src, int count)
{
    constexpr int U = 8;
    for (int base = 0; base < count; base += U * NT) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + (int)threadIdx.x + u * NT;
            v[u] = load_cx<LP, T>(src + (e < count ? e : count - 1));  // always a valid address
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + (int)threadIdx.x + u * NT;
            if (e < count) store_cx<SP, T>(dst + e, v[u]);
        }
    }
}

// LDS view of `rows` padded rows (lines along a row; see LdsRowsIO).
template <typename T> __device__ __forceinline__ LdsRowsIO<T> lds_rows(cx<T>* buf, int Hs)
{
    LdsRowsIO<T> l;
    l.buf = buf;
    l.Hs = Hs;
    return l;
}

// LDS view of the columns of planes of n1 padded rows (lines down a column).
template <typename T>
__device__ __forceinline__ LdsPlaneColsIO<T> lds_plane_cols(cx<T>* buf, int n1, int H, int Hs, uint32_t mgH)
{
    LdsPlaneColsIO<T> l;
    l.buf = buf;
    l.H = H;
    l.Hs = Hs;
    l.plane = n1 * Hs;
    l.mgH = mgH;
    return l;
}

// `rows` contiguous rows of H elements in global memory <-> padded LDS rows,
// 8 loads in flight per thread before the matching stores.  mgH: div_magic(H).
// FP32: two complex values (16 bytes) per lane and access when the run is
// 16-byte aligned and of even length (the usual case), which halves the
// memory instructions.
template <typename T, int NT, int LP = LD_PLAIN>
__device__ __forceinline__ void rows_to_lds(cx<T>* buf, const cx<T>* src, int rows, int H, int Hs, uint32_t mgH)
{
    constexpr int U = 8;
    const int count = rows * H;
    if constexpr (sizeof(T) == 4 && LP == LD_PLAIN) {
        if (((uintptr_t)src & 15) == 0 && (count & 1) == 0) {
            const int pairs = count >> 1;
            const float4* s4 = reinterpret_cast<const float4*>(src);
            for (int base = 0; base < pairs; base += U * NT) {
                float4 v[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = base + (int)threadIdx.x + u * NT;
                    v[u] = s4[e < pairs ? e : pairs - 1];  // always a valid address
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = base + (int)threadIdx.x + u * NT;
                    if (e < pairs) {
                        const int e0 = 2 * e, e1 = e0 + 1;
                        const int q0 = fdiv(e0, mgH), q1 = fdiv(e1, mgH);
                        buf[q0 * Hs + pad16(e0 - q0 * H)] = mk<T>(v[u].x, v[u].y);
                        buf[q1 * Hs + pad16(e1 - q1 * H)] = mk<T>(v[u].z, v[u].w);
                    }
                }
            }
            return;
        }
    }
    for (int base = 0; base < count; base += U * NT) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + (int)threadIdx.x + u * NT;
            v[u] = load_cx<LP, T>(src + (e < count ? e : count - 1));  // always a valid address
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + (int)threadIdx.x + u * NT;
            if (e < count) {
                const int q = fdiv(e, mgH);
                buf[q * Hs + pad16(e - q * H)] = v[u];
            }
        }
    }
}

template <typename T, int NT, int SP = ST_PLAIN>
__device__ __forceinline__ void lds_to_rows(cx<T>* dst, const cx<T>* buf, int rows, int H, int Hs, uint32_t mgH)
{
    const int count = rows * H;
    if constexpr (sizeof(T) == 4 && SP == ST_PLAIN) {
        if (((uintptr_t)dst & 15) == 0 && (count & 1) == 0) {
            const int pairs = count >> 1;
            float4* d4 = reinterpret_cast<float4*>(dst);
            for (int e = (int)threadIdx.x; e < pairs; e += NT) {
                const int e0 = 2 * e, e1 = e0 + 1;
                const int q0 = fdiv(e0, mgH), q1 = fdiv(e1, mgH);
                const cx<T> a = buf[q0 * Hs + pad16(e0 - q0 * H)], b = buf[q1 * Hs + pad16(e1 - q1 * H)];
                d4[e] = make_float4(a.x, a.y, b.x, b.y);
            }
            return;
        }
    }
    for (int e = (int)threadIdx.x; e < count; e += NT) {
        const int q = fdiv(e, mgH);
        store_cx<SP, T>(dst + e, buf[q * Hs + pad16(e - q * H)]);
    }
}

// ---- tiles: the unit of work of every kernel ----

// Length-n transforms down `width` (<= W) consecutive columns of a row-major
// block, row stride S; src and dst may be equal.  LP / SP: cache policies.
template <typename T, int NT, int EPT, bool INV, int LP = LD_PLAIN, int SP = ST_PLAIN>
__device__ __forceinline__ void col_tile(const cx<T>* src, cx<T>* dst, int64_t S, int width, int W,
                                         uint32_t mg_w, const AxisSched& ax, const cx<T>* __restrict__ tw,
                                         cx<T>* buf)
{
    ColTileIO<T, LP, SP> g;
    g.src = src;
    g.dst = dst;
    g.S = S;
    g.width = width;
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

// `rows` real rows of length n2 (read as h = n2/2 complex values
// z[m] = x[2m] + i x[2m+1]) -> `rows` rows of H = h+1 bins, contiguous.
// Hs: padded LDS row stride.  rs: stride of the real rows in complex units
// (0: h, contiguous rows; H for the padded in-place layout).  LP: cache policy of the input loads, SP: of
// the output stores.
template <typename T, int NT, int EPT, int LP = LD_PLAIN, int SP = ST_PLAIN>
__device__ __forceinline__ void rows_r2c_tile(const cx<T>* xz, cx<T>* Xo, int rows, int Hs, const AxisSched& axh,
                                              const cx<T>* __restrict__ tw, const cx<T>* __restrict__ post,
                                              cx<T>* buf, int rs = 0)
{
    const int h = axh.n, H = h + 1;
    RowsIO<T, LP> g;
    g.src = xz;
    g.dst = nullptr;
    g.len = rs ? rs : h;
    const LdsRowsIO<T> l = lds_rows<T>(buf, Hs);
    fft_lines<false, false, NT, EPT, T>(g, l, l, rows, 0u, axh, tw);
    split_rows<NT, T>(buf, rows, Hs, h, axh.mg_pairs, post);
    lds_to_rows<T, NT, SP>(Xo, buf, rows, H, Hs, axh.mg_np1);
}

// `rows` rows of H bins -> `rows` real rows of length n2.  LP: cache policy
// of the bin loads, SP: of the output stores.
template <typename T, int NT, int EPT, int LP = LD_PLAIN, int SP = ST_PLAIN>
__device__ __forceinline__ void rows_c2r_tile(const cx<T>* Xi, cx<T>* yz, int rows, int Hs, const AxisSched& axh,
                                              const cx<T>* __restrict__ tw, const cx<T>* __restrict__ post,
                                              cx<T>* buf, int rs = 0)
{
    const int h = axh.n, H = h + 1;
    rows_to_lds<T, NT, LP>(buf, Xi, rows, H, Hs, axh.mg_np1);
    __syncthreads();
    merge_rows<NT, T>(buf, rows, Hs, h, axh.mg_pairs, post);
    RowsIO<T, LD_PLAIN, SP> g;
    g.src = nullptr;
    g.dst = yz;
    g.len = rs ? rs : h;
    const LdsRowsIO<T> l = lds_rows<T>(buf, Hs);
    fft_lines<true, false, NT, EPT, T>(l, l, g, rows, 0u, axh, tw);
}

// ---- standalone kernels ----

template <typename T, int NT, int EPT, bool INV>
__global__ __launch_bounds__(NT, (cols_waves<T, NT, EPT>())) void k_cols(const cx<T>* in, cx<T>* out, const AxisSched* __restrict__ axp,
                                             const cx<T>* __restrict__ tw, int64_t S, int64_t ncols,
                                             int64_t bstride, int W, uint32_t mg_w, int64_t tiles_per_batch,
                                             int64_t ntiles, int64_t ngroups, int gsize, int reverse)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int64_t t = group_tile(blockIdx.x, ngroups, gsize, reverse);
    if (t >= ntiles) return;  // padding workgroup
    const int64_t b = t / tiles_per_batch;
    const int64_t c0 = (t - b * tiles_per_batch) * W;
    const int64_t rem = ncols - c0;
    const int width = rem < (int64_t)W ? (int)rem : W;
    col_tile<T, NT, EPT, INV>(in + b * bstride + c0, out + b * bstride + c0, S, width, W, mg_w, *axp, tw, buf);
}

// The wide column tiles (128 KB, one workgroup per CU, so no second
// workgroup overlaps one's loads with another's arithmetic) as a persistent
// loop: each workgroup walks the tiles k_cols's grid would hand to workgroups
// blockIdx.x, blockIdx.x + gridDim.x, ... (gridDim.x a multiple of the XCD
// count, so every tile stays on the XCD it had), and loads the next tile's
// first-stage inputs into registers while the current tile runs its LDS
// stages and stores.  R0: the first stage's radix; needs two stages or more,
// the later ones of radix <= kPipeMaxRadix (the registers of the loads in
// flight leave no room for radix-16 code).  Same tiles, same arithmetic and
// results as k_cols.
//
// Vector memory accesses complete on one in-order counter (vmcnt): waiting
// for one load waits for every global or scratch access issued before it.
// So nothing between issuing the next tile's loads and using them may wait
// on such an access: the later stages load nothing from global memory (their
// twiddles sit in LDS after the tile, copied once), the loads are unmasked
// until they are used (first_stage_load), and the kernel must not spill (a
// spill reload is such a wait).  Dynamic LDS: the tile, then
// later_twiddles(ax) complex values.
template <typename T, int NT, int EPT, bool INV, int R0>
__global__ __launch_bounds__(NT, 1) void k_cols_pipe(const cx<T>* in, cx<T>* out, const AxisSched* __restrict__ axp,
                                                     const cx<T>* __restrict__ tw, int64_t S, int64_t ncols,
                                                     int64_t bstride, int W, uint32_t mg_w, int64_t tiles_per_batch,
                                                     int64_t ntiles, int64_t ngroups, int gsize, int reverse,
                                                     int64_t nvirt)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    cx<T>* twl = buf + (int64_t)axp->n * W;
    {
        const int ntw = later_twiddles(*axp);
        for (int i = (int)threadIdx.x; i < ntw; i += NT) twl[i] = tw[i];
        // (the first barrier of the loop orders these writes before any read)
    }
    // What the stages derive from the schedule, the tile width, the
    // twiddles and the thread index is the same for every tile; the compiler
    // would hoist all of it out of the loop and hold it in registers across
    // tiles (spilling).  Every such input is taken once per tile through an
    // offset of zero that the compiler cannot see through (Loop), which keeps
    // that work inside the loop.
    struct Loop {
        const AxisSched* ax;
        const cx<T>* tw;
        int W, gsize;
        uint32_t mg_w;
        int64_t tpb;
    };
    auto loop_inputs = [&]() {
        int zero = 0;
        asm volatile("" : "+s"(zero));
        Loop q;
        q.ax = axp + zero;
        q.tw = twl + zero;
        q.W = W + zero;
        q.gsize = gsize + zero;
        q.mg_w = mg_w + (uint32_t)zero;
        q.tpb = tiles_per_batch + zero;
        return q;
    };
    auto lds_io = [&](const Loop& q) {
        LdsIO<T> l;
        l.buf = buf;
        l.L.nlines = q.W;
        l.L.lpp = q.W;
        l.L.sp = 0;
        l.L.sw = 1;
        l.L.si = q.W;
        l.L.mg_lines = q.mg_w;
        l.L.mg_lpp = q.mg_w;
        return l;
    };
    auto first_arg = [&](const Loop& q) {
        StageArg a;
        a.n = q.ax->n;
        a.nlines = q.W;
        a.Ns = 1;
        a.mg_lines = q.mg_w;
        a.mg_nb = q.ax->mg_nb[0];
        a.mg_ns = q.ax->mg_ns[0];
        return a;
    };
    // the next real tile at or after virtual workgroup index vb (padding
    // indices map past the tile count); nvirt when none is left
    auto next_tile = [&](const Loop& q, int64_t vb, int64_t& t) {
        for (; vb < nvirt; vb += gridDim.x) {
            t = group_tile(vb, ngroups, q.gsize, reverse);
            if (t < ntiles) break;
        }
        return vb;
    };
    auto tile_io = [&](const Loop& q, int64_t t) {
        const int64_t b = t / q.tpb;
        const int64_t c0 = (t - b * q.tpb) * q.W;
        const int64_t rem = ncols - c0;
        ColTileIO<T> g;
        g.src = in + b * bstride + c0;
        g.dst = out + b * bstride + c0;
        g.S = S;
        g.width = rem < (int64_t)q.W ? (int)rem : q.W;
        return g;
    };
    int64_t t = 0;
    Loop q = loop_inputs();
    int64_t vb = next_tile(q, blockIdx.x, t);
    if (vb >= nvirt) return;
    ColTileIO<T> g = tile_io(q, t);
    cx<T> v[FirstStage<R0, NT, EPT>::K][R0];
    first_stage_load<R0, NT, EPT, T>(g, first_arg(q), v);
    for (;;) {
        q = loop_inputs();
        const AxisSched& ax = *q.ax;
        const LdsIO<T> l = lds_io(q);
        const StageArg a0 = first_arg(q);
        // the next tile's index first: the loads in flight complete before
        // anything here that waits on memory (a spill reload) holds them up
        int64_t tn = 0;
        const int64_t vn = next_tile(q, vb + gridDim.x, tn);
        first_stage_finish<R0, INV, NT, EPT, T>(l, a0, v, g.width);
        __syncthreads();
        ColTileIO<T> gn = g;
        if (vn < nvirt) {
            gn = tile_io(q, tn);
            first_stage_load<R0, NT, EPT, T>(gn, a0, v);  // in flight during the stages below
        }
        const int nst = ax.nst;
        for (int s = 1; s < nst - 1; ++s)
            stage_upto<kPipeMaxRadix, INV, true, NT, EPT, true, true, T>(ax, s, q.W, q.mg_w, l, l, q.tw);
        stage_direct_upto<kPipeMaxRadix, INV, true, NT, EPT, T>(ax, nst - 1, q.W, q.mg_w, l, g, q.tw);
        if (vn >= nvirt) break;
        __syncthreads();  // the last stage's LDS reads before the next tile's writes
        vb = vn;
        g = gn;
    }
}

// Split-plane forward: rpw real rows of length n2 -> rpw rows of H bins.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT, (rows_waves<T, EPT, false>())) void k_rows_r2c(const T* x, cx<T>* X, const AxisSched* __restrict__ axp,
                                                 const cx<T>* __restrict__ tw,
                                                 const cx<T>* __restrict__ post, int64_t nrows,
                                                 int rpw, int Hs, int reverse, int rs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& axh = *axp;
    const int H = axh.n + 1;
    const int64_t row0 = (reverse ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x) * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    rows_r2c_tile<T, NT, EPT>(reinterpret_cast<const cx<T>*>(x) + row0 * rs, X + row0 * H, rows, Hs, axh, tw, post,
                              buf, rs);
}

// Split-plane inverse: rpw rows of H bins -> rpw real rows of length n2.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT, (rows_waves<T, EPT, true>())) void k_rows_c2r(const cx<T>* X, T* y, const AxisSched* __restrict__ axp,
                                                 const cx<T>* __restrict__ tw,
                                                 const cx<T>* __restrict__ post, int64_t nrows,
                                                 int rpw, int Hs, int reverse, int rs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& axh = *axp;
    const int H = axh.n + 1;
    const int64_t row0 = (reverse ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x) * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    rows_c2r_tile<T, NT, EPT>(X + row0 * H, reinterpret_cast<cx<T>*>(y) + row0 * rs, rows, Hs, axh, tw, post, buf,
                              rs);
}

// ---- odd n2: two real rows per complex line ----
//
// With n2 odd there is no half-length complex row.  Rows a = 2p and b = 2p+1
// of a tile are transformed together as the complex line z = x_a + i x_b of
// length n2 (Z = DFT z) and then separated, for k = 0 .. H-1 (H = (n2+1)/2):
//   X_a[k] = (Z[k] + conj Z[n2-k]) / 2,   X_b[k] = (Z[k] - conj Z[n2-k]) / (2i)
// (Z[n2-0] read as Z[0]).  The inverse builds the line from the two rows of
// bins, Z[k] = X_a[k] + i X_b[k] and Z[n2-k] = conj X_a[k] + i conj X_b[k]
// for k >= 1, Z[0] = Re X_a[0] + i Re X_b[0] (the imaginary part of the DC
// bin is dropped, as the c2r definition does), and takes y_a = Re z,
// y_b = Im z.  A tile with an odd number of rows pairs its last row with a
// zero row.  In LDS, pair p's line occupies the two padded rows 2p, 2p+1
// (line stride 2*Hs), and the separated bins land in those rows.

// Global real rows read as pair lines: line w, element i = (x_a[i], x_b[i]).
template <typename T> struct PairRowsIn {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    struct Pos {
        int off;
        bool two;  // row b exists
    };
    const T* src;
    int rs, rows;  // rs: real-row stride (n2, or 2H padded)
    __device__ __forceinline__ Pos at(int w, int i) const { return Pos{2 * w * rs + i, 2 * w + 1 < rows}; }
    __device__ __forceinline__ Pos adv(Pos p, int d) const
    {
        p.off += d;
        return p;
    }
    __device__ __forceinline__ cx<T> get(Pos p) const { return mk<T>(src[p.off], p.two ? src[p.off + rs] : (T)0); }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
};

// Pair lines written out as real rows: y_a[i] = Re, y_b[i] = Im.
template <typename T> struct PairRowsOut {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    using Pos = typename PairRowsIn<T>::Pos;
    T* dst;
    int rs, rows;
    __device__ __forceinline__ Pos at(int w, int i) const { return Pos{2 * w * rs + i, 2 * w + 1 < rows}; }
    __device__ __forceinline__ Pos adv(Pos p, int d) const
    {
        p.off += d;
        return p;
    }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const
    {
        dst[p.off] = v.x;
        if (p.two) dst[p.off + rs] = v.y;
    }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

// Separation of the pair lines into rows of H bins (all reads, barrier, all
// writes: the rows overlay the lines).  At most NT * kPairItems (pair, bin)
// items per tile (the plan caps the rows per tile).  mgH = div_magic(H).
template <int NT, typename T>
__device__ __forceinline__ void split_pairs(cx<T>* buf, int rows, int Hs, int n2, int H, uint32_t mgH)
{
    const int total = ((rows + 1) / 2) * H;
    cx<T> xa[kPairItems], xb[kPairItems];
#pragma unroll
    for (int u = 0; u < kPairItems; ++u) {
        const int e = (int)threadIdx.x + u * NT;
        if (e < total) {
            const int p = fdiv(e, mgH), k = e - p * H;
            const cx<T>* Z = buf + 2 * p * Hs;
            const cx<T> A = Z[pad16(k)], B = Z[pad16(k == 0 ? 0 : n2 - k)];
            xa[u] = mk<T>((T)0.5 * (A.x + B.x), (T)0.5 * (A.y - B.y));
            xb[u] = mk<T>((T)0.5 * (A.y + B.y), (T)-0.5 * (A.x - B.x));
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPairItems; ++u) {
        const int e = (int)threadIdx.x + u * NT;
        if (e < total) {
            const int p = fdiv(e, mgH), k = e - p * H;
            buf[2 * p * Hs + pad16(k)] = xa[u];
            if (2 * p + 1 < rows) buf[(2 * p + 1) * Hs + pad16(k)] = xb[u];
        }
    }
    __syncthreads();
}

// The reverse: rows of H bins -> pair lines of n2 elements.
template <int NT, typename T>
__device__ __forceinline__ void merge_pairs(cx<T>* buf, int rows, int Hs, int n2, int H, uint32_t mgH)
{
    const int total = ((rows + 1) / 2) * H;
    cx<T> zk[kPairItems], zm[kPairItems];
#pragma unroll
    for (int u = 0; u < kPairItems; ++u) {
        const int e = (int)threadIdx.x + u * NT;
        if (e < total) {
            const int p = fdiv(e, mgH), k = e - p * H;
            const cx<T> a = buf[2 * p * Hs + pad16(k)];
            const cx<T> b = 2 * p + 1 < rows ? buf[(2 * p + 1) * Hs + pad16(k)] : mk<T>((T)0, (T)0);
            if (k == 0) {
                zk[u] = mk<T>(a.x, b.x);
            } else {
                zk[u] = mk<T>(a.x - b.y, a.y + b.x);
                zm[u] = mk<T>(a.x + b.y, b.x - a.y);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPairItems; ++u) {
        const int e = (int)threadIdx.x + u * NT;
        if (e < total) {
            const int p = fdiv(e, mgH), k = e - p * H;
            cx<T>* Z = buf + 2 * p * Hs;
            Z[pad16(k)] = zk[u];
            if (k > 0) Z[pad16(n2 - k)] = zm[u];
        }
    }
    __syncthreads();
}

// Split-plane forward for odd n2: rpw real rows -> rpw rows of H bins.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_rows_r2c_odd(const T* x, cx<T>* X, const AxisSched* __restrict__ axp,
                                                     const cx<T>* __restrict__ tw, int64_t nrows, int rpw, int Hs,
                                                     uint32_t mgH, int reverse, int rs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& ax = *axp;  // length n2
    const int n2 = ax.n, H = n2 / 2 + 1;
    const int64_t row0 = (reverse ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x) * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    PairRowsIn<T> g;
    g.src = x + row0 * rs;
    g.rs = rs;
    g.rows = rows;
    const LdsRowsIO<T> l = lds_rows<T>(buf, 2 * Hs);
    fft_lines<false, false, NT, EPT, T>(g, l, l, (rows + 1) / 2, 0u, ax, tw);
    split_pairs<NT, T>(buf, rows, Hs, n2, H, mgH);
    lds_to_rows<T, NT>(X + row0 * H, buf, rows, H, Hs, mgH);
}

// Split-plane inverse for odd n2: rpw rows of H bins -> rpw real rows.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_rows_c2r_odd(const cx<T>* X, T* y, const AxisSched* __restrict__ axp,
                                                     const cx<T>* __restrict__ tw, int64_t nrows, int rpw, int Hs,
                                                     uint32_t mgH, int reverse, int rs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const AxisSched& ax = *axp;
    const int n2 = ax.n, H = n2 / 2 + 1;
    const int64_t row0 = (reverse ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x) * rpw;
    const int64_t left = nrows - row0;
    const int rows = left < rpw ? (int)left : rpw;
    rows_to_lds<T, NT>(buf, X + row0 * H, rows, H, Hs, mgH);
    __syncthreads();
    merge_pairs<NT, T>(buf, rows, Hs, n2, H, mgH);
    PairRowsOut<T> g;
    g.dst = y + row0 * rs;
    g.rs = rs;
    g.rows = rows;
    const LdsRowsIO<T> l = lds_rows<T>(buf, 2 * Hs);
    fft_lines<true, false, NT, EPT, T>(l, l, g, (rows + 1) / 2, 0u, ax, tw);
}

// np whole n1 x n2 planes (np <= ppw) held in LDS as padded rows
// [plane][n1][Hs]: forward = rows (from HBM), split, then the n1 columns (to
// HBM); inverse = n1 columns (from HBM), merge, rows (to HBM).  mg_lines =
// div_magic(np * H).
template <typename T, int NT, int EPT>
__device__ __forceinline__ void plane_r2c_tile(const cx<T>* xz, cx<T>* Xo, int np, const AxisSched& axh,
                                               const AxisSched& ax1, const cx<T>* __restrict__ tw2,
                                               const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw1,
                                               int Hs, uint32_t mg_lines, uint32_t mgH, cx<T>* buf, int rs = 0)
{
    const int h = axh.n, H = h + 1, n1 = ax1.n;
    const int rows = np * n1;
    RowsIO<T> gi;
    gi.src = xz;
    gi.dst = nullptr;
    gi.len = rs ? rs : h;
    const LdsRowsIO<T> lr = lds_rows<T>(buf, Hs);
    fft_lines<false, false, NT, EPT, T>(gi, lr, lr, rows, 0u, axh, tw2);
    split_rows<NT, T>(buf, rows, Hs, h, axh.mg_pairs, post);
    PlaneColsIO<T> go;
    go.src = nullptr;
    go.dst = Xo;
    go.H = H;
    go.plane = n1 * H;
    go.mgH = mgH;
    const LdsPlaneColsIO<T> lc = lds_plane_cols<T>(buf, n1, H, Hs, mgH);
    fft_lines<false, true, NT, EPT, T>(lc, lc, go, np * H, mg_lines, ax1, tw1);
}

template <typename T, int NT, int EPT>
__device__ __forceinline__ void plane_c2r_tile(const cx<T>* Xi, cx<T>* yz, int np, const AxisSched& axh,
                                               const AxisSched& ax1, const cx<T>* __restrict__ tw2,
                                               const cx<T>* __restrict__ post, const cx<T>* __restrict__ tw1,
                                               int Hs, uint32_t mg_lines, uint32_t mgH, cx<T>* buf, int rs = 0)
{
    const int h = axh.n, H = h + 1, n1 = ax1.n;
    const int rows = np * n1;
    PlaneColsIO<T> gi;
    gi.src = Xi;
    gi.dst = nullptr;
    gi.H = H;
    gi.plane = n1 * H;
    gi.mgH = mgH;
    const LdsPlaneColsIO<T> lc = lds_plane_cols<T>(buf, n1, H, Hs, mgH);
    fft_lines<true, true, NT, EPT, T>(gi, lc, lc, np * H, mg_lines, ax1, tw1);
    merge_rows<NT, T>(buf, rows, Hs, h, axh.mg_pairs, post);
    RowsIO<T> go;
    go.src = nullptr;
    go.dst = yz;
    go.len = rs ? rs : h;
    const LdsRowsIO<T> lr = lds_rows<T>(buf, Hs);
    fft_lines<true, false, NT, EPT, T>(lr, lr, go, rows, 0u, axh, tw2);
}

// Fused plane kernels: ppw whole planes per workgroup.  Their pointer
// arguments are not declared restrict: with it the compiler keeps more of the
// tables in registers across both axes' stages (163 VGPRs instead of 113 for
// the FP32 small tier, one workgroup a CU instead of two; the big tier
// spilled); measured without it: 96^3 FP64 and 192x192x96 FP32 plane steps
// 11% and 24% faster, the others equal, bits unchanged.
template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_plane_r2c(const T* x, cx<T>* X, const AxisSched* axhp,
                                                  const AxisSched* ax1p,
                                                  const cx<T>* tw2,
                                                  const cx<T>* post,
                                                  const cx<T>* tw1, int64_t nplanes,
                                                  int ppw, int Hs, uint32_t mg_lines, uint32_t mgH, int rs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int H = axhp->n + 1, n1 = ax1p->n;
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int64_t left = nplanes - p0;
    const int np = left < ppw ? (int)left : ppw;
    plane_r2c_tile<T, NT, EPT>(reinterpret_cast<const cx<T>*>(x) + p0 * n1 * rs, X + p0 * n1 * H, np, *axhp, *ax1p,
                               tw2, post, tw1, Hs, np == ppw ? mg_lines : div_magic_dev(np * H), mgH, buf, rs);
}

template <typename T, int NT, int EPT>
__global__ __launch_bounds__(NT) void k_plane_c2r(const cx<T>* X, T* y, const AxisSched* axhp,
                                                  const AxisSched* ax1p,
                                                  const cx<T>* tw2,
                                                  const cx<T>* post,
                                                  const cx<T>* tw1, int64_t nplanes,
                                                  int ppw, int Hs, uint32_t mg_lines, uint32_t mgH, int rs)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const int H = axhp->n + 1, n1 = ax1p->n;
    const int64_t p0 = (int64_t)blockIdx.x * ppw;
    const int64_t left = nplanes - p0;
    const int np = left < ppw ? (int)left : ppw;
    plane_c2r_tile<T, NT, EPT>(X + p0 * n1 * H, reinterpret_cast<cx<T>*>(y) + p0 * n1 * rs, np, *axhp, *ax1p, tw2,
                               post, tw1, Hs, np == ppw ? mg_lines : div_magic_dev(np * H), mgH, buf, rs);
}

// ---- cooperative plane step for planes larger than LDS ----
//
// One persistent launch does the whole plane step.  Each workgroup reads the
// XCD it runs on (hardware register XCC_ID) and takes tickets from that
// XCD's queue.  Tickets come in slots of T = RT + CT tasks.  Slot s first
// holds the first-phase tasks of plane P(s) (forward: RT row tasks, rpw rows
// each: half-length FFT + split, written to X; inverse: CT column tasks, W
// columns of the plane down n1, in place), then the second-phase tasks of
// plane P(s - L) (forward: CT column tasks in place on X; inverse: RT row
// tasks, merge + inverse rows to y).  A second-phase task waits until every
// first-phase task of its plane has counted itself done; the lag of L slots
// gives those tasks time to finish, so workgroups rarely wait.  P(s) is
// claimed by the first ticket of slot s from a global plane counter, in slot
// order within a queue (the claimer waits for slot s-1's claim), so once a
// slot finds no plane left every later slot of the queue is empty too.
// A plane's tasks all run on one XCD, so its intermediate stays in that
// XCD's L2: producers drain their stores to L2 (s_waitcnt) before the count
// goes up, consumers read with device-scope loads that miss L1.  Every wait
// is for a smaller ticket than the waiter's own, held by a workgroup that is
// running, so the kernel cannot deadlock whatever the placement of
// workgroups; every wait is also bounded (spin limit), after which the
// workgroup records an error and leaves.

struct CoopArgs {
    int64_t n0;
    int n1, h, H;
    int rpw, RT;         // rows per row task, row tasks per plane
    int Hs;              // padded LDS row stride
    int W, CT;           // column tile width, column tasks per plane
    uint32_t mg_w;
    int lag;             // L: slots between a plane's two phases
    int nslots;          // slots per queue
    int spin_limit;
    const AxisSched* axh;
    const AxisSched* ax1;
    int64_t off_tw2, off_post, off_tw1;
    int* ctr;  // [claim][error][ticket x kCoopQueues][queue][slot][plane+1 or -1, done]
};

// Bounded waits.  Both give up at once when an earlier wait of the launch has
// already failed (*err != 0), so a failed launch drains in one spin limit
// instead of one per waiting ticket.
__device__ __forceinline__ int coop_wait_nonzero(int* p, const int* err, int limit)
{
    for (int it = 0; it < limit; ++it) {
        const int v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v != 0) return v;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return 0;
        __builtin_amdgcn_s_sleep(2);
    }
    return 0;
}

__device__ __forceinline__ bool coop_wait_geq(int* p, int target, const int* err, int limit)
{
    for (int it = 0; it < limit; ++it) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

enum { kCoopExit = 0, kCoopSkip = 1, kCoopTask = 2 };

template <typename T, int NT, int EPT, bool INV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_plane_coop(const void* in, void* out, const cx<T>* tw, CoopArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    __shared__ int s_task[4];
    const int q = __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kCoopQueues - 1);
    int* ticket = a.ctr + 2 + q;
    int* slots = a.ctr + 2 + kCoopQueues + (int64_t)q * 2 * a.nslots;
    const int first = INV ? a.CT : a.RT;  // first-phase tasks per plane
    const int TT = a.RT + a.CT;
    const cx<T>* tw2 = tw + a.off_tw2;
    const cx<T>* post = tw + a.off_post;
    const cx<T>* tw1 = tw + a.off_tw1;
    const int h = a.h, H = a.H, n1 = a.n1;
    // a workgroup runs each ticket of its queue at most once: more iterations
    // than the queue's tickets end the loop (error bit 8), whatever memory holds
    const int max_iters = a.nslots * TT + 1;
    int iters = 0;
    for (;;) {
        __syncthreads();  // the previous task is done with LDS and s_task
        if (threadIdx.x == 0) {
            int kind = kCoopExit, pl = 0, k = 0, ps = 0;
            const int t = atomicAdd(ticket, 1);
            const int s = t / TT;
            k = t - s * TT;
            if (++iters > max_iters) {
                atomicOr(&a.ctr[1], 8);
            } else if (s >= a.nslots) {
                atomicOr(&a.ctr[1], 4);
            } else if (k < first) {
                // first phase of plane P(s)
                int* slot = slots + 2 * s;
                int v;
                if (k == 0) {
                    const int prev = s > 0 ? coop_wait_nonzero(slot - 2, a.ctr + 1, a.spin_limit) : 1;
                    if (prev == 0) {
                        atomicOr(&a.ctr[1], 1);
                        v = 0;
                    } else if (prev < 0) {
                        v = -1;
                    } else {
                        const int c = atomicAdd(&a.ctr[0], 1);
                        v = c < a.n0 ? c + 1 : -1;
                    }
                    if (v != 0) __hip_atomic_store(slot, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    v = coop_wait_nonzero(slot, a.ctr + 1, a.spin_limit);
                    if (v == 0) atomicOr(&a.ctr[1], 1);
                }
                if (v > 0) {
                    kind = kCoopTask;
                    pl = v - 1;
                    ps = s;
                } else if (v < 0) {
                    kind = kCoopSkip;  // later second-phase tickets may still have work
                }
            } else if (s < a.lag) {
                kind = kCoopSkip;
            } else {
                // second phase of plane P(s - L)
                int* slot = slots + 2 * (s - a.lag);
                const int v = coop_wait_nonzero(slot, a.ctr + 1, a.spin_limit);
                if (v > 0) {
                    if (coop_wait_geq(slot + 1, first, a.ctr + 1, a.spin_limit)) {
                        kind = kCoopTask;
                        pl = v - 1;
                        ps = s - a.lag;
                    } else {
                        atomicOr(&a.ctr[1], 2);
                    }
                } else if (v == 0) {
                    atomicOr(&a.ctr[1], 1);
                }
                // v < 0: no plane there, nor in any later slot: leave
            }
            s_task[0] = kind;
            s_task[1] = pl;
            s_task[2] = k;
            s_task[3] = ps;
        }
        __syncthreads();
        const int kind = s_task[0], pl = s_task[1], k = s_task[2], ps = s_task[3];
        if (kind == kCoopExit) break;
        if (kind == kCoopSkip) continue;
        const int64_t plane = (int64_t)pl * n1 * H;  // complex offset of the plane
        const bool first_phase = k < first;
        const int ktask = first_phase ? k : k - first;
        const bool row_task = INV ? !first_phase : first_phase;
        if (row_task) {
            const int r0 = ktask * a.rpw;
            const int rows = n1 - r0 < a.rpw ? n1 - r0 : a.rpw;
            if (!INV) {
                const cx<T>* xz = reinterpret_cast<const cx<T>*>(in) + ((int64_t)pl * n1 + r0) * h;
                cx<T>* Xo = reinterpret_cast<cx<T>*>(out) + plane + (int64_t)r0 * H;
                // input read once (streamed); the intermediate stays in L2
                rows_r2c_tile<T, NT, EPT, LD_STREAM, ST_PLAIN>(xz, Xo, rows, a.Hs, *a.axh, tw2, post, buf);
            } else {
                const cx<T>* Xi = reinterpret_cast<const cx<T>*>(in) + plane + (int64_t)r0 * H;
                cx<T>* yz = reinterpret_cast<cx<T>*>(out) + ((int64_t)pl * n1 + r0) * h;
                // the intermediate comes from L2; the output is streamed
                rows_c2r_tile<T, NT, EPT, LD_L2, ST_STREAM>(Xi, yz, rows, a.Hs, *a.axh, tw2, post, buf);
            }
        } else {
            const int c0 = ktask * a.W;
            const int width = H - c0 < a.W ? H - c0 : a.W;
            if (!INV) {
                cx<T>* X = reinterpret_cast<cx<T>*>(out) + plane + c0;
                col_tile<T, NT, EPT, false, LD_L2, ST_STREAM>(X, X, H, width, a.W, a.mg_w, *a.ax1, tw1, buf);
            } else {
                cx<T>* B = const_cast<cx<T>*>(reinterpret_cast<const cx<T>*>(in)) + plane + c0;
                col_tile<T, NT, EPT, true, LD_STREAM, ST_PLAIN>(B, B, H, width, a.W, a.mg_w, *a.ax1, tw1, buf);
            }
        }
        if (first_phase) {
            __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
            __syncthreads();                // ... and every wave's
            if (threadIdx.x == 0) atomicAdd(&slots[2 * ps + 1], 1);
        }
    }
}

// Exchange of the two outer axes of an [na][nb][H] array of rows (the
// transpose of the paper's transpose-based method, Sec. 2.1 step 2):
// out[b][a][:] = in[a][b][:].  Rows of H elements stay contiguous, so reads
// and writes are whole-row runs.  Workgroup: rows a0 .. a0+R-1 of column b,
// written as one contiguous run.
template <typename T, int NT>
__global__ __launch_bounds__(NT) void k_swap01(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, int na,
                                              int nb, int H, int R, uint32_t mgH, int tiles_a)
{
    constexpr int U = 8;
    const int b = (int)blockIdx.x / tiles_a;
    const int a0 = ((int)blockIdx.x - b * tiles_a) * R;
    const int rows = na - a0 < R ? na - a0 : R;
    const int count = rows * H;
    const int64_t stride = (int64_t)nb * H;
    const cx<T>* src = in + ((int64_t)a0 * nb + b) * H;
    cx<T>* dst = out + ((int64_t)b * na + a0) * H;
    for (int base = 0; base < count; base += U * NT) {
        cx<T> v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            int e = base + (int)threadIdx.x + u * NT;
            e = e < count ? e : count - 1;  // always a valid address
            const int q = fdiv(e, mgH);
            v[u] = load_cx<LD_STREAM, T>(src + q * stride + (e - q * H));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = base + (int)threadIdx.x + u * NT;
            if (e < count) store_cx<ST_STREAM, T>(dst + e, v[u]);
        }
    }
}

template <int Unused = 0> __global__ void k_zero_ints(int* p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ----------------------------------------------------------- launchers --
// Templates instantiated per dtype in fft3d_kern_{f32,f64}.hip (plain kernels)
// and fft3d_coop_{f32,f64}.hip (cooperative plane kernel).



template <typename T> const cx<T>* table(const Plan& p, int64_t off)
{
    return reinterpret_cast<const cx<T>*>(p.d_tw) + off;
}

// Device copies of the schedules: [n0, n1, n2/2].
inline const AxisSched* dsched(const Plan& p, int axis) { return p.d_sched + axis; }

template <typename K> hipError_t allow_lds(K kernel)
{
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
}

template <typename T> hipError_t init_plain()
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
    FFT3D_ALLOW((k_cols<T, kNtWide, ES, false>));
    FFT3D_ALLOW((k_cols<T, kNtWide, ES, true>));
    FFT3D_ALLOW((k_cols_pipe<T, PipeTier<T>::kNt, PipeTier<T>::kEpt, false, 16>));
    FFT3D_ALLOW((k_cols_pipe<T, PipeTier<T>::kNt, PipeTier<T>::kEpt, true, 16>));
    FFT3D_ALLOW((k_cols_pipe<T, PipeTier<T>::kNt, PipeTier<T>::kEpt, false, 8>));
    FFT3D_ALLOW((k_cols_pipe<T, PipeTier<T>::kNt, PipeTier<T>::kEpt, true, 8>));
    if constexpr (sizeof(T) == 4) {
        FFT3D_ALLOW((k_cols<T, kNtFine, kEptFine, false>));
        FFT3D_ALLOW((k_cols<T, kNtFine, kEptFine, true>));
    }
    FFT3D_ALLOW((k_rows_r2c<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_r2c<T, kNtBig, EB>));
    FFT3D_ALLOW((k_rows_c2r<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_c2r<T, kNtBig, EB>));
    FFT3D_ALLOW((k_rows_r2c_odd<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_r2c_odd<T, kNtBig, EB>));
    FFT3D_ALLOW((k_rows_c2r_odd<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_rows_c2r_odd<T, kNtBig, EB>));
    FFT3D_ALLOW((k_plane_r2c<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_plane_r2c<T, kNtBig, EB>));
    FFT3D_ALLOW((k_plane_c2r<T, kNtSmall, ES>));
    FFT3D_ALLOW((k_plane_c2r<T, kNtBig, EB>));
#undef FFT3D_ALLOW
    return e;
}

template <typename T> hipError_t init_coop()
{
    constexpr int ES = Tier<T>::kEptSmall;
    hipError_t a = allow_lds(k_plane_coop<T, kNtSmall, ES, false>);
    hipError_t b = allow_lds(k_plane_coop<T, kNtSmall, ES, true>);
    return a != hipSuccess ? a : b;
}

// padded: real rows of 2H reals (the in-place layout) instead of n2.
template <typename T>
hipError_t plane_r2c_t(const Plan& p, const void* x, void* X, hipStream_t st, bool padded = false)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const int rs = (int)(padded ? p.H : p.h);
    const unsigned grid = (unsigned)((p.n0 + p.ppw - 1) / p.ppw);
    const T* xi = static_cast<const T*>(x);
    cx<T>* Xo = static_cast<cx<T>*>(X);
    if (p.plane_big)
        hipLaunchKernelGGL((k_plane_r2c<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.plane_lds, st, xi,
                           Xo, dsched(p, 2), dsched(p, 1), table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw, p.plane_Hs,
                           div_magic((uint32_t)(p.ppw * p.H)), div_magic((uint32_t)p.H), rs);
    else
        hipLaunchKernelGGL((k_plane_r2c<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.plane_lds, st,
                           xi, Xo, dsched(p, 2), dsched(p, 1), table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw, p.plane_Hs,
                           div_magic((uint32_t)(p.ppw * p.H)), div_magic((uint32_t)p.H), rs);
    return hipGetLastError();
}

template <typename T>
hipError_t plane_c2r_t(const Plan& p, const void* X, void* y, hipStream_t st, bool padded = false)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const int rs = (int)(padded ? p.H : p.h);
    const unsigned grid = (unsigned)((p.n0 + p.ppw - 1) / p.ppw);
    const cx<T>* Xi = static_cast<const cx<T>*>(X);
    T* yo = static_cast<T*>(y);
    if (p.plane_big)
        hipLaunchKernelGGL((k_plane_c2r<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.plane_lds, st, Xi,
                           yo, dsched(p, 2), dsched(p, 1), table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw, p.plane_Hs,
                           div_magic((uint32_t)(p.ppw * p.H)), div_magic((uint32_t)p.H), rs);
    else
        hipLaunchKernelGGL((k_plane_c2r<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.plane_lds, st,
                           Xi, yo, dsched(p, 2), dsched(p, 1), table<T>(p, p.off_ax2h), table<T>(p, p.off_post),
                           table<T>(p, p.off_ax1), p.n0, p.ppw, p.plane_Hs,
                           div_magic((uint32_t)(p.ppw * p.H)), div_magic((uint32_t)p.H), rs);
    return hipGetLastError();
}

template <typename T>
hipError_t rows_r2c_t(const Plan& p, const void* x, void* X, int64_t nrows, int rev, hipStream_t st,
                      bool padded = false)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const unsigned grid = (unsigned)((nrows + p.rpw - 1) / p.rpw);
    const T* xi = static_cast<const T*>(x);
    cx<T>* Xo = static_cast<cx<T>*>(X);
    if (p.n2 & 1) {
        const uint32_t mgH = div_magic((uint32_t)p.H);
        const int rs = (int)(padded ? 2 * p.H : p.n2);
        if (p.rows_big)
            hipLaunchKernelGGL((k_rows_r2c_odd<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds, st, xi, Xo,
                               dsched(p, 2), table<T>(p, p.off_ax2h), nrows, p.rpw, p.Hs, mgH, rev, rs);
        else
            hipLaunchKernelGGL((k_rows_r2c_odd<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds, st, xi,
                               Xo, dsched(p, 2), table<T>(p, p.off_ax2h), nrows, p.rpw, p.Hs, mgH, rev, rs);
        return hipGetLastError();
    }
    if (p.rows_big)
        hipLaunchKernelGGL((k_rows_r2c<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds, st, xi, Xo,
                           dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw, p.Hs, rev,
                           (int)(padded ? p.H : p.h));
    else
        hipLaunchKernelGGL((k_rows_r2c<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds, st, xi,
                           Xo, dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw, p.Hs, rev,
                           (int)(padded ? p.H : p.h));
    return hipGetLastError();
}

template <typename T>
hipError_t rows_c2r_t(const Plan& p, const void* X, void* y, int64_t nrows, int rev, hipStream_t st,
                      bool padded = false)
{
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    const unsigned grid = (unsigned)((nrows + p.rpw_inv - 1) / p.rpw_inv);
    const cx<T>* Xi = static_cast<const cx<T>*>(X);
    T* yo = static_cast<T*>(y);
    if (p.n2 & 1) {
        const uint32_t mgH = div_magic((uint32_t)p.H);
        const int rs = (int)(padded ? 2 * p.H : p.n2);
        if (p.rows_big)
            hipLaunchKernelGGL((k_rows_c2r_odd<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds_inv, st, Xi, yo,
                               dsched(p, 2), table<T>(p, p.off_ax2h), nrows, p.rpw_inv, p.Hs, mgH, rev, rs);
        else
            hipLaunchKernelGGL((k_rows_c2r_odd<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds_inv, st, Xi,
                               yo, dsched(p, 2), table<T>(p, p.off_ax2h), nrows, p.rpw_inv, p.Hs, mgH, rev, rs);
        return hipGetLastError();
    }
    if (p.rows_big)
        hipLaunchKernelGGL((k_rows_c2r<T, kNtBig, EB>), dim3(grid), dim3(kNtBig), p.rows_lds_inv, st, Xi, yo,
                           dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw_inv, p.Hs, rev,
                           (int)(padded ? p.H : p.h));
    else
        hipLaunchKernelGGL((k_rows_c2r<T, kNtSmall, ES>), dim3(grid), dim3(kNtSmall), p.rows_lds_inv, st, Xi,
                           yo, dsched(p, 2), table<T>(p, p.off_ax2h), table<T>(p, p.off_post), nrows, p.rpw_inv, p.Hs, rev,
                           (int)(padded ? p.H : p.h));
    return hipGetLastError();
}

template <typename T, bool INV>
hipError_t cols_t(const Plan& p, const ColPass& cp, int axis, int64_t tw_off, const void* in, void* out,
                  int rev, hipStream_t st)
{
    const AxisSched* ax = dsched(p, axis);
    constexpr int ES = Tier<T>::kEptSmall, EB = Tier<T>::kEptBig;
    // XCD groups: the tiles of one block (plane) for a batched pass, single
    // tiles for the one-block (n0) pass
    const int64_t ntiles = cp.nbatch * cp.tiles_per_batch;
    const int gsize = cp.nbatch > 1 ? (int)cp.tiles_per_batch : std::max(1, p.n0_group);
    const int64_t ngroups = (ntiles + gsize - 1) / gsize;
    const unsigned grid = (unsigned)group_grid(ngroups, gsize);
    const cx<T>* ci = static_cast<const cx<T>*>(in);
    cx<T>* co = static_cast<cx<T>*>(out);
    if (cp.big)
        hipLaunchKernelGGL((k_cols<T, kNtBig, EB, INV>), dim3(grid), dim3(kNtBig), cp.lds, st, ci, co, ax,
                           table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W,
                           div_magic((uint32_t)cp.W), cp.tiles_per_batch, ntiles, ngroups, gsize, rev);
    else if (cp.wide && cp.pipe) {
        // persistent: one workgroup per CU, at most one per tile group slot
        const int64_t pgrid = pipe_grid(grid, p.cus);
        const AxisSched& hax = axis == 0 ? p.ax0 : p.ax1;
        const int r0 = hax.radix[0];
        const size_t lds = cp.lds + (size_t)later_twiddles(hax) * sizeof(cx<T>);
        if (lds > (size_t)kLdsMax) return hipErrorInvalidConfiguration;
        if (r0 == 16)
            hipLaunchKernelGGL((k_cols_pipe<T, PipeTier<T>::kNt, PipeTier<T>::kEpt, INV, 16>), dim3(pgrid), dim3(PipeTier<T>::kNt), lds, st, ci, co,
                               ax, table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W, div_magic((uint32_t)cp.W),
                               cp.tiles_per_batch, ntiles, ngroups, gsize, rev, (int64_t)grid);
        else if (r0 == 8)
            hipLaunchKernelGGL((k_cols_pipe<T, PipeTier<T>::kNt, PipeTier<T>::kEpt, INV, 8>), dim3(pgrid), dim3(PipeTier<T>::kNt), lds, st, ci, co,
                               ax, table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W, div_magic((uint32_t)cp.W),
                               cp.tiles_per_batch, ntiles, ngroups, gsize, rev, (int64_t)grid);
        else
            return hipErrorInvalidConfiguration;  // the plan marks first stages of radix 16 or 8 only
    } else if (cp.wide)
        hipLaunchKernelGGL((k_cols<T, kNtWide, ES, INV>), dim3(grid), dim3(kNtWide), cp.lds, st, ci, co, ax,
                           table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W,
                           div_magic((uint32_t)cp.W), cp.tiles_per_batch, ntiles, ngroups, gsize, rev);
    else if (cp.fine) {
        if constexpr (sizeof(T) == 4)
            hipLaunchKernelGGL((k_cols<T, kNtFine, kEptFine, INV>), dim3(grid), dim3(kNtFine), cp.lds, st, ci, co,
                               ax, table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W,
                               div_magic((uint32_t)cp.W), cp.tiles_per_batch, ntiles, ngroups, gsize, rev);
        else
            return hipErrorInvalidConfiguration;  // the plan marks FP32 passes only
    } else
        hipLaunchKernelGGL((k_cols<T, kNtSmall, ES, INV>), dim3(grid), dim3(kNtSmall), cp.lds, st, ci, co,
                           ax, table<T>(p, tw_off), cp.S, cp.ncols, cp.bstride, cp.W,
                           div_magic((uint32_t)cp.W), cp.tiles_per_batch, ntiles, ngroups, gsize, rev);
    return hipGetLastError();
}

// in: [na][nb][H] -> out: [nb][na][H]
template <typename T>
hipError_t swap01_t(const Plan& p, const void* in, void* out, int64_t na, int64_t nb, hipStream_t st)
{
    const int H = (int)p.H;
    const int R = std::max(1, 8192 / H);
    const int tiles_a = (int)((na + R - 1) / R);
    const unsigned grid = (unsigned)(nb * tiles_a);
    hipLaunchKernelGGL((k_swap01<T, kNtSmall>), dim3(grid), dim3(kNtSmall), 0, st, static_cast<const cx<T>*>(in),
                       static_cast<cx<T>*>(out), (int)na, (int)nb, H, R, div_magic((uint32_t)H), tiles_a);
    return hipGetLastError();
}

template <typename T> CoopArgs coop_args(const Plan& p)
{
    CoopArgs a;
    a.n0 = p.n0;
    a.n1 = (int)p.n1;
    a.h = (int)p.h;
    a.H = (int)p.H;
    a.rpw = p.coop_rpw;
    a.Hs = p.Hs;
    a.RT = p.coop_rt;
    a.W = p.coop_w;
    a.CT = p.coop_ct;
    a.mg_w = div_magic((uint32_t)p.coop_w);
    a.nslots = p.coop_nslots;
    a.spin_limit = 1 << 22;
    a.axh = dsched(p, 2);
    a.ax1 = dsched(p, 1);
    a.lag = p.coop_lag;
    a.off_tw2 = p.off_ax2h;
    a.off_post = p.off_post;
    a.off_tw1 = p.off_ax1;
    a.ctr = p.d_ctr;
    return a;
}

template <typename T>
hipError_t coop_t(const Plan& p, const void* in, void* out, bool inverse, hipStream_t st)
{
    constexpr int ES = Tier<T>::kEptSmall;
    hipLaunchKernelGGL(k_zero_ints<0>, dim3(64), dim3(256), 0, st, p.d_ctr, p.coop_ctr_count);
    const CoopArgs a = coop_args<T>(p);
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(p.d_tw);
    if (inverse)
        hipLaunchKernelGGL((k_plane_coop<T, kNtSmall, ES, true>), dim3(p.coop_grid), dim3(kNtSmall), p.coop_lds,
                           st, in, out, tw, a);
    else
        hipLaunchKernelGGL((k_plane_coop<T, kNtSmall, ES, false>), dim3(p.coop_grid), dim3(kNtSmall), p.coop_lds,
                           st, in, out, tw, a);
    return hipGetLastError();
}

template <typename T> hipError_t coop_occupancy(const Plan& p, int* per_cu)
{
    constexpr int ES = Tier<T>::kEptSmall;
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &a, reinterpret_cast<const void*>(k_plane_coop<T, kNtSmall, ES, false>), kNtSmall, p.coop_lds);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &b, reinterpret_cast<const void*>(k_plane_coop<T, kNtSmall, ES, true>), kNtSmall, p.coop_lds);
    if (e != hipSuccess) return e;
    *per_cu = a < b ? a : b;
    return hipSuccess;
}


}  // inline namespace FFT3D_KNS
}  // namespace fft3d
