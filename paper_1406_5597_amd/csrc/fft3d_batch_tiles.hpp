// fft3d_batch_tiles.hpp -- one tile of a batch task: the tile functions of
// the single-item kernels, called with the task's own tiling, schedules and
// tables, so that every result is bit-identical to the item run alone.  Used
// by the persistent batched kernel (any kind, by a switch) and by the
// per-kind launches of the level mode.
#pragma once

#include "fft3d_batch.hpp"
#include "fft3d_kernels.hpp"

namespace fft3d {

// A task's addresses re-derived from a pointer the kernel received as an
// argument.  Pointers read from memory are generic to the compiler, and a
// tile would access global memory through them with flat instructions
// (64-bit addresses held in vector registers: FP64 column tiles needed 154
// VGPRs instead of 108, one workgroup a CU instead of two); derived from a
// kernel argument they are global-memory pointers.  The values are unchanged.
template <typename P> __device__ __forceinline__ P* rebase(const char* base, P* p)
{
    return reinterpret_cast<P*>(const_cast<char*>(base) + ((intptr_t)p - (intptr_t)base));
}
__device__ __forceinline__ BatchTask rebased(const BatchTask& t, const void* arg)
{
    const char* base = static_cast<const char*>(arg);
    BatchTask k = t;
    k.in = rebase(base, t.in);
    k.out = rebase(base, t.out);
    k.s0 = rebase(base, t.s0);
    k.s1 = rebase(base, t.s1);
    k.t0 = rebase(base, t.t0);
    k.t1 = rebase(base, t.t1);
    k.t2 = rebase(base, t.t2);
    return k;
}

template <typename T, int EPT, int K>
__device__ __forceinline__ void batch_tile_kind(const BatchTask& k, int tile, unsigned char* smem)
{
    constexpr int NT = kNtSmall;
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem);
    const cx<T>* t0 = static_cast<const cx<T>*>(k.t0);
    const cx<T>* t1 = static_cast<const cx<T>*>(k.t1);
    if constexpr (K == kBkPlaneR2C || K == kBkPlaneC2R) {
        const AxisSched& axh = *k.s0;
        const AxisSched& ax1 = *k.s1;
        const int h = axh.n, H = h + 1, n1 = ax1.n;
        const int64_t p0 = (int64_t)tile * k.a0;
        const int64_t left = k.i0 - p0;
        const int np = left < k.a0 ? (int)left : k.a0;
        const uint32_t mg = np == k.a0 ? k.m0 : div_magic_dev(np * H);
        const cx<T>* t2 = static_cast<const cx<T>*>(k.t2);
        if constexpr (K == kBkPlaneR2C)
            plane_r2c_tile<T, NT, EPT>(static_cast<const cx<T>*>(k.in) + p0 * n1 * h,
                                       static_cast<cx<T>*>(k.out) + p0 * n1 * H, np, axh, ax1, t0, t1, t2, k.a1, mg,
                                       k.m1, buf);
        else
            plane_c2r_tile<T, NT, EPT>(static_cast<const cx<T>*>(k.in) + p0 * n1 * H,
                                       static_cast<cx<T>*>(k.out) + p0 * n1 * h, np, axh, ax1, t0, t1, t2, k.a1, mg,
                                       k.m1, buf);
    } else if constexpr (K == kBkRowsR2C || K == kBkRowsC2R) {
        const AxisSched& axh = *k.s0;
        const int h = axh.n, H = h + 1;
        const int64_t r0 = (int64_t)tile * k.a0;
        const int64_t left = k.i0 - r0;
        const int rows = left < k.a0 ? (int)left : k.a0;
        if constexpr (K == kBkRowsR2C)
            rows_r2c_tile<T, NT, EPT>(static_cast<const cx<T>*>(k.in) + r0 * h, static_cast<cx<T>*>(k.out) + r0 * H,
                                      rows, k.a1, axh, t0, t1, buf);
        else
            rows_c2r_tile<T, NT, EPT>(static_cast<const cx<T>*>(k.in) + r0 * H, static_cast<cx<T>*>(k.out) + r0 * h,
                                      rows, k.a1, axh, t0, t1, buf);
    } else {  // column passes
        const int W = k.a0;
        const int b = tile / k.a1;
        const int64_t c0 = (int64_t)(tile - b * k.a1) * W;
        const int64_t rem = k.i1 - c0;
        const int width = rem < (int64_t)W ? (int)rem : W;
        const int64_t off = (int64_t)b * k.i2 + c0;
        const cx<T>* src = static_cast<const cx<T>*>(k.in) + off;
        cx<T>* dst = static_cast<cx<T>*>(k.out) + off;
        col_tile<T, NT, EPT, K == kBkColsInv>(src, dst, k.i0, width, W, k.m0, *k.s0, t0, buf);
    }
}

}  // namespace fft3d
