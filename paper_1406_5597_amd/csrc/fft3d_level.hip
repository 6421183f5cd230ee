// fft3d_level.hip -- the level mode of the batched launch: one launch per
// pass level, tile kind, tier and dtype.
//
// The host sorts the passes of all items into a sequence of launches such
// that every pass runs in a later launch than the pass it reads from (stream
// order is the only synchronisation: no tickets, counters or waits).  A
// launch runs the tiles of many items' passes of one kind and dtype, one
// workgroup per tile; its kernel holds that one tile kind only, so it needs
// about the registers of the single-item kernel of that kind, not those of
// every kind at once (the persistent kernel's 223 VGPRs allow one 512-thread
// workgroup a CU).  The tile functions are those of the single-item kernels:
// results are bit-identical to the items run alone.
#include "fft3d_batch.hpp"
#include "fft3d_batch_tiles.hpp"
#include "fft3d_kernels.hpp"

namespace fft3d {

// Register bound of a level kernel (waves per SIMD; 1: none): the rows
// kinds take the inverse rows kernel's (FP32: at most 80 VGPRs, three
// workgroups a CU at the batch's rows tiles of up to 48 KB).
template <typename T, int K> constexpr int level_waves()
{
    return (K == kBkRowsR2C || K == kBkRowsC2R) ? Tier<T>::kRowsWavesInv : 1;
}

// Workgroup b runs tile b - firsts[i] of task i, the last task with
// firsts[i] <= b (firsts: the first tile of each of the launch's ntasks
// tasks, ascending; the grid is the launch's total tiles).  BIG: the tiles
// are big-tier fused planes (the plan's own tile for planes of more than
// the small tier's elements; up to the whole LDS).
template <typename T, int K, bool BIG>
__global__ __launch_bounds__(kNtSmall, (level_waves<T, K>())) void k_level(const BatchTask* __restrict__ tasks,
                                                                           const int* __restrict__ firsts,
                                                                           int ntasks)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = (int)blockIdx.x;
    int lo = 0, hi = ntasks;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (firsts[mid] <= b) lo = mid;
        else hi = mid;
    }
    constexpr int EPT = BIG ? Tier<T>::kEptBig : Tier<T>::kEptSmall;
    batch_tile_kind<T, EPT, K>(rebased(tasks[lo], tasks), b - firsts[lo], smem_raw);
}

namespace {

template <typename T> const void* level_kernel_t(int kind, bool big)
{
    if (big) {
        if (kind == kBkPlaneR2C) return reinterpret_cast<const void*>(&k_level<T, kBkPlaneR2C, true>);
        if (kind == kBkPlaneC2R) return reinterpret_cast<const void*>(&k_level<T, kBkPlaneC2R, true>);
        return nullptr;  // big tiles are fused planes only
    }
    switch (kind) {
    case kBkPlaneR2C: return reinterpret_cast<const void*>(&k_level<T, kBkPlaneR2C, false>);
    case kBkPlaneC2R: return reinterpret_cast<const void*>(&k_level<T, kBkPlaneC2R, false>);
    case kBkRowsR2C: return reinterpret_cast<const void*>(&k_level<T, kBkRowsR2C, false>);
    case kBkRowsC2R: return reinterpret_cast<const void*>(&k_level<T, kBkRowsC2R, false>);
    case kBkColsFwd: return reinterpret_cast<const void*>(&k_level<T, kBkColsFwd, false>);
    case kBkColsInv: return reinterpret_cast<const void*>(&k_level<T, kBkColsInv, false>);
    default: return nullptr;
    }
}

}  // namespace

const void* level_kernel(int kind, int f64, int big)
{
    return f64 ? level_kernel_t<double>(kind, big != 0) : level_kernel_t<float>(kind, big != 0);
}

hipError_t init_level()
{
    hipError_t e = hipSuccess;
    for (int f64 = 0; f64 < 2; ++f64)
        for (int big = 0; big < 2; ++big)
            for (int kind = kBkPlaneR2C; kind <= kBkColsInv; ++kind) {
                const void* f = level_kernel(kind, f64, big);
                if (!f) continue;
                const hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, kLdsMax);
                if (r != hipSuccess) e = r;
            }
    return e;
}

hipError_t launch_level(int kind, int f64, int big, unsigned grid, size_t lds, const BatchTask* tasks,
                        const int* firsts, int ntasks, hipStream_t s)
{
    const void* f = level_kernel(kind, f64, big);
    if (!f || grid == 0 || ntasks < 1) return hipErrorInvalidValue;
    void* args[] = {&tasks, &firsts, &ntasks};
    return hipLaunchKernel(f, dim3(grid), dim3(kNtSmall), args, lds, s);
}

}  // namespace fft3d
