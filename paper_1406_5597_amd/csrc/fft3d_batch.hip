// fft3d_batch.hip -- one persistent launch for a whole batch of transforms
// (batch modes 1, 2 and 4; the rule is the level mode of fft3d_level.hip).
//
// Every item of a batch (forward, inverse or both, any supported shape, FP32
// or FP64) becomes a chain of tasks, one per pass of the single-item path:
// the plane step (fused, or rows + n1 columns), the strided n0 column pass,
// and for the inverse the same in reverse order.  The tiles of all tasks are
// numbered in an order where a task's tiles follow those of the task it
// depends on; workgroups take the numbers ("tickets") from one global
// counter, so the kernel runs many small fields at once without a launch per
// pass and with no idle gap between passes.
//
// Dependencies: before its first tile of a task, a workgroup waits until
// every tile of the task's predecessor has counted itself done, then issues
// an agent-scope acquire; a finished tile drains its stores, meets the
// workgroup barrier and counts itself done with an agent-scope release.
// Every wait is for tiles with smaller tickets than the waiter's, and a
// ticket is only ever held by a running workgroup, so the smallest
// unfinished ticket always makes progress: the kernel cannot deadlock,
// whatever the grid.  Waits are bounded anyway (spin limit); a wait that
// runs out records an error bit and the tile is skipped, so every workgroup
// still reaches the end.  The same tile functions as the single-item kernels
// run the work, with the same schedules, so each result is bit-identical to
// the item run alone.  All tiles are small-tier (the host picks such
// tilings), which keeps this one kernel -- every tile kind of both dtypes --
// quick to compile.
#include <mutex>

#include "fft3d_batch.hpp"
#include "fft3d_batch_tiles.hpp"
#include "fft3d_kernels.hpp"

namespace fft3d {

// One tile of any kind (the persistent kernel's dispatch).
template <typename T, int EPT>
__device__ __forceinline__ void batch_tile(const BatchTask& k, int tile, unsigned char* smem)
{
    switch (k.kind) {
    case kBkPlaneR2C: batch_tile_kind<T, EPT, kBkPlaneR2C>(k, tile, smem); break;
    case kBkPlaneC2R: batch_tile_kind<T, EPT, kBkPlaneC2R>(k, tile, smem); break;
    case kBkRowsR2C: batch_tile_kind<T, EPT, kBkRowsR2C>(k, tile, smem); break;
    case kBkRowsC2R: batch_tile_kind<T, EPT, kBkRowsC2R>(k, tile, smem); break;
    case kBkColsFwd: batch_tile_kind<T, EPT, kBkColsFwd>(k, tile, smem); break;
    default: batch_tile_kind<T, EPT, kBkColsInv>(k, tile, smem); break;
    }
}

// Wait until *p >= target; false after `limit` polls, or at once when an
// earlier wait of the launch has already failed (err != 0), so a failed
// launch drains quickly.
__device__ __forceinline__ bool batch_wait(int* p, int target, int* err, int limit)
{
    for (int it = 0; it < limit; ++it) {
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return false;
}

__device__ __forceinline__ int image_offset_tasks(int ntasks, int nqueues)
{
    const int f = (int)sizeof(BatchHeader) + (ntasks + nqueues) * (int)sizeof(int32_t);
    return (f + 255) & ~255;
}

// Every tile of a batch is small-tier (at most 64 KB of data, 80 KB of LDS).
template <int Unused = 0>
__global__ __launch_bounds__(kNtSmall) void k_batch(const void* __restrict__ image, int* ctr, int spin_limit)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_task[3];
    const BatchHeader& hd = *static_cast<const BatchHeader*>(image);
    const int nqueues = hd.nqueues, ntasks = hd.ntasks, pinned = hd.pinned;
    const BatchTask* tasks =
        reinterpret_cast<const BatchTask*>(static_cast<const char*>(image) + image_offset_tasks(ntasks, nqueues));
    // this workgroup's queue: the one of the XCD it runs on (hardware
    // register XCC_ID), or the only one
    const int xcc = __builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kBatchMaxQueues - 1);
    const int q = hd.qmap[xcc];
    int* done = ctr + kBatchCtrHeader;
    int tb = 0, nq = 0;
    const int* firsts = nullptr;
    int* ticket = nullptr;
    if (q >= 0) {
        tb = hd.task_begin[q];
        nq = hd.task_begin[q + 1] - tb;
        firsts = reinterpret_cast<const int*>(&hd + 1) + tb + q;  // nq + 1 entries
        ticket = ctr + kBatchCtrQueueStride * q;
    }
    // the queue's ticket table in LDS when it fits (thread 0 searches it for
    // every ticket)
    __shared__ int s_firsts[kBatchFirstsCache];
    const bool cached = q >= 0 && nq + 1 <= kBatchFirstsCache;
    if (cached)
        for (int i = (int)threadIdx.x; i <= nq; i += kNtSmall) s_firsts[i] = firsts[i];
    __syncthreads();
    auto first_of = [&](int i) { return cached ? s_firsts[i] : firsts[i]; };
    const int total = q >= 0 ? first_of(nq) : 0;
    // thread 0's scheduling state
    int next = 0, cur = 0, checked = -1, failed = -1, iters = 0;
    if (threadIdx.x == 0 && q >= 0) next = atomicAdd(ticket, 1);
    for (;;) {
        if (threadIdx.x == 0) {
            const int t = next;
            int k = -1, tile = 0, skip = 0;
            // Every iteration but the last runs a distinct ticket of the
            // queue, so a workgroup iterates at most total + 1 times.  The
            // bound does not depend on memory: were the ticket state ever to
            // stop advancing, the loop would still end (with an error bit)
            // instead of running one ticket forever.
            if (++iters > total + 1) {
                atomicOr(&ctr[kBatchCtrErr], kBatchErrLoop);
            } else if (t < total) {
                next = atomicAdd(ticket, 1);  // the next ticket, while this one runs
                // task of ticket t: firsts[cur] <= t (tickets only grow)
                if (first_of(cur + 1) <= t) {
                    int lo = cur + 1, step = 1;
                    while (lo + step < nq && first_of(lo + step) <= t) {
                        lo += step;
                        step *= 2;
                    }
                    int hi = lo + step < nq ? lo + step : nq;
                    while (hi - lo > 1) {
                        const int mid = (lo + hi) >> 1;
                        if (first_of(mid) <= t) lo = mid;
                        else hi = mid;
                    }
                    cur = lo;
                }
                k = tb + cur;
                tile = t - first_of(cur);
                if (k != checked) {
                    checked = k;
                    const int dep = tasks[k].dep;
                    if (dep >= 0) {
                        if (!batch_wait(&done[dep], tasks[k].dep_tiles, &ctr[kBatchCtrErr], spin_limit)) {
                            atomicOr(&ctr[kBatchCtrErr], kBatchErrWait);
                            failed = k;
                        }
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                }
                skip = failed == k;
            }
            s_task[0] = k;
            s_task[1] = tile;
            s_task[2] = skip;
        }
        __syncthreads();
        const int k = __builtin_amdgcn_readfirstlane(s_task[0]);
        const int tile = __builtin_amdgcn_readfirstlane(s_task[1]);
        const int skip = __builtin_amdgcn_readfirstlane(s_task[2]);
        if (k < 0) break;
        if (!skip) {
            const BatchTask tk = rebased(tasks[k], image);
            if (tk.f64) batch_tile<double, Tier<double>::kEptSmall>(tk, tile, smem_raw);
            else batch_tile<float, Tier<float>::kEptSmall>(tk, tile, smem_raw);
        }
        __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached L2
        __syncthreads();                // ... and every wave's
        if (threadIdx.x == 0) {
            if (pinned) {
                // the readers of this task's output run on this XCD and read
                // it through this L2: the drained stores are visible to them
                __hip_atomic_fetch_add(&done[k], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                // readers may run on any XCD: release (writes back this L2)
                __hip_atomic_fetch_add(&done[k], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (threadIdx.x == 0) {
        const int prev = __hip_atomic_fetch_add(&ctr[kBatchCtrExit], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == (int)gridDim.x - 1) {
            // every other workgroup has left.  A queue whose tickets were not
            // all taken had no workgroup on its XCD: its items did not run.
            int err = __hip_atomic_load(&ctr[kBatchCtrErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const int* tables = reinterpret_cast<const int*>(&hd + 1);
            for (int i = 0; i < nqueues; ++i) {
                const int b = hd.task_begin[i], n = hd.task_begin[i + 1] - b;
                const int taken = __hip_atomic_load(&ctr[kBatchCtrQueueStride * i], __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
                if (taken < tables[b + i + n]) err |= kBatchErrQueue;
            }
            // clear the block for the next launch
            __hip_atomic_store(&ctr[kBatchCtrStatus], err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr[kBatchCtrErr], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int i = 0; i < kBatchMaxQueues; ++i)
                __hip_atomic_store(&ctr[kBatchCtrQueueStride * i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int i = 0; i < ntasks; ++i) __hip_atomic_store(&done[i], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctr[kBatchCtrExit], 0, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int Unused = 0> __global__ void k_xcc_probe(int* ids)
{
    if (threadIdx.x == 0)
        ids[blockIdx.x] = (int)(__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kBatchMaxQueues - 1));
}

const void* batch_kernel() { return reinterpret_cast<const void*>(&k_batch<0>); }

hipError_t init_batch() { return allow_lds(k_batch<0>); }

hipError_t batch_occupancy(size_t lds, int* per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, batch_kernel(), kNtSmall, lds);
}

hipError_t launch_batch(unsigned grid, size_t lds, const void* image, int* ctr, int spin_limit, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch<0>, dim3(grid), dim3(kNtSmall), lds, s, image, ctr, spin_limit);
    return hipGetLastError();
}

// ---- the allocation-free batched launch ----
//
// Callers that cannot allocate (code under graph capture, serving loops that
// forbid hipMalloc) run a batch through this array: one task image per
// device (the level mode's launches read their tasks from it), held until the
// process ends.  Every launch on a
// device shares the device's copy, which keeps the last launch's contents;
// launches that overlap in time on one device (unordered streams) race.  Host
// code never passes the array's name to a kernel or a copy (in host code it
// is a stand-in, not a device address): it uses the address that
// hipGetSymbolAddress returned on that device.

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kStaticMaxDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kStaticMaxDevices] = {};
}  // namespace

hipError_t static_scratch_setup(int device)
{
    if (device < 0 || device >= kStaticMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_static_mu);
    if (g_static_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the device must be current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_static_ptr[device] = p;
    return hipSuccess;
}

void* static_scratch(int device)
{
    if (device < 0 || device >= kStaticMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_static_mu);
    return g_static_ptr[device];
}

hipError_t stage_static_image(int device, const void* host_image, size_t bytes, const void** dev, hipStream_t s)
{
    unsigned char* base = static_cast<unsigned char*>(static_scratch(device));
    if (!base) return hipErrorNotInitialized;
    if (bytes > kStaticScratchBytes) return hipErrorInvalidValue;
    *dev = base;
    return hipMemcpyAsync(base, host_image, bytes, hipMemcpyHostToDevice, s);
}

hipError_t probe_xcc_ids(int blocks, int* ids)
{
    int* d = nullptr;
    hipError_t e = hipMalloc(&d, (size_t)blocks * sizeof(int));
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_xcc_probe<0>, dim3(blocks), dim3(64), 0, 0, d);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(ids, d, (size_t)blocks * sizeof(int), hipMemcpyDeviceToHost);
    hipError_t f = hipFree(d);
    return e != hipSuccess ? e : f;
}

}  // namespace fft3d
