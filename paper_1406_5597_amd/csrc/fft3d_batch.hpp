// fft3d_batch.hpp -- the work list of the persistent batched launch.
//
// A batch is a list of tasks.  A task is one pass of one item (the plane
// step, a rows pass, a column pass) cut into tiles; the tiles of a task are
// independent, and a task may start only once every tile of the task it
// depends on (the previous pass of the same item) is done.  Tasks are
// numbered so that a task always comes after the task it depends on, and
// workgroups take tiles ("tickets") in that order from one global counter.
// This plain struct is shared by the host builder and the kernel.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "fft3d_sched.hpp"

namespace fft3d {

enum BatchKind : int32_t {
    kBkPlaneR2C = 0,  // fused plane step, forward: real planes -> spectrum planes
    kBkPlaneC2R = 1,  // fused plane step, inverse
    kBkRowsR2C = 2,   // rows pass of the split plane step, forward
    kBkRowsC2R = 3,   // rows pass, inverse
    kBkColsFwd = 4,   // column pass (n1 or n0 axis), forward
    kBkColsInv = 5,   // column pass, inverse
};

struct BatchTask {
    int32_t kind;    // BatchKind
    int32_t f64;     // 1: FP64 data and tables, 0: FP32
    int32_t big;     // 1: a big-tier fused plane tile (level mode only), 0: small tier
    int32_t ntiles;  // tiles of this task
    int32_t dep;     // task this one waits for, or -1
    int32_t dep_tiles;
    int32_t lds;  // dynamic LDS bytes the tile needs (host bookkeeping)
    int32_t pad_;
    // kind-specific:
    //  plane: a0 planes per tile, a1 padded LDS row stride, i0 planes,
    //         m0 div_magic(a0*H), m1 div_magic(H); s0 n2/2 schedule, s1 n1
    //         schedule; t0 n2/2 twiddles, t1 split roots, t2 n1 twiddles
    //  rows:  a0 rows per tile, a1 padded LDS row stride, i0 rows;
    //         s0 n2/2 schedule; t0 n2/2 twiddles, t1 split roots
    //  cols:  a0 tile width W, a1 tiles per block, i0 row stride S,
    //         i1 columns per block, i2 block stride, m0 div_magic(W);
    //         s0 axis schedule; t0 axis twiddles
    int32_t a0, a1;
    uint32_t m0, m1;
    int64_t i0, i1, i2;
    const void* in;
    void* out;
    const AxisSched* s0;
    const AxisSched* s1;
    const void* t0;
    const void* t1;
    const void* t2;
};

// Queues.  A batch has one ticket queue per XCD ("pinned": every task of an
// item is in the queue of one XCD and only that XCD's workgroups take its
// tiles, so a pass's output is read back through the same L2 it was written
// to) or a single queue that every workgroup serves ("spread").
constexpr int kBatchMaxQueues = 16;
// A queue's ticket table is copied to LDS when it has at most this many
// entries (tasks + 1).
constexpr int kBatchFirstsCache = 512;

// Head of the device image of a batch, followed by the per-queue ticket
// tables (queue q: the first ticket of each of its tasks, then its total) and
// the tasks (queue by queue, task_begin[q] .. task_begin[q+1]-1).
struct BatchHeader {
    int32_t nqueues;
    int32_t pinned;                       // 1: per-XCD queues; 0: one queue
    int32_t ntasks;
    int32_t pad0;
    int32_t qmap[kBatchMaxQueues];        // hardware XCC id -> queue, or -1
    int32_t task_begin[kBatchMaxQueues + 1];
    int32_t pad1[3];
};

// Counter block of one batch launch (ints): the ticket counter of queue q at
// kBatchCtrQueueStride*q (a 64-byte line each), then error bits, workgroups
// finished and the status of the last launch, then the done count of every
// task.  The last workgroup to finish clears everything but the status, so
// the block is ready for the next launch (also when that is a graph replay).
constexpr int kBatchCtrQueueStride = 16;
constexpr int kBatchCtrErr = kBatchMaxQueues * kBatchCtrQueueStride;
constexpr int kBatchCtrExit = kBatchCtrErr + 1;
constexpr int kBatchCtrStatus = kBatchCtrErr + 2;
constexpr int kBatchCtrHeader = kBatchCtrErr + 16;
// error bits
constexpr int kBatchErrWait = 1;   // a dependency wait hit its spin limit
constexpr int kBatchErrQueue = 2;  // a queue's XCD had no workgroup: its items did not run
constexpr int kBatchErrLoop = 4;   // a workgroup's ticket loop ran more iterations than its queue has
                                   // tickets (its ticket state stopped advancing) and was ended

// Polls of a dependency wait before it gives up (error bit kBatchErrWait).
constexpr int kBatchSpinLimit = 1 << 20;

// The allocation-free batched launch (fft3d_batch_submit_static) keeps one
// task image per device in a static device array of kStaticScratchBytes (at
// most kStaticTasks passes).
constexpr int kStaticTasks = 4096;
constexpr size_t kStaticScratchBytes = (size_t)1 << 20;

}  // namespace fft3d

#include <hip/hip_runtime_api.h>
#include <stddef.h>

namespace fft3d {

// Device side (fft3d_batch.hip).
hipError_t init_batch();
const void* batch_kernel();
hipError_t batch_occupancy(size_t lds, int* per_cu);
// image: BatchHeader, ticket tables, tasks (see write_batch_image)
hipError_t launch_batch(unsigned grid, size_t lds, const void* image, int* ctr, int spin_limit, hipStream_t s);
// The level mode (fft3d_level.hip): the kernel of one tile kind and dtype,
// and one launch of it over `ntasks` tasks (device pointers: the tasks, and
// the first tile of each) with one workgroup per tile (grid = total tiles).
hipError_t init_level();
const void* level_kernel(int kind, int f64, int big);
hipError_t launch_level(int kind, int f64, int big, unsigned grid, size_t lds, const BatchTask* tasks, const int* firsts,
                        int ntasks, hipStream_t s);
// Hardware XCC id of every workgroup of a `blocks`-block probe launch
// (synchronous; `ids` gets `blocks` values).
hipError_t probe_xcc_ids(int blocks, int* ids);

// The static scratch array of fft3d_batch_submit_static.  Setup resolves its
// address on the current device (once per device; thread-safe); the address
// is then found by device ordinal (nullptr before setup).
hipError_t static_scratch_setup(int device);
void* static_scratch(int device);
// Copy a task image (host, `bytes` <= kStaticScratchBytes) into the
// device's scratch on stream s; *dev receives its device address.
hipError_t stage_static_image(int device, const void* host_image, size_t bytes, const void** dev, hipStream_t s);

}  // namespace fft3d
