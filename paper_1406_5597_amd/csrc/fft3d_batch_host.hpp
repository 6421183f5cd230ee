// fft3d_batch_host.hpp -- host side of the batched launch (fft3d_batch_host.cpp).
#pragma once

#include <mutex>
#include <vector>

#include "fft3d_batch.hpp"
#include "fft3d_internal.hpp"

namespace fft3d {

// One validated item of a batch (pointers as in fft3d_batch_item).
struct BatchSpec {
    const Plan* plan;
    int dir;
    const void* in;
    void* mid;
    void* out;
    void* work;
};

struct BatchOptions {
    // the device's hardware XCC ids (one queue per XCD when pinned)
    std::vector<int> xcc_ids;
    // 0 (the rule) and 3: level mode (one launch per pass level, tile kind
    // and dtype; no queues); the one persistent launch with 1: items pinned
    // to XCDs (a queue per XCD), 2: one queue, 4: pinned when that balances
    // the XCDs, else one queue.  Measured on the 64-field mix: 1.58 ms in
    // level mode (a graph), 2.5-2.6 ms persistent.
    int mode = 0;
    // slots between an item's consecutive passes in the ticket order; 0 means
    // the number of items (pass-major order)
    int lag = 0;
    // small fields get fewer, larger tiles (several planes per plane tile,
    // column tiles widened to the tier); false: the plans' own tile shapes
    bool widen = true;
    // workgroups per CU of the launch; 0: as many as fit
    int wg_per_cu = 0;
    // polls of a dependency wait before it gives up (0: give up at once)
    int spin_limit = kBatchSpinLimit;
};

// One launch of the level mode: tasks task_begin .. task_begin+ntasks-1 (one
// kind and dtype, passes of different items), the first tile of each at
// firsts[firsts_begin ..]; one workgroup per tile.
struct BatchLaunch {
    int kind = 0;
    int f64 = 0;
    int big = 0;  // big-tier fused plane tiles
    int task_begin = 0;
    int ntasks = 0;
    int firsts_begin = 0;
    int64_t tiles = 0;
    size_t lds = 0;
    // earlier launches holding the passes this launch's tasks read (a graph
    // runs the launch after these only; a stream after every earlier one)
    std::vector<int> deps;
};

struct BatchTable {
    // level mode: `launches` in stream order, every pass in a later launch
    // than the pass it reads (firsts: per launch, the first tile of each of
    // its tasks); the queue fields below are unused
    bool levels = false;
    std::vector<BatchLaunch> launches;
    std::vector<BatchTask> tasks;  // queue by queue
    // per queue: the first ticket (within the queue) of each of its tasks,
    // then its total; queue q's entries start at task_begin[q] + q
    std::vector<int32_t> firsts;
    std::vector<int> task_begin;         // nqueues + 1
    std::vector<int64_t> queue_tickets;  // nqueues
    int nqueues = 1;
    bool pinned = false;
    int qmap[kBatchMaxQueues] = {};
    int64_t tickets = 0;
    size_t lds = 0;  // dynamic LDS of the launch (largest tile)
    int wg_per_cu = 0;  // workgroups per CU (0: as many as fit)
    int spin_limit = kBatchSpinLimit;  // polls of a dependency wait
};

// LDS of one batch tile: half a CU's LDS less the kernel's own (scheduling
// words and the cached ticket table), so that two workgroups fit on a CU.
constexpr int64_t kBatchLdsCap = kLdsHalf - 2560;
constexpr int kRingSlots = 16;    // task images fft3d_batch_submit may have in flight per device
constexpr int kRingTasks = 4096;  // tasks per ring slot

// Task list of n items; nullptr or why it cannot be built.
const char* build_batch_table(const BatchSpec* items, int n, const BatchOptions& o, BatchTable& tab);
// Device image of a task list: BatchHeader, the per-queue ticket tables, then
// the tasks (256-byte aligned); level mode: the launches' first-tile tables,
// then the tasks (256-byte aligned).
size_t batch_image_bytes(int ntasks, int nqueues);
size_t batch_image_bytes(const BatchTable& tab);
size_t batch_tasks_offset(int ntasks, int nqueues);
size_t level_tasks_offset(const BatchTable& tab);  // level mode: offset of the tasks
void write_batch_image(const BatchTable& tab, void* dst);
// Workgroups of the launch: every CU times the workgroups that fit on one,
// at most one per ticket.
hipError_t batch_grid(const BatchTable& tab, int device, unsigned* grid);
hipError_t enqueue_batch_image(const BatchTable& tab, unsigned grid, const void* dev_image, int* dev_ctr,
                               hipStream_t s);

// The per-device ring of task images behind fft3d_batch_submit: set up once
// per device (fft3d_init), then each submit stages its image in pinned
// memory, copies it on the stream and launches, with no allocation and no
// wait: a submit that finds no slot free or finished returns at once.
hipError_t ring_init(int device);
bool ring_ready(int device);
// Distinct hardware XCC ids of the device (found by ring_init), or empty.
std::vector<int> device_xcc_ids(int device);
// Slot states of the submit ring as the host sees them.
enum RingSlotState { kSlotFree = 0, kSlotDone = 1, kSlotBusy = 2 };
// Picks up to `needed` slots in ring order from `next`, skipping the ones in
// flight; returns how many it found (their indexes in picked[]).
int ring_pick(const int* state, int nslots, int next, int needed, int* picked);
// Stage and launch ntabs task lists (all or nothing): hipErrorNotReady with
// *why set when fewer than ntabs slots are free or finished, nothing
// enqueued.  *first_seq: sequence number of the first launch (the others
// follow), for ring_status.
hipError_t ring_submit(int device, const BatchTable* tabs, int ntabs, hipStream_t s, int64_t* first_seq,
                       const char** why);
// Error bits (ORed) of the launches first_seq .. first_seq+count-1, once
// finished; FFT3D_ERR_BUSY while one still runs; a negative code if unknown.
int ring_status(int device, int64_t first_seq, int count, const char** why);

}  // namespace fft3d
