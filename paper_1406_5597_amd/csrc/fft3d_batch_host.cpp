// fft3d_batch_host.cpp -- host side of the batched launch: the task list of a
// batch, the per-device ring that fft3d_batch_submit streams task lists
// through, and the launch.
#include "fft3d_batch_host.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>

#include "../../include/fft3d.h"

namespace fft3d {

namespace {

BatchTask base_task(const Plan& p, int kind, const void* in, void* out, int ntiles)
{
    BatchTask t;
    memset(&t, 0, sizeof t);
    t.kind = kind;
    t.f64 = p.dtype == FFT3D_F64;
    t.ntiles = ntiles;
    t.dep = -1;
    t.in = in;
    t.out = out;
    return t;
}

const void* tw_at(const Plan& p, int64_t off)
{
    return static_cast<const char*>(p.d_tw) + off * 2 * p.elem;
}

int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

// Tiling of one item inside a batch: the plan's own where it is small-tier
// (so the passes are the very kernels' tiles of the item run alone), else the
// small-tier alternative with the same radix schedules -- the split plane
// step instead of a big fused plane, narrower column tiles.  Either way the
// arithmetic of every line is the same, so the bits are too.
struct ItemTiling {
    bool fused = false;
    size_t plane_lds = 0;
    int ppw = 1;
    int rpw = 1;
    size_t rows_lds = 0;
    ColPass pass1;
    ColPass pass0;
};

const char* item_tiling(const Plan& p, ItemTiling& t)
{
    if (p.n0 > 1) {
        t.pass0 = p.pass0;
        if (t.pass0.big && !small_colpass(p, 0, t.pass0)) return "n0 too long for a small-tier column tile";
    }
    if (p.fused_plane && !p.plane_big) {
        t.fused = true;
        t.plane_lds = p.plane_lds;
        t.ppw = p.ppw;
        return nullptr;
    }
    bool rows_big = false;
    if (p.fused_plane) {
        if (const char* why = split_tiling(p, t.rpw, rows_big, t.rows_lds, t.pass1)) return why;
    } else {
        // split plans (the cooperative plane step is the split step in one
        // launch; both give the same bits)
        t.rpw = p.rpw;
        rows_big = p.rows_big;
        t.rows_lds = p.rows_lds;
        t.pass1 = p.pass1;
    }
    if (rows_big) return "rows too long for a small-tier tile";
    if (p.n1 > 1 && t.pass1.big && !small_colpass(p, 1, t.pass1)) return "n1 too long for a small-tier column tile";
    return nullptr;
}

void add_cols(std::vector<BatchTask>& chain, const Plan& p, const ColPass& cp, int64_t nbatch, int axis,
              int64_t tw_off, const void* in, void* out, bool inverse)
{
    BatchTask t = base_task(p, inverse ? kBkColsInv : kBkColsFwd, in, out, (int32_t)(nbatch * cp.tiles_per_batch));
    t.a0 = cp.W;
    t.a1 = (int32_t)cp.tiles_per_batch;
    t.i0 = cp.S;
    t.i1 = cp.ncols;
    t.i2 = cp.bstride;
    t.m0 = div_magic((uint32_t)cp.W);
    t.s0 = p.d_sched + axis;
    t.t0 = tw_at(p, tw_off);
    t.lds = (int32_t)cp.lds;
    chain.push_back(t);
}

void add_plane(std::vector<BatchTask>& chain, const Plan& p, const ItemTiling& pt, bool inverse, const void* in,
               void* out)
{
    BatchTask t = base_task(p, inverse ? kBkPlaneC2R : kBkPlaneR2C, in, out, ceil_div(p.n0, pt.ppw));
    t.a0 = pt.ppw;
    t.a1 = p.plane_Hs;
    t.i0 = p.n0;
    t.m0 = div_magic((uint32_t)(pt.ppw * p.H));
    t.m1 = div_magic((uint32_t)p.H);
    t.s0 = p.d_sched + 2;
    t.s1 = p.d_sched + 1;
    t.t0 = tw_at(p, p.off_ax2h);
    t.t1 = tw_at(p, p.off_post);
    t.t2 = tw_at(p, p.off_ax1);
    t.lds = (int32_t)(pt.ppw * pt.plane_lds);
    chain.push_back(t);
}

void add_rows(std::vector<BatchTask>& chain, const Plan& p, const ItemTiling& pt, bool inverse, const void* in,
              void* out)
{
    const int64_t nrows = p.n0 * p.n1;
    BatchTask t = base_task(p, inverse ? kBkRowsC2R : kBkRowsR2C, in, out, ceil_div(nrows, pt.rpw));
    t.a0 = pt.rpw;
    t.a1 = p.Hs;
    t.i0 = nrows;
    t.s0 = p.d_sched + 2;
    t.t0 = tw_at(p, p.off_ax2h);
    t.t1 = tw_at(p, p.off_post);
    t.lds = (int32_t)pt.rows_lds;
    chain.push_back(t);
}

// The passes of the forward transform, as the single-item path runs them.
void chain_r2c(std::vector<BatchTask>& chain, const Plan& p, const ItemTiling& pt, const void* x, void* X)
{
    if (pt.fused) {
        add_plane(chain, p, pt, false, x, X);
    } else {
        add_rows(chain, p, pt, false, x, X);
        if (p.n1 > 1) add_cols(chain, p, pt.pass1, p.n0, 1, p.off_ax1, X, X, false);
    }
    if (p.n0 > 1) add_cols(chain, p, pt.pass0, 1, 0, p.off_ax0, X, X, false);
}

// The passes of the inverse transform; X is preserved iff work is given.
void chain_c2r(std::vector<BatchTask>& chain, const Plan& p, const ItemTiling& pt, void* X, void* y, void* work)
{
    void* scratch = work ? work : X;
    const void* cur = X;
    if (p.n0 > 1) {
        add_cols(chain, p, pt.pass0, 1, 0, p.off_ax0, cur, scratch, true);
        cur = scratch;
    }
    if (pt.fused) {
        add_plane(chain, p, pt, true, cur, y);
    } else {
        if (p.n1 > 1) {
            add_cols(chain, p, pt.pass1, p.n0, 1, p.off_ax1, cur, scratch, true);
            cur = scratch;
        }
        add_rows(chain, p, pt, true, cur, y);
    }
}

}  // namespace

const char* build_batch_table(const BatchSpec* items, int n, const BatchOptions& o, BatchTable& tab)
{
    tab = BatchTable{};
    std::vector<std::vector<BatchTask>> chains((size_t)n);
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        const BatchSpec& it = items[i];
        const Plan& p = *it.plan;
        ItemTiling pt;
        if (const char* why = item_tiling(p, pt)) return why;
        std::vector<BatchTask>& c = chains[(size_t)i];
        switch (it.dir) {
        case FFT3D_R2C: chain_r2c(c, p, pt, it.in, it.out); break;
        case FFT3D_C2R: chain_c2r(c, p, pt, const_cast<void*>(it.in), it.out, it.work); break;
        case FFT3D_ROUNDTRIP:
            chain_r2c(c, p, pt, it.in, it.mid);
            chain_c2r(c, p, pt, it.mid, it.out, it.work);
            break;
        default: return "unknown direction";
        }
        for (const BatchTask& t : c) lds = std::max(lds, (size_t)t.lds);
    }
    // order: item i's pass L goes to slot i + L*lag (lag >= n: pass-major,
    // every item's first pass, then every item's second pass, ...); within a
    // slot, later passes first.  A pass always lands after its predecessor.
    struct Key {
        int64_t slot;
        int level, item;
    };
    std::vector<Key> keys;
    const int64_t lag = o.lag > 0 ? o.lag : std::max(n, 1);
    for (int i = 0; i < n; ++i)
        for (int L = 0; L < (int)chains[(size_t)i].size(); ++L) keys.push_back({i + L * lag, L, i});
    std::stable_sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
        return a.slot != b.slot ? a.slot < b.slot : a.level > b.level;
    });
    std::vector<std::vector<int>> index((size_t)n);
    for (int i = 0; i < n; ++i) index[(size_t)i].assign(chains[(size_t)i].size(), -1);
    int64_t tickets = 0;
    for (const Key& k : keys) {
        BatchTask t = chains[(size_t)k.item][(size_t)k.level];
        if (k.level > 0) {
            const int d = index[(size_t)k.item][(size_t)k.level - 1];
            if (d < 0) return "internal error: a pass ordered before its predecessor";
            t.dep = d;
            t.dep_tiles = tab.tasks[(size_t)d].ntiles;
        }
        index[(size_t)k.item][(size_t)k.level] = (int)tab.tasks.size();
        tab.firsts.push_back((int32_t)tickets);
        tickets += t.ntiles;
        if (tickets > 0x3fffffff) return "too many tiles in one batch";
        tab.tasks.push_back(t);
    }
    tab.firsts.push_back((int32_t)tickets);
    tab.tickets = tickets;
    tab.lds = lds;
    return nullptr;
}

size_t batch_image_bytes(int ntasks)
{
    const size_t f = ((size_t)(ntasks + 1) * sizeof(int32_t) + 255) & ~(size_t)255;
    return f + (size_t)ntasks * sizeof(BatchTask);
}

size_t batch_tasks_offset(int ntasks) { return ((size_t)(ntasks + 1) * sizeof(int32_t) + 255) & ~(size_t)255; }

void write_batch_image(const BatchTable& tab, void* dst)
{
    const int nt = (int)tab.tasks.size();
    memcpy(dst, tab.firsts.data(), (size_t)(nt + 1) * sizeof(int32_t));
    memcpy(static_cast<char*>(dst) + batch_tasks_offset(nt), tab.tasks.data(), (size_t)nt * sizeof(BatchTask));
}

hipError_t batch_grid(const BatchTable& tab, int device, unsigned* grid)
{
    int cus = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = batch_occupancy(tab.lds, &per_cu);
    if (e != hipSuccess) return e;
    int64_t g = (int64_t)cus * std::max(per_cu, 1);
    if (const char* v = getenv("FFT3D_BATCH_WG_PER_CU")) {
        const int w = atoi(v);
        if (w >= 1 && w <= std::max(per_cu, 1)) g = (int64_t)cus * w;
    }
    g = std::min<int64_t>(g, std::max<int64_t>(tab.tickets, 1));
    *grid = (unsigned)g;
    return hipSuccess;
}

hipError_t enqueue_batch_image(const BatchTable& tab, unsigned grid, const void* dev_image, int* dev_ctr,
                               hipStream_t s)
{
    const int nt = (int)tab.tasks.size();
    const int* firsts = static_cast<const int*>(dev_image);
    const BatchTask* tasks =
        reinterpret_cast<const BatchTask*>(static_cast<const char*>(dev_image) + batch_tasks_offset(nt));
    return launch_batch(grid, tab.lds, tasks, firsts, nt, dev_ctr, kBatchSpinLimit, s);
}

// ---------------------------------------------------------------- ring --

namespace {

struct Slot {
    void* host = nullptr;  // pinned staging of the task image
    void* dev = nullptr;   // device task image
    int* ctr = nullptr;    // device counter block (left zeroed by each launch)
    hipEvent_t done = nullptr;
    bool used = false;
};

struct Ring {
    int device = -1;
    int next = 0;
    Slot slots[kRingSlots];
    std::mutex mu;
};

std::mutex g_rings_mu;
std::vector<std::unique_ptr<Ring>> g_rings;

Ring* ring_of(int device)
{
    std::lock_guard<std::mutex> g(g_rings_mu);
    for (auto& r : g_rings)
        if (r->device == device) return r.get();
    return nullptr;
}

}  // namespace

hipError_t ring_init(int device)
{
    std::lock_guard<std::mutex> g(g_rings_mu);
    for (auto& r : g_rings)
        if (r->device == device) return hipSuccess;
    std::unique_ptr<Ring> r(new Ring);
    r->device = device;
    const size_t img = batch_image_bytes(kRingTasks);
    const size_t ctr = (size_t)(kBatchCtrHeader + kRingTasks) * sizeof(int);
    for (Slot& s : r->slots) {
        hipError_t e = hipHostMalloc(&s.host, img, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&s.dev, img);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.ctr), ctr);
        if (e == hipSuccess) e = hipMemset(s.ctr, 0, ctr);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (Slot& q : r->slots) {
                if (q.host) (void)hipHostFree(q.host);
                if (q.dev) (void)hipFree(q.dev);
                if (q.ctr) (void)hipFree(q.ctr);
                if (q.done) (void)hipEventDestroy(q.done);
            }
            return e;
        }
    }
    g_rings.push_back(std::move(r));
    return hipSuccess;
}

hipError_t ring_submit(int device, const BatchTable& tab, hipStream_t s, const char** why)
{
    *why = nullptr;
    Ring* r = ring_of(device);
    if (!r) {
        *why = "no batch ring on this device (create a plan on it first)";
        return hipErrorInvalidValue;
    }
    if ((int)tab.tasks.size() > kRingTasks) {
        *why = "too many tasks for one ring slot";
        return hipErrorInvalidValue;
    }
    unsigned grid = 0;
    hipError_t e = batch_grid(tab, device, &grid);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(r->mu);
    Slot& sl = r->slots[r->next];
    r->next = (r->next + 1) % kRingSlots;
    // the slot's previous launch must be done with its staging and counters
    // (normally long since: the ring is kRingSlots deep)
    if (sl.used && (e = hipEventSynchronize(sl.done)) != hipSuccess) return e;
    write_batch_image(tab, sl.host);
    const size_t bytes = batch_image_bytes((int)tab.tasks.size());
    e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = enqueue_batch_image(tab, grid, sl.dev, sl.ctr, s);
    if (e == hipSuccess) e = hipEventRecord(sl.done, s);
    sl.used = e == hipSuccess;
    return e;
}

}  // namespace fft3d
