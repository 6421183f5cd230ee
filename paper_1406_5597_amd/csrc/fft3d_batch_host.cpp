// fft3d_batch_host.cpp -- host side of the batched launch: the task list of a
// batch, the per-device ring that fft3d_batch_submit streams task lists
// through, and the launch.
#include "fft3d_batch_host.hpp"

#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>

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
    bool plane_big = false;  // the plan's own big-tier fused plane tile (level mode)
    size_t plane_lds = 0;
    int ppw = 1;
    int rpw = 1;
    size_t rows_lds = 0;
    ColPass pass1;
    ColPass pass0;
};

int small_tier_elems(const Plan& p)
{
    return kNtSmall * (p.dtype == FFT3D_F64 ? Tier<double>::kEptSmall : Tier<float>::kEptSmall);
}

// Widest column tile of the small tier: W doubles while the tile (n rows by
// W columns) fits the tier and the batch's LDS budget and W does not pass the
// block's column count.  Small fields get fewer, larger tiles this way.
void widen_cols(ColPass& cp, int64_t n, const Plan& p)
{
    const int64_t es = small_tier_elems(p), cxs = 2 * p.elem;
    while ((int64_t)cp.W * 2 <= cp.ncols && n * cp.W * 2 <= es && n * cp.W * 2 * cxs <= kBatchLdsCap) cp.W *= 2;
    cp.wshift = 0;
    while ((1 << cp.wshift) < cp.W) ++cp.wshift;
    cp.tiles_per_batch = (cp.ncols + cp.W - 1) / cp.W;
    cp.lds = (size_t)(n * cp.W * cxs);
}

// big_planes: a plane that needs the big tier keeps its fused tile (the
// level mode has a kernel for it) instead of taking the split step.
const char* item_tiling(const Plan& p, bool widen, bool big_planes, ItemTiling& t)
{
    if (p.n0 > 1) {
        t.pass0 = p.pass0;
        if ((t.pass0.big || t.pass0.wide) && !small_colpass(p, 0, t.pass0))
            return "n0 too long for a small-tier column tile";
        if (widen) widen_cols(t.pass0, p.n0, p);
    }
    if (p.fused_plane && p.plane_big && big_planes) {
        t.fused = true;
        t.plane_big = true;
        t.plane_lds = p.plane_lds;
        t.ppw = p.ppw;
        return nullptr;
    }
    if (p.fused_plane && !p.plane_big && p.plane_lds <= kBatchLdsCap) {
        t.fused = true;
        t.plane_lds = p.plane_lds;
        t.ppw = p.ppw;
        if (widen) {
            // several small planes per tile, within the tier and the LDS budget
            const int64_t es = small_tier_elems(p), pe = p.n1 * p.H;
            while (t.ppw * 2 <= p.n0 && (t.ppw * 2) * pe <= es && (size_t)(t.ppw * 2) * p.plane_lds <= kBatchLdsCap)
                t.ppw *= 2;
        }
        return nullptr;
    }
    // one rows tile for both directions: the inverse kernel's (its LDS
    // budget has no cut for a fourth workgroup a CU, which the batched
    // kernel's registers never allow)
    bool rows_big = false;
    if (p.fused_plane) {
        int rpw_fwd = 1;
        size_t lds_fwd = 0;
        if (const char* why = split_tiling(p, rpw_fwd, rows_big, lds_fwd, t.rpw, t.rows_lds, t.pass1)) return why;
    } else {
        // split plans (the cooperative plane step is the split step in one
        // launch; both give the same bits)
        t.rpw = p.rpw_inv;
        rows_big = p.rows_big;
        t.rows_lds = p.rows_lds_inv;
        t.pass1 = p.pass1;
    }
    if (rows_big) return "rows too long for a small-tier tile";
    // rows per tile within the batch's LDS budget
    const int64_t row_bytes = (int64_t)p.Hs * 2 * p.elem;
    if ((int64_t)t.rpw * row_bytes > kBatchLdsCap) {
        t.rpw = (int)(kBatchLdsCap / row_bytes);
        if (t.rpw < 1) return "rows too long for a small-tier tile";
        t.rows_lds = (size_t)(t.rpw * row_bytes);
    }
    if (p.n1 > 1 && (t.pass1.big || t.pass1.wide) && !small_colpass(p, 1, t.pass1))
        return "n1 too long for a small-tier column tile";
    if (p.n1 > 1 && widen) widen_cols(t.pass1, p.n1, p);
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
    t.big = pt.plane_big ? 1 : 0;
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

// Rough time of a task on one workgroup, for placing items on XCDs: per tile
// a fixed part (scheduling, load latency, store drain; about 4 us measured on
// MI355X) plus its LDS-sized data at about 16 GB/s per CU; the plane tiles do
// two axes and the split of the real transform, about 1.6x the work.
int64_t task_cost_ns(const BatchTask& t)
{
    int64_t tile = 4000 + t.lds / 16;
    if (t.kind == kBkPlaneR2C || t.kind == kBkPlaneC2R) tile = tile * 8 / 5;
    return (int64_t)t.ntiles * tile;
}

// The level mode's launches: each item's passes in order, pass L in the
// first launch of its kind and dtype after the launch of pass L-1, or in a
// new launch right after that one.  Inserting a launch keeps the order of
// those already placed, so every pass stays after its predecessor.  Items
// with the longest chains go first (they set the skeleton the others fit
// into); within a launch, tasks with more tiles first.
const char* build_levels(const std::vector<std::vector<BatchTask>>& chains, const std::vector<int64_t>& load,
                         BatchTable& tab)
{
    struct Group {
        int kind, f64, big;
        std::vector<const BatchTask*> tasks;
        std::vector<const BatchTask*> preds;  // the pass before each task (or null)
    };
    std::vector<Group> g;
    const int n = (int)chains.size();
    std::vector<int> order((size_t)n);
    for (int i = 0; i < n; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const size_t la = chains[(size_t)a].size(), lb = chains[(size_t)b].size();
        return la != lb ? la > lb : load[(size_t)a] > load[(size_t)b];
    });
    for (int i : order) {
        int prev = -1;
        const BatchTask* pred = nullptr;
        for (const BatchTask& t : chains[(size_t)i]) {
            int j = prev + 1;
            while (j < (int)g.size() &&
                   !(g[(size_t)j].kind == t.kind && g[(size_t)j].f64 == t.f64 && g[(size_t)j].big == t.big))
                ++j;
            if (j == (int)g.size()) {
                j = prev + 1;
                g.insert(g.begin() + j, Group{t.kind, t.f64, t.big, {}, {}});
            }
            g[(size_t)j].tasks.push_back(&t);
            g[(size_t)j].preds.push_back(pred);
            prev = j;
            pred = &t;
        }
    }
    // the launch of every pass, for the launches' dependencies (std::less:
    // a total order on pointers into different chains)
    std::map<const BatchTask*, int, std::less<const BatchTask*>> where;
    for (size_t j = 0; j < g.size(); ++j)
        for (const BatchTask* t : g[j].tasks) where[t] = (int)j;
    auto launch_of = [&](const BatchTask* t) { return where.at(t); };
    for (Group& gr : g) {
        BatchLaunch L;
        for (const BatchTask* pr : gr.preds)
            if (pr) L.deps.push_back(launch_of(pr));
        std::sort(L.deps.begin(), L.deps.end());
        L.deps.erase(std::unique(L.deps.begin(), L.deps.end()), L.deps.end());
        std::stable_sort(gr.tasks.begin(), gr.tasks.end(),
                         [](const BatchTask* a, const BatchTask* b) { return a->ntiles > b->ntiles; });
        L.kind = gr.kind;
        L.f64 = gr.f64;
        L.big = gr.big;
        L.task_begin = (int)tab.tasks.size();
        L.ntasks = (int)gr.tasks.size();
        L.firsts_begin = (int)tab.firsts.size();
        for (const BatchTask* t : gr.tasks) {
            tab.firsts.push_back((int32_t)L.tiles);
            L.tiles += t->ntiles;
            if (L.tiles > 0x3fffffff) return "too many tiles in one launch";
            L.lds = std::max(L.lds, (size_t)t->lds);
            BatchTask c = *t;
            c.dep = -1;
            c.dep_tiles = 0;
            tab.tasks.push_back(c);
        }
        tab.firsts.push_back((int32_t)L.tiles);
        tab.tickets += L.tiles;
        tab.lds = std::max(tab.lds, L.lds);
        tab.launches.push_back(L);
    }
    tab.levels = true;
    tab.nqueues = 0;
    tab.task_begin.assign(1, 0);
    return nullptr;
}

}  // namespace

const char* build_batch_table(const BatchSpec* items, int n, const BatchOptions& o, BatchTable& tab)
{
    tab = BatchTable{};
    std::vector<std::vector<BatchTask>> chains((size_t)n);
    std::vector<int64_t> load((size_t)n, 0);
    size_t lds = 0;
    for (int i = 0; i < n; ++i) {
        const BatchSpec& it = items[i];
        const Plan& p = *it.plan;
        ItemTiling pt;
        const bool levels = o.mode == 0 || o.mode == 3;
        if (const char* why = item_tiling(p, o.widen, levels, pt)) return why;
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
        for (const BatchTask& t : c) {
            lds = std::max(lds, (size_t)t.lds);
            load[(size_t)i] += task_cost_ns(t);
        }
    }

    if (o.mode == 0 || o.mode == 3) {
        tab.wg_per_cu = o.wg_per_cu;
        tab.spin_limit = o.spin_limit;
        return build_levels(chains, load, tab);
    }

    // queues: one per XCD, items placed largest first on the least loaded
    // (pinned) -- when that balances the XCDs; else one queue (spread)
    const int nx = (int)o.xcc_ids.size();
    std::vector<int> queue_of((size_t)n, 0);
    int nq = 1;
    bool pinned = false;
    if (nx > 1 && o.mode != 2 && n > 0) {
        std::vector<int> order((size_t)n);
        for (int i = 0; i < n; ++i) order[(size_t)i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return load[(size_t)a] > load[(size_t)b]; });
        std::vector<int64_t> ql((size_t)nx, 0);
        for (int i : order) {
            const int best = (int)(std::min_element(ql.begin(), ql.end()) - ql.begin());
            queue_of[(size_t)i] = best;
            ql[(size_t)best] += load[(size_t)i];
        }
        const int64_t mx = *std::max_element(ql.begin(), ql.end());
        int64_t sum = 0;
        for (int64_t v : ql) sum += v;
        // auto: pin when the busiest XCD has at most 1/4 more than the mean
        pinned = o.mode == 1 || (int64_t)4 * nx * mx <= (int64_t)5 * sum;
        if (pinned) nq = nx;
    }
    if (!pinned) std::fill(queue_of.begin(), queue_of.end(), 0);
    tab.nqueues = nq;
    tab.pinned = pinned;
    for (int x = 0; x < kBatchMaxQueues; ++x) tab.qmap[x] = pinned ? -1 : 0;
    if (pinned)
        for (int qi = 0; qi < nx; ++qi) tab.qmap[o.xcc_ids[(size_t)qi] & (kBatchMaxQueues - 1)] = qi;

    // order within a queue: item i's pass L goes to slot r + L*lag, r the
    // item's rank in its queue (lag >= items: pass-major, every item's first
    // pass, then every item's second pass, ...); within a slot, later passes
    // first.  A pass always lands after its predecessor.
    std::vector<std::vector<int>> index((size_t)n);
    for (int i = 0; i < n; ++i) index[(size_t)i].assign(chains[(size_t)i].size(), -1);
    tab.task_begin.assign((size_t)nq + 1, 0);
    tab.queue_tickets.assign((size_t)nq, 0);
    for (int qi = 0; qi < nq; ++qi) {
        struct Key {
            int64_t slot;
            int level, item;
        };
        std::vector<Key> keys;
        int rank = 0;
        int nitems = 0;
        for (int i = 0; i < n; ++i) nitems += queue_of[(size_t)i] == qi;
        const int64_t lag = o.lag > 0 ? o.lag : std::max(nitems, 1);
        for (int i = 0; i < n; ++i) {
            if (queue_of[(size_t)i] != qi) continue;
            for (int L = 0; L < (int)chains[(size_t)i].size(); ++L) keys.push_back({rank + L * lag, L, i});
            ++rank;
        }
        std::stable_sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
            return a.slot != b.slot ? a.slot < b.slot : a.level > b.level;
        });
        tab.task_begin[(size_t)qi] = (int)tab.tasks.size();
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
        tab.queue_tickets[(size_t)qi] = tickets;
        tab.tickets += tickets;
    }
    tab.task_begin[(size_t)nq] = (int)tab.tasks.size();
    tab.lds = lds;
    tab.wg_per_cu = o.wg_per_cu;
    tab.spin_limit = o.spin_limit;
    return nullptr;
}

size_t batch_tasks_offset(int ntasks, int nqueues)
{
    return (sizeof(BatchHeader) + (size_t)(ntasks + nqueues) * sizeof(int32_t) + 255) & ~(size_t)255;
}

size_t batch_image_bytes(int ntasks, int nqueues)
{
    return batch_tasks_offset(ntasks, nqueues) + (size_t)ntasks * sizeof(BatchTask);
}

// Level mode: the first-tile tables, then the tasks.
size_t level_tasks_offset(const BatchTable& tab) { return (tab.firsts.size() * sizeof(int32_t) + 255) & ~(size_t)255; }

size_t batch_image_bytes(const BatchTable& tab)
{
    if (tab.levels) return level_tasks_offset(tab) + tab.tasks.size() * sizeof(BatchTask);
    return batch_image_bytes((int)tab.tasks.size(), tab.nqueues);
}

void write_batch_image(const BatchTable& tab, void* dst)
{
    const int nt = (int)tab.tasks.size();
    if (tab.levels) {
        char* d = static_cast<char*>(dst);
        const size_t off = level_tasks_offset(tab);
        memset(d, 0, off);
        memcpy(d, tab.firsts.data(), tab.firsts.size() * sizeof(int32_t));
        memcpy(d + off, tab.tasks.data(), (size_t)nt * sizeof(BatchTask));
        return;
    }
    BatchHeader h;
    memset(&h, 0, sizeof h);
    h.nqueues = tab.nqueues;
    h.pinned = tab.pinned ? 1 : 0;
    h.ntasks = nt;
    for (int x = 0; x < kBatchMaxQueues; ++x) h.qmap[x] = tab.qmap[x];
    for (int q = 0; q <= tab.nqueues; ++q) h.task_begin[q] = tab.task_begin[(size_t)q];
    char* d = static_cast<char*>(dst);
    memcpy(d, &h, sizeof h);
    memcpy(d + sizeof h, tab.firsts.data(), tab.firsts.size() * sizeof(int32_t));
    memcpy(d + batch_tasks_offset(nt, tab.nqueues), tab.tasks.data(), (size_t)nt * sizeof(BatchTask));
}

hipError_t batch_grid(const BatchTable& tab, int device, unsigned* grid)
{
    int cus = 0, per_cu = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) e = batch_occupancy(tab.lds, &per_cu);
    if (e != hipSuccess) return e;
    int64_t g = (int64_t)cus * std::max(per_cu, 1);
    if (tab.wg_per_cu >= 1 && tab.wg_per_cu <= std::max(per_cu, 1)) g = (int64_t)cus * tab.wg_per_cu;
    // one queue: no more workgroups than tickets; per-XCD queues: every XCD
    // must get workgroups (blocks go to the XCDs in turn), so keep them all
    if (!tab.pinned) g = std::min<int64_t>(g, std::max<int64_t>(tab.tickets, 1));
    *grid = (unsigned)g;
    return hipSuccess;
}

hipError_t enqueue_batch_image(const BatchTable& tab, unsigned grid, const void* dev_image, int* dev_ctr,
                               hipStream_t s)
{
    if (tab.levels) {
        const int32_t* firsts = static_cast<const int32_t*>(dev_image);
        const BatchTask* tasks = reinterpret_cast<const BatchTask*>(static_cast<const char*>(dev_image) +
                                                                    level_tasks_offset(tab));
        for (const BatchLaunch& L : tab.launches) {
            const hipError_t e = launch_level(L.kind, L.f64, L.big, (unsigned)L.tiles, L.lds, tasks + L.task_begin,
                                              firsts + L.firsts_begin, L.ntasks, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    return launch_batch(grid, tab.lds, dev_image, dev_ctr, tab.spin_limit, s);
}

// ---------------------------------------------------------------- ring --

namespace {

struct Slot {
    void* host = nullptr;  // pinned staging of the task image
    void* dev = nullptr;   // device task image
    int* ctr = nullptr;    // device counter block (left zeroed by each launch)
    int* hstat = nullptr;  // pinned: the launch's error bits, copied back behind it
    hipEvent_t done = nullptr;
    bool used = false;
    int64_t seq = -1;      // sequence number of the slot's last launch
};

// Error bits of completed launches whose slots were reused since, by
// sequence number (the last kRingHistory of them).
constexpr int kRingHistory = 256;

struct Ring {
    int device = -1;
    int next = 0;
    int64_t seq = 0;           // launches staged so far
    std::vector<int> xcc_ids;  // distinct hardware XCC ids of the device
    Slot slots[kRingSlots];
    int64_t hist_seq[kRingHistory];
    int hist_err[kRingHistory];
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

void free_slots(Ring& r)
{
    for (Slot& q : r.slots) {
        if (q.host) (void)hipHostFree(q.host);
        if (q.hstat) (void)hipHostFree(q.hstat);
        if (q.dev) (void)hipFree(q.dev);
        if (q.ctr) (void)hipFree(q.ctr);
        if (q.done) (void)hipEventDestroy(q.done);
        q = Slot{};
    }
}

// State of a slot as the host sees it, without waiting.
int slot_state(const Slot& sl, hipError_t* err)
{
    *err = hipSuccess;
    if (!sl.used) return kSlotFree;
    const hipError_t e = hipEventQuery(sl.done);
    if (e == hipErrorNotReady) return kSlotBusy;
    if (e != hipSuccess) *err = e;
    return kSlotDone;
}

// Record the error bits of a slot's completed launch before it is reused.
void retire(Ring& r, Slot& sl)
{
    if (!sl.used || sl.seq < 0) return;
    const int i = (int)(sl.seq % kRingHistory);
    r.hist_seq[i] = sl.seq;
    r.hist_err[i] = *sl.hstat;
    sl.used = false;
}

}  // namespace

hipError_t ring_init(int device)
{
    std::lock_guard<std::mutex> g(g_rings_mu);
    for (auto& r : g_rings)
        if (r->device == device) return hipSuccess;
    std::unique_ptr<Ring> r(new Ring);
    r->device = device;
    for (int i = 0; i < kRingHistory; ++i) {
        r->hist_seq[i] = -1;
        r->hist_err[i] = 0;
    }
    // the XCDs the device dispatches to (a probe launch of 1024 workgroups)
    std::vector<int> ids(1024);
    hipError_t pe = probe_xcc_ids(1024, ids.data());
    if (pe != hipSuccess) return pe;
    std::sort(ids.begin(), ids.end());
    ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
    r->xcc_ids = ids;
    const size_t img = batch_image_bytes(kRingTasks, kBatchMaxQueues);
    const size_t ctr = (size_t)(kBatchCtrHeader + kRingTasks) * sizeof(int);
    for (Slot& s : r->slots) {
        hipError_t e = hipHostMalloc(&s.host, img, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&s.hstat), sizeof(int), hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc(&s.dev, img);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&s.ctr), ctr);
        if (e == hipSuccess) e = hipMemset(s.ctr, 0, ctr);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            free_slots(*r);
            return e;
        }
        *s.hstat = 0;
    }
    g_rings.push_back(std::move(r));
    return hipSuccess;
}

bool ring_ready(int device) { return ring_of(device) != nullptr; }

std::vector<int> device_xcc_ids(int device)
{
    Ring* r = ring_of(device);
    return r ? r->xcc_ids : std::vector<int>();
}

int ring_pick(const int* state, int nslots, int next, int needed, int* picked)
{
    int got = 0;
    for (int k = 0; k < nslots && got < needed; ++k) {
        const int i = (next + k) % nslots;
        if (state[i] != kSlotBusy) picked[got++] = i;
    }
    return got;
}

hipError_t ring_submit(int device, const BatchTable* tabs, int ntabs, hipStream_t s, int64_t* first_seq,
                       const char** why)
{
    *why = nullptr;
    Ring* r = ring_of(device);
    if (!r) {
        *why = "the device has no batch ring: call fft3d_init() on it first";
        return hipErrorInvalidValue;
    }
    if (ntabs < 1 || ntabs > kRingSlots) {
        *why = "batch needs more ring slots than the ring has";
        return hipErrorInvalidValue;
    }
    std::vector<unsigned> grids((size_t)ntabs);
    for (int t = 0; t < ntabs; ++t) {
        if ((int)tabs[t].tasks.size() > kRingTasks ||
            batch_image_bytes(tabs[t]) > batch_image_bytes(kRingTasks, kBatchMaxQueues)) {
            *why = "too many tasks for one ring slot";
            return hipErrorInvalidValue;
        }
        hipError_t e = batch_grid(tabs[t], device, &grids[(size_t)t]);
        if (e != hipSuccess) return e;
    }
    std::lock_guard<std::mutex> g(r->mu);
    // every slot this submit needs must be free or finished: a slot still in
    // flight is never waited for (all or nothing: nothing is enqueued then)
    int state[kRingSlots], picked[kRingSlots];
    for (int i = 0; i < kRingSlots; ++i) {
        hipError_t qe;
        state[i] = slot_state(r->slots[i], &qe);
        if (qe != hipSuccess) return qe;
    }
    if (ring_pick(state, kRingSlots, r->next, ntabs, picked) < ntabs) {
        *why = "every ring slot is still in flight";
        return hipErrorNotReady;
    }
    *first_seq = r->seq;
    for (int t = 0; t < ntabs; ++t) {
        Slot& sl = r->slots[picked[t]];
        retire(*r, sl);
        write_batch_image(tabs[t], sl.host);
        const size_t bytes = batch_image_bytes(tabs[t]);
        hipError_t e = hipMemcpyAsync(sl.dev, sl.host, bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = enqueue_batch_image(tabs[t], grids[(size_t)t], sl.dev, sl.ctr, s);
        // the launch's error bits, back to the host behind it (the level
        // mode has no waits and no error bits)
        *sl.hstat = 0;
        if (e == hipSuccess && !tabs[t].levels)
            e = hipMemcpyAsync(sl.hstat, sl.ctr + kBatchCtrStatus, sizeof(int), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipEventRecord(sl.done, s);
        if (e != hipSuccess) return e;
        sl.used = true;
        sl.seq = r->seq++;
        r->next = (picked[t] + 1) % kRingSlots;
    }
    return hipSuccess;
}

int ring_status(int device, int64_t first_seq, int count, const char** why)
{
    *why = nullptr;
    Ring* r = ring_of(device);
    if (!r) {
        *why = "the device has no batch ring";
        return FFT3D_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> g(r->mu);
    int err = 0;
    for (int64_t q = first_seq; q < first_seq + count; ++q) {
        bool found = false;
        for (Slot& sl : r->slots) {
            if (sl.used && sl.seq == q) {
                hipError_t qe;
                const int st = slot_state(sl, &qe);
                if (qe != hipSuccess) {
                    *why = hipGetErrorString(qe);
                    return FFT3D_ERR_HIP;
                }
                if (st == kSlotBusy) return FFT3D_ERR_BUSY;
                err |= *sl.hstat;
                found = true;
                break;
            }
        }
        if (found) continue;
        const int i = (int)(q % kRingHistory);
        if (q < 0 || q >= r->seq || r->hist_seq[i] != q) {
            *why = "unknown or expired batch token";
            return FFT3D_ERR_INVALID_ARG;
        }
        err |= r->hist_err[i];
    }
    return err;
}

}  // namespace fft3d
