// batch_sim.cpp -- CPU check of the batched launch's task lists and of its
// ticket protocol (test infrastructure; built by tests/test_batch_host.py).
//
// Reads items from stdin, one per line: "n0 n1 n2 dtype dir work" (dtype 0
// FP32 / 1 FP64, dir 0 R2C / 1 C2R / 2 ROUNDTRIP, work 0/1), and optional
// lines "lag L", "mode M" (4 auto, the default here; 1 pinned, 2 spread; 0 and 3
// levels), "xcds X" (the device
// has XCC ids 0..X-1; default 8).  Builds host-only plans and the batch's
// task list with the library's own host code (fake, disjoint device
// addresses), then:
//  1. checks the table: tickets numbered in order, every task after the task
//     it waits for (the previous pass of its item), tile LDS within budget;
//  2. checks every tile's memory footprint (the index arithmetic the kernel
//     uses) against the item's buffers;
//  3. runs the kernel's scheduling loop -- a ticket counter per queue, the
//     next ticket taken before the current tile runs, the task found by a
//     galloping search, a wait for the dependency before a task's first tile
//     -- on G host threads (thread g on XCD g mod X, as blocks are dealt to
//     the XCDs in turn), and checks that it ends with every tile run exactly
//     once, after all tiles of its dependency, and, when items are pinned,
//     with every pass of an item on the item's XCD.
// Prints "ok <tasks> <tickets> <lds> <pinned>" or "FAIL: why" (exit 1).
//
// Level mode ("mode 3"): checks 1 and 2 only -- every launch of one tile kind
// and dtype, every item's passes those of the persistent table in the same
// order and each in a later launch than its predecessor -- and prints
// "ok levels <tasks> <launches> <tiles> <lds>".
//
// "state lost" models thread 0's next-ticket word kept where it does not
// hold its value -- an LDS address past the launch's LDS allocation, which
// reads as zero and drops writes on this hardware -- and "bound 0" drops the
// kernel's iteration bound (a workgroup runs at most its queue's tickets + 1
// iterations).  With the state lost, the loop keeps running ticket 0: with
// the bound every workgroup still leaves and the loop error bit is set
// ("bounded <iterations>", exit 0); without it the simulation stops each
// workgroup after 1000 times its queue's tickets and reports "unbounded"
// (exit 3) -- the way such a launch never ends on the device.
//
// "spin N" gives every dependency wait the kernel's bound of N polls (N = 0:
// none): a wait that runs out sets the error bit, its task's tiles are
// skipped, and every later wait gives up at once.  The run must still end
// with every workgroup gone; it prints "errbit <skipped tiles>" (exit 0).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <chrono>
#include <string>
#include <thread>
#include <vector>

#include "../include/fft3d.h"
#include "../paper_1406_5597_amd/csrc/fft3d_batch_host.hpp"

using namespace fft3d;

// The device half of the library is not linked: these are never called.
namespace fft3d {
hipError_t batch_occupancy(size_t, int* per_cu)
{
    *per_cu = 1;
    return hipSuccess;
}
hipError_t launch_batch(unsigned, size_t, const void*, int*, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_level(int, int, int, unsigned, size_t, const BatchTask*, const int*, int, hipStream_t)
{
    return hipErrorNotSupported;
}
hipError_t probe_xcc_ids(int, int*) { return hipErrorNotSupported; }
}  // namespace fft3d

static int fail(const std::string& m)
{
    printf("FAIL: %s\n", m.c_str());
    return 1;
}

struct Buf {
    uintptr_t base;
    size_t bytes;
};

struct ItemBufs {
    Buf in, mid, out, work;
};

static bool inside(uintptr_t a, size_t n, const Buf& b) { return b.base && a >= b.base && a + n <= b.base + b.bytes; }

// Byte range [lo, hi) of `count` elements at element offset `off` with
// stride 1, of `es` bytes each, from `ptr`.
static void span(const void* ptr, int64_t off, int64_t count, int es, uintptr_t& lo, size_t& n)
{
    lo = (uintptr_t)ptr + (uintptr_t)(off * es);
    n = (size_t)(count * es);
}

// "ring": the slot choice of the submit ring (ring_pick) on fixed slot
// states.  A submit must take only free or finished slots, in ring order
// from the next one, and report a shortfall instead of waiting for a slot in
// flight.
static int ring_check()
{
    const int F = kSlotFree, D = kSlotDone, B = kSlotBusy;
    int picked[8];
    {
        const int st[4] = {B, B, B, B};  // all in flight: nothing to take
        if (ring_pick(st, 4, 1, 1, picked) != 0) return fail("ring: took a slot in flight");
    }
    {
        const int st[4] = {B, D, B, F};  // from slot 2: 3 (free), then 1 (finished)
        if (ring_pick(st, 4, 2, 2, picked) != 2 || picked[0] != 3 || picked[1] != 1)
            return fail("ring: wrong slots for a two-slot submit");
        if (ring_pick(st, 4, 2, 3, picked) != 2) return fail("ring: three slots found where two are usable");
    }
    {
        const int st[4] = {F, F, F, F};
        if (ring_pick(st, 4, 3, 4, picked) != 4 || picked[0] != 3 || picked[1] != 0 || picked[3] != 2)
            return fail("ring: free slots not taken in ring order");
    }
    printf("ok ring\n");
    return 0;
}

int main(int argc, char** argv)
{
    if (argc > 1 && !strcmp(argv[1], "ring")) return ring_check();
    int G = argc > 1 ? atoi(argv[1]) : 64;
    std::vector<Plan> plans;
    std::vector<int> dirs, works;
    BatchOptions o;
    o.mode = 4;  // the persistent launch (pinned when balanced) unless "mode M" says otherwise
    int xcds = 8;
    bool state_lost = false, bounded = true;
    int spin = -1;  // polls of a dependency wait; -1: wait (up to 60 s)
    char line[256];
    while (fgets(line, sizeof line, stdin)) {
        long long n0, n1, n2;
        int dt, dir, work;
        int lag;
        if (sscanf(line, "lag %d", &lag) == 1) {
            o.lag = lag;
            continue;
        }
        if (sscanf(line, "mode %d", &lag) == 1) {
            o.mode = lag;
            continue;
        }
        if (sscanf(line, "xcds %d", &lag) == 1) {
            xcds = lag;
            continue;
        }
        if (!strncmp(line, "state lost", 10)) {
            state_lost = true;
            continue;
        }
        if (sscanf(line, "bound %d", &lag) == 1) {
            bounded = lag != 0;
            continue;
        }
        if (sscanf(line, "spin %d", &lag) == 1) {
            spin = lag;
            continue;
        }
        if (sscanf(line, "%lld %lld %lld %d %d %d", &n0, &n1, &n2, &dt, &dir, &work) != 6) continue;
        Plan p;
        std::string why;
        if (plan_build_host(p, n0, n1, n2, dt, 0, nullptr, why)) return fail("plan: " + why);
        plans.push_back(p);
        dirs.push_back(dir);
        works.push_back(work);
    }
    const int n = (int)plans.size();
    // fake device memory: every plan's tables and every buffer disjoint
    uintptr_t next = 1ull << 32;
    auto take = [&](size_t bytes) {
        uintptr_t a = next;
        next += (bytes + 4095) / 4096 * 4096 + 4096;
        return a;
    };
    std::vector<ItemBufs> bufs((size_t)n);
    std::vector<BatchSpec> specs((size_t)n);
    for (int i = 0; i < n; ++i) {
        Plan& p = plans[(size_t)i];
        p.d_sched = reinterpret_cast<AxisSched*>(take(3 * sizeof(AxisSched)));
        p.d_tw = reinterpret_cast<void*>(take((size_t)p.tw_count * 2 * p.elem));
        p.has_device = true;
        const size_t rb = (size_t)p.N * p.elem, cb = (size_t)p.M * 2 * p.elem;
        ItemBufs& b = bufs[(size_t)i];
        memset(&b, 0, sizeof b);
        if (dirs[(size_t)i] == FFT3D_C2R) {
            b.in = {take(cb), cb};
            b.out = {take(rb), rb};
        } else if (dirs[(size_t)i] == FFT3D_R2C) {
            b.in = {take(rb), rb};
            b.out = {take(cb), cb};
        } else {
            b.in = {take(rb), rb};
            b.mid = {take(cb), cb};
            b.out = {take(rb), rb};
        }
        if (works[(size_t)i] && dirs[(size_t)i] != FFT3D_R2C) b.work = {take(cb), cb};
        specs[(size_t)i] = {&p, dirs[(size_t)i], (const void*)b.in.base, (void*)b.mid.base, (void*)b.out.base,
                            (void*)b.work.base};
    }
    for (int x = 0; x < xcds; ++x) o.xcc_ids.push_back(x);
    BatchTable tab;
    if (const char* why = build_batch_table(specs.data(), n, o, tab)) return fail(why);
    const int nt = (int)tab.tasks.size();
    const int nq = tab.nqueues;

    auto owner_of = [&](const void* p) -> int {
        for (int i = 0; i < n; ++i) {
            const ItemBufs& b = bufs[(size_t)i];
            for (const Buf* x : {&b.in, &b.mid, &b.out, &b.work})
                if (x->base && (uintptr_t)p >= x->base && (uintptr_t)p < x->base + x->bytes) return i;
        }
        return -1;
    };
    // 1. the table
    if (tab.levels) {
        // level mode: every launch of one kind and dtype, its first-tile table
        // counting its tasks' tiles; every item's passes those of the
        // persistent table of the same items, in the same order, each in a
        // later launch than the one before
        const int nl = (int)tab.launches.size();
        if ((int)tab.firsts.size() != nt + nl) return fail("levels: first-tile table size");
        int64_t all = 0;
        int next_task = 0;
        std::vector<std::vector<std::pair<int, int>>> got((size_t)n);
        for (int j = 0; j < nl; ++j) {
            const BatchLaunch& L = tab.launches[(size_t)j];
            if (L.ntasks < 1 || L.task_begin != next_task) return fail("levels: launch task ranges");
            for (int d : L.deps)
                if (d < 0 || d >= j) return fail("levels: a launch depends on a later one");
            next_task += L.ntasks;
            const int32_t* f = tab.firsts.data() + L.firsts_begin;
            if (L.firsts_begin != L.task_begin + j || f[0] != 0) return fail("levels: first-tile table layout");
            for (int k = L.task_begin; k < L.task_begin + L.ntasks; ++k) {
                const BatchTask& t = tab.tasks[(size_t)k];
                if (t.kind != L.kind || t.f64 != L.f64) return fail("levels: a launch mixes kinds or dtypes");
                if (t.ntiles < 1 || f[k - L.task_begin + 1] - f[k - L.task_begin] != t.ntiles)
                    return fail("levels: first-tile table does not count tiles");
                if ((size_t)t.lds > L.lds || (int64_t)L.lds > (L.big ? kLdsMax : kBatchLdsCap))
                    return fail("levels: LDS over budget");
                if (t.big != L.big) return fail("levels: a launch mixes tiers");
                const int item = owner_of(t.in);
                if (item < 0) return fail("levels: task of no item");
                got[(size_t)item].push_back({j, k});
            }
            if (f[L.ntasks] != L.tiles) return fail("levels: launch tiles");
            all += L.tiles;
        }
        if (next_task != nt || all != tab.tickets) return fail("levels: task or tile totals");
        // each item's passes, in launch order, are the chain the single-item
        // path runs: the plane step (fused, or rows + n1 columns) and the n0
        // columns, reversed for the inverse; each pass reads what the pass
        // before wrote, from the item's input to its output; each is in a
        // later launch than the pass before, and that launch is among its
        // launch's dependencies
        for (int i = 0; i < n; ++i) {
            const auto& g = got[(size_t)i];
            const Plan& p = plans[(size_t)i];
            const ItemBufs& bb = bufs[(size_t)i];
            const int dir = dirs[(size_t)i];
            const std::string who = "levels: item " + std::to_string(i);
            std::vector<std::pair<int, int>> want;  // (kind, column axis or -1)
            size_t at = 0;
            auto kind_at = [&](size_t L) { return L < g.size() ? tab.tasks[(size_t)g[L].second].kind : -1; };
            if (dir != FFT3D_C2R) {
                if (kind_at(at) == kBkPlaneR2C) {
                    want.push_back({kBkPlaneR2C, -1});
                } else {
                    want.push_back({kBkRowsR2C, -1});
                    if (p.n1 > 1) want.push_back({kBkColsFwd, 1});
                }
                if (p.n0 > 1) want.push_back({kBkColsFwd, 0});
                at = want.size();
            }
            if (dir != FFT3D_R2C) {
                if (p.n0 > 1) want.push_back({kBkColsInv, 0});
                const size_t k = at + (p.n0 > 1 ? 1 : 0);
                if (kind_at(k) == kBkPlaneC2R) {
                    want.push_back({kBkPlaneC2R, -1});
                } else {
                    if (p.n1 > 1) want.push_back({kBkColsInv, 1});
                    want.push_back({kBkRowsC2R, -1});
                }
            }
            if (g.size() != want.size()) return fail(who + " has a wrong pass count");
            const void* cur = (const void*)bb.in.base;
            for (size_t L = 0; L < g.size(); ++L) {
                const BatchTask& a = tab.tasks[(size_t)g[L].second];
                const int axis = (a.kind == kBkColsFwd || a.kind == kBkColsInv) ? (int)(a.s0 - p.d_sched) : -1;
                if (a.kind != want[L].first || axis != want[L].second)
                    return fail(who + " pass " + std::to_string(L) + " is not the pass the item runs there");
                if (a.in != cur) return fail(who + " pass " + std::to_string(L) + " does not read the previous output");
                cur = a.out;
                if (dir == FFT3D_ROUNDTRIP && L + 1 == at && cur != (const void*)bb.mid.base)
                    return fail(who + ": the forward half does not end in mid");
                if (a.big && (a.kind != kBkPlaneR2C && a.kind != kBkPlaneC2R))
                    return fail(who + ": a big tile that is not a fused plane");
                if (L > 0 && g[L].first <= g[L - 1].first)
                    return fail(who + " pass " + std::to_string(L) + " not in a later launch than its predecessor");
                if (L > 0) {
                    const std::vector<int>& d = tab.launches[(size_t)g[L].first].deps;
                    if (std::find(d.begin(), d.end(), g[L - 1].first) == d.end())
                        return fail("levels: a launch does not depend on its tasks' predecessors' launch");
                }
            }
            if (cur != (const void*)bb.out.base) return fail(who + ": the last pass does not write the output");
        }
    } else {
        if ((int)tab.task_begin.size() != nq + 1 || tab.task_begin[0] != 0 || tab.task_begin[(size_t)nq] != nt)
            return fail("queue task ranges");
        if ((int)tab.firsts.size() != nt + nq) return fail("ticket table size");
        std::vector<int> qof((size_t)nt, -1);
        int64_t all = 0;
        for (int q = 0; q < nq; ++q) {
            const int b = tab.task_begin[(size_t)q], e = tab.task_begin[(size_t)q + 1];
            const int32_t* f = tab.firsts.data() + b + q;
            if (f[0] != 0) return fail("queue tickets do not start at 0");
            for (int k = b; k < e; ++k) {
                qof[(size_t)k] = q;
                const BatchTask& t = tab.tasks[(size_t)k];
                if (t.ntiles < 1) return fail("empty task");
                if (f[k - b + 1] - f[k - b] != t.ntiles) return fail("ticket table does not count tiles");
                if (t.dep >= 0 && (t.dep < b || t.dep >= k)) return fail("task waits for a later task or another queue");
                if (t.dep >= 0 && t.dep_tiles != tab.tasks[(size_t)t.dep].ntiles) return fail("dep_tiles");
                if ((size_t)t.lds > tab.lds || (int64_t)tab.lds > kBatchLdsCap) return fail("LDS over budget");
            }
            if (f[e - b] != tab.queue_tickets[(size_t)q]) return fail("queue total");
            all += f[e - b];
        }
        if (all != tab.tickets) return fail("ticket total");
        if (tab.pinned ? nq != xcds : nq != 1) return fail("queue count");
        for (int x = 0; x < xcds; ++x)
            if (tab.qmap[x] < 0 || tab.qmap[x] >= nq) return fail("an XCD without a queue");
    }

    // 2. tile footprints against the buffers of the item that owns the task
    auto owner = [&](const void* p) -> int {
        for (int i = 0; i < n; ++i) {
            const ItemBufs& b = bufs[(size_t)i];
            for (const Buf* x : {&b.in, &b.mid, &b.out, &b.work})
                if (x->base && (uintptr_t)p >= x->base && (uintptr_t)p < x->base + x->bytes) return i;
        }
        return -1;
    };
    auto ok_range = [&](int item, uintptr_t lo, size_t len) {
        const ItemBufs& b = bufs[(size_t)item];
        return inside(lo, len, b.in) || inside(lo, len, b.mid) || inside(lo, len, b.out) || inside(lo, len, b.work);
    };
    for (int k = 0; k < nt; ++k) {
        const BatchTask& t = tab.tasks[(size_t)k];
        const int item = owner(t.in);
        if (item < 0 || owner(t.out) != item) return fail("task buffers belong to no item / two items");
        const Plan& p = plans[(size_t)item];
        const int es = 2 * p.elem;  // complex element
        for (int tile = 0; tile < t.ntiles; ++tile) {
            uintptr_t lo;
            size_t len;
            bool good = true;
            switch (t.kind) {
            case kBkPlaneR2C:
            case kBkPlaneC2R: {
                const int64_t p0 = (int64_t)tile * t.a0;
                const int64_t np = std::min<int64_t>(t.a0, t.i0 - p0);
                if (np < 1) return fail("plane tile past the end");
                const int64_t rin = t.kind == kBkPlaneR2C ? p.n1 * p.h : p.n1 * p.H;
                const int64_t rout = t.kind == kBkPlaneR2C ? p.n1 * p.H : p.n1 * p.h;
                span(t.in, p0 * rin, np * rin, es, lo, len);
                good = good && ok_range(item, lo, len);
                span(t.out, p0 * rout, np * rout, es, lo, len);
                good = good && ok_range(item, lo, len);
                const int64_t ept = t.big ? (p.elem == 8 ? Tier<double>::kEptBig : Tier<float>::kEptBig)
                                          : (p.elem == 8 ? 8 : 16);
                if (np * p.n1 * p.H > (int64_t)kNtSmall * ept) return fail("plane tile too big");
                break;
            }
            case kBkRowsR2C:
            case kBkRowsC2R: {
                const int64_t r0 = (int64_t)tile * t.a0;
                const int64_t rows = std::min<int64_t>(t.a0, t.i0 - r0);
                if (rows < 1) return fail("rows tile past the end");
                const int64_t win = t.kind == kBkRowsR2C ? p.h : p.H, wout = t.kind == kBkRowsR2C ? p.H : p.h;
                span(t.in, r0 * win, rows * win, es, lo, len);
                good = good && ok_range(item, lo, len);
                span(t.out, r0 * wout, rows * wout, es, lo, len);
                good = good && ok_range(item, lo, len);
                if (rows * p.h > (int64_t)kNtSmall * (p.elem == 8 ? 8 : 16)) return fail("rows tile too big");
                if ((int64_t)rows * p.Hs * es > (int64_t)tab.lds) return fail("rows tile over its LDS");
                break;
            }
            default: {
                const int W = t.a0;
                const int b = tile / t.a1;
                const int64_t c0 = (int64_t)(tile - b * t.a1) * W;
                const int64_t width = std::min<int64_t>(W, t.i1 - c0);
                if (width < 1) return fail("column tile past the end");
                const int64_t nrows = (t.s0 == p.d_sched) ? p.n0 : p.n1;
                const int64_t off = (int64_t)b * t.i2 + c0;
                span(t.in, off, (nrows - 1) * t.i0 + width, es, lo, len);
                good = good && ok_range(item, lo, len);
                span(t.out, off, (nrows - 1) * t.i0 + width, es, lo, len);
                good = good && ok_range(item, lo, len);
                if (nrows * W > (int64_t)kNtSmall * (p.elem == 8 ? 8 : 16)) return fail("column tile too big");
                break;
            }
            }
            if (!good) return fail("task " + std::to_string(k) + " tile " + std::to_string(tile) + " outside its buffers");
        }
    }

    if (tab.levels) {
        // stream order is the level mode's only synchronisation: nothing to run
        printf("ok levels %d %d %lld %zu\n", nt, (int)tab.launches.size(), (long long)tab.tickets, tab.lds);
        return 0;
    }

    // 3. the ticket protocol on G threads
    std::vector<std::atomic<int>> ticket((size_t)nq);
    std::atomic<int> exited{0}, err{0}, loop_err{0}, unbounded{0}, wait_err{0}, skipped{0};
    std::atomic<long long> iterations{0};
    std::vector<std::atomic<int>> done((size_t)nt);
    std::vector<std::vector<std::atomic<int>>> runs((size_t)nq);
    for (auto& t : ticket) t.store(0);
    for (auto& d : done) d.store(0);
    for (int q = 0; q < nq; ++q) {
        std::vector<std::atomic<int>> v((size_t)tab.queue_tickets[(size_t)q]);
        for (auto& r : v) r.store(0);
        runs[(size_t)q].swap(v);
    }
    std::vector<int> item_xcd((size_t)n, -1);  // XCD that ran the item's first tile (pinned check)
    std::vector<int> task_item((size_t)nt, -1);
    for (int k = 0; k < nt; ++k) task_item[(size_t)k] = owner(tab.tasks[(size_t)k].in);
    std::mutex mu;
    const auto t0 = std::chrono::steady_clock::now();
    auto wg = [&](int g) {
        const int xcc = g % xcds;
        const int q = tab.qmap[xcc];
        const int tb = tab.task_begin[(size_t)q], nqk = tab.task_begin[(size_t)q + 1] - tb;
        const int32_t* firsts = tab.firsts.data() + tb + q;
        const int total = firsts[nqk];
        // thread 0's next-ticket word: kept (registers), or lost (reads 0,
        // writes dropped)
        struct Word {
            bool lost;
            int v;
            int get() const { return lost ? 0 : v; }
            void set(int x) { if (!lost) v = x; }
        } nxt{state_lost, 0};
        nxt.set(ticket[(size_t)q].fetch_add(1));
        int cur = 0, checked = -1, failed = -1;
        long long iters = 0;
        for (;;) {
            ++iters;
            if (bounded && iters > (long long)total + 1) {
                loop_err.fetch_add(1);  // the kernel's bound: error bit, leave
                break;
            }
            if (!bounded && iters > 1000LL * (total + 1)) {
                unbounded.fetch_add(1);
                break;
            }
            const int t = nxt.get();
            if (t >= total) break;
            nxt.set(ticket[(size_t)q].fetch_add(1));
            if (state_lost) cur = 0;  // the search state is lost the same way
            if (firsts[cur + 1] <= t) {
                int lo = cur + 1, step = 1;
                while (lo + step < nqk && firsts[lo + step] <= t) {
                    lo += step;
                    step *= 2;
                }
                int hi = lo + step < nqk ? lo + step : nqk;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (firsts[mid] <= t) lo = mid;
                    else hi = mid;
                }
                cur = lo;
            }
            if (!(firsts[cur] <= t && t < firsts[cur + 1])) {
                err.store(1);
                break;
            }
            const int k = tb + cur;
            const BatchTask& tk = tab.tasks[(size_t)k];
            if (k != checked) {
                checked = k;
                if (tk.dep >= 0 && spin >= 0) {
                    // the kernel's bounded wait
                    bool ok = false;
                    for (int it = 0; it < spin; ++it) {
                        if (done[(size_t)tk.dep].load() >= tk.dep_tiles) {
                            ok = true;
                            break;
                        }
                        if (wait_err.load()) break;
                        std::this_thread::yield();
                    }
                    if (!ok) {
                        wait_err.store(1);
                        failed = k;
                    }
                } else if (tk.dep >= 0) {
                    while (done[(size_t)tk.dep].load() < tk.dep_tiles) {
                        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(60)) {
                            err.store(2);
                            exited.fetch_add(1);
                            return;
                        }
                        std::this_thread::yield();
                    }
                }
            }
            if (failed == k) {
                // the tile is skipped and still counts itself done
                skipped.fetch_add(1);
                done[(size_t)k].fetch_add(1);
                runs[(size_t)q][(size_t)t].fetch_add(1);
                continue;
            }
            if (tk.dep >= 0 && done[(size_t)tk.dep].load() != tk.dep_tiles) err.store(3);
            if (tab.pinned) {
                std::lock_guard<std::mutex> lk(mu);
                int& x = item_xcd[(size_t)task_item[(size_t)k]];
                if (x < 0) x = xcc;
                else if (x != xcc) err.store(4);
            }
            runs[(size_t)q][(size_t)t].fetch_add(1);
            done[(size_t)k].fetch_add(1);
        }
        iterations.fetch_add(iters);
        exited.fetch_add(1);
    };
    std::vector<std::thread> th;
    for (int g = 0; g < G; ++g) th.emplace_back(wg, g);
    for (auto& x : th) x.join();
    if (state_lost) {
        if (exited.load() != G) return fail("a workgroup did not leave");
        if (unbounded.load()) {
            printf("unbounded %d\n", unbounded.load());
            return 3;
        }
        if (loop_err.load() != G) return fail("lost state without the loop error bit");
        printf("bounded %lld\n", iterations.load());
        return 0;
    }
    if (loop_err.load() || unbounded.load()) return fail("the iteration bound ended a correct launch");
    if (spin >= 0) {
        if (exited.load() != G) return fail("a workgroup did not leave");
        if (err.load()) return fail("protocol error " + std::to_string(err.load()));
        for (int q = 0; q < nq; ++q)
            for (size_t t = 0; t < runs[(size_t)q].size(); ++t)
                if (runs[(size_t)q][t].load() != 1) return fail("a ticket ran more or less than once");
        if (wait_err.load()) {
            printf("errbit %d\n", skipped.load());
            return 0;
        }
    }
    if (err.load()) return fail("protocol error " + std::to_string(err.load()));
    if (exited.load() != G) return fail("a workgroup did not leave");
    for (int q = 0; q < nq; ++q)
        for (size_t t = 0; t < runs[(size_t)q].size(); ++t)
            if (runs[(size_t)q][t].load() != 1)
                return fail("queue " + std::to_string(q) + " ticket " + std::to_string(t) + " ran " +
                            std::to_string(runs[(size_t)q][t].load()) + " times");
    for (int k = 0; k < nt; ++k)
        if (done[(size_t)k].load() != tab.tasks[(size_t)k].ntiles) return fail("task not complete");
    printf("ok %d %lld %zu %d\n", nt, (long long)tab.tickets, tab.lds, tab.pinned ? 1 : 0);
    return 0;
}
