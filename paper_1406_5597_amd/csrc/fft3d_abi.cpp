// fft3d_abi.cpp -- the extern "C" entry points of libfft3d (see include/fft3d.h).
//
// Validation, error codes and thread-local messages; plan creation (the only
// place the library allocates device memory); and the call sequences of the
// forward and inverse transforms.  Nothing here synchronises the device
// except plan creation, which uploads the twiddle table.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fft3d.h"
#include "fft3d_batch_host.hpp"
#include "fft3d_internal.hpp"

struct fft3d_batch_s {
    int nitems = 0;
    int device = -1;
    fft3d::BatchTable tab;
    unsigned grid = 0;
    void* image = nullptr;  // task image (device)
    int* ctr = nullptr;     // counter block (device)
    struct {
        const void* image;
        int* ctr;
        int spin;
    } args{};
    // level mode: the arguments of each launch's graph node
    struct LevelArgs {
        const void* tasks;
        const void* firsts;
        int ntasks;
    };
    std::vector<LevelArgs> level_args;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~fft3d_batch_s()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (image) (void)hipFree(image);
        if (ctr) (void)hipFree(ctr);
    }
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg)
{
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    std::string m = std::string(where) + ": " + hipGetErrorString(e);
    return fail(FFT3D_ERR_HIP, m);
}

std::once_flag g_init_once;
hipError_t g_init_status = hipSuccess;

bool overlaps(const void* a, size_t na, const void* b, size_t nb)
{
    uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Checks shared by the transforms: a plan with device state, used on its own
// device.
int check_plan(const fft3d_plan_s* h, const char* who)
{
    if (!h) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": plan is NULL");
    if (!h->p.has_device)
        return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": plan was created host-only");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, who);
    if (dev != h->p.device) {
        char b[160];
        snprintf(b, sizeof b, "%s: plan belongs to device %d but device %d is current", who, h->p.device, dev);
        return fail(FFT3D_ERR_INVALID_ARG, b);
    }
    return FFT3D_OK;
}

int check_ptr(const void* ptr, int align, const char* who, const char* name)
{
    if (!ptr) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": " + name + " is NULL");
    if ((uintptr_t)ptr % (uintptr_t)align)
        return fail(FFT3D_ERR_ALIGN, std::string(who) + ": " + name + " is not aligned to the complex type");
    return FFT3D_OK;
}

size_t real_bytes(const fft3d::Plan& p) { return (size_t)p.N * (size_t)p.elem; }
size_t cplx_bytes(const fft3d::Plan& p) { return (size_t)p.M * 2 * (size_t)p.elem; }

int validate_r2c(const fft3d_plan_s* h, const void* x, const void* X)
{
    const char* who = "fft3d_r2c";
    int rc = check_plan(h, who);
    if (rc) return rc;
    const int a = 2 * h->p.elem;
    if ((rc = check_ptr(x, a, who, "x"))) return rc;
    if ((rc = check_ptr(X, a, who, "X"))) return rc;
    if (overlaps(x, real_bytes(h->p), X, cplx_bytes(h->p)))
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_r2c: x and X overlap (out-of-place only)");
    return FFT3D_OK;
}

int validate_c2r(const fft3d_plan_s* h, const void* X, const void* y, const void* work)
{
    const char* who = "fft3d_c2r";
    int rc = check_plan(h, who);
    if (rc) return rc;
    const int a = 2 * h->p.elem;
    if ((rc = check_ptr(X, a, who, "X"))) return rc;
    if ((rc = check_ptr(y, a, who, "y"))) return rc;
    const size_t cb = cplx_bytes(h->p), rb = real_bytes(h->p);
    if (overlaps(X, cb, y, rb)) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_c2r: X and y overlap");
    if (work) {
        if ((rc = check_ptr(work, a, who, "work"))) return rc;
        if (overlaps(work, cb, X, cb) || overlaps(work, cb, y, rb))
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_c2r: work overlaps X or y");
    }
    return FFT3D_OK;
}

// Forward: step 1 (plane r2c), then step 3 (n0 columns, in place on X).
int enqueue_r2c(const fft3d::Plan& p, const void* x, void* X, hipStream_t s)
{
    hipError_t e;
    if (p.fused_plane) {
        e = fft3d::launch_plane_r2c(p, x, X, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_r2c plane kernel");
    } else if (p.coop) {
        e = fft3d::launch_plane_coop(p, x, X, false, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_r2c cooperative plane kernel");
    } else {
        // rows kernel, then the n1 columns of the planes in place
        e = fft3d::launch_rows_r2c(p, x, X, p.n0 * p.n1, p.rev & 1, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_r2c rows kernel");
        if (p.n1 > 1) {
            e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, X, X, false, (p.rev >> 1) & 1, s);
            if (e != hipSuccess) return hip_fail(e, "fft3d_r2c n1 columns kernel");
        }
    }
    if (p.n0 > 1) {
        e = fft3d::launch_cols(p, p.pass0, 0, p.off_ax0, X, X, false, (p.rev >> 2) & 1, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_r2c n0 columns kernel");
    }
    return FFT3D_OK;
}

// Inverse: step 3 reversed (n0 columns, into work or in place), then step 1
// reversed (plane c2r).
int enqueue_c2r(const fft3d::Plan& p, void* X, void* y, void* work, hipStream_t s)
{
    hipError_t e;
    void* scratch = work ? work : X;
    const void* cur = X;
    if (p.n0 > 1) {
        e = fft3d::launch_cols(p, p.pass0, 0, p.off_ax0, cur, scratch, true, (p.rev >> 3) & 1, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_c2r n0 columns kernel");
        cur = scratch;
    }
    if (p.fused_plane) {
        e = fft3d::launch_plane_c2r(p, cur, y, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_c2r plane kernel");
    } else if (p.coop) {
        // the cooperative kernel transforms the n1 columns in place: with
        // work, first bring the spectrum there if the n0 pass did not
        if (cur == X && work) {
            e = hipMemcpyAsync(work, X, cplx_bytes(p), hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return hip_fail(e, "fft3d_c2r copy to work");
            cur = work;
        }
        e = fft3d::launch_plane_coop(p, cur, y, true, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_c2r cooperative plane kernel");
    } else {
        const void* src = cur;
        if (p.n1 > 1) {
            e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, src, scratch, true, (p.rev >> 4) & 1, s);
            if (e != hipSuccess) return hip_fail(e, "fft3d_c2r n1 columns kernel");
            src = scratch;
        }
        e = fft3d::launch_rows_c2r(p, src, y, p.n0 * p.n1, (p.rev >> 5) & 1, s);
        if (e != hipSuccess) return hip_fail(e, "fft3d_c2r rows kernel");
    }
    return FFT3D_OK;
}

template <typename T> void round_table(const std::vector<long double>& src, std::vector<T>& dst)
{
    dst.resize(src.size());
    for (size_t i = 0; i < src.size(); ++i) dst[i] = (T)src[i];
}

// Buffers an item writes and reads, for the cross-item overlap check.
struct Range {
    const void* p;
    size_t n;
    bool written;
};

void item_ranges(const fft3d_batch_item& it, std::vector<Range>& r)
{
    const fft3d::Plan& p = it.plan->p;
    const size_t rb = real_bytes(p), cb = cplx_bytes(p);
    switch (it.dir) {
    case FFT3D_R2C:
        r.push_back({it.in, rb, false});
        r.push_back({it.out, cb, true});
        break;
    case FFT3D_C2R:
        r.push_back({it.in, cb, it.work == nullptr});
        r.push_back({it.out, rb, true});
        if (it.work) r.push_back({it.work, cb, true});
        break;
    default:
        r.push_back({it.in, rb, false});
        r.push_back({it.mid, cb, true});
        r.push_back({it.out, rb, true});
        if (it.work) r.push_back({it.work, cb, true});
        break;
    }
}

// Every item valid on its own, and no item writes memory another item uses.
int validate_batch(const fft3d_batch_item* items, int n, const char* who)
{
    if (n < 0 || (n > 0 && !items)) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": bad item array");
    for (int i = 0; i < n; ++i) {
        const fft3d_batch_item& it = items[i];
        int rc;
        switch (it.dir) {
        case FFT3D_R2C: rc = validate_r2c(it.plan, it.in, it.out); break;
        case FFT3D_C2R: rc = validate_c2r(it.plan, it.in, it.out, it.work); break;
        case FFT3D_ROUNDTRIP:
            rc = validate_r2c(it.plan, it.in, it.mid);
            if (!rc) rc = validate_c2r(it.plan, it.mid, it.out, it.work);
            if (!rc && it.plan && overlaps(it.in, real_bytes(it.plan->p), it.out, real_bytes(it.plan->p)))
                rc = fail(FFT3D_ERR_INVALID_ARG, "in and out overlap");
            break;
        default: rc = fail(FFT3D_ERR_INVALID_ARG, "unknown direction"); break;
        }
        if (rc) {
            char b[96];
            snprintf(b, sizeof b, "%s: item %d: ", who, i);
            g_last_error = b + g_last_error;
            return rc;
        }
    }
    // sweep over the ranges in address order: each range against the ranges
    // that start before it ends
    std::vector<Range> all;
    std::vector<int> owner;
    for (int i = 0; i < n; ++i) {
        item_ranges(items[i], all);
        owner.resize(all.size(), i);
    }
    std::vector<size_t> order(all.size());
    for (size_t a = 0; a < order.size(); ++a) order[a] = a;
    std::sort(order.begin(), order.end(),
              [&](size_t a, size_t b) { return (uintptr_t)all[a].p < (uintptr_t)all[b].p; });
    for (size_t u = 0; u < order.size(); ++u) {
        const Range& ra = all[order[u]];
        const uintptr_t end = (uintptr_t)ra.p + ra.n;
        for (size_t v = u + 1; v < order.size() && (uintptr_t)all[order[v]].p < end; ++v) {
            const Range& rb = all[order[v]];
            const int ia = owner[order[u]], ib = owner[order[v]];
            if (ia != ib && (ra.written || rb.written)) {
                char m[160];
                snprintf(m, sizeof m, "%s: item %d writes memory that item %d uses (items run concurrently)", who,
                         ra.written ? ia : ib, ra.written ? ib : ia);
                return fail(FFT3D_ERR_INVALID_ARG, m);
            }
        }
    }
    return FFT3D_OK;
}

std::vector<fft3d::BatchSpec> batch_specs(const fft3d_batch_item* items, int n)
{
    std::vector<fft3d::BatchSpec> v((size_t)n);
    for (int i = 0; i < n; ++i)
        v[(size_t)i] = {&items[i].plan->p, items[i].dir, items[i].in, items[i].mid, items[i].out, items[i].work};
    return v;
}

// Batch options for a device: its XCDs, and the batch tuning's launch shape
// (mode, ticket order, tile widening, workgroups per CU, spin limit).
fft3d::BatchOptions batch_options(int device, const fft3d_batch_tuning* bt = nullptr)
{
    fft3d::BatchOptions o;
    o.xcc_ids = fft3d::device_xcc_ids(device);
    if (bt) {
        o.mode = bt->mode;
        o.lag = bt->lag;
        o.widen = bt->widen != 2;
        o.wg_per_cu = bt->wg_per_cu;
        o.spin_limit = bt->spin_limit == 0 ? fft3d::kBatchSpinLimit : std::max(0, bt->spin_limit);
    }
    return o;
}

int check_batch_tuning(const fft3d_batch_tuning* bt, const char* who)
{
    if (!bt) return FFT3D_OK;
    if (bt->mode < 0 || bt->mode > 4) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": mode must be 0..4");
    if (bt->lag < 0) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": lag must be >= 0");
    if (bt->widen < 0 || bt->widen > 2) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": widen must be 0, 1 or 2");
    if (bt->wg_per_cu < 0 || bt->wg_per_cu > 16)
        return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": wg_per_cu must be 0..16");
    return FFT3D_OK;
}

}  // namespace

namespace fft3d {
void set_last_error(const std::string& m) { g_last_error = m; }
}  // namespace fft3d

extern "C" {

int fft3d_version(void) { return 100; }

int fft3d_plan_tuned(int64_t n0, int64_t n1, int64_t n2, int dtype, int flags, const fft3d_tuning* t,
                     fft3d_plan_t* out)
{
    if (!out) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_plan: out is NULL");
    *out = nullptr;
    if (flags & ~(FFT3D_PLAN_HOST_ONLY | FFT3D_PLAN_COOP_PLANE | FFT3D_PLAN_TUNED))
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_plan: unknown flags");
    // FFT3D_PLAN_TUNED: the process's tuning table entry for this shape on
    // the current device's architecture, if there is one
    fft3d_tuning looked{};
    if (!t && (flags & FFT3D_PLAN_TUNED) && fft3d_tune_lookup(n0, n1, n2, dtype, &looked) == 1) t = &looked;
    fft3d_plan_s* h = new (std::nothrow) fft3d_plan_s;
    if (!h) return fail(FFT3D_ERR_NOMEM, "fft3d_plan: out of host memory");
    std::string why;
    int rc = fft3d::plan_build_host(h->p, n0, n1, n2, dtype, flags, t, why);
    if (rc) {
        delete h;
        return fail(rc, "fft3d_plan: " + why);
    }
    if (!(flags & FFT3D_PLAN_HOST_ONLY)) {
        std::call_once(g_init_once, [] { g_init_status = fft3d::kernels_init(); });
        if (g_init_status != hipSuccess) {
            delete h;
            return hip_fail(g_init_status, "fft3d_plan: kernel set-up");
        }
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) {
            delete h;
            return hip_fail(e, "fft3d_plan: hipGetDevice");
        }
        const fft3d::Plan& p = h->p;
        size_t bytes = (size_t)std::max<int64_t>(p.tw_count, 1) * 2 * (size_t)p.elem;
        std::vector<float> tf;
        std::vector<double> td;
        const void* host;
        if (p.dtype == FFT3D_F64) {
            round_table(p.tw_host, td);
            td.resize(bytes / sizeof(double), 0.0);
            host = td.data();
        } else {
            round_table(p.tw_host, tf);
            tf.resize(bytes / sizeof(float), 0.0f);
            host = tf.data();
        }
        void* d = nullptr;
        e = hipMalloc(&d, bytes);
        if (e != hipSuccess) {
            delete h;
            return fail(FFT3D_ERR_NOMEM, std::string("fft3d_plan: hipMalloc of twiddles: ") + hipGetErrorString(e));
        }
        e = hipMemcpy(d, host, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(d);
            delete h;
            return hip_fail(e, "fft3d_plan: twiddle upload");
        }
        h->p.d_tw = d;
        h->p.device = dev;
        h->p.has_device = true;
        e = hipDeviceGetAttribute(&h->p.cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e != hipSuccess) {
            fft3d_plan_destroy(h);
            return hip_fail(e, "fft3d_plan: device attributes");
        }
        const fft3d::AxisSched sched[3] = {p.ax0, p.ax1, p.ax2h};
        e = hipMalloc(&h->p.d_sched, sizeof sched);
        if (e != hipSuccess) {
            fft3d_plan_destroy(h);
            return fail(FFT3D_ERR_NOMEM, std::string("fft3d_plan: hipMalloc of schedules: ") + hipGetErrorString(e));
        }
        e = hipMemcpy(h->p.d_sched, sched, sizeof sched, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            fft3d_plan_destroy(h);
            return hip_fail(e, "fft3d_plan: schedule upload");
        }
        e = fft3d::coop_setup(h->p);
        if (e != hipSuccess) {
            fft3d_plan_destroy(h);
            return hip_fail(e, "fft3d_plan: cooperative plane step set-up");
        }
    }
    *out = h;
    return FFT3D_OK;
}

int fft3d_plan_ex(int64_t n0, int64_t n1, int64_t n2, int dtype, int flags, fft3d_plan_t* out)
{
    return fft3d_plan_tuned(n0, n1, n2, dtype, flags, nullptr, out);
}

int fft3d_plan(int64_t n0, int64_t n1, int64_t n2, int dtype, fft3d_plan_t* out)
{
    return fft3d_plan_ex(n0, n1, n2, dtype, 0, out);
}

int fft3d_plan_destroy(fft3d_plan_t h)
{
    if (!h) return FFT3D_OK;
    int rc = FFT3D_OK;
    if (h->p.d_tw) {
        hipError_t e = hipFree(h->p.d_tw);
        if (e != hipSuccess) rc = hip_fail(e, "fft3d_plan_destroy");
    }
    if (h->p.d_ctr) {
        hipError_t e = hipFree(h->p.d_ctr);
        if (e != hipSuccess) rc = hip_fail(e, "fft3d_plan_destroy");
    }
    if (h->p.d_sched) {
        hipError_t e = hipFree(h->p.d_sched);
        if (e != hipSuccess) rc = hip_fail(e, "fft3d_plan_destroy");
    }
    delete h;
    return rc;
}

size_t fft3d_work_bytes(fft3d_plan_t h) { return h ? cplx_bytes(h->p) : 0; }
size_t fft3d_real_bytes(fft3d_plan_t h) { return h ? real_bytes(h->p) : 0; }
size_t fft3d_complex_bytes(fft3d_plan_t h) { return h ? cplx_bytes(h->p) : 0; }

int fft3d_r2c(fft3d_plan_t h, const void* x, void* X, hipStream_t s)
{
    int rc = validate_r2c(h, x, X);
    if (rc) return rc;
    return enqueue_r2c(h->p, x, X, s);
}

int fft3d_c2r(fft3d_plan_t h, void* X, void* y, void* work, hipStream_t s)
{
    int rc = validate_c2r(h, X, y, work);
    if (rc) return rc;
    return enqueue_c2r(h->p, X, y, work, s);
}

int fft3d_r2c_transposed(fft3d_plan_t h, const void* x, void* Xt, void* work, hipStream_t s)
{
    const char* who = "fft3d_r2c_transposed";
    int rc = validate_r2c(h, x, Xt);
    if (rc) return rc;
    const fft3d::Plan& p = h->p;
    if ((rc = check_ptr(work, 2 * p.elem, who, "work"))) return rc;
    const size_t cb = cplx_bytes(p);
    if (overlaps(work, cb, Xt, cb) || overlaps(work, cb, x, real_bytes(p)))
        return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": work overlaps x or Xt");
    // step 1 into work: the plane step of the transpose-free path (its own
    // n0 pass is left out)
    hipError_t e;
    if (p.fused_plane) {
        e = fft3d::launch_plane_r2c(p, x, work, s);
    } else if (p.coop) {
        e = fft3d::launch_plane_coop(p, x, work, false, s);
    } else {
        e = fft3d::launch_rows_r2c(p, x, work, p.n0 * p.n1, 0, s);
        if (e == hipSuccess && p.n1 > 1) e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, work, work, false, 1, s);
    }
    // step 2: the transpose; step 3: n0 columns of the transposed layout
    if (e == hipSuccess) e = fft3d::launch_swap01(p, work, Xt, p.n0, p.n1, s);
    if (e == hipSuccess && p.n0 > 1) e = fft3d::launch_cols(p, p.pass0t, 0, p.off_ax0, Xt, Xt, false, 1, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

int fft3d_c2r_transposed(fft3d_plan_t h, void* Xt, void* y, void* work, hipStream_t s)
{
    const char* who = "fft3d_c2r_transposed";
    int rc = validate_c2r(h, Xt, y, work);
    if (rc) return rc;
    if (!work) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": work is required");
    const fft3d::Plan& p = h->p;
    hipError_t e = hipSuccess;
    const void* t = Xt;
    if (p.n0 > 1) {
        e = fft3d::launch_cols(p, p.pass0t, 0, p.off_ax0, Xt, work, true, 1, s);
        t = work;
    }
    if (e == hipSuccess) e = fft3d::launch_swap01(p, t, t == work ? Xt : work, p.n1, p.n0, s);
    void* nat = t == work ? Xt : work;  // natural-order spectrum after the exchange
    if (e == hipSuccess) {
        if (p.fused_plane) {
            e = fft3d::launch_plane_c2r(p, nat, y, s);
        } else if (p.coop) {
            e = fft3d::launch_plane_coop(p, nat, y, true, s);
        } else {
            if (p.n1 > 1) e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, nat, nat, true, 1, s);
            if (e == hipSuccess) e = fft3d::launch_rows_c2r(p, nat, y, p.n0 * p.n1, 0, s);
        }
    }
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

namespace {

// kmax -> the kernels' box: an axis whose cut keeps every index is not cut.
int pruned_box(const fft3d::Plan& p, const int64_t* kmax, const char* who, fft3d::PrunedBox& b)
{
    if (!kmax) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": kmax is NULL");
    if (p.n2 % 2 != 0) return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": odd n2 is not supported");
    const int64_t K0 = kmax[0], K1 = kmax[1], K2 = kmax[2];
    b.K0 = (K0 < 0 || 2 * K0 + 1 >= p.n0) ? -1 : (int)K0;
    b.K1 = (K1 < 0 || 2 * K1 + 1 >= p.n1) ? -1 : (int)K1;
    b.K2 = (K2 < 0 || K2 >= p.h) ? (int)p.h : (int)K2;
    return FFT3D_OK;
}

}  // namespace

int fft3d_r2c_pruned(fft3d_plan_t h, const void* x, void* X, const int64_t kmax[3], hipStream_t s)
{
    const char* who = "fft3d_r2c_pruned";
    int rc = validate_r2c(h, x, X);
    if (rc) return rc;
    fft3d::PrunedBox b;
    if ((rc = pruned_box(h->p, kmax, who, b))) return rc;
    const hipError_t e = fft3d::launch_pruned_r2c(h->p, x, X, b, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

int fft3d_c2r_pruned(fft3d_plan_t h, void* X, void* y, void* work, const int64_t kmax[3], hipStream_t s)
{
    const char* who = "fft3d_c2r_pruned";
    int rc = validate_c2r(h, X, y, work);
    if (rc) return rc;
    fft3d::PrunedBox b;
    if ((rc = pruned_box(h->p, kmax, who, b))) return rc;
    const hipError_t e = fft3d::launch_pruned_c2r(h->p, X, y, work, b, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

int fft3d_r2c_inplace(fft3d_plan_t h, void* buf, hipStream_t s)
{
    const char* who = "fft3d_r2c_inplace";
    int rc = check_plan(h, who);
    if (rc) return rc;
    const fft3d::Plan& p = h->p;
    if ((rc = check_ptr(buf, 2 * p.elem, who, "buf"))) return rc;
    // each rows / plane tile reads all of its rows before it writes them back
    // as bins, and the column passes run in place anyway
    hipError_t e;
    if (p.fused_plane) {
        e = fft3d::launch_plane_r2c(p, buf, buf, s, true);
    } else {
        e = fft3d::launch_rows_r2c(p, buf, buf, p.n0 * p.n1, p.rev & 1, s, true);
        if (e == hipSuccess && p.n1 > 1)
            e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, buf, buf, false, (p.rev >> 1) & 1, s);
    }
    if (e == hipSuccess && p.n0 > 1)
        e = fft3d::launch_cols(p, p.pass0, 0, p.off_ax0, buf, buf, false, (p.rev >> 2) & 1, s);
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

int fft3d_c2r_inplace(fft3d_plan_t h, void* buf, hipStream_t s)
{
    const char* who = "fft3d_c2r_inplace";
    int rc = check_plan(h, who);
    if (rc) return rc;
    const fft3d::Plan& p = h->p;
    if ((rc = check_ptr(buf, 2 * p.elem, who, "buf"))) return rc;
    hipError_t e = hipSuccess;
    if (p.n0 > 1) e = fft3d::launch_cols(p, p.pass0, 0, p.off_ax0, buf, buf, true, (p.rev >> 3) & 1, s);
    if (e == hipSuccess) {
        if (p.fused_plane) {
            e = fft3d::launch_plane_c2r(p, buf, buf, s, true);
        } else {
            if (p.n1 > 1) e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, buf, buf, true, (p.rev >> 4) & 1, s);
            if (e == hipSuccess) e = fft3d::launch_rows_c2r(p, buf, buf, p.n0 * p.n1, (p.rev >> 5) & 1, s, true);
        }
    }
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

int fft3d_init(void)
{
    std::call_once(g_init_once, [] { g_init_status = fft3d::kernels_init(); });
    if (g_init_status != hipSuccess) return hip_fail(g_init_status, "fft3d_init: kernel set-up");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "fft3d_init: hipGetDevice");
    e = fft3d::ring_init(dev);
    if (e != hipSuccess) return fail(FFT3D_ERR_NOMEM, std::string("fft3d_init: batch ring: ") + hipGetErrorString(e));
    // the address of this device's copy of the static batch scratch
    e = fft3d::static_scratch_setup(dev);
    if (e != hipSuccess) return hip_fail(e, "fft3d_init: static batch scratch");
    return FFT3D_OK;
}

int fft3d_batch_submit(const fft3d_batch_item* items, int n, hipStream_t s)
{
    return fft3d_batch_submit_ex(items, n, 0, s);
}

namespace {

// The batched launch of fft3d_batch_submit_ex / _checked; *token (if not
// NULL) names the ring launches it staged, or -1 when it staged none.
int batch_submit_impl(const fft3d_batch_item* items, int n, int flags, hipStream_t s, int64_t* token)
{
    const char* who = "fft3d_batch_submit";
    if (token) *token = -1;
    if (flags & ~FFT3D_BATCH_SEQUENTIAL)
        return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": unknown flags");
    int rc = validate_batch(items, n, who);
    if (rc || n == 0) return rc;
    auto run_alone = [&](const fft3d_batch_item& it) {
        if (it.dir == FFT3D_R2C) return enqueue_r2c(it.plan->p, it.in, it.out, s);
        if (it.dir == FFT3D_C2R) return enqueue_c2r(it.plan->p, const_cast<void*>(it.in), it.out, it.work, s);
        int r = enqueue_r2c(it.plan->p, it.in, it.mid, s);
        return r ? r : enqueue_c2r(it.plan->p, it.mid, it.out, it.work, s);
    };
    if (flags & FFT3D_BATCH_SEQUENTIAL) {
        for (int i = 0; i < n; ++i)
            if ((rc = run_alone(items[i]))) return rc;
        return FFT3D_OK;
    }
    // items with radix-5/7 extents or odd n2 run their own kernels, after
    // the batched launch of the others (the batched kernel has only the 2/3
    // stages and the half-length rows)
    std::vector<fft3d_batch_item> even;
    even.reserve(n);
    for (int i = 0; i < n; ++i)
        if (items[i].plan->p.batchable()) even.push_back(items[i]);
    const int device = items[0].plan->p.device;
    if (!even.empty()) {
        if (!fft3d::ring_ready(device))
            return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": fft3d_init() has not been called on device " +
                                                   std::to_string(device));
        const fft3d::BatchOptions o = batch_options(device);
        // items in chunks whose task lists fit a ring slot (6 passes per item at most)
        const int chunk = fft3d::kRingTasks / 6;
        const int m = (int)even.size();
        std::vector<fft3d::BatchTable> tabs;
        for (int i0 = 0; i0 < m; i0 += chunk) {
            const int k = std::min(chunk, m - i0);
            std::vector<fft3d::BatchSpec> specs = batch_specs(even.data() + i0, k);
            tabs.emplace_back();
            if (const char* why = fft3d::build_batch_table(specs.data(), k, o, tabs.back()))
                return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": " + why);
        }
        const char* why = nullptr;
        int64_t seq = -1;
        hipError_t e = fft3d::ring_submit(device, tabs.data(), (int)tabs.size(), s, &seq, &why);
        if (e == hipErrorNotReady) return fail(FFT3D_ERR_BUSY, std::string(who) + ": " + why);
        if (why) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": " + why);
        if (e != hipSuccess) return hip_fail(e, who);
        if (token) *token = ((int64_t)device << 56) | ((int64_t)tabs.size() << 48) | seq;
    }
    for (int i = 0; i < n; ++i)
        if (!items[i].plan->p.batchable() && (rc = run_alone(items[i]))) return rc;
    return FFT3D_OK;
}

}  // namespace

int fft3d_batch_submit_ex(const fft3d_batch_item* items, int n, int flags, hipStream_t s)
{
    return batch_submit_impl(items, n, flags, s, nullptr);
}

int fft3d_batch_submit_checked(const fft3d_batch_item* items, int n, hipStream_t s, int64_t* token)
{
    if (!token) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_batch_submit_checked: token is NULL");
    return batch_submit_impl(items, n, 0, s, token);
}

int fft3d_batch_submit_static(const fft3d_batch_item* items, int n, int* status, hipStream_t s)
{
    const char* who = "fft3d_batch_submit_static";
    int rc = validate_batch(items, n, who);
    if (rc) return rc;
    if (status && ((uintptr_t)status & 3))
        return fail(FFT3D_ERR_ALIGN, std::string(who) + ": status is not aligned to int");
    if (n == 0) return FFT3D_OK;
    std::vector<fft3d_batch_item> even;
    even.reserve(n);
    for (int i = 0; i < n; ++i)
        if (items[i].plan->p.batchable()) even.push_back(items[i]);
    const int device = items[0].plan->p.device;
    hipError_t e = hipSuccess;
    if (!even.empty()) {
        if (!fft3d::static_scratch(device) || !fft3d::ring_ready(device))
            return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": fft3d_init() has not been called on device " +
                                                   std::to_string(device));
        const fft3d::BatchOptions o = batch_options(device);
        std::vector<fft3d::BatchSpec> specs = batch_specs(even.data(), (int)even.size());
        fft3d::BatchTable tab;
        if (const char* why = fft3d::build_batch_table(specs.data(), (int)even.size(), o, tab))
            return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": " + why);
        const int nt = (int)tab.tasks.size();
        if (nt > fft3d::kStaticTasks)
            return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": " + std::to_string(nt) +
                                                   " passes, more than the static scratch holds (" +
                                                   std::to_string(fft3d::kStaticTasks) + ")");
        const size_t img = fft3d::batch_image_bytes(tab);
        if (!tab.levels)  // the rule; the persistent form would need a counter block
            return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": runs the level mode only");
        if (img > fft3d::kStaticScratchBytes)
            return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": task image larger than the static scratch");
        // host staging: this thread's buffer (no device or pinned memory)
        thread_local std::vector<char> host;
        host.resize(img);
        fft3d::write_batch_image(tab, host.data());
        // the image, the level mode's launches (the rule; no counters, no
        // waits), and a clean status
        const void* dev = nullptr;
        static const int zero = 0;
        if ((e = fft3d::stage_static_image(device, host.data(), img, &dev, s)) != hipSuccess ||
            (e = fft3d::enqueue_batch_image(tab, 0, dev, nullptr, s)) != hipSuccess ||
            (status && (e = hipMemcpyAsync(status, &zero, sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess))
            return hip_fail(e, who);
    } else if (status) {
        // no batched launch: report a clean launch
        static const int zero = 0;
        if ((e = hipMemcpyAsync(status, &zero, sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
            return hip_fail(e, who);
    }
    for (int i = 0; i < n; ++i) {
        const fft3d_batch_item& it = items[i];
        if (it.plan->p.batchable()) continue;
        if (it.dir == FFT3D_R2C) rc = enqueue_r2c(it.plan->p, it.in, it.out, s);
        else if (it.dir == FFT3D_C2R) rc = enqueue_c2r(it.plan->p, const_cast<void*>(it.in), it.out, it.work, s);
        else {
            rc = enqueue_r2c(it.plan->p, it.in, it.mid, s);
            if (!rc) rc = enqueue_c2r(it.plan->p, it.mid, it.out, it.work, s);
        }
        if (rc) return rc;
    }
    return FFT3D_OK;
}

int fft3d_batch_check(int64_t token)
{
    if (token == -1) return 0;  // nothing was staged through the ring
    if (token < 0) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_batch_check: bad token");
    const int device = (int)(token >> 56);
    const int count = (int)((token >> 48) & 0xff);
    const int64_t seq = token & (((int64_t)1 << 48) - 1);
    const char* why = nullptr;
    const int r = fft3d::ring_status(device, seq, count, &why);
    if (r < 0 && why) return fail(r, std::string("fft3d_batch_check: ") + why);
    if (r == FFT3D_ERR_BUSY) return fail(r, "fft3d_batch_check: the launch has not finished");
    return r;
}

int fft3d_batch_create(const fft3d_batch_item* items, int n, int flags, fft3d_batch_t* out)
{
    return fft3d_batch_create_tuned(items, n, flags, nullptr, out);
}

int fft3d_batch_create_tuned(const fft3d_batch_item* items, int n, int flags, const fft3d_batch_tuning* bt,
                             fft3d_batch_t* out)
{
    const char* who = "fft3d_batch_create";
    if (!out) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": out is NULL");
    *out = nullptr;
    if (int rc = check_batch_tuning(bt, who)) return rc;
    if (flags & ~FFT3D_BATCH_DIRECT)
        return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": unknown flags");
    if (n < 1) return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": empty batch");
    int rc = validate_batch(items, n, who);
    if (rc) return rc;
    for (int i = 0; i < n; ++i)
        if (!items[i].plan->p.batchable())
            return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": item " + std::to_string(i) +
                                                   " has radix-5/7 extents or odd n2 (use fft3d_batch_submit)");
    if (!fft3d::ring_ready(items[0].plan->p.device))
        return fail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": fft3d_init() has not been called on device " +
                                               std::to_string(items[0].plan->p.device));
    fft3d::BatchOptions o = batch_options(items[0].plan->p.device, bt);
    std::unique_ptr<fft3d_batch_s> b(new (std::nothrow) fft3d_batch_s);
    if (!b) return fail(FFT3D_ERR_NOMEM, std::string(who) + ": out of host memory");
    b->nitems = n;
    b->device = items[0].plan->p.device;
    std::vector<fft3d::BatchSpec> specs = batch_specs(items, n);
    if (const char* why = fft3d::build_batch_table(specs.data(), n, o, b->tab))
        return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": " + why);
    const int nt = (int)b->tab.tasks.size();
    if (nt > fft3d::kRingTasks) return fail(FFT3D_ERR_UNSUPPORTED, std::string(who) + ": more than 4096 passes");
    // the persistent launch's workgroups (the level mode launches one per tile)
    hipError_t e = b->tab.levels ? hipSuccess : fft3d::batch_grid(b->tab, b->device, &b->grid);
    if (e != hipSuccess) return hip_fail(e, who);
    const size_t img = fft3d::batch_image_bytes(b->tab);
    const size_t ctr = (size_t)(fft3d::kBatchCtrHeader + nt) * sizeof(int);
    std::vector<char> host(img);
    fft3d::write_batch_image(b->tab, host.data());
    if ((e = hipMalloc(&b->image, img)) != hipSuccess || (e = hipMalloc(reinterpret_cast<void**>(&b->ctr), ctr)) != hipSuccess)
        return fail(FFT3D_ERR_NOMEM, std::string(who) + ": hipMalloc: " + hipGetErrorString(e));
    if ((e = hipMemcpy(b->image, host.data(), img, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(b->ctr, 0, ctr)) != hipSuccess)
        return hip_fail(e, who);
    if (!(flags & FFT3D_BATCH_DIRECT) && b->tab.levels) {
        // one kernel node per launch, each after the one before
        const size_t toff = fft3d::level_tasks_offset(b->tab);
        const fft3d::BatchTask* tasks =
            reinterpret_cast<const fft3d::BatchTask*>(static_cast<const char*>(b->image) + toff);
        const int32_t* firsts = static_cast<const int32_t*>(b->image);
        b->level_args.resize(b->tab.launches.size());
        if ((e = hipGraphCreate(&b->graph, 0)) != hipSuccess) return hip_fail(e, "fft3d_batch_create: graph");
        // each launch after the launches it reads from only: independent
        // chains (the two dtypes, fused and split items) are parallel branches
        std::vector<hipGraphNode_t> nodes;
        for (size_t i = 0; i < b->tab.launches.size(); ++i) {
            const fft3d::BatchLaunch& L = b->tab.launches[i];
            fft3d_batch_s::LevelArgs& a = b->level_args[i];
            a.tasks = tasks + L.task_begin;
            a.firsts = firsts + L.firsts_begin;
            a.ntasks = L.ntasks;
            void* params[] = {&a.tasks, &a.firsts, &a.ntasks};
            hipKernelNodeParams kp;
            memset(&kp, 0, sizeof kp);
            kp.func = const_cast<void*>(fft3d::level_kernel(L.kind, L.f64, L.big));
            kp.gridDim = dim3((unsigned)L.tiles);
            kp.blockDim = dim3(fft3d::kNtSmall);
            kp.sharedMemBytes = (unsigned)L.lds;
            kp.kernelParams = params;
            std::vector<hipGraphNode_t> deps;
            for (int d : L.deps) deps.push_back(nodes[(size_t)d]);
            hipGraphNode_t node;
            if ((e = hipGraphAddKernelNode(&node, b->graph, deps.empty() ? nullptr : deps.data(), deps.size(), &kp)) !=
                hipSuccess)
                return hip_fail(e, "fft3d_batch_create: graph");
            nodes.push_back(node);
        }
        if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
            return hip_fail(e, "fft3d_batch_create: graph");
    } else if (!(flags & FFT3D_BATCH_DIRECT)) {
        b->args.image = b->image;
        b->args.ctr = b->ctr;
        b->args.spin = b->tab.spin_limit;
        void* params[] = {&b->args.image, &b->args.ctr, &b->args.spin};
        hipKernelNodeParams kp;
        memset(&kp, 0, sizeof kp);
        kp.func = const_cast<void*>(fft3d::batch_kernel());
        kp.gridDim = dim3(b->grid);
        kp.blockDim = dim3(fft3d::kNtSmall);
        kp.sharedMemBytes = (unsigned)b->tab.lds;
        kp.kernelParams = params;
        hipGraphNode_t node;
        if ((e = hipGraphCreate(&b->graph, 0)) != hipSuccess ||
            (e = hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp)) != hipSuccess ||
            (e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess)
            return hip_fail(e, "fft3d_batch_create: graph");
    }
    *out = b.release();
    return FFT3D_OK;
}

int fft3d_batch_launch(fft3d_batch_t b, hipStream_t s)
{
    if (!b) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_batch_launch: batch is NULL");
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "fft3d_batch_launch");
    if (dev != b->device) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_batch_launch: batch belongs to another device");
    if (b->exec) e = hipGraphLaunch(b->exec, s);
    else e = fft3d::enqueue_batch_image(b->tab, b->grid, b->image, b->ctr, s);
    if (e != hipSuccess) return hip_fail(e, "fft3d_batch_launch");
    return FFT3D_OK;
}

int fft3d_batch_status(fft3d_batch_t b)
{
    if (!b) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_batch_status: batch is NULL");
    hipError_t e = hipDeviceSynchronize();
    int v = 0;
    if (e == hipSuccess) e = hipMemcpy(&v, b->ctr + fft3d::kBatchCtrStatus, sizeof v, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "fft3d_batch_status");
    return v;
}

int fft3d_batch_describe(fft3d_batch_t b, char* buf, size_t len)
{
    if (!b) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_batch_describe: batch is NULL");
    static const char* kinds[] = {"plane_r2c", "plane_c2r", "rows_r2c", "rows_c2r", "cols_fwd", "cols_inv"};
    std::string d = "{\"items\": " + std::to_string(b->nitems) + ", \"tickets\": " + std::to_string(b->tab.tickets) +
                    ", \"grid\": " + std::to_string(b->grid) + ", \"lds\": " + std::to_string(b->tab.lds) +
                    ", \"graph\": " + (b->exec ? "true" : "false") + ", \"mode\": \"" +
                    (b->tab.levels ? "levels" : b->tab.pinned ? "pinned" : "spread") + "\", \"queue_tickets\": [";
    for (int q = 0; q < b->tab.nqueues; ++q)
        d += (q ? ", " : "") + std::to_string(b->tab.queue_tickets[(size_t)q]);
    d += "], \"launches\": [";
    for (size_t i = 0; i < b->tab.launches.size(); ++i) {
        const fft3d::BatchLaunch& L = b->tab.launches[i];
        d += (i ? ", " : "");
        d += "[\"" + std::string(kinds[L.kind]) + "\", \"" + (L.f64 ? "f64" : "f32") + "\", " + std::to_string(L.ntasks) +
             ", " + std::to_string(L.tiles) + ", " + std::to_string(L.lds) + "]";
    }
    d += "], \"tasks\": [";
    for (size_t i = 0; i < b->tab.tasks.size(); ++i) {
        const fft3d::BatchTask& t = b->tab.tasks[i];
        d += (i ? ", " : "");
        d += "[\"" + std::string(kinds[t.kind]) + "\", \"" + (t.f64 ? "f64" : "f32") + "\", " +
             std::to_string(t.ntiles) + ", " + std::to_string(t.dep) + ", " + std::to_string(t.lds) + "]";
    }
    d += "]}";
    if (buf && len) {
        size_t m = std::min(len - 1, d.size());
        memcpy(buf, d.data(), m);
        buf[m] = '\0';
    }
    return (int)d.size();
}

int fft3d_batch_destroy(fft3d_batch_t b)
{
    if (!b) return FFT3D_OK;
    delete b;
    return FFT3D_OK;
}

int fft3d_run_pass(fft3d_plan_t h, int pass, const void* in, void* out, hipStream_t s)
{
    const char* who = "fft3d_run_pass";
    int rc = check_plan(h, who);
    if (rc) return rc;
    const fft3d::Plan& p = h->p;
    const int a = 2 * p.elem;
    if ((rc = check_ptr(in, a, who, "in"))) return rc;
    if ((rc = check_ptr(out, a, who, "out"))) return rc;
    const size_t cb = cplx_bytes(p), rb = real_bytes(p);
    hipError_t e = hipSuccess;
    switch (pass) {
    case FFT3D_PASS_PLANE_R2C:
        if (overlaps(in, rb, out, cb)) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: in and out overlap");
        e = p.fused_plane ? fft3d::launch_plane_r2c(p, in, out, s)
            : p.coop      ? fft3d::launch_plane_coop(p, in, out, false, s)
                          : fft3d::launch_rows_r2c(p, in, out, p.n0 * p.n1, p.rev & 1, s);
        break;
    case FFT3D_PASS_PLANE_C2R:
        // the cooperative plane c2r transforms the n1 columns of `in` in place
        if (overlaps(in, cb, out, rb)) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: in and out overlap");
        e = p.fused_plane ? fft3d::launch_plane_c2r(p, in, out, s)
            : p.coop      ? fft3d::launch_plane_coop(p, in, out, true, s)
                          : fft3d::launch_rows_c2r(p, in, out, p.n0 * p.n1, (p.rev >> 5) & 1, s);
        break;
    case FFT3D_PASS_N1_FWD:
    case FFT3D_PASS_N1_INV:
        if (p.fused_plane || p.coop || p.n1 == 1)
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: plan has no n1 pass");
        if (in != out && overlaps(in, cb, out, cb))
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: in and out partially overlap");
        e = fft3d::launch_cols(p, p.pass1, 1, p.off_ax1, in, out, pass == FFT3D_PASS_N1_INV,
                               pass == FFT3D_PASS_N1_INV ? (p.rev >> 4) & 1 : (p.rev >> 1) & 1, s);
        break;
    case FFT3D_PASS_N0_FWD:
    case FFT3D_PASS_N0_INV:
        if (p.n0 == 1) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: plan has no n0 pass");
        if (in != out && overlaps(in, cb, out, cb))
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: in and out partially overlap");
        e = fft3d::launch_cols(p, p.pass0, 0, p.off_ax0, in, out, pass == FFT3D_PASS_N0_INV,
                               pass == FFT3D_PASS_N0_INV ? (p.rev >> 3) & 1 : (p.rev >> 2) & 1, s);
        break;
    case FFT3D_PASS_SWAP01:
    case FFT3D_PASS_SWAP10:
        if (overlaps(in, cb, out, cb)) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: in and out overlap");
        e = pass == FFT3D_PASS_SWAP01 ? fft3d::launch_swap01(p, in, out, p.n0, p.n1, s)
                                      : fft3d::launch_swap01(p, in, out, p.n1, p.n0, s);
        break;
    case FFT3D_PASS_N0T_FWD:
    case FFT3D_PASS_N0T_INV:
        if (p.n0 == 1) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: plan has no n0 pass");
        if (in != out && overlaps(in, cb, out, cb))
            return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: in and out partially overlap");
        e = fft3d::launch_cols(p, p.pass0t, 0, p.off_ax0, in, out, pass == FFT3D_PASS_N0T_INV, 1, s);
        break;
    default: return fail(FFT3D_ERR_INVALID_ARG, "fft3d_run_pass: unknown pass");
    }
    if (e != hipSuccess) return hip_fail(e, who);
    return FFT3D_OK;
}

const char* fft3d_strerror(int code)
{
    switch (code) {
    case FFT3D_OK: return "success";
    case FFT3D_ERR_INVALID_ARG: return "invalid argument";
    case FFT3D_ERR_UNSUPPORTED: return "unsupported extents";
    case FFT3D_ERR_NOMEM: return "out of memory";
    case FFT3D_ERR_HIP: return "HIP runtime error";
    case FFT3D_ERR_BUDGET: return "over the memory budget";
    case FFT3D_ERR_ALIGN: return "misaligned pointer";
    case FFT3D_ERR_BUSY: return "busy: try again later";
    default: return "unknown error code";
    }
}

const char* fft3d_last_error(void) { return g_last_error.c_str(); }

int fft3d_plan_describe(fft3d_plan_t h, char* buf, size_t len)
{
    if (!h) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_plan_describe: plan is NULL");
    std::string d = h->p.describe();
    if (buf && len) {
        size_t n = std::min(len - 1, d.size());
        memcpy(buf, d.data(), n);
        buf[n] = '\0';
    }
    return (int)d.size();
}

int64_t fft3d_plan_twiddles(fft3d_plan_t h, int which, double* out, int64_t count)
{
    if (!h) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_plan_twiddles: plan is NULL");
    const fft3d::Plan& p = h->p;
    int64_t off, cnt;
    switch (which) {
    case 0: off = p.off_ax0; cnt = p.tw_count - p.off_ax0; break;
    case 1: off = p.off_ax1; cnt = p.off_ax0 - p.off_ax1; break;
    case 2: off = p.off_ax2h; cnt = p.off_post - p.off_ax2h; break;
    case 3: off = p.off_post; cnt = p.h + 1; break;
    default: return fail(FFT3D_ERR_INVALID_ARG, "fft3d_plan_twiddles: which must be 0..3");
    }
    if (count < 0 || (count > 0 && !out)) return fail(FFT3D_ERR_INVALID_ARG, "fft3d_plan_twiddles: bad output");
    const int64_t m = std::min(count, cnt);
    for (int64_t i = 0; i < 2 * m; ++i) {
        long double v = p.tw_host[2 * off + i];
        out[i] = p.dtype == FFT3D_F64 ? (double)v : (double)(float)v;
    }
    return cnt;
}

int fft3d_exchange_block(int64_t n0, int64_t ncols, int64_t np, int64_t src, int64_t dst, int64_t* out)
{
    if (!out || np < 1 || n0 < 1 || ncols < 1 || n0 % np || ncols % np || src < 0 || src >= np || dst < 0 ||
        dst >= np)
        return fail(FFT3D_ERR_INVALID_ARG, "fft3d_exchange_block: bad arguments");
    const int64_t r = n0 / np, c = ncols / np;
    out[0] = dst * c;  // sender: columns of dst within its r x ncols slab
    out[1] = r;
    out[2] = c;
    out[3] = ncols;
    out[4] = src * r * c;  // receiver: rows of src within its n0 x c column slab
    out[5] = r;
    out[6] = c;
    out[7] = c;
    return FFT3D_OK;
}

}  // extern "C"
