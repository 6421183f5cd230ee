// fft3d_tune.cpp -- the autotuner: times candidate tile shapes and radix
// schedules of a plan (and launch shapes of a batch) on the device with the
// library's own kernels, keeps the winners in the process's tuning table,
// and reads and writes that table as a JSON file.
//
// What is tuned never changes what is computed (the paper's two steps, Sec.
// 2.1 items 1 and 3, cut into launches); a different radix schedule changes
// only the rounding.
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fft3d.h"
#include "fft3d_internal.hpp"

namespace fft3d {
namespace {

int tfail(int code, const std::string& m)
{
    set_last_error(m);
    return code;
}

int copy_out(const std::string& s, char* buf, size_t len)
{
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, s.size());
        memcpy(buf, s.data(), n);
        buf[n] = 0;
    }
    return (int)std::min<size_t>(s.size(), 0x7fffffff);
}

// ------------------------------------------------------------ the table --

struct Key {
    std::string arch;
    int64_t n0, n1, n2;
    int dtype;
    bool operator<(const Key& o) const
    {
        return std::tie(arch, n0, n1, n2, dtype) < std::tie(o.arch, o.n0, o.n1, o.n2, o.dtype);
    }
};

struct Entry {
    fft3d_tuning t{};
    double ms_rule = 0, ms_tuned = 0;  // r2c+c2r pair, when measured
};

std::mutex g_mu;
std::map<Key, Entry> g_table;

// The GPU architecture of a device ("gfx950"), without feature suffixes.
bool device_arch(std::string& arch)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    static std::mutex mu;
    static std::map<int, std::string> cache;
    std::lock_guard<std::mutex> g(mu);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        hipDeviceProp_t pr;
        if (hipGetDeviceProperties(&pr, dev) != hipSuccess) return false;
        std::string a = pr.gcnArchName;
        const size_t c = a.find(':');
        if (c != std::string::npos) a.resize(c);
        it = cache.emplace(dev, a).first;
    }
    arch = it->second;
    return true;
}

// ------------------------------------------------------------- JSON out --

void put_tuning(std::string& o, const fft3d_tuning& t)
{
    char b[384];
    snprintf(b, sizeof b,
             "{\"plane\": %d, \"rows_rpw\": %d, \"rows_rpw_inv\": %d, \"n1_w\": %d, \"n0_w\": %d, "
             "\"n0_group\": %d, \"walk\": %d, \"coop_lag\": %d, \"coop_rpw\": %d, \"coop_w\": %d, "
             "\"cols_pipe\": %d, \"radix\": [",
             t.plane, t.rows_rpw, t.rows_rpw_inv, t.n1_w, t.n0_w, t.n0_group, t.walk, t.coop_lag, t.coop_rpw,
             t.coop_w, t.cols_pipe);
    o += b;
    for (int a = 0; a < 3; ++a) {
        o += a ? ", [" : "[";
        for (int i = 0; i < 8 && t.radix[a][i]; ++i) o += (i ? ", " : "") + std::to_string(t.radix[a][i]);
        o += "]";
    }
    o += "]}";
}

std::string fmt_ms(double ms)
{
    char b[48];
    snprintf(b, sizeof b, "%.5f", ms);
    return b;
}

// -------------------------------------------------------------- JSON in --
// A small reader for the files fft3d_tune_save writes (objects, arrays,
// numbers, strings, true/false/null).

struct JVal {
    enum Kind { Null, Num, Str, Arr, Obj } k = Null;
    double num = 0;
    std::string str;
    std::vector<JVal> arr;
    std::vector<std::pair<std::string, JVal>> obj;
    const JVal* get(const char* name) const
    {
        for (const auto& kv : obj)
            if (kv.first == name) return &kv.second;
        return nullptr;
    }
};

struct JParser {
    const char* p;
    const char* e;
    int depth = 0;
    void ws()
    {
        while (p < e && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
    }
    bool lit(const char* w)
    {
        const size_t n = strlen(w);
        if ((size_t)(e - p) < n || strncmp(p, w, n) != 0) return false;
        p += n;
        return true;
    }
    bool string(std::string& out)
    {
        if (p >= e || *p != '"') return false;
        ++p;
        out.clear();
        while (p < e && *p != '"') {
            if (*p == '\\') {
                ++p;
                if (p >= e) return false;
                const char c = *p;
                out += c == 'n' ? '\n' : c == 't' ? '\t' : c;
            } else {
                out += *p;
            }
            ++p;
        }
        if (p >= e) return false;
        ++p;
        return true;
    }
    bool value(JVal& v)
    {
        if (++depth > 64) return false;
        ws();
        bool ok = false;
        if (p >= e) {
            ok = false;
        } else if (*p == '{') {
            ++p;
            v.k = JVal::Obj;
            ws();
            if (p < e && *p == '}') {
                ++p;
                ok = true;
            } else {
                for (;;) {
                    ws();
                    std::string key;
                    if (!string(key)) break;
                    ws();
                    if (p >= e || *p != ':') break;
                    ++p;
                    JVal child;
                    if (!value(child)) break;
                    v.obj.emplace_back(key, std::move(child));
                    ws();
                    if (p < e && *p == ',') {
                        ++p;
                        continue;
                    }
                    if (p < e && *p == '}') {
                        ++p;
                        ok = true;
                    }
                    break;
                }
            }
        } else if (*p == '[') {
            ++p;
            v.k = JVal::Arr;
            ws();
            if (p < e && *p == ']') {
                ++p;
                ok = true;
            } else {
                for (;;) {
                    JVal child;
                    if (!value(child)) break;
                    v.arr.push_back(std::move(child));
                    ws();
                    if (p < e && *p == ',') {
                        ++p;
                        continue;
                    }
                    if (p < e && *p == ']') {
                        ++p;
                        ok = true;
                    }
                    break;
                }
            }
        } else if (*p == '"') {
            v.k = JVal::Str;
            ok = string(v.str);
        } else if (lit("true")) {
            v.k = JVal::Num;
            v.num = 1;
            ok = true;
        } else if (lit("false")) {
            v.k = JVal::Num;
            v.num = 0;
            ok = true;
        } else if (lit("null")) {
            v.k = JVal::Null;
            ok = true;
        } else {
            char* end = nullptr;
            std::string tok(p, (size_t)std::min<ptrdiff_t>(e - p, 64));
            const double d = strtod(tok.c_str(), &end);
            if (end && end != tok.c_str()) {
                v.k = JVal::Num;
                v.num = d;
                p += end - tok.c_str();
                ok = true;
            }
        }
        --depth;
        return ok;
    }
};

bool int_field(const JVal& o, const char* name, int32_t& out)
{
    const JVal* v = o.get(name);
    if (!v) return true;  // absent: the rule
    if (v->k != JVal::Num || v->num != (double)(int32_t)v->num) return false;
    out = (int32_t)v->num;
    return true;
}

bool read_tuning(const JVal& o, fft3d_tuning& t)
{
    if (o.k != JVal::Obj) return false;
    t = fft3d_tuning{};
    if (!int_field(o, "plane", t.plane) || !int_field(o, "rows_rpw", t.rows_rpw) ||
        !int_field(o, "rows_rpw_inv", t.rows_rpw_inv) || !int_field(o, "n1_w", t.n1_w) ||
        !int_field(o, "n0_w", t.n0_w) || !int_field(o, "n0_group", t.n0_group) || !int_field(o, "walk", t.walk) ||
        !int_field(o, "coop_lag", t.coop_lag) || !int_field(o, "coop_rpw", t.coop_rpw) ||
        !int_field(o, "coop_w", t.coop_w) || !int_field(o, "cols_pipe", t.cols_pipe))
        return false;
    if (const JVal* r = o.get("radix")) {
        if (r->k != JVal::Arr || r->arr.size() != 3) return false;
        for (int a = 0; a < 3; ++a) {
            const JVal& l = r->arr[(size_t)a];
            if (l.k != JVal::Arr || l.arr.size() > 7) return false;
            for (size_t i = 0; i < l.arr.size(); ++i) {
                if (l.arr[i].k != JVal::Num) return false;
                t.radix[a][i] = (int32_t)l.arr[i].num;
            }
        }
    }
    return true;
}

// ----------------------------------------------------------- timing --

struct Bufs {
    void* x = nullptr;  // real input
    void* X = nullptr;  // spectrum
    void* Y = nullptr;  // real output
    void* W = nullptr;  // c2r work
    size_t rb = 0, cb = 0;
};

void free_bufs(Bufs& b)
{
    for (void* q : {b.x, b.X, b.Y, b.W})
        if (q) (void)hipFree(q);
    b = Bufs{};
}

struct Clock {
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    bool ok = false;
    Clock()
    {
        ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess && hipEventCreate(&a) == hipSuccess &&
             hipEventCreate(&b) == hipSuccess;
    }
    ~Clock()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (s) (void)hipStreamDestroy(s);
    }
};

// One pass of the plan on the timing buffers (in/out as the pass needs).
int run_pass_on(fft3d_plan_t h, int pass, const Bufs& b, hipStream_t s)
{
    switch (pass) {
    case FFT3D_PASS_PLANE_R2C: return fft3d_run_pass(h, pass, b.x, b.X, s);
    case FFT3D_PASS_PLANE_C2R: return fft3d_run_pass(h, pass, b.X, b.Y, s);
    default: return fft3d_run_pass(h, pass, b.X, b.X, s);
    }
}

// Milliseconds per repetition of the pass list (pass < 0: a whole
// r2c + c2r pair), the least of three timed blocks of `reps` repetitions
// after one warm-up repetition.  Negative on a failed launch.
double time_list(fft3d_plan_t h, const std::vector<int>& passes, const Bufs& b, Clock& c, int reps)
{
    auto once = [&]() -> int {
        for (int ps : passes) {
            int rc;
            if (ps < 0) {
                rc = fft3d_r2c(h, b.x, b.X, c.s);
                if (!rc) rc = fft3d_c2r(h, b.X, b.Y, b.W, c.s);
            } else {
                rc = run_pass_on(h, ps, b, c.s);
            }
            if (rc) return rc;
        }
        return 0;
    };
    if (once()) return -1;
    if (hipStreamSynchronize(c.s) != hipSuccess) return -1;
    double best = -1;
    for (int blk = 0; blk < 3; ++blk) {
        if (hipEventRecord(c.a, c.s) != hipSuccess) return -1;
        for (int r = 0; r < reps; ++r)
            if (once()) return -1;
        if (hipEventRecord(c.b, c.s) != hipSuccess || hipEventSynchronize(c.b) != hipSuccess) return -1;
        float ms = 0;
        if (hipEventElapsedTime(&ms, c.a, c.b) != hipSuccess) return -1;
        const double per = ms / reps;
        if (best < 0 || per < best) best = per;
    }
    return best;
}

// ------------------------------------------------------ the candidates --

// Radix lists of length n: the power-of-two part 2^a as stages from
// {16, 8, 4, 2} (fewest stages, or one more; at most one radix-2 stage),
// largest first or smallest first, with the odd radices after (and, for
// one list, before).  The rule's own schedule is among them.
std::vector<std::vector<int>> radix_lists(int64_t n, int limit)
{
    std::vector<std::vector<int>> out;
    if (n <= 1) return out;
    int64_t m = n;
    int a = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++a;
    }
    std::vector<int> odd;
    for (int p : {3, 5, 7})
        while (m % p == 0) {
            m /= p;
            odd.push_back(p);
        }
    if (m != 1) return out;
    std::vector<std::vector<int>> sets;  // non-increasing multisets of {16,8,4,2} summing (in log2) to a
    const int smin = (a + 3) / 4;
    std::vector<int> cur;
    // depth-first over non-increasing sequences
    struct Rec {
        static void go(int left, int maxlog, int stages_left, std::vector<int>& cur, std::vector<std::vector<int>>& sets)
        {
            if (left == 0) {
                int twos = 0;
                for (int r : cur) twos += r == 2;
                if (twos <= 1) sets.push_back(cur);
                return;
            }
            if (stages_left == 0) return;
            for (int lg = std::min(maxlog, left); lg >= 1; --lg) {
                cur.push_back(1 << lg);
                go(left - lg, lg, stages_left - 1, cur, sets);
                cur.pop_back();
            }
        }
    };
    if (a > 0) {
        for (int st = smin; st <= smin + 1; ++st) {
            std::vector<std::vector<int>> s1;
            Rec::go(a, 4, st, cur, s1);
            for (auto& v : s1)
                if ((int)v.size() == st) sets.push_back(v);
        }
    } else {
        sets.push_back({});
    }
    auto add = [&](const std::vector<int>& v) {
        if (v.empty()) return;
        for (const auto& o : out)
            if (o == v) return;
        out.push_back(v);
    };
    for (const auto& s : sets) {
        std::vector<int> d = s;  // largest first
        d.insert(d.end(), odd.begin(), odd.end());
        add(d);
        std::vector<int> u(s.rbegin(), s.rend());  // smallest first
        u.insert(u.end(), odd.begin(), odd.end());
        add(u);
    }
    if (!odd.empty() && !sets.empty()) {
        std::vector<int> f = odd;
        f.insert(f.end(), sets[0].begin(), sets[0].end());
        add(f);
    }
    if ((int)out.size() > limit) out.resize((size_t)limit);
    return out;
}

void set_radix(fft3d_tuning& t, int axis, const std::vector<int>& r)
{
    for (int i = 0; i < 8; ++i) t.radix[axis][i] = i < (int)r.size() ? r[(size_t)i] : 0;
}

std::string radix_str(const std::vector<int>& r)
{
    std::string s = "[";
    for (size_t i = 0; i < r.size(); ++i) s += (i ? ", " : "") + std::to_string(r[i]);
    return s + "]";
}

struct Search {
    int64_t n0, n1, n2;
    int dtype;
    int effort;
    Bufs b;
    Clock c;
    int reps = 5;
    std::string log;  // JSON array items
    int count = 0;

    // Time the pass list with tuning t: ms, or -1 if t is not valid for the
    // shape (or a launch failed; the candidate is then skipped).
    double eval(const fft3d_tuning& t, const std::vector<int>& passes, const char* stage, const std::string& what)
    {
        fft3d_plan_t h = nullptr;
        double ms = -1;
        if (fft3d_plan_tuned(n0, n1, n2, dtype, 0, &t, &h) == FFT3D_OK) {
            ms = time_list(h, passes, b, c, reps);
            (void)fft3d_plan_destroy(h);
        }
        log += std::string(count++ ? ", " : "") + "{\"stage\": \"" + stage + "\", \"candidate\": " + what +
               ", \"ms\": " + (ms < 0 ? std::string("null") : fmt_ms(ms)) + "}";
        return ms;
    }
};

// The passes of a plan's plane step and of its n1 pass, by the plan's kind.
void plane_passes(const Plan& p, std::vector<int>& plane, std::vector<int>& n1p)
{
    plane = {FFT3D_PASS_PLANE_R2C, FFT3D_PASS_PLANE_C2R};
    n1p.clear();
    if (!p.fused_plane && !p.coop && p.n1 > 1) n1p = {FFT3D_PASS_N1_FWD, FFT3D_PASS_N1_INV};
}

}  // namespace
}  // namespace fft3d

using namespace fft3d;

int fft3d_tune_lookup(int64_t n0, int64_t n1, int64_t n2, int dtype, fft3d_tuning* t)
{
    if (!t) return tfail(FFT3D_ERR_INVALID_ARG, "fft3d_tune_lookup: t is NULL");
    std::string arch;
    if (!device_arch(arch)) return 0;
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_table.find(Key{arch, n0, n1, n2, dtype});
    if (it == g_table.end()) return 0;
    *t = it->second.t;
    return 1;
}

int fft3d_tune_save(const char* path)
{
    if (!path) return tfail(FFT3D_ERR_INVALID_ARG, "fft3d_tune_save: path is NULL");
    std::string o = "{\"version\": 1, \"entries\": [";
    {
        std::lock_guard<std::mutex> g(g_mu);
        bool first = true;
        for (const auto& kv : g_table) {
            const Key& k = kv.first;
            const Entry& e = kv.second;
            char b[256];
            snprintf(b, sizeof b, "%s\n  {\"arch\": \"%s\", \"shape\": [%lld, %lld, %lld], \"dtype\": \"%s\", ",
                     first ? "" : ",", k.arch.c_str(), (long long)k.n0, (long long)k.n1, (long long)k.n2,
                     k.dtype ? "f64" : "f32");
            o += b;
            o += "\"pair_ms_rule\": " + fmt_ms(e.ms_rule) + ", \"pair_ms_tuned\": " + fmt_ms(e.ms_tuned) +
                 ", \"tuning\": ";
            put_tuning(o, e.t);
            o += "}";
            first = false;
        }
    }
    o += "\n]}\n";
    FILE* f = fopen(path, "w");
    if (!f) return tfail(FFT3D_ERR_INVALID_ARG, std::string("fft3d_tune_save: cannot open ") + path);
    const bool ok = fwrite(o.data(), 1, o.size(), f) == o.size();
    if (fclose(f) != 0 || !ok) return tfail(FFT3D_ERR_INVALID_ARG, std::string("fft3d_tune_save: write failed: ") + path);
    return FFT3D_OK;
}

int fft3d_tune_load(const char* path)
{
    if (!path) return tfail(FFT3D_ERR_INVALID_ARG, "fft3d_tune_load: path is NULL");
    FILE* f = fopen(path, "r");
    if (!f) return tfail(FFT3D_ERR_INVALID_ARG, std::string("fft3d_tune_load: cannot open ") + path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    JParser ps{text.data(), text.data() + text.size()};
    JVal root;
    const std::string bad = std::string("fft3d_tune_load: not a tuning file: ") + path;
    if (!ps.value(root) || root.k != JVal::Obj) return tfail(FFT3D_ERR_INVALID_ARG, bad);
    const JVal* ver = root.get("version");
    const JVal* ents = root.get("entries");
    if (!ver || ver->k != JVal::Num || ver->num != 1 || !ents || ents->k != JVal::Arr)
        return tfail(FFT3D_ERR_INVALID_ARG, bad);
    std::vector<std::pair<Key, Entry>> got_entries;
    for (const JVal& e : ents->arr) {
        const JVal* arch = e.get("arch");
        const JVal* shape = e.get("shape");
        const JVal* dt = e.get("dtype");
        const JVal* tu = e.get("tuning");
        if (!arch || arch->k != JVal::Str || !shape || shape->k != JVal::Arr || shape->arr.size() != 3 || !dt ||
            dt->k != JVal::Str || (dt->str != "f32" && dt->str != "f64") || !tu)
            return tfail(FFT3D_ERR_INVALID_ARG, bad + " (entry fields)");
        Key k{arch->str, 0, 0, 0, dt->str == "f64" ? 1 : 0};
        int64_t* ns[3] = {&k.n0, &k.n1, &k.n2};
        for (int i = 0; i < 3; ++i) {
            const JVal& v = shape->arr[(size_t)i];
            if (v.k != JVal::Num || v.num < 1 || v.num > 1e9 || v.num != (double)(int64_t)v.num)
                return tfail(FFT3D_ERR_INVALID_ARG, bad + " (shape)");
            *ns[i] = (int64_t)v.num;
        }
        Entry en;
        if (!read_tuning(*tu, en.t)) return tfail(FFT3D_ERR_INVALID_ARG, bad + " (tuning)");
        // the tuning must make a valid plan of the shape (host only)
        fft3d_plan_t h = nullptr;
        if (fft3d_plan_tuned(k.n0, k.n1, k.n2, k.dtype, FFT3D_PLAN_HOST_ONLY, &en.t, &h) != FFT3D_OK)
            return tfail(FFT3D_ERR_INVALID_ARG, bad + " (a tuning that does not fit its shape)");
        (void)fft3d_plan_destroy(h);
        if (const JVal* v = e.get("pair_ms_rule"))
            if (v->k == JVal::Num) en.ms_rule = v->num;
        if (const JVal* v = e.get("pair_ms_tuned"))
            if (v->k == JVal::Num) en.ms_tuned = v->num;
        got_entries.emplace_back(k, en);
    }
    std::lock_guard<std::mutex> g(g_mu);
    for (auto& kv : got_entries) g_table[kv.first] = kv.second;
    return FFT3D_OK;
}

int fft3d_autotune(int64_t n0, int64_t n1, int64_t n2, int dtype, int effort, fft3d_tuning* best, char* report,
                   size_t len)
{
    const char* who = "fft3d_autotune";
    if (!best) return tfail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": best is NULL");
    if (effort < 0 || effort > 1) return tfail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": effort must be 0 or 1");
    *best = fft3d_tuning{};
    // the rule plan (validates the shape)
    fft3d_plan_t rule = nullptr;
    int rc = fft3d_plan(n0, n1, n2, dtype, &rule);
    if (rc) return rc;
    const Plan rp = rule->p;
    (void)fft3d_plan_destroy(rule);
    std::string arch;
    if (!device_arch(arch)) return tfail(FFT3D_ERR_HIP, std::string(who) + ": no device");

    Search S;
    S.n0 = n0;
    S.n1 = n1;
    S.n2 = n2;
    S.dtype = dtype;
    S.effort = effort;
    if (!S.c.ok) return tfail(FFT3D_ERR_HIP, std::string(who) + ": stream/event creation failed");
    S.b.rb = (size_t)rp.N * rp.elem;
    S.b.cb = (size_t)rp.M * 2 * rp.elem;
    hipError_t e = hipMalloc(&S.b.x, S.b.rb);
    if (e == hipSuccess) e = hipMalloc(&S.b.X, S.b.cb);
    if (e == hipSuccess) e = hipMalloc(&S.b.Y, S.b.rb);
    if (e == hipSuccess) e = hipMalloc(&S.b.W, S.b.cb);
    // any finite values do: 0.5 in every FP32 word (FP64: a small normal number)
    if (e == hipSuccess) e = hipMemsetD32(S.b.x, 0x3f000000, S.b.rb / 4);
    if (e == hipSuccess) e = hipMemsetD32(S.b.X, 0, S.b.cb / 4);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_bufs(S.b);
        return tfail(FFT3D_ERR_NOMEM, std::string(who) + ": buffers: " + hipGetErrorString(e));
    }
    // repetitions per timed block: about 2 ms of one sweep of the spectrum
    // at 4 TB/s, between 3 and 200
    const double sweep_ms = (double)(S.b.cb * 2) / 4e9;
    S.reps = (int)std::min(200.0, std::max(3.0, 2.0 / std::max(sweep_ms, 1e-4)));

    fft3d_tuning cur{};  // the choices so far (zero: the rule)
    std::vector<int> plane, n1p;
    plane_passes(rp, plane, n1p);
    const std::vector<int> n0p = n0 > 1 ? std::vector<int>{FFT3D_PASS_N0_FWD, FFT3D_PASS_N0_INV} : std::vector<int>{};
    // keep a candidate only if it beats the incumbent by 1% (timing noise)
    auto better = [](double ms, double inc) { return ms > 0 && (inc < 0 || ms < 0.99 * inc); };
    char w[160];

    // 1. radix schedules, axis by axis
    const int64_t lens[3] = {n0, n1, n2 % 2 ? n2 : n2 / 2};
    for (int ax = 2; ax >= 0; --ax) {
        const std::vector<int>& ps = ax == 0 ? n0p : ax == 1 ? (n1p.empty() ? plane : n1p) : plane;
        if (ps.empty()) continue;
        const auto lists = radix_lists(lens[ax], effort ? 12 : 5);
        if (lists.size() < 2) continue;
        double inc = S.eval(cur, ps, "radix", "{\"axis\": " + std::to_string(ax) + ", \"radix\": \"rule\"}");
        std::vector<int> pick;
        for (const auto& l : lists) {
            fft3d_tuning t = cur;
            set_radix(t, ax, l);
            const double ms = S.eval(t, ps, "radix", "{\"axis\": " + std::to_string(ax) + ", \"radix\": " + radix_str(l) + "}");
            if (better(ms, inc)) {
                inc = ms;
                pick = l;
            }
        }
        if (!pick.empty()) set_radix(cur, ax, pick);
    }
    // 2. rows per tile of the forward and of the inverse rows kernel (split
    //    plane step), each timed on its own pass
    if (!rp.fused_plane) {
        for (int inv = 0; inv < 2; ++inv) {
            const std::vector<int> ps = {inv ? FFT3D_PASS_PLANE_C2R : FFT3D_PASS_PLANE_R2C};
            const char* field = inv ? "rows_rpw_inv" : "rows_rpw";
            const int rule = inv ? rp.rpw_inv : rp.rpw;
            double inc = S.eval(cur, ps, field, std::string("{\"") + field + "\": \"rule\"}");
            int pick = 0;
            for (int r : {2, 4, 6, 8, 10, 12, 14, 16, 18, 20, 24, 32, 48, 64}) {
                if (r == rule) continue;
                if (!effort && (r == 6 || r == 10 || r == 14 || r == 18 || r == 48)) continue;
                fft3d_tuning t = cur;
                (inv ? t.rows_rpw_inv : t.rows_rpw) = r;
                snprintf(w, sizeof w, "{\"%s\": %d}", field, r);
                const double ms = S.eval(t, ps, field, w);
                if (better(ms, inc)) {
                    inc = ms;
                    pick = r;
                }
            }
            (inv ? cur.rows_rpw_inv : cur.rows_rpw) = pick;
        }
    }
    // 3. n1 tile width (split plane step)
    if (!n1p.empty()) {
        double inc = S.eval(cur, n1p, "n1_w", "{\"n1_w\": \"rule\"}");
        int pick = 0;
        for (int W = 1; W <= 64; W *= 2) {
            if (W == rp.pass1.W) continue;
            fft3d_tuning t = cur;
            t.n1_w = W;
            snprintf(w, sizeof w, "{\"n1_w\": %d}", W);
            const double ms = S.eval(t, n1p, "n1_w", w);
            if (better(ms, inc)) {
                inc = ms;
                pick = W;
            }
        }
        cur.n1_w = pick;
    }
    // 4. n0 tile width and XCD grouping
    if (!n0p.empty()) {
        double inc = S.eval(cur, n0p, "n0", "{\"n0_w\": \"rule\", \"n0_group\": \"rule\"}");
        int pw = 0, pg = 0;
        for (int W = 1; W <= 64; W *= 2) {
            for (int G : {0, 1, 2, 4, 8, 16, 32}) {
                if (W == rp.pass0.W && G == 0) continue;
                if (!effort && G != 0 && G != 1 && G != 8) continue;
                fft3d_tuning t = cur;
                t.n0_w = W == rp.pass0.W ? 0 : W;
                t.n0_group = G;
                snprintf(w, sizeof w, "{\"n0_w\": %d, \"n0_group\": %d}", W, G);
                const double ms = S.eval(t, n0p, "n0", w);
                if (better(ms, inc)) {
                    inc = ms;
                    pw = t.n0_w;
                    pg = G;
                }
            }
        }
        cur.n0_w = pw;
        cur.n0_group = pg;
    }
    // 5. the plane step: split against cooperative (planes larger than LDS),
    //    fused against split (planes that fit)
    if (!rp.fused_plane && n1 > 1) {
        std::vector<int> split_ps = plane;
        split_ps.insert(split_ps.end(), n1p.begin(), n1p.end());
        double inc = S.eval(cur, split_ps, "plane", "{\"plane\": \"split\"}");
        fft3d_tuning pick = cur;
        bool coop = false;
        const std::vector<int> lags = effort ? std::vector<int>{1, 2, 3, 4, 6, 8, 12, 16, 24, 32}
                                             : std::vector<int>{2, 4, 8, 16, 32};
        for (int lag : lags)
            for (int halve_r = 0; halve_r < (effort ? 2 : 1); ++halve_r)
                for (int halve_w = 0; halve_w < (effort ? 2 : 1); ++halve_w) {
                    fft3d_tuning t = cur;
                    t.plane = FFT3D_TUNE_COOP;
                    t.coop_lag = lag;
                    // row / column tasks of the chosen split tiling, or half of them
                    fft3d_plan_t h = nullptr;
                    if (fft3d_plan_tuned(n0, n1, n2, dtype, FFT3D_PLAN_HOST_ONLY, &cur, &h) != FFT3D_OK) continue;
                    const int r = h->p.rpw, W = h->p.pass1.W;
                    (void)fft3d_plan_destroy(h);
                    t.coop_rpw = halve_r ? std::max(1, r / 2) : 0;
                    t.coop_w = halve_w ? std::max(1, W / 2) : 0;
                    snprintf(w, sizeof w, "{\"plane\": \"coop\", \"coop_lag\": %d, \"coop_rpw\": %d, \"coop_w\": %d}",
                             lag, t.coop_rpw ? t.coop_rpw : r, t.coop_w ? t.coop_w : W);
                    const double ms = S.eval(t, plane, "plane", w);
                    if (better(ms, inc)) {
                        inc = ms;
                        pick = t;
                        coop = true;
                    }
                }
        if (coop) cur = pick;
    } else if (rp.fused_plane && n1 > 1) {
        const double inc = S.eval(cur, plane, "plane", "{\"plane\": \"fused\"}");
        fft3d_tuning t = cur;
        t.plane = FFT3D_TUNE_SPLIT;
        std::vector<int> split_ps = plane;
        split_ps.push_back(FFT3D_PASS_N1_FWD);
        split_ps.push_back(FFT3D_PASS_N1_INV);
        const double ms = S.eval(t, split_ps, "plane", "{\"plane\": \"split\"}");
        if (better(ms, inc)) cur = t;
    }
    // 6. wide column passes: the persistent loop that loads a tile ahead
    //    against one tile per workgroup, on whole pairs
    const std::vector<int> pair = {-1};
    {
        bool pipe = false;
        fft3d_plan_t h = nullptr;
        if (fft3d_plan_tuned(n0, n1, n2, dtype, FFT3D_PLAN_HOST_ONLY, &cur, &h) == FFT3D_OK) {
            pipe = h->p.pass0.pipe || (!h->p.fused_plane && h->p.pass1.pipe);
            (void)fft3d_plan_destroy(h);
        }
        if (pipe) {
            const double inc = S.eval(cur, pair, "cols_pipe", "{\"cols_pipe\": \"rule\"}");
            fft3d_tuning t = cur;
            t.cols_pipe = 1;
            const double ms = S.eval(t, pair, "cols_pipe", "{\"cols_pipe\": 1}");
            if (better(ms, inc)) cur = t;
        }
    }
    // 7. walk order, on whole pairs
    {
        double inc = S.eval(cur, pair, "walk", "{\"walk\": \"rule\"}");
        int pick = 0;
        const std::vector<int> walks = effort ? std::vector<int>{0, 63, 2, 8, 16, 2 | 16, 4 | 8, 1 | 32}
                                              : std::vector<int>{0, 63};
        for (int bits : walks) {
            if (bits == rp.rev) continue;
            fft3d_tuning t = cur;
            t.walk = 64 + bits;
            snprintf(w, sizeof w, "{\"walk\": %d}", 64 + bits);
            const double ms = S.eval(t, pair, "walk", w);
            if (better(ms, inc)) {
                inc = ms;
                pick = 64 + bits;
            }
        }
        cur.walk = pick;
    }
    // 8. the rule plan against the tuned one, whole pairs
    const fft3d_tuning zero{};
    const double ms_rule = S.eval(zero, pair, "final", "{\"plan\": \"rule\"}");
    std::string tj;
    put_tuning(tj, cur);
    const double ms_tuned = S.eval(cur, pair, "final", "{\"plan\": \"tuned\", \"tuning\": " + tj + "}");
    free_bufs(S.b);
    if (ms_rule < 0) return tfail(FFT3D_ERR_HIP, std::string(who) + ": the rule plan failed to run");
    const bool keep = ms_tuned > 0 && ms_tuned < ms_rule;
    if (keep) *best = cur;
    {
        std::lock_guard<std::mutex> g(g_mu);
        Entry en;
        en.t = *best;
        en.ms_rule = ms_rule;
        en.ms_tuned = keep ? ms_tuned : ms_rule;
        g_table[Key{arch, n0, n1, n2, dtype}] = en;
    }
    std::string out;
    char b[256];
    snprintf(b, sizeof b,
             "{\"arch\": \"%s\", \"shape\": [%lld, %lld, %lld], \"dtype\": \"%s\", \"effort\": %d, \"reps\": %d, "
             "\"pair_ms_rule\": %s, \"pair_ms_tuned\": %s, \"kept\": \"%s\", \"best\": ",
             arch.c_str(), (long long)n0, (long long)n1, (long long)n2, dtype ? "f64" : "f32", effort, S.reps,
             fmt_ms(ms_rule).c_str(), ms_tuned < 0 ? "null" : fmt_ms(ms_tuned).c_str(), keep ? "tuned" : "rule");
    out = b;
    put_tuning(out, *best);
    out += ", \"candidates\": [" + S.log + "]}";
    return copy_out(out, report, len);
}

int fft3d_batch_autotune(const fft3d_batch_item* items, int n, int effort, fft3d_batch_tuning* best, char* report,
                         size_t len)
{
    const char* who = "fft3d_batch_autotune";
    if (!best) return tfail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": best is NULL");
    if (effort < 0 || effort > 1) return tfail(FFT3D_ERR_INVALID_ARG, std::string(who) + ": effort must be 0 or 1");
    *best = fft3d_batch_tuning{};
    Clock c;
    if (!c.ok) return tfail(FFT3D_ERR_HIP, std::string(who) + ": stream/event creation failed");
    std::string log;
    int count = 0;
    auto eval = [&](const fft3d_batch_tuning& bt) -> double {
        fft3d_batch_t b = nullptr;
        double ms = -1;
        if (fft3d_batch_create_tuned(items, n, FFT3D_BATCH_DIRECT, &bt, &b) == FFT3D_OK) {
            // warm-up, then the least of three blocks of 5 launches
            if (fft3d_batch_launch(b, c.s) == FFT3D_OK && hipStreamSynchronize(c.s) == hipSuccess) {
                for (int blk = 0; blk < 3; ++blk) {
                    if (hipEventRecord(c.a, c.s) != hipSuccess) break;
                    bool ok = true;
                    for (int r = 0; r < 5 && ok; ++r) ok = fft3d_batch_launch(b, c.s) == FFT3D_OK;
                    float t = 0;
                    if (!ok || hipEventRecord(c.b, c.s) != hipSuccess || hipEventSynchronize(c.b) != hipSuccess ||
                        hipEventElapsedTime(&t, c.a, c.b) != hipSuccess)
                        break;
                    if (ms < 0 || t / 5 < ms) ms = t / 5;
                }
            }
            (void)fft3d_batch_destroy(b);
        }
        char w[200];
        snprintf(w, sizeof w, "%s{\"mode\": %d, \"lag\": %d, \"widen\": %d, \"wg_per_cu\": %d, \"ms\": %s}",
                 count++ ? ", " : "", bt.mode, bt.lag, bt.widen, bt.wg_per_cu,
                 ms < 0 ? "null" : fmt_ms(ms).c_str());
        log += w;
        return ms;
    };
    const fft3d_batch_tuning rule{};
    const double ms_rule = eval(rule);
    if (ms_rule < 0) {
        std::string why = std::string(who) + ": the rule batch failed: ";
        return tfail(FFT3D_ERR_INVALID_ARG, why + fft3d_last_error());
    }
    double inc = ms_rule;
    fft3d_batch_tuning pick = rule;
    std::vector<int> lags = {0};
    if (effort)
        for (int l : {1, 2, 4, 8, 16}) lags.push_back(l);
    for (int mode : {0, 1, 2, 4})
        for (int widen = 1; widen <= 2; ++widen)
            for (int wg = 0; wg <= 2; ++wg)
                for (int lag : lags) {
                    fft3d_batch_tuning bt{mode, lag, widen, wg, 0};
                    if (mode == 0 && widen == 1 && wg == 0 && lag == 0) continue;
                    if (mode == 0 && (wg != 0 || lag != 0)) continue;  // level mode: no queues, a workgroup per tile
                    const double ms = eval(bt);
                    if (ms > 0 && ms < 0.99 * inc) {
                        inc = ms;
                        pick = bt;
                    }
                }
    *best = pick;
    char b[256];
    snprintf(b, sizeof b,
             "{\"items\": %d, \"effort\": %d, \"ms_rule\": %s, \"ms_tuned\": %s, \"best\": {\"mode\": %d, \"lag\": %d, "
             "\"widen\": %d, \"wg_per_cu\": %d, \"spin_limit\": %d}, \"candidates\": [",
             n, effort, fmt_ms(ms_rule).c_str(), fmt_ms(inc).c_str(), pick.mode, pick.lag, pick.widen, pick.wg_per_cu,
             pick.spin_limit);
    return copy_out(std::string(b) + log + "]}", report, len);
}
