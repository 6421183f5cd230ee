// host_sanitize.cpp -- drives the library's host code under the host
// sanitizers (test infrastructure; built by tests/test_sanitizers.py with
// g++ and AddressSanitizer + UndefinedBehaviorSanitizer, or ThreadSanitizer,
// linked with tests/host_stubs.cpp in place of the device half).
//
//   host_sanitize plans          host-only plans of many shapes, flags and
//                                tunings; descriptions and twiddle tables
//                                into buffers of every small size
//   host_sanitize table <dir>    the tuning-table file reader on a valid
//                                file, every truncation of it, seeded byte
//                                mutations and deep nesting; save / load
//   host_sanitize server         the server in its no-device mode: four
//                                client threads submitting, waiting,
//                                reading and releasing requests while a
//                                fifth reads the counters
// Exit status 0 and "ok <part>" when every call returned as documented.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "../include/fft3d.h"

static int g_fail = 0;

static void check(bool ok, const char* what)
{
    if (!ok) {
        fprintf(stderr, "FAIL: %s (%s)\n", what, fft3d_last_error());
        g_fail = 1;
    }
}

// ------------------------------------------------------------------ plans --

static void one_plan(int64_t n0, int64_t n1, int64_t n2, int dt, int flags, const fft3d_tuning* t)
{
    fft3d_plan_t p = nullptr;
    const int rc = t ? fft3d_plan_tuned(n0, n1, n2, dt, flags, t, &p) : fft3d_plan_ex(n0, n1, n2, dt, flags, &p);
    if (rc != FFT3D_OK) {
        check(p == nullptr && rc < 0 && fft3d_last_error()[0] != 0, "a refused plan leaves out NULL and a message");
        return;
    }
    const int need = fft3d_plan_describe(p, nullptr, 0);
    check(need > 0, "describe length");
    for (size_t len : {(size_t)1, (size_t)2, (size_t)17, (size_t)need, (size_t)need + 1}) {
        std::vector<char> b(len, 'x');
        check(fft3d_plan_describe(p, b.data(), len) == need, "describe returns the full length");
        check(b[std::min(len - 1, (size_t)need)] == 0, "describe is NUL-terminated");
    }
    for (int which = 0; which < 4; ++which) {
        const int64_t n = fft3d_plan_twiddles(p, which, nullptr, 0);
        check(n >= 0, "twiddle count");
        for (int64_t cnt : {(int64_t)1, n}) {
            if (cnt < 1) continue;
            std::vector<double> tw((size_t)(2 * cnt));
            check(fft3d_plan_twiddles(p, which, tw.data(), cnt) == n, "twiddle copy");
        }
    }
    check(fft3d_work_bytes(p) == fft3d_complex_bytes(p), "work bytes");
    check(fft3d_plan_destroy(p) == FFT3D_OK, "destroy");
}

static int run_plans()
{
    const int64_t shapes[][3] = {{1, 1, 1},    {1, 1, 2},     {2, 3, 4},      {7, 5, 9},      {30, 42, 50},
                                 {96, 128, 384}, {512, 512, 512}, {64, 64, 64},  {1024, 64, 1024}, {4096, 4096, 8192},
                                 {4096, 1, 8192}, {3, 2401, 7},  {16, 128, 243}, {11, 4, 4},     {4, 4, 16384},
                                 {0, 4, 4},     {4, -3, 4},     {8192, 8, 8},   {625, 2, 10},   {2, 2, 8191}};
    for (const auto& s : shapes)
        for (int dt = 0; dt < 3; ++dt)
            for (int flags : {(int)FFT3D_PLAN_HOST_ONLY, FFT3D_PLAN_HOST_ONLY | FFT3D_PLAN_COOP_PLANE, 8 | 1})
                one_plan(s[0], s[1], s[2], dt, flags, nullptr);
    // tunings, valid and not, on a split and a fused shape
    std::vector<fft3d_tuning> ts;
    fft3d_tuning t{};
    ts.push_back(t);
    const int vals[] = {-2147483647 - 1, -1, 0, 1, 2, 3, 4, 5, 16, 63, 64, 65, 127, 128, 256, 257, 2147483647};
    for (int v : vals) {
        for (int f = 0; f < 9; ++f) {
            fft3d_tuning u{};
            int32_t* fields[] = {&u.plane, &u.rows_rpw, &u.n1_w, &u.n0_w, &u.n0_group,
                                 &u.walk,  &u.coop_lag, &u.coop_rpw, &u.coop_w};
            *fields[f] = v;
            if (f >= 6) u.plane = FFT3D_TUNE_COOP;
            ts.push_back(u);
        }
    }
    const int lists[][8] = {{16, 16, 2}, {2, 16, 16}, {8, 8, 8}, {16, 8, 4}, {4, 4, 4, 8}, {16, 16, 4},
                            {3, 0, 5},   {7, 7},      {5, 5, 5, 4}, {-16, -32}, {2, 2, 2, 2, 2, 2, 2, 2}};
    for (const auto& l : lists)
        for (int a = 0; a < 3; ++a) {
            fft3d_tuning u{};
            memcpy(u.radix[a], l, sizeof l);
            ts.push_back(u);
        }
    for (const fft3d_tuning& u : ts)
        for (const auto& s : {std::vector<int64_t>{512, 512, 512}, std::vector<int64_t>{64, 64, 64},
                              std::vector<int64_t>{40, 49, 100}, std::vector<int64_t>{16, 16, 243}})
            for (int dt = 0; dt < 2; ++dt) one_plan(s[0], s[1], s[2], dt, FFT3D_PLAN_HOST_ONLY, &u);
    int64_t out[8];
    for (int64_t p = 1; p <= 8; p *= 2)
        for (int64_t a = 0; a < p; ++a)
            for (int64_t b = 0; b < p; ++b) check(fft3d_exchange_block(64, 4096, p, a, b, out) == FFT3D_OK, "exchange");
    check(fft3d_exchange_block(63, 4096, 2, 0, 0, out) < 0, "exchange refuses n0 % p");
    check(fft3d_plan_describe(nullptr, nullptr, 0) < 0, "describe of NULL");
    puts(g_fail ? "FAIL plans" : "ok plans");
    return g_fail;
}

// ------------------------------------------------------------------ table --

static bool write_file(const std::string& path, const std::string& text)
{
    FILE* f = fopen(path.c_str(), "wb");
    if (!f) return false;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    return fclose(f) == 0 && ok;
}

static int run_table(const char* dir)
{
    const std::string good =
        "{\"version\": 1, \"entries\": [\n"
        "  {\"arch\": \"gfx950\", \"shape\": [512, 512, 512], \"dtype\": \"f32\", \"pair_ms_rule\": 1.38, "
        "\"pair_ms_tuned\": 1.2, \"tuning\": {\"plane\": 3, \"coop_lag\": 16, \"n0_w\": 32, \"n0_group\": 4, "
        "\"walk\": 64, \"radix\": [[16, 16, 2], [], [16, 16]]}},\n"
        "  {\"arch\": \"gfx950\", \"shape\": [64, 64, 64], \"dtype\": \"f64\", \"tuning\": {\"plane\": 2}},\n"
        "  {\"arch\": \"gfx942\", \"shape\": [96, 128, 384], \"dtype\": \"f32\", \"tuning\": {\"rows_rpw\": 6, "
        "\"n1_w\": 8, \"note\": \"x\\\"y\"}}\n"
        "]}\n";
    const std::string p = std::string(dir) + "/t.json";
    check(write_file(p, good), "write");
    check(fft3d_tune_load(p.c_str()) == FFT3D_OK, "load a valid file");
    const std::string q = std::string(dir) + "/saved.json";
    check(fft3d_tune_save(q.c_str()) == FFT3D_OK, "save");
    check(fft3d_tune_load(q.c_str()) == FFT3D_OK, "load what was saved");
    // every truncation: refused (or, for the whole text less its newline, accepted)
    for (size_t n = 0; n + 1 < good.size(); ++n) {
        check(write_file(p, good.substr(0, n)), "write");
        const int rc = fft3d_tune_load(p.c_str());
        check(rc == FFT3D_ERR_INVALID_ARG || rc == FFT3D_OK, "truncated file: refused or read");
    }
    // seeded byte mutations: whatever the result, no memory error
    uint64_t s = 12345;
    for (int it = 0; it < 3000; ++it) {
        std::string m = good;
        for (int k = 0; k < 1 + it % 4; ++k) {
            s = s * 6364136223846793005ull + 1442695040888963407ull;
            const size_t pos = (size_t)((s >> 33) % m.size());
            m[pos] = (char)(s >> 24);
        }
        check(write_file(p, m), "write");
        const int rc = fft3d_tune_load(p.c_str());
        check(rc == FFT3D_ERR_INVALID_ARG || rc == FFT3D_OK, "mutated file: refused or read");
    }
    // deep nesting and a long number
    check(write_file(p, std::string(100000, '[')), "write");
    check(fft3d_tune_load(p.c_str()) == FFT3D_ERR_INVALID_ARG, "deep nesting refused");
    check(write_file(p, "{\"version\": 1" + std::string(5000, '0') + ", \"entries\": []}"), "write");
    (void)fft3d_tune_load(p.c_str());
    check(fft3d_tune_load((std::string(dir) + "/missing.json").c_str()) == FFT3D_ERR_INVALID_ARG, "missing file");
    check(fft3d_tune_load(nullptr) == FFT3D_ERR_INVALID_ARG, "NULL path");
    check(fft3d_tune_save((std::string(dir) + "/no/such/dir/x.json").c_str()) == FFT3D_ERR_INVALID_ARG,
          "unwritable path");
    puts(g_fail ? "FAIL table" : "ok table");
    return g_fail;
}

// ----------------------------------------------------------------- server --

static int run_server()
{
    fft3d_server_config cfg{};
    cfg.budget_bytes = (size_t)64 << 20;
    cfg.nstreams = 4;
    cfg.batch_points = 4096;
    cfg.max_batch_items = 5;
    cfg.flags = FFT3D_SERVER_NO_DEVICE;
    fft3d_server_t srv = nullptr;
    check(fft3d_server_create(&cfg, &srv) == FFT3D_OK, "server create");
    if (!srv) return 1;
    std::atomic<bool> stop{false};
    std::atomic<int> done{0};
    std::thread reader([&] {
        while (!stop.load()) {
            fft3d_server_counters st;
            check(fft3d_server_stats(srv, &st) == FFT3D_OK, "stats");
            check(st.reserved_bytes <= st.budget_bytes, "reserved within the budget");
        }
    });
    std::vector<std::thread> clients;
    for (int c = 0; c < 4; ++c) {
        clients.emplace_back([&, c] {
            const int64_t shapes[][3] = {{8, 8, 8}, {16, 16, 16}, {32, 32, 32}, {16, 12, 30}, {8, 8, 7}};
            for (int i = 0; i < 60; ++i) {
                const auto& s = shapes[(c + i) % 5];
                fft3d_request r{};
                r.n0 = s[0];
                r.n1 = s[1];
                r.n2 = s[2];
                r.dtype = (i / 5) % 2;
                r.dir = (i / 2) % 2;
                r.ncomp = 1 + i % 3;
                for (int k = 0; k < r.ncomp; ++k) r.in[k] = (const void*)(uintptr_t)(0x100000 + 0x10000 * k);
                int64_t id = -1;
                if (fft3d_server_submit(srv, &r, &id) != FFT3D_OK) {
                    check(false, "submit");
                    continue;
                }
                check(fft3d_server_wait(srv, id, 20.0) == 1, "wait");
                void* out[FFT3D_SERVER_MAX_COMP];
                double times[4];
                check(fft3d_server_result(srv, id, out, times) == FFT3D_OK, "result");
                check(times[0] <= times[3], "times in order");
                check(fft3d_server_release(srv, id) == FFT3D_OK, "release");
                check(fft3d_server_release(srv, id) < 0, "second release refused");
                done.fetch_add(1);
            }
        });
    }
    for (auto& t : clients) t.join();
    stop.store(true);
    reader.join();
    fft3d_request big{};
    big.n0 = big.n1 = big.n2 = 512;
    big.ncomp = 3;
    for (int k = 0; k < 3; ++k) big.in[k] = (const void*)(uintptr_t)0x100000;
    int64_t id = -1;
    check(fft3d_server_submit(srv, &big, &id) == FFT3D_ERR_BUDGET, "over-budget request refused");
    fft3d_server_counters st;
    check(fft3d_server_stats(srv, &st) == FFT3D_OK && st.completed == 240 && st.released == 240 &&
              st.reserved_bytes == 0,
          "all requests completed and released");
    check(done.load() == 240, "every client request done");
    check(fft3d_server_destroy(srv) == FFT3D_OK, "server destroy");
    puts(g_fail ? "FAIL server" : "ok server");
    return g_fail;
}

int main(int argc, char** argv)
{
    if (argc < 2) return 2;
    const std::string part = argv[1];
    if (part == "plans") return run_plans();
    if (part == "table" && argc > 2) return run_table(argv[2]);
    if (part == "server") return run_server();
    return 2;
}
