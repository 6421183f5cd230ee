// fft3d_internal.hpp -- host-side plan of the 3D r2c/c2r library and the
// kernel launchers it drives.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/fft3d.h"
#include "fft3d_sched.hpp"

namespace fft3d {

// LDS per workgroup on gfx950, and the budget for a tile when two
// workgroups should share a compute unit.
constexpr int kLdsMax = 160 * 1024;
constexpr int kLdsHalf = 80 * 1024;

// Thread counts / elements-per-thread of the two kernel tiers.  A tile of
// NT*EPT elements; every thread holds EPT elements in registers during a
// stage.  Small tier: 64 KB tiles, two workgroups per CU; big tier: up to the
// whole 160 KB of LDS.
constexpr int kNtSmall = 512;
constexpr int kNtBig = 512;
// Wide tier of the column kernels: the small tier's elements per thread on
// 1024 threads -- tiles as large as 128 KB (long columns at full 128-byte
// width) at the small tier's register budget, sixteen waves per CU.
constexpr int kNtWide = 1024;
template <typename T> struct Tier;
template <> struct Tier<float> {
    static constexpr int kEptSmall = 16;  // 8192 elements, 64 KB
    static constexpr int kEptBig = 40;    // 20480 elements, 160 KB
    // Waves per SIMD the small-tier rows kernels of even n2 are compiled for
    // (a register bound): the forward kernel eight (64 VGPRs, four 512-thread
    // workgroups a CU), the inverse six (80 VGPRs, three).  Measured at 512^3:
    // rows r2c 226 -> 215 us (16 rows a tile), rows c2r 252 -> 222 us (it had
    // needed 81 VGPRs, two workgroups a CU).
    static constexpr int kRowsWavesFwd = 8;
    static constexpr int kRowsWavesInv = 6;
};
template <> struct Tier<double> {
    static constexpr int kEptSmall = 8;   // 4096 elements, 64 KB
    static constexpr int kEptBig = 20;    // 10240 elements, 160 KB
    // no bound: six waves spill the forward kernel and were slower both ways
    static constexpr int kRowsWavesFwd = 1;
    static constexpr int kRowsWavesInv = 1;
};
// The wide tier's tiles walked by a persistent loop (k_cols_pipe), whose
// registers hold the next tile's loads beside the current tile's stages.
// FP32: the wide tier's 1024 threads of 16 elements (at most 128 VGPRs).
// FP64: 512 threads of 16 elements (two waves per SIMD, at most 256 VGPRs;
// on 1024 threads the FP64 kernel spilled some 100 registers and ran 40%
// slower than the one-tile kernel).  Measured at 1024^3 with 512 threads
// for both, FP32 pairs were 12.6 ms against 12.0 ms on 1024.
template <typename T> struct PipeTier;
template <> struct PipeTier<float> {
    static constexpr int kNt = kNtWide;
    static constexpr int kEpt = Tier<float>::kEptSmall;
};
template <> struct PipeTier<double> {
    static constexpr int kNt = kNtWide / 2;
    static constexpr int kEpt = 2 * Tier<double>::kEptSmall;
};

// Waves-per-SIMD bound of a rows kernel: the small tier's, none for the big.
template <typename T, int EPT, bool INV> constexpr int rows_waves()
{
    return EPT == Tier<T>::kEptSmall ? (INV ? Tier<T>::kRowsWavesInv : Tier<T>::kRowsWavesFwd) : 1;
}
// ... of a column kernel: eight for the fine tier, none otherwise.
template <typename T, int NT, int EPT> constexpr int cols_waves()
{
    return (sizeof(T) == 4 && NT == kNtFine && EPT == kEptFine) ? 8 : 1;
}

// Strided line pass over an array viewed as nbatch blocks of n rows by ncols
// columns: element (b, i, c) at b*bstride + i*S + c.  Tiles are W consecutive
// columns by all n rows of one block.
struct ColPass {
    int64_t S = 0;        // row stride (elements)
    int64_t ncols = 0;    // columns per block
    int64_t nbatch = 0;   // blocks
    int64_t bstride = 0;  // block stride (elements)
    int W = 0;            // tile width (power of two)
    int wshift = 0;       // log2(W)
    int64_t tiles_per_batch = 0;
    bool big = false;     // kernel tier: big, or
    bool wide = false;    // ... wide (column kernels only), else small
    bool fine = false;    // small tile on the fine tier (FP32, radix <= 8)
    bool pipe = false;    // wide tiles walked by a persistent loop (k_cols_pipe)
    size_t lds = 0;       // dynamic LDS bytes
};

struct Plan {
    int64_t n0 = 0, n1 = 0, n2 = 0;
    int64_t h = 0, H = 0;     // h = n2/2, H = h+1
    int Hs = 0;               // padded LDS row stride of the rows kernels
    int plane_Hs = 0;         // padded LDS row stride of the fused plane kernels
    int64_t C = 0;            // n1*H, columns of the n0 pass
    int64_t M = 0;            // n0*n1*H complex outputs
    int64_t N = 0;            // n0*n1*n2 real inputs
    int dtype = 0;            // 0 FP32, 1 FP64
    bool odd = false;         // a schedule has radix-5/7 stages: the kernels built with them

    // The batched kernel takes the plan's items (2/3 stages, even n2).
    bool batchable() const { return !odd && n2 % 2 == 0; }
    int elem = 4;             // bytes per real scalar

    AxisSched ax0{}, ax1{}, ax2h{};  // stage schedules: n0, n1, and the rows: h = n2/2 (n2 even) or n2 (odd)
    // Twiddle table (forward roots of unity) in long double, interleaved re, im;
    // offsets in complex elements.  Rounded once to the plan's dtype on upload.
    std::vector<long double> tw_host;
    int64_t off_ax2h = 0, off_post = 0, off_ax1 = 0, off_ax0 = 0, tw_count = 0;

    // plane step
    bool fused_plane = false;  // whole n1 x H plane in LDS
    int ppw = 1;               // planes per workgroup (fused)
    bool plane_big = false;
    size_t plane_lds = 0;
    int rpw = 1;               // rows per workgroup (split), forward rows kernel
    bool rows_big = false;
    size_t rows_lds = 0;
    int rpw_inv = 1;           // ... and of the inverse rows kernel (its own LDS budget)
    size_t rows_lds_inv = 0;
    ColPass pass1;             // n1 columns of each plane (split)
    ColPass pass0;             // n0 columns over C (the strided step)
    ColPass pass0t;            // n0 columns of the transposed layout [n1][n0][H] (transpose-based method)

    // cooperative plane step (split planes done in one launch, see k_plane_coop)
    bool coop = false;
    int coop_rt = 0, coop_ct = 0;  // row / column tasks per plane
    int coop_rpw = 0, coop_w = 0;  // rows per row task, columns per column task
    size_t coop_lds = 0;
    int coop_grid = 0;             // set with the device state
    int coop_nslots = 0;
    int coop_lag = 2;              // slots between a plane's two phases
    int n0_group = 1;              // n0-pass tiles sent together to one XCD (see plan_build_host)
    // Passes that walk their tiles in reverse (each XCD from its last group),
    // one bit per pass: 1 rows r2c, 2 n1 forward, 4 n0 forward, 8 n0 inverse,
    // 16 n1 inverse, 32 rows c2r.  A pass that reads what the previous pass
    // wrote last first finds more of it still in the memory-side cache
    // (measured at 512^3: the n1 passes and the inverse n0 pass reversed,
    // 0.7% faster pairs than the n1 passes alone).
    int rev = 2 | 8 | 16;
    int64_t coop_ctr_count = 0;
    int* d_ctr = nullptr;
    AxisSched* d_sched = nullptr;  // device copies of ax0, ax1, ax2h

    // the tuning the plan was built with (fft3d_plan_tuned), if any
    bool tuned = false;
    fft3d_tuning tuning{};

    // device state
    bool has_device = false;
    int device = -1;
    int cus = 0;               // compute units of the device
    void* d_tw = nullptr;

    std::string describe() const;
};

// Build the host part of a plan (schedules, tables, strategy).  Returns an
// FFT3D_* code; `why` receives a message on failure.
int plan_build_host(Plan& p, int64_t n0, int64_t n1, int64_t n2, int dtype, int flags, const fft3d_tuning* t,
                    std::string& why);

// Tiling of the split plane step (rows kernel + n1 column pass) for the
// plan's shape and dtype, also for plans that fuse the plane step.  Returns
// nullptr, or why the shape does not fit.
// rpw / rows_lds: the forward rows kernel's tile; rpw_inv / rows_lds_inv the
// inverse kernel's (same tier).
const char* split_tiling(const Plan& p, int& rpw, bool& rows_big, size_t& rows_lds, int& rpw_inv,
                         size_t& rows_lds_inv, ColPass& pass1);
// Small-tier tiling of the column pass along axis 0 (n0, over all C columns)
// or 1 (n1, per plane): the widest power-of-two W whose tile fits the small
// tier.  False if not even one column does.
bool small_colpass(const Plan& p, int axis, ColPass& cp);

// Factor n = 2^a 3^b 5^c 7^d into stages; false if n has another prime factor.
bool make_schedule(int64_t n, AxisSched& s);
// The schedule of an explicit radix list (first stage first); false unless
// every radix is 2, 3, 4, 8, 16, 5 or 7 and their product is n.
bool fill_schedule(int64_t n, const int* radices, int cnt, AxisSched& s);

// e^{-2 pi i e/m}, quadrant-reduced, in long double.
void root_of_unity_ld(int64_t e, int64_t m, long double* c, long double* s);

// Work queues of the cooperative plane step: one per XCD (8 on MI355X; the
// queue index is the hardware XCC id masked to this many).
constexpr int kCoopQueues = 16;

// Odd n2: (pair, bin) items per thread in the separation of two real rows
// from one complex line; the plan caps rows per tile so a tile has at most
// kNtSmall * kPairItems of them.
constexpr int kPairItems = 8;

// Box of kept modes of the pruned transforms: |k0| <= K0, |k1| <= K1,
// 0 <= k2 <= K2.  K0, K1 < 0 keep the whole axis; K2 is in [0, h].
struct PrunedBox {
    int K0 = -1, K1 = -1, K2 = 0;
};

// Per-dtype entry points (fft3d_kern_*.hip, fft3d_coop_*.hip, fft3d_pruned_*.hip).
#define FFT3D_DECLARE_DTYPE(sfx)                                                                            \
    hipError_t init_plain_##sfx();                                                                         \
    hipError_t init_coop_##sfx();                                                                          \
    hipError_t coop_occupancy_##sfx(const Plan& p, int* per_cu);                                           \
    hipError_t launch_plane_coop_##sfx(const Plan& p, const void* in, void* out, bool inverse, hipStream_t s); \
    hipError_t launch_plane_r2c_##sfx(const Plan& p, const void* x, void* X, hipStream_t s, bool padded);  \
    hipError_t launch_plane_c2r_##sfx(const Plan& p, const void* X, void* y, hipStream_t s, bool padded);  \
    hipError_t launch_rows_r2c_##sfx(const Plan& p, const void* x, void* X, int64_t nrows, int rev,        \
                                     hipStream_t s, bool padded);                                          \
    hipError_t launch_rows_c2r_##sfx(const Plan& p, const void* X, void* y, int64_t nrows, int rev,        \
                                     hipStream_t s, bool padded);                                          \
    hipError_t launch_cols_##sfx(const Plan& p, const ColPass& cp, int axis, int64_t tw_off, const void* in, \
                                 void* out, bool inverse, int rev, hipStream_t s);                         \
    hipError_t launch_swap01_##sfx(const Plan& p, const void* in, void* out, int64_t na, int64_t nb, hipStream_t s); \
    hipError_t init_pruned_##sfx();                                                                        \
    hipError_t launch_pruned_r2c_##sfx(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t s); \
    hipError_t launch_pruned_c2r_##sfx(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b,   \
                                       hipStream_t s);
FFT3D_DECLARE_DTYPE(f32)
FFT3D_DECLARE_DTYPE(f64)
// the kernels compiled with radix-5/7 stages (fft3d_kern_*_odd.hip, fft3d_pruned_*_odd.hip;
// no cooperative kernel)
FFT3D_DECLARE_DTYPE(f32_odd)
FFT3D_DECLARE_DTYPE(f64_odd)
#undef FFT3D_DECLARE_DTYPE

// Launchers (enqueue on `stream`, no allocation, no synchronisation).
// padded: the real array in the in-place layout (rows of 2H reals, n2 used)
// instead of contiguous rows of n2.
hipError_t launch_plane_r2c(const Plan& p, const void* x, void* X, hipStream_t stream, bool padded = false);
hipError_t launch_plane_c2r(const Plan& p, const void* X, void* y, hipStream_t stream, bool padded = false);
// rev: walk each XCD's chunk of tiles from its end (see xcd_tile).
// nrows: rows to transform from the given pointers (n0*n1 for a whole array).
hipError_t launch_rows_r2c(const Plan& p, const void* x, void* X, int64_t nrows, int rev, hipStream_t stream,
                           bool padded = false);
hipError_t launch_rows_c2r(const Plan& p, const void* X, void* y, int64_t nrows, int rev, hipStream_t stream,
                           bool padded = false);
// axis: 0 = n0, 1 = n1 (index into the plan's device schedules).
hipError_t launch_cols(const Plan& p, const ColPass& cp, int axis, int64_t tw_off, const void* in, void* out,
                       bool inverse, int rev, hipStream_t stream);
hipError_t launch_plane_coop(const Plan& p, const void* in, void* out, bool inverse, hipStream_t stream);
// Exchange of the two outer axes of an [na][nb][H] array of complex rows
// (the explicit transpose of the transpose-based method).
hipError_t launch_swap01(const Plan& p, const void* in, void* out, int64_t na, int64_t nb, hipStream_t stream);
// Pruned transforms (the whole path, enqueued): forward writes the kept box
// of X only; inverse reads the kept box of X only (see fft3d_pruned.hpp).
hipError_t launch_pruned_r2c(const Plan& p, const void* x, void* X, const PrunedBox& b, hipStream_t stream);
hipError_t launch_pruned_c2r(const Plan& p, const void* X, void* y, void* work, const PrunedBox& b,
                             hipStream_t stream);
// The message fft3d_last_error() returns on this thread.
void set_last_error(const std::string& m);
// Raise the dynamic-LDS limit of every kernel once per process.
hipError_t kernels_init();
// Device part of the cooperative plane step: grid from occupancy on the
// current device, counter block allocation.  No-op unless p.coop.
hipError_t coop_setup(Plan& p);

}  // namespace fft3d

// The opaque plan handle of the C interface.
struct fft3d_plan_s {
    fft3d::Plan p;
};
