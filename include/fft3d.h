/*
 * fft3d.h -- C interface of libfft3d, a 3D real-to-complex / complex-to-real
 * FFT for one AMD Instinct MI355X (gfx950).
 *
 * The operation (paper: Chatterjee, Verma & Chaudhuri, "Transpose-free Fast
 * Fourier Transform for Turbulence Simulation", Sec. 2, problem statement):
 * the forward transform (r2c) takes a real n0 x n1 x n2 array x to the complex
 * n0 x n1 x (n2/2+1) array
 *
 *   X[k0,k1,k2] = sum_{j0,j1,j2} x[j0,j1,j2] exp(-2 pi i (k0 j0/n0 + k1 j1/n1 + k2 j2/n2)),
 *
 * 0 <= k2 <= n2/2; the inverse (c2r) maps such an array back to a real one.
 * It is computed the transpose-free way (Sec. 2.1 items 1 and 3, Sec. 2.2):
 * 2D r2c transforms of the n0 planes, then a length-n0 c2c transform that
 * reads the strided n0 columns of the natural-order spectrum in place; the
 * inverse runs the steps in reverse order.
 *
 * Conventions (the paper is silent; these are FFTW's, which it builds on):
 *   - minus sign forward, plus sign inverse, no normalisation:
 *     c2r(r2c(x)) = n0*n1*n2 * x;
 *   - C order (n2 fastest); complex values interleaved (re, im) in the real
 *     type of the plan (float2 / double2);
 *   - the spectrum is in natural order: X[k0,k1,k2] at offset
 *     (k0*n1 + k1)*(n2/2+1) + k2, index k >= n/2 standing for k - n;
 *   - c2r of an arbitrary half spectrum X returns Re(IDFT3(E(X))), where E
 *     completes the k2 axis with E[k0,k1,n2-k2] = conj(X[-k0,-k1,k2]) and
 *     keeps the k2 = 0 plane (and, for even n2, the k2 = n2/2 plane) as given
 *     (equivalently: the imaginary parts of those bins of each row are
 *     dropped after the n0 and n1 inverse passes).
 *
 * Memory and threads:
 *   - every array is device memory owned by the caller; a plan owns only its
 *     twiddle table (device) and its host description;
 *   - fft3d_r2c, fft3d_c2r and fft3d_batch_submit allocate nothing and
 *     never wait for the device: they enqueue kernels on the given stream
 *     and return (fft3d_batch_submit returns FFT3D_ERR_BUSY, enqueuing
 *     nothing, when all 16 slots of its staging ring are still in flight);
 *   - the library allocates device or pinned memory only in fft3d_init (the
 *     device's batch ring: about 9 MB device + 9 MB pinned host, kept until
 *     the process ends), fft3d_plan / fft3d_plan_ex (the plan's tables),
 *     fft3d_batch_create and fft3d_server_create;
 *   - a plan is immutable after creation and may be used from several
 *     streams or host threads at once, as long as every concurrent call has
 *     its own output and work buffers -- except a plan whose plane step is
 *     cooperative (fft3d_plan_describe reports plane.kind "coop": planes
 *     larger than LDS): it owns a small device counter block, so its calls
 *     must not overlap in time (issue them on one stream, or order them with
 *     events; use one plan per concurrently used stream);
 *   - a plan belongs to the device that was current when it was created;
 *     calls must be made with that device current.
 *
 * Errors are returned as negative codes, never thrown; fft3d_last_error()
 * gives a thread-local message for the last failing call on this thread.
 */
#ifndef FFT3D_H
#define FFT3D_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fft3d_plan_s* fft3d_plan_t;

/* Real type of a plan.  All arithmetic of the plan's kernels is in this type;
 * twiddle factors are computed in extended precision on the host and rounded
 * to it once. */
typedef enum { FFT3D_F32 = 0, FFT3D_F64 = 1 } fft3d_dtype;

enum {
    FFT3D_OK = 0,
    FFT3D_ERR_INVALID_ARG = -1, /* null/overlapping pointers, bad sizes or dtype */
    FFT3D_ERR_UNSUPPORTED = -2, /* extents the GPU path does not cover */
    FFT3D_ERR_NOMEM = -3,       /* plan table allocation failed */
    FFT3D_ERR_HIP = -4,         /* a HIP runtime call failed (no device, launch error) */
    FFT3D_ERR_BUDGET = -5,      /* a server request needs more than the server's memory budget */
    FFT3D_ERR_ALIGN = -6,       /* a pointer is not aligned to the plan's complex type */
    FFT3D_ERR_BUSY = -7         /* every slot of the batch staging ring is in flight, or a batched
                                   launch asked about has not finished: nothing was done, try again */
};

/* Transform directions of a batch item. */
enum { FFT3D_R2C = 0, FFT3D_C2R = 1, FFT3D_ROUNDTRIP = 2 };

/* Plan flags for fft3d_plan_ex. */
enum {
    FFT3D_PLAN_HOST_ONLY = 1,  /* build schedules/tables on the host only; cannot execute */
    FFT3D_PLAN_COOP_PLANE = 2, /* planes larger than LDS: one cooperative persistent launch
                                  for the plane step (rows + n1 columns through the L2 of
                                  one XCD) instead of the default rows kernel + n1 column
                                  kernel */
    FFT3D_PLAN_TUNED = 4       /* tile shapes and schedules from the process's tuning table
                                  (fft3d_autotune, fft3d_tune_load) when it has an entry for
                                  the shape on this GPU architecture, else the rule */
};

/* Library version (major*10000 + minor*100 + patch). */
int fft3d_version(void);

/* Set up the current device for batched launches (the batched form of the
 * paper's two steps, Sec. 2.1-2.2, over many fields): finds the device's
 * XCDs (one probe launch, synchronous) and allocates the staging ring of
 * fft3d_batch_submit (16 slots of a task image and a counter block: about
 * 9 MB of device memory and 9 MB of pinned host memory, kept until the
 * process ends).  Call it once per device, with that device current, before
 * fft3d_batch_submit / fft3d_batch_create on it (they return
 * FFT3D_ERR_INVALID_ARG otherwise); further calls do nothing.  Plans and the
 * single-field transforms do not need it; fft3d_server_create calls it.
 * Returns FFT3D_OK, FFT3D_ERR_HIP or FFT3D_ERR_NOMEM. */
int fft3d_init(void);

/* Create a plan for the transforms of an n0 x n1 x n2 real array in the
 * given dtype (the operation of Sec. 2; like the FFTW plans the paper's
 * implementation builds its two steps on, Sec. 2.2, a plan is made once per
 * shape and reused).
 * Supported extents: every n >= 1 whose prime factors are 2, 3, 5 and 7, with
 * n0, n1 <= 4096 and n2 <= 8192 (n2 odd or even).  Other extents return
 * FFT3D_ERR_UNSUPPORTED; n < 1, a bad dtype or out == NULL return
 * FFT3D_ERR_INVALID_ARG.  Builds the radix schedules and the twiddle table
 * (host, FP64 via long double) and uploads the table to the current device
 * (hipMalloc + hipMemcpy, synchronous).  The library allocates only here, in
 * fft3d_init, fft3d_batch_create and fft3d_server_create: the transforms
 * themselves allocate nothing.
 * On success *out receives the plan. */
int fft3d_plan(int64_t n0, int64_t n1, int64_t n2, int dtype, fft3d_plan_t* out);

/* As fft3d_plan, with flags: FFT3D_PLAN_HOST_ONLY builds no device state
 * (usable for fft3d_plan_describe / fft3d_plan_twiddles, not for transforms);
 * FFT3D_PLAN_COOP_PLANE selects the cooperative plane step for large planes,
 * which allocates its counter block (some KB) here. */
int fft3d_plan_ex(int64_t n0, int64_t n1, int64_t n2, int dtype, int flags, fft3d_plan_t* out);

/* ---- Tuning: the tile shapes and radix schedules of a plan --------------
 *
 * How a plan cuts the paper's two steps (Sec. 2.1 items 1 and 3) into kernel
 * launches: the plane step fused (a whole plane in LDS), split (rows kernel +
 * n1 column pass) or cooperative (both in one persistent launch through the
 * L2 of one XCD); the rows per tile of the rows kernels; the width of the
 * column tiles of the n1 pass and of the strided n0 pass; how n0 tiles are
 * grouped onto XCDs; the order in which each pass walks its tiles; and the
 * radix schedule of every axis.  None of this changes what is computed; a
 * different radix schedule changes the rounding (results stay within the
 * plan's accuracy bound), the rest gives bit-identical results.
 *
 * fft3d_plan picks all of it by rule.  fft3d_plan_tuned takes it from a
 * tuning (a zero field keeps the rule for that field); fft3d_autotune times
 * the candidates on the current device and returns the fastest. */
typedef struct {
    int32_t plane;       /* 0 rule; FFT3D_TUNE_FUSED, FFT3D_TUNE_SPLIT or FFT3D_TUNE_COOP */
    int32_t rows_rpw;    /* rows per tile of the forward rows kernel (split / cooperative plane
                            step) and of the cooperative step's row tasks */
    int32_t n1_w;        /* columns per tile of the n1 pass (power of two, <= 64) */
    int32_t n0_w;        /* columns per tile of the n0 pass (power of two, <= 64) */
    int32_t n0_group;    /* n0-pass tiles sent together to one XCD (>= 1) */
    int32_t walk;        /* 0 rule, else 64 + walk-order bits: a set bit reverses the tile order of
                            1 rows r2c, 2 n1 forward, 4 n0 forward, 8 n0 inverse, 16 n1 inverse,
                            32 rows c2r */
    int32_t coop_lag;    /* cooperative plane step: slots between a plane's two phases (1..256) */
    int32_t coop_rpw;    /* ... rows per row task */
    int32_t coop_w;      /* ... columns per column task (power of two) */
    int32_t radix[3][8]; /* radix schedule of axis 0 (n0), 1 (n1), 2 (the rows: length n2/2 for
                            even n2, n2 for odd n2), first stage first, 0-terminated; radices 2, 3,
                            4, 8, 16, 5, 7 with product the axis length; all zero: rule */
    int32_t rows_rpw_inv; /* rows per tile of the inverse rows kernel (split plane step) */
    int32_t cols_pipe;    /* column passes on the wide tier (tiles of up to 128 KB, one workgroup
                             per CU): 0 rule, 1 one tile per workgroup, 2 one workgroup per CU that
                             walks its tiles and loads each one ahead */
} fft3d_tuning;

enum { FFT3D_TUNE_FUSED = 1, FFT3D_TUNE_SPLIT = 2, FFT3D_TUNE_COOP = 3 };

/* As fft3d_plan_ex with the plan's tile shapes and schedules from *t (NULL:
 * the rule).  A field that cannot apply to the shape (a fused plane step for
 * a plane larger than LDS, a tile that fits no kernel tier, a radix list
 * whose product is not the axis length) is FFT3D_ERR_INVALID_ARG, with the
 * field named by fft3d_last_error(). */
int fft3d_plan_tuned(int64_t n0, int64_t n1, int64_t n2, int dtype, int flags, const fft3d_tuning* t,
                     fft3d_plan_t* out);

/* Time the candidate tunings of an n0 x n1 x n2 plan of the given dtype on
 * the current device and return the fastest in *best (fields the search
 * left at the rule are 0).  The search, pass by pass with the plan's own
 * kernels (fft3d_run_pass): rows per tile of each rows kernel; n1 and n0 tile widths and
 * the n0 XCD grouping; the radix schedule of every axis; the plane step
 * (split against cooperative over lags 1..32 and task sizes); the wide
 * column passes' persistent loop against one tile per workgroup; the walk
 * order; then whole r2c+c2r pairs of the rule plan against the tuned one (the
 * rule is kept unless the tuned plan is faster).  effort 0: a short search;
 * 1: the full one.  Allocates its own buffers (about 4 x the spectrum's
 * bytes), synchronises the device, takes seconds.  The winner is also kept in
 * the process's tuning table (key: GPU architecture, extents, dtype), from
 * which fft3d_plan_ex with FFT3D_PLAN_TUNED takes it.  report: NULL, or a
 * buffer for a JSON account of every candidate timed (truncated to len;
 * the return value is the full length needed, as fft3d_plan_describe). */
int fft3d_autotune(int64_t n0, int64_t n1, int64_t n2, int dtype, int effort, fft3d_tuning* best, char* report,
                   size_t len);

/* The tuning table of the process (what fft3d_autotune found, and what
 * fft3d_tune_load read), keyed by (GPU architecture, n0, n1, n2, dtype).
 * fft3d_tune_lookup: 1 and *t filled when the current device's architecture
 * has an entry for the shape, else 0.  fft3d_tune_save writes the table as
 * JSON to a file; fft3d_tune_load merges a file written so into the table
 * (entries of the file replace equal keys).  FFT3D_ERR_INVALID_ARG for a
 * file that cannot be opened or parsed (the table is unchanged then). */
int fft3d_tune_lookup(int64_t n0, int64_t n1, int64_t n2, int dtype, fft3d_tuning* t);
int fft3d_tune_save(const char* path);
int fft3d_tune_load(const char* path);

/* Free a plan and its device table.  NULL is accepted.  The caller must make
 * sure no enqueued work still uses the plan. */
int fft3d_plan_destroy(fft3d_plan_t p);

/* Bytes of the optional c2r work buffer: n0*n1*(n2/2+1) complex values --
 * the spectrum's size (Sec. 2: n0 x n1 x (n2/2+1) complex), into which the
 * inverse's first step (the n0 columns, Sec. 2.1 run in reverse) writes when
 * the input spectrum is to be kept.  0 for a NULL plan. */
size_t fft3d_work_bytes(fft3d_plan_t p);
/* Bytes of the real array (n0*n1*n2 reals) and of the spectrum. */
size_t fft3d_real_bytes(fft3d_plan_t p);
size_t fft3d_complex_bytes(fft3d_plan_t p);

/* Forward transform (paper Sec. 2.1 steps 1 and 3, Sec. 2.2).
 * x: device, n0*n1*n2 reals, C order, not modified.
 * X: device, n0*n1*(n2/2+1) complex, written in natural order.
 * x and X must not overlap; both aligned to the complex type (8 or 16 bytes).
 * Enqueued on `stream` (0 = the null stream). */
int fft3d_r2c(fft3d_plan_t p, const void* x, void* X, hipStream_t stream);

/* Inverse transform (the same steps in reverse order, Sec. 2.1).
 * X: device, n0*n1*(n2/2+1) complex.  y: device, n0*n1*n2 reals.
 * work: device buffer of fft3d_work_bytes(p), or NULL.  With work, X is
 * preserved; without, X is used as scratch and overwritten.  X, y and work
 * must not overlap; all aligned to the complex type. */
int fft3d_c2r(fft3d_plan_t p, void* X, void* y, void* work, hipStream_t stream);

/* One item of a batch.
 *   R2C:       in = x (real), out = X (complex); mid, work unused.
 *   C2R:       in = X (complex), out = y (real); work optional as in fft3d_c2r.
 *   ROUNDTRIP: in = x, mid = X (receives r2c(x)), out = y = c2r(X); work
 *              optional (with work, mid keeps the spectrum). */
typedef struct {
    fft3d_plan_t plan;
    int dir;
    const void* in;
    void* mid;
    void* out;
    void* work;
} fft3d_batch_item;

/* Run every item in a few batched launches on `stream` (the batched form of
 * the plane step and the strided n0 step, Sec. 2.1 items 1 and 3, Sec. 2.2,
 * over many fields at once).  Requires fft3d_init on the items' device.
 * Each item becomes a chain of passes (the ones fft3d_r2c / fft3d_c2r would
 * launch).  By rule (level mode, see fft3d_batch_tuning) the passes go into
 * one launch per pass level, tile kind and dtype, each launch running that
 * pass of many items at once, every pass in a later launch than the pass
 * it reads.  The alternative is one persistent launch whose workgroups take
 * tiles of all chains from ticket counters, a pass waiting for the previous
 * pass of the same item.  Every result is bit-identical to the item run
 * alone.
 * Items run CONCURRENTLY: a buffer one item writes (out, mid, work, and in
 * for C2R without work) must not overlap any buffer of another item; inputs
 * that are only read may be shared.  Plans must outlive the launch.
 * All items are validated first; if any is invalid nothing is enqueued (all
 * or nothing) and fft3d_last_error() names the first bad item.
 * No allocation and no wait: the task list is staged through the ring of
 * pinned/device buffers fft3d_init set up (16 launches deep); a submit that
 * finds fewer free slots than it needs returns FFT3D_ERR_BUSY and enqueues
 * nothing.  Batches of more than 4096 passes are split into several
 * launches (one slot each).  The persistent kernel's error bits (see
 * fft3d_batch_status; the level mode has none) are kept per launch:
 * fft3d_batch_submit_checked returns a token to read them with.
 * Items whose extents have a factor 5 or 7, or an odd n2, run their own
 * kernels (as fft3d_r2c / fft3d_c2r), on the same stream after the batched
 * launch. */
int fft3d_batch_submit(const fft3d_batch_item* items, int n, hipStream_t stream);

/* flags of fft3d_batch_submit_ex / fft3d_batch_create */
enum {
    FFT3D_BATCH_SEQUENTIAL = 2, /* fft3d_batch_submit_ex only: no batched kernel; the items' own kernels,
                                   item after item (the per-field launch sequence) */
    FFT3D_BATCH_DIRECT = 4      /* fft3d_batch_create only: launch with hipLaunchKernel instead of a graph */
};
int fft3d_batch_submit_ex(const fft3d_batch_item* items, int n, int flags, hipStream_t stream);

/* As fft3d_batch_submit; *token receives a number for fft3d_batch_check (-1
 * when no batched launch was staged, e.g. only radix-5/7 or odd-n2 items). */
int fft3d_batch_submit_checked(const fft3d_batch_item* items, int n, hipStream_t stream, int64_t* token);
/* Error bits of the batched launch(es) a token names, without waiting: 0
 * clean, else bit 1 (a dependency wait hit its spin limit: tiles skipped),
 * bit 2 (a ticket queue had no workgroup on its XCD: its items did not run)
 * and/or bit 4 (a workgroup's ticket loop ran more iterations than its queue
 * has tickets and was ended) -- the results of such a launch are not
 * valid.  FFT3D_ERR_BUSY
 * while the launch has not finished; FFT3D_ERR_INVALID_ARG for an unknown
 * token or one older than the last 256 ring launches of its device. */
int fft3d_batch_check(int64_t token);

/* For callers that cannot allocate device or pinned memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * fft3d_batch_submit (level mode) with the task image of the batched
 * launches in a static device array of the library (1 MiB per device, held
 * until the process ends) instead of the ring.  Allocates nothing: copies the
 * task image (from a host buffer of the calling thread, pageable) into the
 * array and enqueues the launches that read it, all on `stream`.
 * Requires fft3d_init on the items' device (which finds the array's address
 * there).  Items, validation (all or nothing), results (bit-identical to
 * fft3d_batch_submit's) and the handling of radix-5/7 or odd-n2 items as
 * fft3d_batch_submit.  Limit: one task image of at most 4096 passes
 * (about 680 ROUNDTRIP items with split planes); a larger batch returns
 * FFT3D_ERR_UNSUPPORTED and enqueues nothing.  status: NULL, or a device int
 * that receives the launch's error bits behind it on the stream (always 0:
 * the level mode has no waits that could give up).  Every call on a device shares that device's array: calls on one
 * device must not overlap in time (issue them on one stream, or order them
 * with events); overlapping calls race and give wrong results. */
int fft3d_batch_submit_static(const fft3d_batch_item* items, int n, int* status, hipStream_t stream);

/* A batch built once and launched many times: the task list and its counters
 * live in device memory owned by the handle (allocated here, synchronously),
 * and the launch is a hipGraph (instantiated here: in level mode one kernel
 * node per launch, each after the launches it reads from; persistent: one
 * node) unless FFT3D_BATCH_DIRECT (the launches in order on the stream).  The item pointers are fixed at creation.  The same
 * concurrency rules as fft3d_batch_submit apply; at most 4096 passes.
 * Items whose extents have a factor 5 or 7, or an odd n2, are refused here
 * (FFT3D_ERR_UNSUPPORTED): the batched kernel has only the radix-2/3 stages
 * and the half-length rows of even n2;
 * fft3d_batch_submit runs such items with their own kernels, after the
 * batched launch of the others.
 * Launches of one handle must not overlap in time (same stream, or ordered);
 * the kernel leaves its counters cleared for the next launch. */
typedef struct fft3d_batch_s* fft3d_batch_t;
int fft3d_batch_create(const fft3d_batch_item* items, int n, int flags, fft3d_batch_t* out);
int fft3d_batch_launch(fft3d_batch_t b, hipStream_t stream);
/* Error bits of the last finished launch (synchronises the device):
 * 0 = clean, bit 1 = a dependency wait hit its spin limit (its tiles
 * skipped), bit 2 = a ticket queue had no workgroup on its XCD (its items
 * did not run), bit 4 = a workgroup's ticket loop ran more iterations than
 * its queue has tickets and was ended.  The bits come from the persistent
 * launch; in level mode (the rule) there are no waits or queues and the
 * status is always 0. */
int fft3d_batch_status(fft3d_batch_t b);
/* JSON: items, tickets (tiles), grid (the persistent launch's workgroups; 0
 * in level mode), LDS bytes, graph, mode, the level mode's launches as
 * [kind, dtype, tasks, tiles, LDS bytes], and the tasks in ticket (level
 * mode: launch) order as [kind, dtype, tiles, index of the task waited for,
 * LDS bytes].  Same return convention as fft3d_plan_describe. */
int fft3d_batch_describe(fft3d_batch_t b, char* buf, size_t len);
int fft3d_batch_destroy(fft3d_batch_t b);

/* Launch shape of the batched kernel (what fft3d_batch_autotune chooses;
 * a zero field keeps the rule):
 *   mode: 0 (rule) or 3 level mode: one launch per pass level, tile kind
 *         and dtype, each launch's kernel holding only its tile kind, each
 *         pass in a later launch than the pass it reads (a batch handle's
 *         graph runs a launch after the launches it reads from only; on a
 *         stream, launch order is the only dependency), so lag, wg_per_cu
 *         and spin_limit do not apply and the status is always 0;
 *         the one persistent launch (ticket queues, bounded dependency
 *         waits) with 1 every item pinned to one XCD (one ticket queue per
 *         XCD), 2 one queue for all workgroups, 4 pinned when that balances
 *         the XCDs, else one queue;
 *   lag: slots between an item's consecutive passes in the ticket order
 *        (rule: the number of items, i.e. every item's first pass, then
 *        every item's second pass, ...);
 *   widen: 1 small fields get fewer, larger tiles (several planes per plane
 *          tile, column tiles widened to the tier; the rule), 2 the plans'
 *          own tile shapes;
 *   wg_per_cu: workgroups per CU (rule: as many as fit);
 *   spin_limit: polls of a dependency wait before it gives up (error bit 1:
 *               the waiting task's tiles are skipped, every later wait gives
 *               up at once, the launch still ends); rule 2^20; negative: no
 *               poll at all -- every dependent task fails at once, which
 *               tests the error path without a slow or stuck launch. */
typedef struct {
    int32_t mode;
    int32_t lag;
    int32_t widen;
    int32_t wg_per_cu;
    int32_t spin_limit;
} fft3d_batch_tuning;

/* fft3d_batch_create with a launch shape (bt NULL: the rule).  Out-of-range
 * fields are FFT3D_ERR_INVALID_ARG. */
int fft3d_batch_create_tuned(const fft3d_batch_item* items, int n, int flags, const fft3d_batch_tuning* bt,
                             fft3d_batch_t* out);

/* Time candidate launch shapes of the batch of these items on the current
 * device (each as a directly launched batch handle, several launches each)
 * and return the fastest in *best (the rule is kept unless a candidate is
 * faster).  The items run many times: their outputs are overwritten, and so
 * are the inputs of C2R items without work.  Synchronises the device.
 * report: NULL or a buffer for a JSON account of the candidates (return
 * value: the full length, as fft3d_plan_describe). */
int fft3d_batch_autotune(const fft3d_batch_item* items, int n, int effort, fft3d_batch_tuning* best, char* report,
                         size_t len);

/* The transpose-based method of the paper's Sec. 2.1, for comparison with
 * the transpose-free path (Sec. 2.2): step 1 (the same plane step) into
 * `work`, step 2 an explicit exchange of the n0 and n1 axes (rows of n2/2+1
 * complex values stay contiguous) into Xt, step 3 the n0 columns of that
 * layout (stride n2/2+1) in place.  Xt: n1 x n0 x (n2/2+1) complex, i.e.
 * Xt[k1][k0][k2] = X[k0][k1][k2] -- FFTW's "transposed out" order; bit for bit
 * the transpose of fft3d_r2c's output.  work: fft3d_work_bytes(p), required.
 * fft3d_c2r_transposed inverts it in reverse order (n0 columns of Xt into
 * work, exchange back into Xt, plane step to y): Xt is overwritten. */
int fft3d_r2c_transposed(fft3d_plan_t p, const void* x, void* Xt, void* work, hipStream_t stream);
int fft3d_c2r_transposed(fft3d_plan_t p, void* Xt, void* y, void* work, hipStream_t stream);

/* Pruned transforms for the dealiased pseudo-spectral solver the path serves
 * (Sec. 1): the solver keeps only the modes of a box -- with the two-thirds
 * rule, |k| <= n/3 on every axis -- and sets the rest to zero, so its forward
 * transforms need only the box's modes and its inverse transforms read only
 * those.  kmax = {K0, K1, K2} (host array) keeps |k0| <= K0, |k1| <= K1 (the
 * signed index: k for k <= n/2, k - n above) and 0 <= k2 <= K2.  K0 or K1
 * negative, or with 2K+1 >= n, keeps that whole axis; K2 negative or >= n2/2
 * keeps every bin.  Every pass skips the lines and rows outside the box, so
 * the pair moves fewer bytes (about 41% fewer at 512^3 with K = n/3).
 *   fft3d_r2c_pruned: X holds fft3d_r2c's values on the kept modes, bit for
 *     bit; its other elements are unspecified (what X held, or intermediate
 *     values of the passes): the caller treats them as zero.
 *   fft3d_c2r_pruned: y = fft3d_c2r of the spectrum that equals X on the kept
 *     modes and is zero elsewhere (equal value for value); X's elements
 *     outside the box are never read.  With work (fft3d_work_bytes), X is
 *     left unchanged; without, X is overwritten.
 * Arguments, alignment and overlap rules, and errors as fft3d_r2c /
 * fft3d_c2r; a NULL kmax is FFT3D_ERR_INVALID_ARG; plans with odd n2 return
 * FFT3D_ERR_UNSUPPORTED. */
int fft3d_r2c_pruned(fft3d_plan_t p, const void* x, void* X, const int64_t kmax[3], hipStream_t stream);
int fft3d_c2r_pruned(fft3d_plan_t p, void* X, void* y, void* work, const int64_t kmax[3], hipStream_t stream);

/* In-place transforms in FFTW's padded layout: buf holds n0 x n1 rows of
 * 2*(n2/2+1) reals each, of which the first n2 are the row (the rest is
 * padding, never read) -- exactly the bytes of the n0 x n1 x (n2/2+1)
 * complex spectrum, which replaces them (fft3d_r2c_inplace); the reverse for
 * fft3d_c2r_inplace (the padding of the output rows is left unspecified).
 * Same kernels as fft3d_r2c / fft3d_c2r (without work): the results are bit
 * for bit theirs.  Plans with the cooperative plane step run the two-kernel
 * plane step here.  buf must be aligned to the complex type. */
int fft3d_r2c_inplace(fft3d_plan_t p, void* buf, hipStream_t stream);
int fft3d_c2r_inplace(fft3d_plan_t p, void* buf, hipStream_t stream);

/* The passes a transform is made of, for fft3d_run_pass.  The forward
 * transform is PLANE_R2C, N1_FWD (split plans only), N0_FWD (n0 > 1); the
 * inverse is N0_INV (n0 > 1), N1_INV (split plans only), PLANE_C2R.  A plan's
 * plane step is "fused" when a whole n1 x (n2/2+1) plane fits in LDS (one
 * kernel does both in-plane axes), "split" for larger planes (rows kernel +
 * N1 pass), or "coop" with FFT3D_PLAN_COOP_PLANE (one cooperative launch
 * does both); fft3d_plan_describe reports which, and the pass lists of both
 * directions. */
enum {
    FFT3D_PASS_PLANE_R2C = 0, /* in: real x; out: spectrum (after the plane step) */
    FFT3D_PASS_N1_FWD = 1,    /* in/out: spectrum (in == out allowed) */
    FFT3D_PASS_N0_FWD = 2,    /* in/out: spectrum (in == out allowed); paper step 3 */
    FFT3D_PASS_N0_INV = 3,    /* in/out: spectrum (in == out allowed) */
    FFT3D_PASS_N1_INV = 4,    /* in/out: spectrum (in == out allowed) */
    FFT3D_PASS_PLANE_C2R = 5, /* in: spectrum; out: real y */
    /* the transpose-based method (fft3d_r2c_transposed): */
    FFT3D_PASS_SWAP01 = 6,    /* in: natural-order spectrum [n0][n1][H]; out: transposed [n1][n0][H] */
    FFT3D_PASS_SWAP10 = 7,    /* in: transposed; out: natural order */
    FFT3D_PASS_N0T_FWD = 8,   /* in/out: transposed spectrum (in == out allowed) */
    FFT3D_PASS_N0T_INV = 9    /* in/out: transposed spectrum (in == out allowed) */
};

/* Enqueue one pass of the plan on `stream` (no allocation, no sync): the same
 * kernel and launch shape the transforms use.  Pointers as for fft3d_r2c /
 * fft3d_c2r; spectrum in/out may be equal, real/spectrum must not overlap.
 * Returns FFT3D_ERR_INVALID_ARG for a pass the plan does not have. */
int fft3d_run_pass(fft3d_plan_t p, int pass, const void* in, void* out, hipStream_t stream);

/* Static message for an error code (the failure conventions of every entry
 * point above). */
const char* fft3d_strerror(int code);
/* Thread-local message of the last failing call on this thread ("" if none);
 * valid until the next failing call on the thread. */
const char* fft3d_last_error(void);

/* JSON description of the plan (extents, schedules, strategy, tile widths,
 * launch grids) written to buf (NUL-terminated, truncated to len).  Returns
 * the full length needed, excluding the NUL, or a negative code. */
int fft3d_plan_describe(fft3d_plan_t p, char* buf, size_t len);

/* Copy the plan's twiddle table for one axis to host memory, as FP64 values of
 * the table exactly as the kernels use it (rounded to the plan's dtype).
 * which: 0 = n0 stages, 1 = n1 stages, 2 = row stages (length n2/2 for even
 * n2, n2 for odd n2), 3 = r2c split roots exp(-2 pi i k/n2) for k = 0..n2/2
 * (used for even n2 only).  out: 2*count doubles (re, im).
 * Returns the number of complex entries of that table, or a negative code;
 * copies min(count, entries). */
int64_t fft3d_plan_twiddles(fft3d_plan_t p, int which, double* out, int64_t count);

/* Slab decomposition over p devices (design of the multi-device form of the
 * paper's exchange, Sec. 2.2, Fig. 3): device q holds rows [q*n0/p, (q+1)*n0/p)
 * of the n0 x ncols natural-order array after step 1 and owns columns
 * [r*ncols/p, (r+1)*ncols/p) for step 3.  The block device src sends to device
 * dst is the strided vector: first element offset (within src's slab), count
 * rows, blocklen contiguous elements per row, stride between rows -- the
 * analogue of an MPI vector type.  out[4] = {first, count, blocklen, stride};
 * the same block lands at offset out[4+0] of dst's natural-order column slab
 * (n0 rows of ncols/p) with stride out[4+3]: out has 8 entries.
 * Requires p >= 1, n0 % p == 0, ncols % p == 0, 0 <= src, dst < p. */
int fft3d_exchange_block(int64_t n0, int64_t ncols, int64_t p, int64_t src, int64_t dst, int64_t* out);

/* ---- Serving: continuous batching of transform requests ----------------
 *
 * A server owns a device arena of `budget_bytes` (allocated once, at
 * creation) from which it places every request's outputs and work buffers,
 * a cache of plans, a dispatcher thread and `nstreams` streams.  A request --
 * r2c or c2r of `ncomp` fields of one shape and dtype (say the three
 * components of a velocity field) -- is admitted when its bytes fit in what
 * the arena has free (first come, first served: a request waits behind an
 * earlier one that does not fit yet), then launched at once on the stream
 * with the least work in flight: requests of at most `batch_points` real
 * points per field go, with
 * every other such request admitted in the same round, through one batched
 * launch (fft3d_batch_submit), larger ones through fft3d_r2c / fft3d_c2r per
 * field.  Requests that arrive while others run are admitted and launched as
 * memory frees up, so their work overlaps on the device.  Every result is
 * bit-identical to the same transform run alone.  A request's outputs stay in
 * the arena until fft3d_server_release; its work buffers are freed when it
 * completes.  Inputs are the caller's (device, not modified, valid until the
 * request completes). */
typedef struct fft3d_server_s* fft3d_server_t;

enum { FFT3D_SERVER_NO_DEVICE = 1 }; /* host logic only: the arena is address
                                        arithmetic, plans are host-only, no
                                        kernel runs and a request completes as
                                        soon as it is launched (for tests) */

typedef struct {
    size_t budget_bytes;  /* arena size (outputs + work buffers of admitted requests) */
    int nstreams;         /* 1..16 streams (0: 4) */
    int64_t batch_points; /* per-field size limit of batched requests (0: 2^21 real points) */
    int max_batch_items;  /* fields per batched launch (0: 192) */
    int flags;            /* FFT3D_SERVER_* */
} fft3d_server_config;

#define FFT3D_SERVER_MAX_COMP 8

typedef struct {
    int64_t n0, n1, n2;
    int dtype; /* FFT3D_F32 / FFT3D_F64 */
    int dir;   /* FFT3D_R2C (in: real fields, out: spectra) or FFT3D_C2R (in: spectra, out: real fields) */
    int ncomp; /* 1..FFT3D_SERVER_MAX_COMP fields */
    const void* in[FFT3D_SERVER_MAX_COMP];
} fft3d_request;

typedef struct {
    int64_t submitted, admitted, completed, released, waiting, in_flight;
    int64_t batched_launches, single_launches;
    size_t reserved_bytes, peak_reserved_bytes, budget_bytes;
} fft3d_server_counters;

/* Create a server on the current device (allocates the arena, streams and the
 * dispatcher thread).  FFT3D_ERR_NOMEM if the arena cannot be allocated. */
int fft3d_server_create(const fft3d_server_config* cfg, fft3d_server_t* out);
/* Queue a request (thread-safe, returns at once; its arrival time is now).
 * *id receives the request's id.  FFT3D_ERR_BUDGET if the request alone needs
 * more than the whole budget; FFT3D_ERR_UNSUPPORTED for a shape no plan can
 * take. */
int fft3d_server_submit(fft3d_server_t s, const fft3d_request* r, int64_t* id);
/* Wait until the request has completed: 1 done, 0 timed out (timeout_s < 0:
 * no limit), negative on error (unknown id, a failed launch). */
int fft3d_server_wait(fft3d_server_t s, int64_t id, double timeout_s);
/* Outputs of a completed request (out: ncomp device pointers into the arena)
 * and its times in seconds on the server's clock (times: arrive, admit,
 * launch, done).  Either may be NULL.  FFT3D_ERR_INVALID_ARG until done. */
int fft3d_server_result(fft3d_server_t s, int64_t id, void** out, double* times);
/* Free a completed request's outputs (waiting requests may then be admitted). */
int fft3d_server_release(fft3d_server_t s, int64_t id);
int fft3d_server_stats(fft3d_server_t s, fft3d_server_counters* st);
/* Stop accepting, finish what was admitted, free everything. */
int fft3d_server_destroy(fft3d_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* FFT3D_H */
