// fft3d_device.hpp -- device building blocks of the 3D r2c/c2r library (gfx950).
//
// Complex arithmetic with explicit fused multiply-adds (the library is built
// with -ffp-contract=off, so the rounding of every expression is fixed by the
// source and identical in every kernel that inlines it), the radix-2/3/4/5/7/8/16
// DFT butterflies held in registers, and a Stockham autosort stage that runs on
// lines held in LDS.
//
// Stage convention (Stockham, natural-order output).  For a line of length n
// and a stage of radix R whose preceding stages have product Ns, butterfly
// j in [0, n/R) reads the R inputs at j + r*(n/R), multiplies input r by the
// twiddle w_{Ns*R}^{r*(j mod Ns)}, runs the length-R DFT, and writes output r
// to (j div Ns)*Ns*R + (j mod Ns) + r*Ns.  After the last stage the line holds
// the DFT in natural order.  w_m = exp(-2 pi i/m) forward, its conjugate for
// the inverse.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft3d_sched.hpp"

// Radix-5 and radix-7 stages are compiled into the kernels only when
// FFT3D_ODD_RADICES is 1: their extra cases in the stage dispatch raise the
// register count of every kernel, so 2^a 3^b extents keep kernels without
// them.  The two compilations live in different inline namespaces, so both sets of
// kernels link into one library.
#ifndef FFT3D_ODD_RADICES
#define FFT3D_ODD_RADICES 0
#endif
#if FFT3D_ODD_RADICES
#define FFT3D_KNS k2357
#else
#define FFT3D_KNS k23
#endif

namespace fft3d {
inline namespace FFT3D_KNS {

template <typename T> struct cx_of;
template <> struct cx_of<float> { using type = float2; };
template <> struct cx_of<double> { using type = double2; };
template <typename T> using cx = typename cx_of<T>::type;

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename T> __device__ __forceinline__ cx<T> mk(T a, T b)
{
    cx<T> r;
    r.x = a;
    r.y = b;
    return r;
}
template <typename T> __device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ cx<T> cconj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }

// a * w
template <typename T> __device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> w)
{
    return mk<T>(fmaT(a.x, w.x, -(a.y * w.y)), fmaT(a.x, w.y, a.y * w.x));
}
// a * conj(w)
template <typename T> __device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> w)
{
    return mk<T>(fmaT(a.x, w.x, a.y * w.y), fmaT(a.y, w.x, -(a.x * w.y)));
}
// multiply by w_4 = -i (forward) or +i (inverse)
template <bool INV, typename T> __device__ __forceinline__ cx<T> rot4(cx<T> a)
{
    return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
// multiply by w twiddle from a forward table: w (forward) or conj(w) (inverse)
template <bool INV, typename T> __device__ __forceinline__ cx<T> twmul(cx<T> a, cx<T> w)
{
    return INV ? cmulc<T>(a, w) : cmul<T>(a, w);
}

// ------------------------------------------------------------ butterflies --
// In-place length-R DFT of v[0..R): v[k] <- sum_r v[r] w_R^{rk}.

template <bool INV, typename T> __device__ __forceinline__ void dft2(cx<T>* v)
{
    cx<T> a = v[0], b = v[1];
    v[0] = cadd<T>(a, b);
    v[1] = csub<T>(a, b);
}

template <bool INV, typename T> __device__ __forceinline__ void dft3(cx<T>* v)
{
    const T s = (T)0.86602540378443864676372317075293618; // sin(2 pi/3)
    cx<T> t = cadd<T>(v[1], v[2]);
    cx<T> d = csub<T>(v[1], v[2]);
    cx<T> x0 = v[0];
    v[0] = cadd<T>(x0, t);
    cx<T> m = mk<T>(fmaT((T)-0.5, t.x, x0.x), fmaT((T)-0.5, t.y, x0.y));
    // forward: w_3 = -1/2 - i s, so X1 = m - i s d, X2 = m + i s d
    cx<T> isd = INV ? mk<T>(-s * d.y, s * d.x) : mk<T>(s * d.y, -s * d.x);
    v[1] = cadd<T>(m, isd);
    v[2] = csub<T>(m, isd);
}

template <bool INV, typename T> __device__ __forceinline__ void dft4(cx<T>* v)
{
    cx<T> t0 = cadd<T>(v[0], v[2]);
    cx<T> t1 = csub<T>(v[0], v[2]);
    cx<T> t2 = cadd<T>(v[1], v[3]);
    cx<T> t3 = rot4<INV, T>(csub<T>(v[1], v[3]));
    v[0] = cadd<T>(t0, t2);
    v[2] = csub<T>(t0, t2);
    v[1] = cadd<T>(t1, t3);
    v[3] = csub<T>(t1, t3);
}

// z * w_8 (forward w_8 = (c, -c)), inverse conj
template <bool INV, typename T> __device__ __forceinline__ cx<T> rot8(cx<T> z)
{
    const T c = (T)0.70710678118654752440084436210484904;
    return INV ? mk<T>(c * (z.x - z.y), c * (z.x + z.y)) : mk<T>(c * (z.x + z.y), c * (z.y - z.x));
}
// z * w_8^3 (forward (-c, -c)), inverse conj
template <bool INV, typename T> __device__ __forceinline__ cx<T> rot8_3(cx<T> z)
{
    const T c = (T)0.70710678118654752440084436210484904;
    return INV ? mk<T>(-c * (z.x + z.y), c * (z.x - z.y)) : mk<T>(c * (z.y - z.x), -c * (z.x + z.y));
}

template <bool INV, typename T> __device__ __forceinline__ void dft8(cx<T>* v)
{
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    dft4<INV, T>(e);
    dft4<INV, T>(o);
    o[1] = rot8<INV, T>(o[1]);
    o[2] = rot4<INV, T>(o[2]);
    o[3] = rot8_3<INV, T>(o[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[k] = cadd<T>(e[k], o[k]);
        v[k + 4] = csub<T>(e[k], o[k]);
    }
}

// Length 16 as 4 x 4: Y_r = DFT4 of v[r + 4m]; Y_r[k1] *= w_16^{r k1};
// X[k1 + 4 k2] = DFT4 over r of Y_r[k1].
template <bool INV, typename T> __device__ __forceinline__ void dft16(cx<T>* v)
{
    const T c1 = (T)0.92387953251128675612818318939678829; // cos(pi/8)
    const T s1 = (T)0.38268343236508977172845998403039887; // sin(pi/8)
    cx<T> y[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        y[r][0] = v[r];
        y[r][1] = v[r + 4];
        y[r][2] = v[r + 8];
        y[r][3] = v[r + 12];
        dft4<INV, T>(y[r]);
    }
    // twiddles w_16^{r k1}, r, k1 in 1..3 (forward table values; inverse conjugates)
    const cx<T> w1 = mk<T>(c1, -s1);  // w_16^1
    const cx<T> w3 = mk<T>(s1, -c1);  // w_16^3
    const cx<T> w9 = mk<T>(-c1, s1);  // w_16^9
    y[1][1] = twmul<INV, T>(y[1][1], w1);
    y[1][2] = rot8<INV, T>(y[1][2]);
    y[1][3] = twmul<INV, T>(y[1][3], w3);
    y[2][1] = rot8<INV, T>(y[2][1]);
    y[2][2] = rot4<INV, T>(y[2][2]);
    y[2][3] = rot8_3<INV, T>(y[2][3]);
    y[3][1] = twmul<INV, T>(y[3][1], w3);
    y[3][2] = rot8_3<INV, T>(y[3][2]);
    y[3][3] = twmul<INV, T>(y[3][3], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cx<T> z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        dft4<INV, T>(z);
        v[k1] = z[0];
        v[k1 + 4] = z[1];
        v[k1 + 8] = z[2];
        v[k1 + 12] = z[3];
    }
}

// cos and sin of 2 pi m / P for the odd radices 5 and 7, m in [0, P).
template <int P> __device__ __forceinline__ constexpr long double cos_2pi(int m)
{
    const int r = m <= P / 2 ? m : P - m;  // cos is even about P/2
    if constexpr (P == 5) {
        return r == 0 ? 1.0L : r == 1 ? 0.309016994374947424102293417182819059L : -0.809016994374947424102293417182819059L;
    } else {
        return r == 0 ? 1.0L
             : r == 1 ? 0.623489801858733530525004884004239811L
             : r == 2 ? -0.222520933956314404288902564496794759L
                      : -0.900968867902419126236102319507445051L;
    }
}
template <int P> __device__ __forceinline__ constexpr long double sin_2pi(int m)
{
    const int r = m <= P / 2 ? m : P - m;  // sin is odd about P/2
    const long double v = P == 5 ? (r == 0   ? 0.0L
                                    : r == 1 ? 0.951056516295153572116439333379382143L
                                             : 0.587785252292473129168705954639072769L)
                                 : (r == 0   ? 0.0L
                                    : r == 1 ? 0.781831482468029808708444526674057750L
                                    : r == 2 ? 0.974927912181823607018131682993931217L
                                             : 0.433883739117558120475768332848358755L);
    return m <= P / 2 ? v : -v;
}

// Length-P DFT for odd P (5, 7) by the symmetric pairs of inputs:
// a_j = x_j + x_{P-j}, b_j = x_j - x_{P-j} (j = 1 .. (P-1)/2);
// X_k = x_0 + sum_j a_j cos(2 pi jk/P) -/+ i sum_j b_j sin(2 pi jk/P), and
// X_{P-k} the same with the opposite sign of the sine part (forward: minus
// for X_k).
template <int P, bool INV, typename T> __device__ __forceinline__ void dft_odd(cx<T>* v)
{
    constexpr int Hh = (P - 1) / 2;
    cx<T> a[Hh + 1], b[Hh + 1];
#pragma unroll
    for (int j = 1; j <= Hh; ++j) {
        a[j] = cadd<T>(v[j], v[P - j]);
        b[j] = csub<T>(v[j], v[P - j]);
    }
    const cx<T> x0 = v[0];
    cx<T> s0 = x0;
#pragma unroll
    for (int j = 1; j <= Hh; ++j) s0 = cadd<T>(s0, a[j]);
#pragma unroll
    for (int k = 1; k <= Hh; ++k) {
        cx<T> A = x0, B = mk<T>((T)0, (T)0);
#pragma unroll
        for (int j = 1; j <= Hh; ++j) {
            const int m = (j * k) % P;
            const T c = (T)cos_2pi<P>(m), sn = (T)sin_2pi<P>(m);
            A = mk<T>(fmaT(a[j].x, c, A.x), fmaT(a[j].y, c, A.y));
            B = mk<T>(fmaT(b[j].x, sn, B.x), fmaT(b[j].y, sn, B.y));
        }
        // forward: X_k = A - i B, X_{P-k} = A + i B; inverse the reverse
        const cx<T> miB = mk<T>(B.y, -B.x);
        v[k] = INV ? csub<T>(A, miB) : cadd<T>(A, miB);
        v[P - k] = INV ? cadd<T>(A, miB) : csub<T>(A, miB);
    }
    v[0] = s0;
}

template <int R, bool INV, typename T> __device__ __forceinline__ void dftR(cx<T>* v)
{
    if constexpr (R == 2) dft2<INV, T>(v);
    else if constexpr (R == 3) dft3<INV, T>(v);
    else if constexpr (R == 5 || R == 7) dft_odd<R, INV, T>(v);
    else if constexpr (R == 4) dft4<INV, T>(v);
    else if constexpr (R == 8) dft8<INV, T>(v);
    else if constexpr (R == 16) dft16<INV, T>(v);
}

// n / d for n * d < 2^32, with mg = div_magic(d) (0 for d == 1).
__device__ __forceinline__ int fdiv(int n, uint32_t mg)
{
    return mg ? (int)__umulhi((uint32_t)n, mg) : n;
}

__device__ __forceinline__ int lds_addr(const LdsLines& L, int w, int i)
{
    if (L.lpp >= L.nlines) return w * L.sw + i * L.si;  // one panel (uniform branch)
    const int p = fdiv(w, L.mg_lpp);
    const int q = w - p * L.lpp;
    return p * L.sp + q * L.sw + i * L.si;
}

// ----------------------------------------------------- XCD-aware order --
// The hardware hands workgroup b to XCD (b mod 8).  Tiles come in groups of g
// consecutive tiles (e.g. the column tiles of one plane, which share the cache
// lines at their edges); group_tile sends every group whole to one XCD --
// group j to XCD (j mod 8) -- so those lines meet in one L2, while the groups
// in flight at the same time stay neighbours in memory.  The grid is padded to
// kXcds * g * ceil(groups / kXcds) workgroups; a padding workgroup gets a tile
// index >= the tile count and leaves.  `reverse` walks the groups of each XCD
// from the last (the data the previous pass wrote last come first).
constexpr int kXcds = 8;

__host__ __device__ inline int64_t group_grid(int64_t groups, int64_t g)
{
    return (int64_t)kXcds * g * ((groups + kXcds - 1) / kXcds);
}

// Workgroups of a persistent loop over the `virt` indices of such a padded
// grid: one per CU, a multiple of kXcds (so that indices b and b + k*grid
// sit on one XCD), at most virt (itself a multiple of kXcds).
__host__ __device__ inline int64_t pipe_grid(int64_t virt, int cus)
{
    int64_t g = cus > kXcds ? cus - cus % kXcds : kXcds;
    return g < virt ? g : virt;
}

__device__ __forceinline__ int64_t group_tile(int64_t b, int64_t groups, int64_t g, bool reverse)
{
    const int64_t x = b % kXcds, k = b / kXcds;
    const int64_t per_xcd = (groups + kXcds - 1) / kXcds;
    int64_t j = k / g;
    if (reverse) j = per_xcd - 1 - j;
    return (x + (int64_t)kXcds * j) * g + (k - (k / g) * g);
}

// ------------------------------------------------------ line accessors --
// A stage addresses element i of line w through a position: at(w, i) gives
// the position of that element, adv(p, d) the position d elements further
// along the same line (d is uniform across the workgroup, so the stride
// arithmetic stays scalar), get/put read and write at a position.  kLds tells
// the stage driver whether the accessor is the LDS tile (which decides where
// barriers are needed).

// Column tiles in LDS (lines laid out by LdsLines; linear in the element
// index, so positions advance by a uniform stride).
template <typename T> struct LdsIO {
    static constexpr bool kLds = true;
    static constexpr bool kLinear = true;
    using Pos = int;
    cx<T>* buf;
    LdsLines L;
    __device__ __forceinline__ Pos at(int w, int i) const { return lds_addr(L, w, i); }
    __device__ __forceinline__ Pos adv(Pos p, int d) const { return p + d * L.si; }
    __device__ __forceinline__ cx<T> get(Pos p) const { return buf[p]; }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const { buf[p] = v; }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// Rows in LDS with padded positions: element i of row w at w*Hs + pad16(i)
// (Hs: padded row stride).  Lines along a row.
template <typename T> struct LdsRowsIO {
    static constexpr bool kLds = true;
    static constexpr bool kLinear = false;
    using Pos = int;
    cx<T>* buf;
    int Hs;
    __device__ __forceinline__ Pos at(int w, int i) const { return w * Hs + pad16(i); }
    __device__ __forceinline__ cx<T> get(Pos p) const { return buf[p]; }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const { buf[p] = v; }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

// The columns of np planes of n1 padded rows in LDS: line w = column
// (w mod H) of plane (w div H), element i = row i.  Linear in i (stride Hs).
template <typename T> struct LdsPlaneColsIO {
    static constexpr bool kLds = true;
    static constexpr bool kLinear = true;
    using Pos = int;
    cx<T>* buf;
    int H, Hs;
    int plane;     // n1 * Hs
    uint32_t mgH;  // div_magic(H)
    __device__ __forceinline__ Pos at(int w, int i) const
    {
        const int p = fdiv(w, mgH);
        return p * plane + i * Hs + pad16(w - p * H);
    }
    __device__ __forceinline__ Pos adv(Pos p, int d) const { return p + d * Hs; }
    __device__ __forceinline__ cx<T> get(Pos p) const { return buf[p]; }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const { buf[p] = v; }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

// Device-scope loads: they miss the CU's L1 and read the XCD's L2.  Used for
// data that another CU of the same XCD wrote earlier in the same kernel (the
// writer drained its stores to L2 before signalling).
__device__ __forceinline__ float2 load_l2(const float2* p)
{
    const uint64_t u = __hip_atomic_load(reinterpret_cast<uint64_t*>(const_cast<float2*>(p)), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    return __builtin_bit_cast(float2, u);
}
__device__ __forceinline__ double2 load_l2(const double2* p)
{
    uint64_t* q = reinterpret_cast<uint64_t*>(const_cast<double2*>(p));
    const uint64_t a = __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t b = __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double2 r;
    r.x = __builtin_bit_cast(double, a);
    r.y = __builtin_bit_cast(double, b);
    return r;
}
// Cache policies of global accesses.  Loads: plain; LD_L2 (device scope,
// misses L1, see load_l2); LD_STREAM (non-temporal: data read once, kept out
// of the way of data the cache should hold).  Stores: plain; ST_STREAM
// (non-temporal: data not read again soon).
enum { LD_PLAIN = 0, LD_L2 = 1, LD_STREAM = 2 };
enum { ST_PLAIN = 0, ST_STREAM = 1 };

typedef float f2v_t __attribute__((ext_vector_type(2)));
typedef double d2v_t __attribute__((ext_vector_type(2)));
template <typename T> struct native2;
template <> struct native2<float> { using type = f2v_t; };
template <> struct native2<double> { using type = d2v_t; };

template <int LP, typename T> __device__ __forceinline__ cx<T> load_cx(const cx<T>* p)
{
    if constexpr (LP == LD_L2) {
        return load_l2(p);
    } else if constexpr (LP == LD_STREAM) {
        using V = typename native2<T>::type;
        const V v = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
        return mk<T>(v.x, v.y);
    } else {
        return *p;
    }
}

template <int SP, typename T> __device__ __forceinline__ void store_cx(cx<T>* p, cx<T> v)
{
    if constexpr (SP == ST_STREAM) {
        using V = typename native2<T>::type;
        V w;
        w.x = v.x;
        w.y = v.y;
        __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
    } else {
        *p = v;
    }
}

// Lane-pair exchange (lanes 2i and 2i+1 swap a value; DPP quad_perm
// [1,0,3,2], no LDS).  Global IO of FP32 complex values uses it to move two
// neighbouring values (16 bytes) per lane and access: each lane of a pair
// loads or stores both values of one of two positions, and the pair swaps
// one value each, so that every lane still ends with its own values.
__device__ __forceinline__ float swap_pair_lane(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));
}
__device__ __forceinline__ double swap_pair_lane(double x) { return x; }  // never called: FP32 only
template <typename T> __device__ __forceinline__ cx<T> swap_pair_lane_cx(cx<T> v)
{
    return mk<T>(swap_pair_lane(v.x), swap_pair_lane(v.y));
}

// Whether a global IO accessor offers the paired 16-byte accesses.
template <class O, class = void> struct io_pairs {
    static constexpr bool value = false;
};
template <class O> struct io_pairs<O, decltype((void)O::kPair, void())> {
    static constexpr bool value = O::kPair;
};

// W consecutive columns of a row-major block: line w = column w (only the
// first `width` exist; the others read as zero and are not written),
// element i = row i at stride S.  src and dst may be equal.  LP / SP: cache
// policies of the loads and stores.
template <typename T, int LP = LD_PLAIN, int SP = ST_PLAIN> struct ColTileIO {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    struct Pos {
        int64_t off;  // element offset, column clamped to a valid one
        bool ok;      // the column exists
    };
    const cx<T>* src;
    cx<T>* dst;
    int64_t S;
    int width;
    __device__ __forceinline__ Pos at(int w, int i) const
    {
        Pos p;
        p.ok = w < width;
        p.off = (int64_t)i * S + (p.ok ? w : width - 1);
        return p;
    }
    __device__ __forceinline__ Pos adv(Pos p, int d) const
    {
        p.off += (int64_t)d * S;
        return p;
    }
    // always a valid address (clamped column), then masked
    __device__ __forceinline__ cx<T> get(Pos p) const
    {
        const cx<T> v = load_cx<LP, T>(src + p.off);
        return p.ok ? v : mk<T>((T)0, (T)0);
    }
    // the same load unmasked: a column past `width` reads column width-1
    __device__ __forceinline__ cx<T> get_unmasked(Pos p) const { return load_cx<LP, T>(src + p.off); }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const
    {
        if (p.ok) store_cx<SP, T>(dst + p.off, v);
    }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
    // Paired access: columns w (even) and w + 1 of a row as one 16-byte
    // access (needs an even number of existing columns, so that a pair is
    // whole or absent, an even row stride and 16-byte aligned tile
    // pointers).  Off: a paired access then touches two rows nb apart (eight
    // row segments per wave instead of four), and the FP32 n0 passes at
    // 512^3 ran 16-25% slower with it (218 -> 275 us forward).
    static constexpr bool kPair = false;
    __device__ __forceinline__ bool pair_ld_ok() const
    {
        return (width & 1) == 0 && (S & 1) == 0 && ((uintptr_t)src & 15) == 0;
    }
    __device__ __forceinline__ bool pair_st_ok() const
    {
        return (width & 1) == 0 && (S & 1) == 0 && ((uintptr_t)dst & 15) == 0;
    }
    __device__ __forceinline__ bool pair_valid(Pos p) const { return p.ok; }
    __device__ __forceinline__ float4 get2(Pos p) const { return *reinterpret_cast<const float4*>(src + p.off); }
    __device__ __forceinline__ void put2(Pos p, cx<T> lo, cx<T> hi) const
    {
        *reinterpret_cast<float4*>(dst + p.off) = make_float4(lo.x, lo.y, hi.x, hi.y);
    }
};

// Contiguous lines of `len` elements: line q, element i at q*len + i.
template <typename T, int LP = LD_PLAIN, int SP = ST_PLAIN> struct RowsIO {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    using Pos = int;
    const cx<T>* src;
    cx<T>* dst;
    int len;
    __device__ __forceinline__ Pos at(int q, int i) const { return q * len + i; }
    __device__ __forceinline__ Pos adv(Pos p, int d) const { return p + d; }
    __device__ __forceinline__ cx<T> get(Pos p) const { return load_cx<LP, T>(src + p); }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const { store_cx<SP, T>(dst + p, v); }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
    // Paired access (FP32, plain policies): elements i (even) and i + 1 of a
    // line as one 16-byte access; needs an even line length and 16-byte
    // aligned pointers.
    static constexpr bool kPair = sizeof(T) == 4 && LP == LD_PLAIN && SP == ST_PLAIN;
    __device__ __forceinline__ bool pair_ld_ok() const { return (len & 1) == 0 && ((uintptr_t)src & 15) == 0; }
    __device__ __forceinline__ bool pair_st_ok() const { return (len & 1) == 0 && ((uintptr_t)dst & 15) == 0; }
    __device__ __forceinline__ bool pair_valid(Pos) const { return true; }
    __device__ __forceinline__ float4 get2(Pos p) const { return *reinterpret_cast<const float4*>(src + p); }
    __device__ __forceinline__ void put2(Pos p, cx<T> lo, cx<T> hi) const
    {
        *reinterpret_cast<float4*>(dst + p) = make_float4(lo.x, lo.y, hi.x, hi.y);
    }
};

// Whole n1 x H planes, contiguous: line w = column (w mod H) of plane
// (w div H), element i = row i (stride H).
template <typename T> struct PlaneColsIO {
    static constexpr bool kLds = false;
    static constexpr bool kLinear = true;
    using Pos = int;
    const cx<T>* src;
    cx<T>* dst;
    int H;
    int plane;     // n1 * H
    uint32_t mgH;  // div_magic(H)
    __device__ __forceinline__ Pos at(int w, int i) const
    {
        const int p = fdiv(w, mgH);
        return p * plane + (w - p * H) + i * H;
    }
    __device__ __forceinline__ Pos adv(Pos p, int d) const { return p + d * H; }
    __device__ __forceinline__ cx<T> get(Pos p) const { return src[p]; }
    __device__ __forceinline__ void put(Pos p, cx<T> v) const { dst[p] = v; }
    __device__ __forceinline__ cx<T> ld(int w, int i) const { return get(at(w, i)); }
    __device__ __forceinline__ void st(int w, int i, cx<T> v) const { put(at(w, i), v); }
};

// Per-stage constants for stage().
struct StageArg {
    int n, nlines, Ns;
    uint32_t mg_lines, mg_nb, mg_ns;
};

template <int R, bool LINES_FAST>
__device__ __forceinline__ void butterfly_of(int b, const StageArg& a, int& j, int& w)
{
    if (LINES_FAST) {
        j = fdiv(b, a.mg_lines);
        w = b - j * a.nlines;
    } else {
        w = fdiv(b, a.mg_nb);
        j = b - w * (a.n / R);
    }
}

template <int R, bool INV, bool LINES_FAST, int NT, int EPT, bool MID, bool END, typename T, class In,
          class Out>
__device__ __forceinline__ void stage(const In& in, const Out& out, const StageArg& a,
                                      const cx<T>* __restrict__ tw)
{
    constexpr int KMAX = (EPT + R - 1) / R;
    const int nb = a.n / R;         // butterflies per line
    const int B = nb * a.nlines;    // butterflies in the tile
    const int Ns = a.Ns;
    // Paired 16-byte global accesses (see swap_pair_lane): lanes 2i, 2i+1
    // hold neighbouring lines (LINES_FAST) or neighbouring butterflies of a
    // line, whose values are neighbours in memory -- on input always, on
    // output when the stage's Ns is even (rows) -- given an even count of
    // lines (butterflies per line).  Both lanes of a pair are active or
    // neither (B is even then).  The arithmetic is unchanged.
    constexpr bool kPairIn = io_pairs<In>::value && R % 2 == 0;
    constexpr bool kPairOut = io_pairs<Out>::value && R % 2 == 0;
    const bool even_pairs = LINES_FAST ? (a.nlines & 1) == 0 : (nb & 1) == 0;
    bool pair_in = false, pair_out = false;
    if constexpr (kPairIn) pair_in = even_pairs && in.pair_ld_ok();
    if constexpr (kPairOut) pair_out = even_pairs && (LINES_FAST || (Ns & 1) == 0) && out.pair_st_ok();
    cx<T> v[KMAX][R];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = (int)threadIdx.x + k * NT;
        if (b < B) {
            int j, w;
            butterfly_of<R, LINES_FAST>(b, a, j, w);
            if constexpr (In::kLinear) {
                bool done = false;
                if constexpr (kPairIn) {
                    if (pair_in) {
                        const int odd = b & 1;
                        const auto p0 = LINES_FAST ? in.at(w - odd, j) : in.at(w, j - odd);
                        const bool ok = in.pair_valid(p0);
#pragma unroll
                        for (int r = 0; r < R; r += 2) {
                            float4 q = make_float4(0.f, 0.f, 0.f, 0.f);
                            if (ok) q = in.get2(in.adv(p0, (r + odd) * nb));
                            const cx<T> lo = mk<T>(q.x, q.y), hi = mk<T>(q.z, q.w);
                            const cx<T> recv = swap_pair_lane_cx<T>(odd ? lo : hi);
                            v[k][r] = odd ? recv : lo;
                            v[k][r + 1] = odd ? hi : recv;
                        }
                        done = true;
                    }
                }
                if (!done) {
                    const auto p0 = in.at(w, j);
#pragma unroll
                    for (int r = 0; r < R; ++r) v[k][r] = in.get(in.adv(p0, r * nb));
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[k][r] = in.ld(w, j + r * nb);
            }
            if (Ns > 1) {
                const int m = j - fdiv(j, a.mg_ns) * Ns;
                const cx<T>* t = tw + m * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) v[k][r] = twmul<INV, T>(v[k][r], t[r - 1]);
            }
            dftR<R, INV, T>(v[k]);
        }
    }
    if (MID) __syncthreads();
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = (int)threadIdx.x + k * NT;
        if (b < B) {
            int j, w;
            butterfly_of<R, LINES_FAST>(b, a, j, w);
            const int m = j - fdiv(j, a.mg_ns) * Ns;
            const int base = (j - m) * R + m;
            if constexpr (Out::kLinear) {
                bool done = false;
                if constexpr (kPairOut) {
                    if (pair_out) {
                        const int odd = b & 1;
                        const auto q0 = LINES_FAST ? out.at(w - odd, base) : out.at(w, base - odd);
                        const bool ok = out.pair_valid(q0);
#pragma unroll
                        for (int r = 0; r < R; r += 2) {
                            const cx<T> recv = swap_pair_lane_cx<T>(odd ? v[k][r] : v[k][r + 1]);
                            const cx<T> lo = odd ? recv : v[k][r];
                            const cx<T> hi = odd ? v[k][r + 1] : recv;
                            if (ok) out.put2(out.adv(q0, (r + odd) * Ns), lo, hi);
                        }
                        done = true;
                    }
                }
                if (!done) {
                    const auto q0 = out.at(w, base);
#pragma unroll
                    for (int r = 0; r < R; ++r) out.put(out.adv(q0, r * Ns), v[k][r]);
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) out.st(w, base + r * Ns, v[k][r]);
            }
        }
    }
    if (END) __syncthreads();
}

// A stage whose input and output cannot alias (no barrier between reads and
// writes), one butterfly at a time: load, twiddle, butterfly, store.  The
// same arithmetic as stage(), which first computes all of a thread's
// butterflies and then stores them; this form holds one butterfly's values
// in registers instead of EPT, for kernels that keep other values live
// across the stage (k_cols_pipe).  Plain (unpaired) accesses only.
template <int R, bool INV, bool LINES_FAST, int NT, int EPT, typename T, class In, class Out>
__device__ __forceinline__ void stage_direct(const In& in, const Out& out, const StageArg& a,
                                             const cx<T>* __restrict__ tw)
{
    constexpr int KMAX = (EPT + R - 1) / R;
    const int nb = a.n / R;
    const int B = nb * a.nlines;
    const int Ns = a.Ns;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = (int)threadIdx.x + k * NT;
        if (b < B) {
            int j, w;
            butterfly_of<R, LINES_FAST>(b, a, j, w);
            cx<T> v[R];
            if constexpr (In::kLinear) {
                const auto p0 = in.at(w, j);
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = in.get(in.adv(p0, r * nb));
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[r] = in.ld(w, j + r * nb);
            }
            const int m = j - fdiv(j, a.mg_ns) * Ns;
            if (Ns > 1) {
                const cx<T>* t = tw + m * (R - 1);
#pragma unroll
                for (int r = 1; r < R; ++r) v[r] = twmul<INV, T>(v[r], t[r - 1]);
            }
            dftR<R, INV, T>(v);
            const int base = (j - m) * R + m;
            if constexpr (Out::kLinear) {
                const auto q0 = out.at(w, base);
#pragma unroll
                for (int r = 0; r < R; ++r) out.put(out.adv(q0, r * Ns), v[r]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) out.st(w, base + r * Ns, v[r]);
            }
        }
    }
}

// A first stage (Ns = 1) in two halves, for column tiles (ColTileIO) whose
// lines are fast (consecutive threads take consecutive columns; no paired
// accesses): the loads of a thread's butterflies into registers, then the
// butterflies and their stores.  stage() does both in one; a persistent loop
// uses the halves to issue one tile's loads ahead of the previous tile's
// later stages.  The loads are unmasked and the second half zeroes the
// columns past the tile's width (what ColTileIO::get does at the load), so
// that nothing between the two halves waits for the loaded values.
template <int R, int NT, int EPT> struct FirstStage {
    static constexpr int K = (EPT + R - 1) / R;
};

template <int R, int NT, int EPT, typename T, class In>
__device__ __forceinline__ void first_stage_load(const In& in, const StageArg& a,
                                                 cx<T> (&v)[FirstStage<R, NT, EPT>::K][R])
{
    constexpr int KMAX = FirstStage<R, NT, EPT>::K;
    const int nb = a.n / R;
    const int B = nb * a.nlines;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = (int)threadIdx.x + k * NT;
        if (b < B) {
            int j, w;
            butterfly_of<R, true>(b, a, j, w);
            const auto p0 = in.at(w, j);
#pragma unroll
            for (int r = 0; r < R; ++r) v[k][r] = in.get_unmasked(in.adv(p0, r * nb));
        }
    }
}

template <int R, bool INV, int NT, int EPT, typename T, class Out>
__device__ __forceinline__ void first_stage_finish(const Out& out, const StageArg& a,
                                                   cx<T> (&v)[FirstStage<R, NT, EPT>::K][R], int width)
{
    constexpr int KMAX = FirstStage<R, NT, EPT>::K;
    const int nb = a.n / R;
    const int B = nb * a.nlines;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        const int b = (int)threadIdx.x + k * NT;
        if (b < B) {
            int j, w;
            butterfly_of<R, true>(b, a, j, w);
            if (w >= width) {
#pragma unroll
                for (int r = 0; r < R; ++r) v[k][r] = mk<T>((T)0, (T)0);
            }
            dftR<R, INV, T>(v[k]);
            const auto q0 = out.at(w, j * R);
#pragma unroll
            for (int r = 0; r < R; ++r) out.put(out.adv(q0, r), v[k][r]);
        }
    }
}

// Largest radix a kernel instantiation carries code for: the fine column
// tier leaves radix 16 out (the plan gives it radix <= 8 schedules only).
template <typename T, int NT, int EPT> constexpr int max_radix()
{
    return (sizeof(T) == 4 && NT == kNtFine && EPT == kEptFine) ? kFineMaxRadix : 16;
}

// One stage of any radix the schedule may hold, up to RMAX (code for larger
// radices is left out).
template <int RMAX, bool INV, bool LINES_FAST, int NT, int EPT, bool MID, bool END, typename T, class In, class Out>
__device__ __forceinline__ void stage_upto(const AxisSched& S, int s, int nlines, uint32_t mg_lines,
                                           const In& in, const Out& out, const cx<T>* __restrict__ tw)
{
    StageArg a;
    a.n = S.n;
    a.nlines = nlines;
    a.Ns = S.ns[s];
    a.mg_lines = mg_lines;
    a.mg_nb = S.mg_nb[s];
    a.mg_ns = S.mg_ns[s];
    const cx<T>* t = tw + S.twoff[s];
    switch (S.radix[s]) {
    case 16:
        if constexpr (RMAX >= 16) stage<16, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t);
        break;
    case 8: stage<8, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t); break;
    case 4: stage<4, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t); break;
    case 3: stage<3, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t); break;
#if FFT3D_ODD_RADICES
    case 5: stage<5, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t); break;
    case 7: stage<7, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t); break;
#endif
    default: stage<2, INV, LINES_FAST, NT, EPT, MID, END, T>(in, out, a, t); break;
    }
}

// stage_direct of any radix up to RMAX.
template <int RMAX, bool INV, bool LINES_FAST, int NT, int EPT, typename T, class In, class Out>
__device__ __forceinline__ void stage_direct_upto(const AxisSched& S, int s, int nlines, uint32_t mg_lines,
                                                  const In& in, const Out& out, const cx<T>* __restrict__ tw)
{
    StageArg a;
    a.n = S.n;
    a.nlines = nlines;
    a.Ns = S.ns[s];
    a.mg_lines = mg_lines;
    a.mg_nb = S.mg_nb[s];
    a.mg_ns = S.mg_ns[s];
    const cx<T>* t = tw + S.twoff[s];
    switch (S.radix[s]) {
    case 16:
        if constexpr (RMAX >= 16) stage_direct<16, INV, LINES_FAST, NT, EPT, T>(in, out, a, t);
        break;
    case 8: stage_direct<8, INV, LINES_FAST, NT, EPT, T>(in, out, a, t); break;
    case 4: stage_direct<4, INV, LINES_FAST, NT, EPT, T>(in, out, a, t); break;
    case 3: stage_direct<3, INV, LINES_FAST, NT, EPT, T>(in, out, a, t); break;
#if FFT3D_ODD_RADICES
    case 5: stage_direct<5, INV, LINES_FAST, NT, EPT, T>(in, out, a, t); break;
    case 7: stage_direct<7, INV, LINES_FAST, NT, EPT, T>(in, out, a, t); break;
#endif
    default: stage_direct<2, INV, LINES_FAST, NT, EPT, T>(in, out, a, t); break;
    }
}

template <bool INV, bool LINES_FAST, int NT, int EPT, bool MID, bool END, typename T, class In, class Out>
__device__ __forceinline__ void stage_any(const AxisSched& S, int s, int nlines, uint32_t mg_lines,
                                          const In& in, const Out& out, const cx<T>* __restrict__ tw)
{
    stage_upto<max_radix<T, NT, EPT>(), INV, LINES_FAST, NT, EPT, MID, END, T>(S, s, nlines, mg_lines, in, out, tw);
}

// All stages of one axis over `nlines` lines: the first stage reads through
// `in`, the last writes through `out`, the stages between exchange through
// the LDS tile `lds`.  mgl = div_magic(nlines) (used when LINES_FAST).  in/out may themselves be the LDS tile.  Barriers are
// placed from the accessor kinds: a stage that writes LDS ends with one; a
// stage whose input and output may alias has one between reads and writes.
// The caller guarantees the tile is ready (barrier) before the call.
// n == 1 (no stages) is a plain copy from in to out.
template <bool INV, bool LINES_FAST, int NT, int EPT, typename T, class In, class Lds, class Out>
__device__ __forceinline__ void fft_lines(const In& in, const Lds& lds, const Out& out, int nlines,
                                          uint32_t mgl, const AxisSched& S, const cx<T>* __restrict__ tw)
{
    constexpr bool IL = In::kLds, OL = Out::kLds;
    const int nst = S.nst;
    if (nst == 0) {  // n == 1: a copy, unless in and out are the same tile
        if (!(IL && OL)) {
            for (int w = (int)threadIdx.x; w < nlines; w += NT) out.st(w, 0, in.ld(w, 0));
            if (OL) __syncthreads();
        }
        return;
    }
    if (nst == 1) {
        // single stage: in -> out; global in place needs the middle barrier too
        stage_any<INV, LINES_FAST, NT, EPT, (IL == OL), OL, T>(S, 0, nlines, mgl, in, out, tw);
        return;
    }
    stage_any<INV, LINES_FAST, NT, EPT, IL, true, T>(S, 0, nlines, mgl, in, lds, tw);
    for (int s = 1; s < nst - 1; ++s)
        stage_any<INV, LINES_FAST, NT, EPT, true, true, T>(S, s, nlines, mgl, lds, lds, tw);
    stage_any<INV, LINES_FAST, NT, EPT, OL, OL, T>(S, nst - 1, nlines, mgl, lds, out, tw);
}

// ------------------------------------------------- real <-> half-length --
// Rows are held as H = h+1 slots (h = n2/2) at padded positions (pad16) of
// rows Hs apart.  The forward split turns the
// length-h DFT Z of z[m] = x[2m] + i x[2m+1] into the bins X[0..h] of the
// real row; the inverse merge does the reverse.  Each thread owns the pair of
// slots (k, h-k), so both run in place.
//   forward: P = (Z[k] + conj Z[h-k]) / 2,  Q = w^k (Z[k] - conj Z[h-k]) / (2i),
//            X[k] = P + Q,  X[h-k] = conj(P - Q),  X[0] = Re Z0 + Im Z0,
//            X[h] = Re Z0 - Im Z0  (w = exp(-2 pi i/n2))
//   inverse: A = X[k] + conj X[h-k],  B = i w^{-k} (X[k] - conj X[h-k]),
//            Z[k] = A + B,  Z[h-k] = conj(A - B),
//            Z[0] = (Re X0 + Re Xh) + i (Re X0 - Re Xh)
//            (the imaginary parts of X[0] and X[h] are never read).
template <int NT, typename T>
__device__ __forceinline__ void split_rows(cx<T>* buf, int rows, int Hs, int h, uint32_t mg_pairs,
                                           const cx<T>* __restrict__ post)
{
    const int npair = h / 2 + 1;  // k = 0 .. h/2
    const int total = rows * npair;
    for (int e = (int)threadIdx.x; e < total; e += NT) {
        const int q = fdiv(e, mg_pairs);
        const int k = e - q * npair;
        cx<T>* Zr = buf + q * Hs;  // row q, element k at Zr[pad16(k)]
        if (k == 0) {
            cx<T> z0 = Zr[pad16(0)];
            Zr[pad16(0)] = mk<T>(z0.x + z0.y, (T)0);
            Zr[pad16(h)] = mk<T>(z0.x - z0.y, (T)0);
        } else {
            cx<T> a = Zr[pad16(k)], b = Zr[pad16(h - k)];
            cx<T> P = mk<T>((T)0.5 * (a.x + b.x), (T)0.5 * (a.y - b.y));
            // (a - conj b) / (2i) = ((a.y + b.y) - i (a.x - b.x)) / 2
            cx<T> O = mk<T>((T)0.5 * (a.y + b.y), (T)-0.5 * (a.x - b.x));
            cx<T> Q = cmul<T>(O, post[k]);
            Zr[pad16(k)] = cadd<T>(P, Q);
            if (2 * k != h) Zr[pad16(h - k)] = cconj<T>(csub<T>(P, Q));
        }
    }
    __syncthreads();
}

template <int NT, typename T>
__device__ __forceinline__ void merge_rows(cx<T>* buf, int rows, int Hs, int h, uint32_t mg_pairs,
                                           const cx<T>* __restrict__ post)
{
    const int npair = h / 2 + 1;
    const int total = rows * npair;
    for (int e = (int)threadIdx.x; e < total; e += NT) {
        const int q = fdiv(e, mg_pairs);
        const int k = e - q * npair;
        cx<T>* Zr = buf + q * Hs;  // row q, element k at Zr[pad16(k)]
        if (k == 0) {
            T a0 = Zr[pad16(0)].x, bh = Zr[pad16(h)].x;
            Zr[pad16(0)] = mk<T>(a0 + bh, a0 - bh);
        } else {
            cx<T> a = Zr[pad16(k)], b = Zr[pad16(h - k)];
            cx<T> A = mk<T>(a.x + b.x, a.y - b.y);
            cx<T> D = mk<T>(a.x - b.x, a.y + b.y);
            // i * conj(w^k) * D
            cx<T> wD = cmulc<T>(D, post[k]);
            cx<T> Bv = mk<T>(-wD.y, wD.x);
            Zr[pad16(k)] = cadd<T>(A, Bv);
            if (2 * k != h) Zr[pad16(h - k)] = cconj<T>(csub<T>(A, Bv));
        }
    }
    __syncthreads();
}

}  // inline namespace FFT3D_KNS
}  // namespace fft3d
