// fft3d_plan.cpp -- host part of a plan: radix schedules, twiddle tables and
// the choice of kernels and tile shapes.  Runs once per (shape, dtype).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <string>

#include "../../include/fft3d.h"
#include "fft3d_internal.hpp"

namespace fft3d {

// ------------------------------------------------------------ schedules --

// n = 2^a 3^b 5^c 7^d.  The power-of-two part takes ceil(a/4) stages with
// radices as equal as possible (512 = 8*8*8, 1024 = 16*8*8, 256 = 16*16,
// 32 = 8*4), followed by one radix-3, -5 or -7 stage per odd factor.
bool make_schedule(int64_t n, AxisSched& s)
{
    s = AxisSched{};
    if (n < 1 || n > (int64_t(1) << 30)) return false;
    s.n = (int32_t)n;
    int64_t m = n;
    int a = 0, b = 0;
    while (m % 2 == 0) {
        m /= 2;
        ++a;
    }
    while (m % 3 == 0) {
        m /= 3;
        ++b;
    }
    int c5 = 0, c7 = 0;
    while (m % 5 == 0) {
        m /= 5;
        ++c5;
    }
    while (m % 7 == 0) {
        m /= 7;
        ++c7;
    }
    if (m != 1) return false;
    int radices[kMaxStages];
    int cnt = 0;
    if (a > 0) {
        const int s2 = (a + 3) / 4;
        const int base = a / s2, extra = a % s2;
        for (int i = 0; i < s2; ++i) {
            if (cnt >= kMaxStages) return false;
            radices[cnt++] = 1 << (base + (i < extra ? 1 : 0));
        }
    }
    for (int i = 0; i < b; ++i) {
        if (cnt >= kMaxStages) return false;
        radices[cnt++] = 3;
    }
    for (int i = 0; i < c5; ++i) {
        if (cnt >= kMaxStages) return false;
        radices[cnt++] = 5;
    }
    for (int i = 0; i < c7; ++i) {
        if (cnt >= kMaxStages) return false;
        radices[cnt++] = 7;
    }
    return fill_schedule(n, radices, cnt, s);
}

bool fill_schedule(int64_t n, const int* radices, int cnt, AxisSched& s)
{
    s = AxisSched{};
    if (n < 1 || n > (int64_t(1) << 30) || cnt < 0 || cnt > kMaxStages) return false;
    int64_t prod = 1;
    for (int i = 0; i < cnt; ++i) {
        const int r = radices[i];
        if (r != 2 && r != 3 && r != 4 && r != 8 && r != 16 && r != 5 && r != 7) return false;
        prod *= r;
    }
    if (prod != n) return false;
    s.n = (int32_t)n;
    int32_t ns = 1, off = 0;
    for (int i = 0; i < cnt; ++i) {
        s.radix[i] = radices[i];
        s.ns[i] = ns;
        s.twoff[i] = off;
        s.mg_ns[i] = div_magic((uint32_t)ns);
        s.mg_nb[i] = div_magic((uint32_t)(n / radices[i]));
        if (ns > 1) off += ns * (radices[i] - 1);
        ns *= radices[i];
    }
    s.nst = cnt;
    s.mg_n = div_magic((uint32_t)n);
    s.mg_pairs = div_magic((uint32_t)(n / 2 + 1));
    s.mg_np1 = div_magic((uint32_t)(n + 1));
    return true;
}

static int64_t stage_twiddle_count(const AxisSched& s)
{
    int64_t c = 0;
    for (int i = 0; i < s.nst; ++i)
        if (s.ns[i] > 1) c += (int64_t)s.ns[i] * (s.radix[i] - 1);
    return c;
}

// e^{-2 pi i e/m}.  The angle is reduced exactly in integers: 4e = q m + r,
// angle = (pi/2)(q + r/m); the base angle is folded to [0, pi/4] (sin/cos of
// at most pi/4), the quadrant q applied by exact sign/swap.  Multiples of
// pi/2 are exact, odd multiples of pi/4 are sqrt(1/2).
void root_of_unity_ld(int64_t e, int64_t m, long double* c, long double* s)
{
    const long double HALF_PI = 1.570796326794896619231321691639751442L;
    e %= m;
    if (e < 0) e += m;
    const int64_t q = (4 * e) / m;
    const int64_t r = (4 * e) % m;
    long double cb, sb;  // cos, sin of the base angle (pi/2) r/m
    if (r == 0) {
        cb = 1.0L;
        sb = 0.0L;
    } else if (2 * r == m) {
        cb = sb = sqrtl(0.5L);
    } else if (2 * r < m) {
        long double phi = HALF_PI * (long double)r / (long double)m;
        cb = cosl(phi);
        sb = sinl(phi);
    } else {
        long double phi = HALF_PI * (long double)(m - r) / (long double)m;
        cb = sinl(phi);
        sb = cosl(phi);
    }
    long double ct, st;  // cos, sin of the full angle
    switch (q & 3) {
    case 0: ct = cb; st = sb; break;
    case 1: ct = -sb; st = cb; break;
    case 2: ct = -cb; st = -sb; break;
    default: ct = sb; st = -cb; break;
    }
    *c = ct;
    *s = -st;  // forward root: exp(-i angle)
}

static void fill_stage_twiddles(const AxisSched& s, long double* out)
{
    for (int i = 0; i < s.nst; ++i) {
        const int R = s.radix[i], Ns = s.ns[i];
        if (Ns == 1) continue;
        long double* t = out + 2 * (int64_t)s.twoff[i];
        for (int m = 0; m < Ns; ++m)
            for (int r = 1; r < R; ++r) {
                long double c, sn;
                root_of_unity_ld((int64_t)r * m, (int64_t)Ns * R, &c, &sn);
                t[2 * (m * (R - 1) + (r - 1))] = c;
                t[2 * (m * (R - 1) + (r - 1)) + 1] = sn;
            }
    }
}

// ------------------------------------------------------------- strategy --

// LDS row stride for rows of H elements at padded positions (pad16).  With
// bank_round the stride is also made 16 mod 32, so that the two rows a wave
// touches at once in a stage fall in disjoint banks too.
static int padded_stride(int64_t H, bool bank_round)
{
    int m = pad16_host((int)H - 1) + 1;
    if (bank_round)
        while (m % 32 != 16) ++m;
    return m;
}

static int ilog2(int v)
{
    int s = 0;
    while ((1 << s) < v) ++s;
    return s;
}

// Tile width W (columns per tile) for a pass of length-n lines over ncols
// columns: aim for rows of >= 128 contiguous bytes, widen for short lines so
// a tile still carries >= 2048 elements, keep within one tier.
static bool make_colpass(ColPass& cp, int64_t n, int64_t S, int64_t ncols, int64_t nbatch, int64_t bstride,
                         int cxs, int es, int eb, bool allow_big = true)
{
    cp = ColPass{};
    cp.S = S;
    cp.ncols = ncols;
    cp.nbatch = nbatch;
    cp.bstride = bstride;
    const int target = std::max(1, 128 / cxs);
    int64_t cap = 1;
    while (cap < ncols && cap < 64) cap *= 2;
    int W = std::min<int64_t>(target, cap);
    while (W < 64 && W < cap && n * W < 2048 && n * W * 2 <= es) W *= 2;
    bool big = false, wide = false;
    const int64_t ew = (int64_t)es / kNtSmall * kNtWide;
    if (!allow_big) {
        while (W > 1 && n * W > es) W /= 2;
        if (n * W > es || n * W * cxs > kLdsHalf) return false;
    } else if (n * W > es) {
        // prefer a larger tier at the target width over narrow segments: the
        // wide one (same registers per thread) if it holds the tile, else big
        if (n * W <= ew && n * W * cxs <= kLdsMax) {
            wide = true;
        } else if (n * W <= eb && n * W * cxs <= kLdsMax) {
            big = true;
        } else {
            while (W > 1 && n * W > es) W /= 2;
            if (n * W > es) {
                big = true;
                while (W > 1 && (n * W > eb || n * W * cxs > kLdsMax)) W /= 2;
                if (n * W > eb || n * W * cxs > kLdsMax) return false;
            }
        }
    }
    cp.W = W;
    cp.wshift = ilog2(W);
    cp.big = big;
    cp.wide = wide;
    cp.tiles_per_batch = (ncols + W - 1) / W;
    cp.lds = (size_t)(n * W * cxs);
    return true;
}

// Set a column pass's tile width to W (a power of two, at most 64): the
// tier is the smallest that holds n rows of W columns (small, wide, big).
// False if W is not such a width or no tier holds the tile.
static bool width_colpass(ColPass& cp, int64_t n, int W, int cxs, int es, int eb)
{
    if (W < 1 || W > 64 || (W & (W - 1))) return false;
    const int64_t ew = (int64_t)es / kNtSmall * kNtWide;
    const int64_t e = n * W, bytes = e * cxs;
    bool big = false, wide = false;
    if (e <= es && bytes <= kLdsHalf) {
    } else if (e <= ew && bytes <= kLdsMax) {
        wide = true;
    } else if (e <= eb && bytes <= kLdsMax) {
        big = true;
    } else {
        return false;
    }
    cp.W = W;
    cp.wshift = ilog2(W);
    cp.big = big;
    cp.wide = wide;
    cp.tiles_per_batch = (cp.ncols + W - 1) / W;
    cp.lds = (size_t)bytes;
    return true;
}

// A small FP32 column tile goes to the fine tier when every stage of its
// schedule has radix <= 8 (the tile is the same 8192 elements).
static void mark_fine(ColPass& cp, const AxisSched& ax)
{
    bool ok = !cp.big && !cp.wide && ax.nst > 0;
    for (int i = 0; i < ax.nst; ++i) ok = ok && ax.radix[i] <= kFineMaxRadix;
    cp.fine = ok;
}

// A wide tile of a schedule whose first stage has radix 16 or 8, with more
// stages after it of radix <= kPipeMaxRadix, runs as the persistent loop of
// k_cols_pipe when the tile and the later stages' twiddles fit LDS together.
static void mark_pipe(ColPass& cp, const AxisSched& ax, bool on, int cxs)
{
    bool ok = on && cp.wide && ax.nst >= 2 && (ax.radix[0] == 16 || ax.radix[0] == 8) &&
              cp.lds + (size_t)later_twiddles(ax) * (size_t)cxs <= (size_t)kLdsMax;
    for (int i = 1; i < ax.nst; ++i) ok = ok && ax.radix[i] <= kPipeMaxRadix;
    cp.pipe = ok;
}

bool small_colpass(const Plan& p, int axis, ColPass& cp)
{
    const int cxs = 2 * p.elem;
    const int es = kNtSmall * (p.dtype ? Tier<double>::kEptSmall : Tier<float>::kEptSmall);
    if (axis == 0) return make_colpass(cp, p.n0, p.C, p.C, 1, 0, cxs, es, es, false);
    return make_colpass(cp, p.n1, p.H, p.H, p.n0, p.n1 * p.H, cxs, es, es, false);
}

const char* split_tiling(const Plan& p, int& rpw, bool& rows_big, size_t& rows_lds, int& rpw_inv,
                         size_t& rows_lds_inv, ColPass& pass1)
{
    const int cxs = 2 * p.elem;
    const int es = kNtSmall * (p.dtype ? Tier<double>::kEptSmall : Tier<float>::kEptSmall);
    const int eb = kNtBig * (p.dtype ? Tier<double>::kEptBig : Tier<float>::kEptBig);
    // rows per tile: what the small tier holds, within an LDS budget that
    // lets as many workgroups share a CU as the kernel's registers allow:
    // FP32 three (the forward kernel of even n2 four), FP64 two -- measured
    // at 512^3: FP32 rows kernels 4.35 -> 4.72 TB/s with 16 rows instead of
    // 32 (three a CU), the forward one 226 -> 215 us at four a CU
    const int64_t budget = p.dtype == FFT3D_F64 ? 60 * 1024 : 48 * 1024;
    const int64_t budget_fwd = p.dtype == FFT3D_F32 && p.n2 % 2 == 0 ? 40 * 1024 : budget;
    if (p.n2 % 2 != 0) {
        // odd n2: pairs of rows per complex line of n2 elements, an even
        // number of rows per tile (the last tile pairs its odd row with a
        // zero row in the slot after it), at most kPairItems (pair, bin)
        // items per thread in the separation
        const int64_t pair_cap = std::max<int64_t>(1, (int64_t)kNtSmall * kPairItems / p.H);
        int64_t pairs = std::min<int64_t>({es / p.n2, budget / (2 * (int64_t)p.Hs * cxs), pair_cap});
        rows_big = false;
        if (pairs < 1) {
            pairs = std::min<int64_t>({eb / p.n2, kLdsMax / (2 * (int64_t)p.Hs * cxs), pair_cap});
            rows_big = true;
        }
        if (pairs < 1) return "n2 too large for one pair of rows in LDS";
        rpw = (int)std::min<int64_t>(2 * pairs, p.n0 * p.n1);
        rows_lds = (size_t)((rpw + (rpw & 1)) * p.Hs * cxs);
        rpw_inv = rpw;
        rows_lds_inv = rows_lds;
        if (!make_colpass(pass1, p.n1, p.H, p.H, p.n0, p.n1 * p.H, cxs, es, eb))
            return "n1 too large for a column tile";
        return nullptr;
    }
    // both directions take the same tier: the budgets differ only below
    // what one small-tier row needs (FP32 rows of up to 4096 bins take
    // 34 KB padded)
    const int64_t per_row = (int64_t)p.Hs * cxs;
    int64_t r = std::min<int64_t>(es / p.h, budget_fwd / per_row);
    int64_t ri = std::min<int64_t>(es / p.h, budget / per_row);
    rows_big = false;
    if (r < 1 || ri < 1) {
        r = ri = std::min<int64_t>(eb / p.h, kLdsMax / per_row);
        rows_big = true;
    }
    if (r < 1) return "n2 too large for one row in LDS";
    rpw = (int)std::min<int64_t>(r, p.n0 * p.n1);
    rows_lds = (size_t)(rpw * per_row);
    rpw_inv = (int)std::min<int64_t>(ri, p.n0 * p.n1);
    rows_lds_inv = (size_t)(rpw_inv * per_row);
    if (!make_colpass(pass1, p.n1, p.H, p.H, p.n0, p.n1 * p.H, cxs, es, eb)) return "n1 too large for a column tile";
    return nullptr;
}

int plan_build_host(Plan& p, int64_t n0, int64_t n1, int64_t n2, int dtype, int flags, const fft3d_tuning* t,
                    std::string& why)
{
    char msg[256];
    if (n0 < 1 || n1 < 1 || n2 < 1) {
        why = "extents must be >= 1";
        return FFT3D_ERR_INVALID_ARG;
    }
    if (dtype != FFT3D_F32 && dtype != FFT3D_F64) {
        why = "dtype must be FFT3D_F32 or FFT3D_F64";
        return FFT3D_ERR_INVALID_ARG;
    }
    if (n0 > 4096 || n1 > 4096 || n2 > 8192) {
        why = "extents above n0, n1 <= 4096, n2 <= 8192 are not supported";
        return FFT3D_ERR_UNSUPPORTED;
    }
    p = Plan{};
    p.n0 = n0;
    p.n1 = n1;
    p.n2 = n2;
    p.h = n2 / 2;
    p.H = p.h + 1;
    p.C = n1 * p.H;
    p.M = n0 * p.C;
    p.N = n0 * n1 * n2;
    p.dtype = dtype;
    p.elem = dtype == FFT3D_F64 ? 8 : 4;
    // rows: a half-length complex FFT of h = n2/2 for even n2, a full-length
    // one of n2 (two real rows per complex line) for odd n2
    const bool n2_odd = n2 % 2 != 0;
    if (!make_schedule(n0, p.ax0) || !make_schedule(n1, p.ax1) || !make_schedule(n2_odd ? n2 : p.h, p.ax2h)) {
        snprintf(msg, sizeof msg, "extents %lld x %lld x %lld: n0, n1 and n2 (n2/2 for even n2) must have no prime factor other than 2, 3, 5 and 7",
                 (long long)n0, (long long)n1, (long long)n2);
        why = msg;
        return FFT3D_ERR_UNSUPPORTED;
    }
    if (t) {
        p.tuned = true;
        p.tuning = *t;
        AxisSched* axes[3] = {&p.ax0, &p.ax1, &p.ax2h};
        const int64_t lens[3] = {n0, n1, n2_odd ? n2 : p.h};
        for (int a = 0; a < 3; ++a) {
            if (t->radix[a][0] == 0) continue;
            int cnt = 0;
            while (cnt < 8 && t->radix[a][cnt] != 0) ++cnt;
            if (!fill_schedule(lens[a], t->radix[a], cnt, *axes[a])) {
                snprintf(msg, sizeof msg,
                         "tuning: radix[%d] is not a schedule of length %lld (radices 2, 3, 4, 8, 16, 5, 7 "
                         "whose product is the length)",
                         a, (long long)lens[a]);
                why = msg;
                return FFT3D_ERR_INVALID_ARG;
            }
        }
    }
    const fft3d_tuning tz{};
    const fft3d_tuning& tu = t ? *t : tz;

    for (const AxisSched* a : {&p.ax0, &p.ax1, &p.ax2h})
        for (int i = 0; i < a->nst; ++i)
            if (a->radix[i] == 5 || a->radix[i] == 7) p.odd = true;

    // twiddle table: [n2/2 stages | split roots k = 0..h | n1 stages | n0 stages]
    p.off_ax2h = 0;
    p.off_post = p.off_ax2h + stage_twiddle_count(p.ax2h);
    p.off_ax1 = p.off_post + (p.h + 1);
    p.off_ax0 = p.off_ax1 + stage_twiddle_count(p.ax1);
    p.tw_count = p.off_ax0 + stage_twiddle_count(p.ax0);
    p.tw_host.assign(2 * (size_t)p.tw_count, 0.0L);
    fill_stage_twiddles(p.ax2h, p.tw_host.data() + 2 * p.off_ax2h);
    for (int64_t k = 0; k <= p.h; ++k) {
        long double c, s;
        root_of_unity_ld(k, n2, &c, &s);
        p.tw_host[2 * (p.off_post + k)] = c;
        p.tw_host[2 * (p.off_post + k) + 1] = s;
    }
    fill_stage_twiddles(p.ax1, p.tw_host.data() + 2 * p.off_ax1);
    fill_stage_twiddles(p.ax0, p.tw_host.data() + 2 * p.off_ax0);

    // kernel choice
    const int cxs = 2 * p.elem;
    const int es = kNtSmall * (dtype ? Tier<double>::kEptSmall : Tier<float>::kEptSmall);
    const int eb = kNtBig * (dtype ? Tier<double>::kEptBig : Tier<float>::kEptBig);
    const int64_t plane_elems = n1 * p.H;  // >= n1*h: bounds both plane phases
    // a whole plane in LDS as padded rows: bank-friendly stride if it fits,
    // else the smallest padded stride
    const int hs_bank = padded_stride(p.H, true), hs_min = padded_stride(p.H, false);
    p.Hs = hs_bank;
    bool fused = false;
    for (int big = 0; big < 2 && !fused && !n2_odd; ++big) {
        const int64_t emax = big ? eb : es, lmax = big ? kLdsMax : kLdsHalf;
        for (int hs : {hs_bank, hs_min}) {
            if (plane_elems <= emax && n1 * hs * cxs <= lmax) {
                fused = true;
                p.plane_big = big;
                p.plane_Hs = hs;
                p.plane_lds = (size_t)(n1 * hs * cxs);
                break;
            }
        }
    }
    if (tu.plane < 0 || tu.plane > FFT3D_TUNE_COOP) {
        why = "tuning: plane must be 0, FFT3D_TUNE_FUSED, FFT3D_TUNE_SPLIT or FFT3D_TUNE_COOP";
        return FFT3D_ERR_INVALID_ARG;
    }
    if (tu.plane == FFT3D_TUNE_FUSED && !fused) {
        why = "tuning: plane FUSED, but the plane does not fit in LDS (or n2 is odd)";
        return FFT3D_ERR_INVALID_ARG;
    }
    if (tu.plane == FFT3D_TUNE_SPLIT || tu.plane == FFT3D_TUNE_COOP) fused = false;
    if (fused) {
        p.fused_plane = true;
        p.ppw = 1;
        if (tu.rows_rpw || tu.rows_rpw_inv || tu.n1_w || tu.coop_lag || tu.coop_rpw || tu.coop_w) {
            why = "tuning: rows_rpw, rows_rpw_inv, n1_w and coop_* apply to split or cooperative plane steps only";
            return FFT3D_ERR_INVALID_ARG;
        }
    } else {
        p.fused_plane = false;
        const char* err = split_tiling(p, p.rpw, p.rows_big, p.rows_lds, p.rpw_inv, p.rows_lds_inv, p.pass1);
        if (err) {
            why = err;
            return FFT3D_ERR_UNSUPPORTED;
        }
        // rows per tile, forward and inverse: up to what the rows kernel's
        // tier holds (the rule keeps an LDS budget below that, for occupancy)
        const int64_t per_row = (int64_t)p.Hs * cxs;
        const int64_t emax = p.rows_big ? eb : es, lmax = p.rows_big ? kLdsMax : kLdsHalf;
        const int64_t rows_cap = n2_odd ? std::min<int64_t>(emax / n2, (int64_t)kNtSmall * kPairItems / p.H) * 2
                                        : emax / p.h;
        for (int inv = 0; inv < 2; ++inv) {
            const int r = inv ? tu.rows_rpw_inv : tu.rows_rpw;
            if (!r) continue;
            const int64_t rr = (int64_t)r + (n2_odd ? (r & 1) : 0);
            if (r < 1 || (n2_odd && (r & 1)) || r > rows_cap || rr * per_row > lmax) {
                snprintf(msg, sizeof msg, "tuning: %s %d does not fit the rows kernel (1..%lld%s)",
                         inv ? "rows_rpw_inv" : "rows_rpw", r,
                         (long long)std::min<int64_t>(rows_cap, lmax / per_row), n2_odd ? ", even" : "");
                why = msg;
                return FFT3D_ERR_INVALID_ARG;
            }
            int& rp = inv ? p.rpw_inv : p.rpw;
            size_t& rl = inv ? p.rows_lds_inv : p.rows_lds;
            rp = (int)std::min<int64_t>(r, n0 * n1);
            rl = (size_t)((rp + (n2_odd ? (rp & 1) : 0)) * per_row);
        }
        if (tu.n1_w) {
            if (!width_colpass(p.pass1, n1, tu.n1_w, cxs, es, eb)) {
                snprintf(msg, sizeof msg, "tuning: n1_w %d is not a power of two <= 64 whose tile fits a tier",
                         tu.n1_w);
                why = msg;
                return FFT3D_ERR_INVALID_ARG;
            }
        }
        // one cooperative launch for the plane step when both task kinds fit
        // the small tier
        const bool coop_ok = !p.rows_big && !p.pass1.big && !p.pass1.wide && n1 > 1 && !p.odd && !n2_odd;
        if (tu.plane == FFT3D_TUNE_COOP && !coop_ok) {
            why = "tuning: plane COOP needs rows and n1 tiles of the small tier, n1 > 1, even n2 and radix 2/3 "
                  "schedules";
            return FFT3D_ERR_INVALID_ARG;
        }
        const bool want_coop = tu.plane == FFT3D_TUNE_COOP || (tu.plane == 0 && (flags & FFT3D_PLAN_COOP_PLANE));
        if (!(want_coop && coop_ok) && (tu.coop_lag || tu.coop_rpw || tu.coop_w)) {
            why = "tuning: coop_* apply to the cooperative plane step only";
            return FFT3D_ERR_INVALID_ARG;
        }
        if (want_coop && coop_ok) {
            p.coop = true;
            p.coop_rpw = p.rpw;
            p.coop_w = p.pass1.W;
            if (tu.coop_rpw) {
                if (tu.coop_rpw < 1 || tu.coop_rpw > p.rpw) {
                    why = "tuning: coop_rpw must be 1..rows per rows tile";
                    return FFT3D_ERR_INVALID_ARG;
                }
                p.coop_rpw = tu.coop_rpw;
            }
            if (tu.coop_w) {
                if (tu.coop_w < 1 || tu.coop_w > p.pass1.W || (tu.coop_w & (tu.coop_w - 1))) {
                    why = "tuning: coop_w must be a power of two up to the n1 tile width";
                    return FFT3D_ERR_INVALID_ARG;
                }
                p.coop_w = tu.coop_w;
            }
            if (tu.coop_lag) {
                if (tu.coop_lag < 1 || tu.coop_lag > 256) {
                    why = "tuning: coop_lag must be 1..256";
                    return FFT3D_ERR_INVALID_ARG;
                }
                p.coop_lag = tu.coop_lag;
            }
            p.coop_rt = (int)((n1 + p.coop_rpw - 1) / p.coop_rpw);
            p.coop_ct = (int)((p.H + p.coop_w - 1) / p.coop_w);
            p.coop_lds = (size_t)std::max<int64_t>((int64_t)p.coop_rpw * p.Hs * cxs, n1 * p.coop_w * cxs);
        }
    }
    if (!make_colpass(p.pass0, n0, p.C, p.C, 1, 0, cxs, es, eb)) {
        why = "n0 too large for a column tile";
        return FFT3D_ERR_UNSUPPORTED;
    }
    // the n0 pass of the transpose-based method: length-n0 columns of the
    // [n1][n0][H] layout, one block per k1
    if (!make_colpass(p.pass0t, n0, p.H, p.H, n1, n0 * p.H, cxs, es, eb)) {
        why = "n0 too large for a column tile";
        return FFT3D_ERR_UNSUPPORTED;
    }
    // n0-pass tiles per XCD group: neighbouring column tiles read and write
    // neighbouring 128-byte segments of every row; keeping 8 (FP32) / 16
    // (FP64) of them on one XCD measured 1.5-3% faster pairs at 512^3
    p.n0_group = dtype == FFT3D_F64 ? 16 : 8;
    if (tu.n0_group) {
        if (tu.n0_group < 1) {
            why = "tuning: n0_group must be >= 1";
            return FFT3D_ERR_INVALID_ARG;
        }
        p.n0_group = tu.n0_group;
    }
    if (tu.walk) {
        if (tu.walk < 64 || tu.walk > 127) {
            why = "tuning: walk must be 0 or 64 + bits (0..63)";
            return FFT3D_ERR_INVALID_ARG;
        }
        p.rev = tu.walk & 63;
    }
    if (tu.n0_w) {
        if (!width_colpass(p.pass0, n0, tu.n0_w, cxs, es, eb)) {
            snprintf(msg, sizeof msg, "tuning: n0_w %d is not a power of two <= 64 whose tile fits a tier", tu.n0_w);
            why = msg;
            return FFT3D_ERR_INVALID_ARG;
        }
    }
    // FP32 small column tiles of radix <= 8 schedules run on the fine tier
    // (measured at 512^3: n1 passes 238 -> 234 us, pairs 1.3% faster)
    if (dtype == FFT3D_F32) {
        mark_fine(p.pass0, p.ax0);
        mark_fine(p.pass0t, p.ax0);
        if (!p.fused_plane) mark_fine(p.pass1, p.ax1);
    }
    if (tu.cols_pipe < 0 || tu.cols_pipe > 2) {
        why = "tuning: cols_pipe must be 0, 1 or 2";
        return FFT3D_ERR_INVALID_ARG;
    }
    const bool pipe = tu.cols_pipe != 1;
    mark_pipe(p.pass0, p.ax0, pipe, cxs);
    mark_pipe(p.pass0t, p.ax0, pipe, cxs);
    if (!p.fused_plane) mark_pipe(p.pass1, p.ax1, pipe, cxs);
    return FFT3D_OK;
}

// ------------------------------------------------------------- describe --

static std::string sched_json(const AxisSched& s)
{
    std::string r = "{\"n\": " + std::to_string(s.n) + ", \"radices\": [";
    for (int i = 0; i < s.nst; ++i) r += (i ? ", " : "") + std::to_string(s.radix[i]);
    return r + "]}";
}

static std::string pass_json(const ColPass& c)
{
    char b[384];
    snprintf(b, sizeof b,
             "{\"row_stride\": %lld, \"ncols\": %lld, \"nbatch\": %lld, \"batch_stride\": %lld, "
             "\"W\": %d, \"tier\": \"%s\", \"grid\": %lld, \"lds\": %zu, \"pipe\": %s}",
             (long long)c.S, (long long)c.ncols, (long long)c.nbatch, (long long)c.bstride, c.W,
             c.big ? "big" : (c.wide ? "wide" : (c.fine ? "fine" : "small")), (long long)(c.nbatch * c.tiles_per_batch),
             c.lds, c.pipe ? "true" : "false");
    return b;
}

std::string Plan::describe() const
{
    char b[512];
    snprintf(b, sizeof b,
             "{\"n0\": %lld, \"n1\": %lld, \"n2\": %lld, \"dtype\": \"%s\", \"H\": %lld, \"columns\": %lld, "
             "\"device\": %d, \"twiddles\": %lld, ",
             (long long)n0, (long long)n1, (long long)n2, dtype ? "f64" : "f32", (long long)H, (long long)C,
             has_device ? device : -1, (long long)tw_count);
    std::string r = b;
    r += "\"schedules\": {\"n0\": " + sched_json(ax0) + ", \"n1\": " + sched_json(ax1) +
         ", \"n2_half\": " + sched_json(ax2h) + "}, ";
    if (fused_plane) {
        snprintf(b, sizeof b,
                 "\"plane\": {\"kind\": \"fused\", \"planes_per_wg\": %d, \"tier\": \"%s\", \"grid\": %lld, "
                 "\"lds\": %zu}, ",
                 ppw, plane_big ? "big" : "small", (long long)((n0 + ppw - 1) / ppw), plane_lds);
        r += b;
    } else {
        snprintf(b, sizeof b,
                 "\"plane\": {\"kind\": \"%s\", \"rows_per_wg\": %d, \"tier\": \"%s\", \"grid\": %lld, "
                 "\"lds\": %zu, \"rows_per_wg_inv\": %d, \"grid_inv\": %lld, \"lds_inv\": %zu, ",
                 coop ? "coop" : "split", rpw, rows_big ? "big" : "small",
                 (long long)((n0 * n1 + rpw - 1) / rpw), rows_lds, rpw_inv,
                 (long long)((n0 * n1 + rpw_inv - 1) / rpw_inv), rows_lds_inv);
        r += b;
        if (coop) {
            snprintf(b, sizeof b,
                     "\"coop\": {\"row_tasks\": %d, \"col_tasks\": %d, \"rows_per_task\": %d, "
                     "\"cols_per_task\": %d, \"lag\": %d, \"grid\": %d, \"lds\": %zu, \"slots\": %d}, ",
                     coop_rt, coop_ct, coop_rpw, coop_w, coop_lag, coop_grid, coop_lds, coop_nslots);
            r += b;
        }
        r += "\"n1_pass\": " + pass_json(pass1) + "}, ";
    }
    r += "\"n0_pass\": " + pass_json(pass0) + ", \"n0_group\": " + std::to_string(n0_group) + ", \"rev\": " + std::to_string(rev) + ", \"radix57\": " + (odd ? "true" : "false") + ", ";
    // pass lists (FFT3D_PASS_* ids) of the two directions
    std::string f = "[0", i = "[";
    const bool n1_pass = !fused_plane && !coop && n1 > 1;
    if (n1_pass) f += ", 1";
    if (n0 > 1) {
        f += ", 2";
        i += "3, ";
    }
    if (n1_pass) i += "4, ";
    r += "\"r2c_passes\": " + f + "], \"c2r_passes\": " + i + "5], ";
    // the tuning the plan was built with (fft3d_plan_tuned), or null
    if (tuned) {
        char t[384];
        snprintf(t, sizeof t,
                 "\"tuning\": {\"plane\": %d, \"rows_rpw\": %d, \"rows_rpw_inv\": %d, \"n1_w\": %d, \"n0_w\": %d, "
                 "\"n0_group\": %d, \"walk\": %d, \"coop_lag\": %d, \"coop_rpw\": %d, \"coop_w\": %d, "
                 "\"cols_pipe\": %d, \"radix\": [",
                 tuning.plane, tuning.rows_rpw, tuning.rows_rpw_inv, tuning.n1_w, tuning.n0_w, tuning.n0_group,
                 tuning.walk, tuning.coop_lag, tuning.coop_rpw, tuning.coop_w, tuning.cols_pipe);
        r += t;
        for (int a = 0; a < 3; ++a) {
            r += a ? ", [" : "[";
            for (int k = 0; k < 8 && tuning.radix[a][k]; ++k) r += (k ? ", " : "") + std::to_string(tuning.radix[a][k]);
            r += "]";
        }
        r += "]}}";
    } else {
        r += "\"tuning\": null}";
    }
    return r;
}

}  // namespace fft3d
