// fft3d_sched.hpp -- plain data shared by the host plan and the kernels:
// the radix schedule of one line length and the layout of lines in LDS.
#pragma once

#include <stdint.h>

namespace fft3d {

constexpr int kMaxStages = 12;

// Fine tier of the FP32 column kernels: a small-tier tile (8192 elements) on
// 1024 threads of 8 elements each, for schedules of radix <= 8 only.  Its
// kernels carry no radix-16 code, which keeps them at eight waves per SIMD
// (two 1024-thread workgroups on a CU).
constexpr int kNtFine = 1024;
constexpr int kEptFine = 8;
constexpr int kFineMaxRadix = 8;
// Largest radix after the first stage of a pipelined wide column pass
// (k_cols_pipe).
constexpr int kPipeMaxRadix = 8;

// Division by an invariant d in [1, 2^16) of an index n with n*d < 2^32:
// n / d = mulhi32(n, magic(d)) with magic(d) = floor(2^32/d) + 1, and
// magic(1) = 0 meaning "n / 1 = n".  Exactness: n*magic/2^32 exceeds n/d by
// at most n/2^32 < 1/d, which cannot carry past the next integer.
inline uint32_t div_magic(uint32_t d) { return d <= 1 ? 0u : (uint32_t)((1ull << 32) / d + 1); }

// Radix schedule of one line length, as the kernels see it.
struct AxisSched {
    int32_t n;                   // line length
    int32_t nst;                 // number of stages (0 for n == 1)
    int32_t radix[kMaxStages];   // radix of each stage
    int32_t ns[kMaxStages];      // product of the radices before the stage
    int32_t twoff[kMaxStages];   // offset of the stage's twiddles in the axis table
    uint32_t mg_ns[kMaxStages];  // div_magic(ns)
    uint32_t mg_nb[kMaxStages];  // div_magic(n / radix): butterflies per line
    uint32_t mg_n;               // div_magic(n)
    uint32_t mg_pairs;           // div_magic(n/2 + 1): (k, n-k) pairs of a real split
    uint32_t mg_np1;             // div_magic(n + 1): bins of a real row of length 2n
};

// Padded position of element i of a row held in LDS: one spare slot after
// every 16 elements, so the stride-R writes of a Stockham stage fall in
// different LDS banks.
inline constexpr int pad16_host(int i) { return i + (i >> 4); }

// Twiddles of the stages after the first of an axis schedule (the first has
// none): complex values from the start of the axis's table.
inline constexpr int later_twiddles(const AxisSched& ax)
{
    return ax.nst > 1 ? ax.twoff[ax.nst - 1] + ax.ns[ax.nst - 1] * (ax.radix[ax.nst - 1] - 1) : 0;
}

// Lines in LDS: element i of line w lives at
//   (w / lpp) * sp + (w % lpp) * sw + i * si.
// LINES_FAST: consecutive threads take consecutive lines (use when sw == 1),
// otherwise consecutive positions along a line (use when si == 1).
struct LdsLines {
    int32_t nlines;
    int32_t lpp;        // lines per panel
    int32_t sp;         // panel stride
    int32_t sw;         // line stride within a panel
    int32_t si;         // element stride along a line
    uint32_t mg_lines;  // div_magic(nlines)
    uint32_t mg_lpp;    // div_magic(lpp)
};

}  // namespace fft3d
