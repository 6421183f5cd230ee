// fft3d_sched.hpp -- plain data shared by the host plan and the kernels:
// the radix schedule of one line length and the layout of lines in LDS.
#pragma once

#include <stdint.h>

namespace fft3d {

constexpr int kMaxStages = 12;

// Radix schedule of one line length, as the kernels see it.
struct AxisSched {
    int32_t n;                  // line length
    int32_t nst;                // number of stages (0 for n == 1)
    int32_t radix[kMaxStages];  // radix of each stage
    int32_t ns[kMaxStages];     // product of the radices before the stage
    int32_t twoff[kMaxStages];  // offset of the stage's twiddles in the axis table
};

// Lines in LDS: element i of line w lives at
//   (w / lpp) * sp + (w % lpp) * sw + i * si.
// LINES_FAST: consecutive threads take consecutive lines (use when sw == 1),
// otherwise consecutive positions along a line (use when si == 1).
struct LdsLines {
    int32_t nlines;
    int32_t lpp;  // lines per panel
    int32_t sp;   // panel stride
    int32_t sw;   // line stride within a panel
    int32_t si;   // element stride along a line
};

}  // namespace fft3d
