// fft3d_pruned_f64_odd.hip -- the pruned transforms with the radix-5 and radix-7 stages
// compiled in, for plans whose extents have those factors.
#define FFT3D_ODD_RADICES 1
#include "fft3d_pruned_f64.hip"
