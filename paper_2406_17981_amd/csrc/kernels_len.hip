// One pencil length's kernels, built once per entry of lengths.def with
// -DSFFT_LEN=<L>; exports sfft_ops_<L>(dtype) for the runtime's table.
#include "axis_kernels.hpp"

#ifndef SFFT_LEN
#error "build with -DSFFT_LEN=<pencil length>"
#endif
#define SFFT_CAT2(a, b) a##b
#define SFFT_CAT(a, b) SFFT_CAT2(a, b)

extern "C" const sfft::AxisOps* SFFT_CAT(sfft_ops_, SFFT_LEN)(int dtype) {
  return dtype == 0 ? sfft::make_ops<float, SFFT_LEN>() : sfft::make_ops<double, SFFT_LEN>();
}
