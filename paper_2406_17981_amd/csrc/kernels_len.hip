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

// Radices of this length's pass kernels (leaf = 0) or leaf kernel (leaf = 1)
// in the given dtype, outermost stage first; returns how many (at most 8).
extern "C" int SFFT_CAT(sfft_radix_, SFFT_LEN)(int dtype, int leaf, int* rads) {
  int n = 0;
  auto put = [&](const int* r, int s) {
    for (int i = 0; i < s && i < 8; ++i) rads[n++] = r[i];
  };
  if (!leaf) put(sfft::Shape<SFFT_LEN>::rads, sfft::Shape<SFFT_LEN>::S);
  else if (dtype == 0) put(sfft::Geo<float, SFFT_LEN>::LSh::rads, sfft::Geo<float, SFFT_LEN>::LSh::S);
  else put(sfft::Geo<double, SFFT_LEN>::LSh::rads, sfft::Geo<double, SFFT_LEN>::LSh::S);
  return n;
}
