// inst.hip - the launch tables of one FFT length; compiled once per length
// with -DLB_N=<length>.
#include <type_traits>
#include "launch.hpp"

#ifndef LB_N
#error "compile with -DLB_N=<FFT length>"
#endif

#define LB_CAT2(a, b) a##b
#define LB_CAT(a, b) LB_CAT2(a, b)

namespace lb {
const NFuncs *LB_CAT(funcs_, LB_N)(int prec) {
  static const NFuncs f64 = Impl<double, LB_N>::table();
  static const NFuncs f32 = Impl<float, LB_N>::table();
  return prec == 0 ? &f64 : &f32;
}
}  // namespace lb
