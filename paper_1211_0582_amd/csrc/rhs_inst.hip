// One order's instantiation of the right-hand-side kernels; the build compiles
// this file once per order N = 1..9 with -DDG_ORDER=N (parallel builds, small
// objects).
#include "rhs_valu.hpp"

#ifndef DG_ORDER
#error "DG_ORDER must be defined"
#endif

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

namespace dgd {

RhsLauncher DG_CAT(rhs_launcher_n, DG_ORDER)(int precision) {
  return precision == 0 ? &launch_rhs_valu<DG_ORDER, double> : &launch_rhs_valu<DG_ORDER, float>;
}

int DG_CAT(rhs_tile_n, DG_ORDER)(int) { return valu_tile<DG_ORDER>(); }

}  // namespace dgd
