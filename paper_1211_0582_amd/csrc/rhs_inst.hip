// One order's instantiation of the right-hand-side kernels; the build compiles
// this file once per order N = 1..9 with -DDG_ORDER=N (parallel builds, small
// objects).
#include "rhs_mfma.hpp"
#include "rhs_valu.hpp"

#ifndef DG_ORDER
#error "DG_ORDER must be defined"
#endif

#define DG_CAT2(a, b) a##b
#define DG_CAT(a, b) DG_CAT2(a, b)

namespace dgd {

namespace {
template <typename T>
KernelSet make(int variant) {
  constexpr int N = DG_ORDER;
  KernelSet k;
  if (variant == kVariantValu) {
    k.rhs = &launch_rhs_valu<N, T>;
    k.tile = valu_tile<N>();
  } else if (variant == kVariantMfma) {
    if constexpr (mfma_supported<N, T>()) {
      k.rhs = &launch_rhs_mfma<N, T>;
      k.rk = &launch_rk_mfma<N, T>;
      k.tile = 16;
      k.frag_count = MfmaShape<N>::frag_count;
    }
  }
  return k;
}
}  // namespace

KernelSet DG_CAT(kernels_n, DG_ORDER)(int precision, int variant) {
  return precision == 0 ? make<double>(variant) : make<float>(variant);
}

}  // namespace dgd
