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
// material: per-element eps and mu (FP64 and FP32; the vector kernel handles
// both flux forms at run time).
template <typename T>
KernelSet make(int variant, bool material) {
  constexpr int N = DG_ORDER;
  KernelSet k;
  if (variant == kVariantValu) {
    k.rhs = &launch_rhs_valu<N, T>;
    k.tile = valu_tile<N>();
  } else if (variant == kVariantMfma) {
    if constexpr (mfma_supported<N, T>()) {
      if (material) {
        k.rhs = &launch_rhs_mfma<N, T, 0, true>;
        k.rk = &launch_rk_mfma<N, T, 0, true>;
      } else {
        k.rhs = &launch_rhs_mfma<N, T>;
        k.rk = &launch_rk_mfma<N, T>;
        k.batch = &launch_rk_mfma_batch<N, T>;
      }
      k.tile = 16;
      k.frag_count = MfmaShape<N>::frag_count;
    }
  }
  return k;
}

// Split 16-bit contraction (FP32 state): matrix-core variants only, vacuum
// flux only.
template <int MIX>
KernelSet make_mixed(int variant, bool material) {
  constexpr int N = DG_ORDER;
  KernelSet k;
  if (variant == kVariantMfma && !material) {
    if constexpr (mfma_supported<N, float>()) {
      k.rhs = &launch_rhs_mfma<N, float, MIX>;
      k.rk = &launch_rk_mfma<N, float, MIX>;
      k.tile = 16;
      k.frag16_bytes = MixedShape<N>::frag_bytes;
    }
  }
  return k;
}
}  // namespace

// precision: 0 FP64, 1 FP32, 2 BF16x3, 3 FP16x3, 4 BF16, 5 FP16, 6 BF16x2, 7 FP16x2
KernelSet DG_CAT(kernels_n, DG_ORDER)(int precision, int variant, bool material) {
  switch (precision) {
    case 0: return make<double>(variant, material);
    case 1: return make<float>(variant, material);
    case 2: return make_mixed<3>(variant, material);
    case 3: return make_mixed<6>(variant, material);
    case 4: return make_mixed<1>(variant, material);
    case 5: return make_mixed<4>(variant, material);
    case 6: return make_mixed<2>(variant, material);
    case 7: return make_mixed<5>(variant, material);
    default: return KernelSet{};
  }
}

}  // namespace dgd
