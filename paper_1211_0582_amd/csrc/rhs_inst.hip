// One (order, precision group) instantiation of the right-hand-side kernels;
// the build compiles this file for every order N = 1..9 (-DDG_ORDER=N) and
// precision group (-DDG_GROUP=0: FP64, 1: FP32, 2: the split 16-bit forms),
// so the objects build in parallel.
#include "rhs_mfma.hpp"
#include "rhs_valu.hpp"

#ifndef DG_ORDER
#error "DG_ORDER must be defined"
#endif
#ifndef DG_GROUP
#error "DG_GROUP must be defined"
#endif

#define DG_CAT3(a, b, c, d) a##b##c##d
#define DG_NAME(n, g) DG_CAT3(kernels_n, n, _g, g)

namespace dgd {

namespace {
constexpr int N = DG_ORDER;

// Matrix-core kernels of tuning configuration CFG (variant kVariantMfma + CFG).
template <typename T, int MIX, int CFG>
KernelSet make_mfma(bool material) {
  KernelSet k;
  if constexpr (config_built<N, T, MIX, CFG>()) {
    if (material) {
      if constexpr (MIX == 0 && CFG == kCfgDefault) {
        k.rhs = &launch_rhs_mfma<N, T, 0, true>;
        k.rk = &launch_rk_mfma<N, T, 0, true>;
      }
    } else {
      k.rhs = &launch_rhs_mfma<N, T, MIX, false, CFG>;
      k.rk = &launch_rk_mfma<N, T, MIX, false, CFG>;
      if constexpr (MIX == 0 && CFG == kCfgDefault) k.batch = &launch_rk_mfma_batch<N, T>;
    }
    if (k.rhs) {
      k.tile = 16;
      k.frag_count = MfmaShape<N>::frag_count;
      k.frag16_bytes = MIX ? SplitShape<N>::frag_bytes : 0;
    }
  }
  return k;
}

template <typename T, int MIX>
KernelSet make(int variant, bool material) {
  KernelSet k;
  if (variant == kVariantValu) {
    if constexpr (MIX == 0) {
      k.rhs = &launch_rhs_valu<N, T>;
      k.tile = valu_tile<N>();
    }
    return k;
  }
  switch (variant - kVariantMfma) {
    case kCfgDefault: return make_mfma<T, MIX, kCfgDefault>(material);
    case kCfgWaves: return make_mfma<T, MIX, kCfgWaves>(material);
    case kCfgPrefetch: return make_mfma<T, MIX, kCfgPrefetch>(material);
    case kCfgOccupancy: return make_mfma<T, MIX, kCfgOccupancy>(material);
    // the flux interleave, split lift and 4-row tail exist for FP64 / FP32 only
    case kCfgInterleave: if constexpr (MIX == 0) return make_mfma<T, MIX, kCfgInterleave>(material); else return k;
    case kCfgLift: if constexpr (MIX == 0) return make_mfma<T, MIX, kCfgLift>(material); else return k;
    case kCfgTail: if constexpr (MIX == 0) return make_mfma<T, MIX, kCfgTail>(material); else return k;
    default: return k;
  }
}
}  // namespace

// precision: 0 FP64, 1 FP32, 2 BF16x3, 3 FP16x3, 4 BF16, 5 FP16, 6 BF16x2, 7 FP16x2
KernelSet DG_NAME(DG_ORDER, DG_GROUP)(int precision, int variant, bool material) {
#if DG_GROUP == 0
  if (precision == 0) return make<double, 0>(variant, material);
#elif DG_GROUP == 1
  if (precision == 1) return make<float, 0>(variant, material);
#else
  // Split 16-bit contraction (FP32 state), vacuum flux only; the tuning
  // configurations are built for the x3 forms, the others take the default.
  if (material) return KernelSet{};
  const bool tuned = precision == 2 || precision == 3 || variant <= kVariantMfma;
  if (!tuned) return KernelSet{};
  switch (precision) {
    case 2: return make<float, 3>(variant, false);
    case 3: return make<float, 6>(variant, false);
    case 4: return make<float, 1>(variant, false);
    case 5: return make<float, 4>(variant, false);
    case 6: return make<float, 2>(variant, false);
    case 7: return make<float, 5>(variant, false);
    default: break;
  }
#endif
  return KernelSet{};
}

}  // namespace dgd
