// Tuned starting variants (the autotuner's table for gfx950, compiled into
// the library by the build): the kernel variant a new problem of precision
// p, order N and size bucket (large: K >= 20000 elements) starts with.
#pragma once

namespace dgd {

struct TunedVariant {
  int precision, N, large, variant;
};
extern const TunedVariant kTunedVariants[];
extern const int kTunedCount;

// Variant recorded for (precision, N, K), or -1.
inline int tuned_variant(int precision, int N, long long K) {
  const int large = K >= 20000 ? 1 : 0;
  for (int i = 0; i < kTunedCount; ++i)
    if (kTunedVariants[i].precision == precision && kTunedVariants[i].N == N && kTunedVariants[i].large == large)
      return kTunedVariants[i].variant;
  return -1;
}

}  // namespace dgd
