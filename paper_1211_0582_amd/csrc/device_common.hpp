// Device-side declarations shared by the kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace dgd {

// Per-element geometry record on the device: 25 scalars,
//   [0..8]   rx ry rz sx sy sz tx ty tz
//   [9+4f .. 12+4f] face f: nx ny nz Fscale
constexpr int kGeoStride = 25;

// Per-element material record (problems whose eps or mu differ from 1):
// 18 scalars,
//   [0] 1 / eps, [1] 1 / mu,
//   [2+4f .. 5+4f] face f: Fscale Z+ / ((Z- + Z+) eps), Fscale Y+ / ((Y- + Y+) mu),
//                  alpha / Z+, alpha Z+
// with Z = sqrt(mu / eps), Y = 1 / Z of the own (-) and neighbour (+)
// element (a boundary face's exterior has the own material).  With these the
// material flux is fE = s_E [ -n x dH + a_E (n (n.dE) - dE) ] and
// fH = s_H [ n x dE + a_H (n (n.dH) - dH) ], already divided by eps / mu; for
// eps = mu = 1 the record reproduces the vacuum flux exactly.
constexpr int kMatStride = 18;

// Exterior-state factors of a face from its connectivity word c: interior
// (c >= 0) reads the neighbour trace (1, 1); a boundary face (c = -1 - b)
// mirrors the own trace, E+ = s_E E-, H+ = s_H H-: conducting (-1, 1),
// magnetic-conducting (1, -1), absorbing (0, 0).
template <typename T>
__device__ __host__ inline void exterior_factors(int32_t c, T& sE, T& sH) {
  sE = c >= 0 ? T(1) : (c == -1 ? T(-1) : (c == -2 ? T(1) : T(0)));
  sH = c >= -1 ? T(1) : (c == -2 ? T(-1) : T(0));
}

// Arguments of one right-hand-side evaluation (or one fused Runge-Kutta stage).
struct RhsArgs {
  const void* u;          // state, [6][field_stride], element-major inside a field
  void* rhs;              // output, same layout (right-hand-side mode)
  const void* geo;        // K x kGeoStride
  const int32_t* conn;    // K x 4, nbr*32 + nbr_face*6 + orient, or -1 - bc on a boundary face
  const void* mat;        // K x kMatStride material records, or nullptr (eps = mu = 1)
  const void* ops;        // Dr^T, Ds^T, Dt^T (Np x Np each, [j][i]), LIFT^T (4Nfp x Np, [m][i])
  const void* ops_frag;   // [Dr|Ds|Dt|LIFT] as 16x4 MFMA A-fragments [row block][depth step][lane]
  const void* ops_frag16; // same operator split into 16-bit heads and tails, 16x16x32 A-fragments
  const uint8_t* nbr;     // 4 x 24 x Nfp neighbour volume node per (face, code, j)
  const int32_t* fmask;   // 4 x Nfp
  int64_t K;
  int64_t fs;             // field stride in scalars
  double alpha;
  // Runge-Kutta stage mode: res <- rk_a res + rk_dt rhs; u_out <- u + rk_b res.
  void* res;
  void* u_out;
  double rk_a, rk_b, rk_dt;
  int32_t stream_out;     // 1: outputs written with non-temporal (streaming) stores
  const int32_t* tile_order;  // tile processed by the i-th workgroup slot, or nullptr (tile i)
};

// One problem of a batch (device descriptor table entry).
struct BatchProblem {
  void* u;               // caller's state
  void* res;             // caller's residual
  void* u2;              // library-owned second state buffer
  const void* geo;
  const int32_t* conn;
  int64_t K, fs;
  double dt, alpha;
};

// One batched Runge-Kutta stage over the problems of one order N.
struct BatchArgs {
  const BatchProblem* probs;
  const int2* items;      // (problem, tile) pairs
  int64_t n_items;
  const void* ops_frag;   // operator fragments of order N (shared by the group)
  const void* ops_frag16;
  const uint8_t* nbr;
  const int32_t* fmask;
  int parity;
  double rk_a, rk_b;
  int32_t stream_out;     // 1: outputs written with non-temporal (streaming) stores
};
using BatchLauncher = hipError_t (*)(const BatchArgs&, hipStream_t);

// Arguments of one LSERK stage update: res <- a res + dt rhs; u <- u + b res
// (res not read when a = 0).
struct UpdateArgs {
  void* u;
  void* res;
  const void* rhs;
  int64_t n;              // K * Np scalars per field
  int64_t fs;
  int nfields;
  double a, b, dt;
};

using RhsLauncher = hipError_t (*)(const RhsArgs&, hipStream_t);

// Kernel variants of the right-hand side: the vector-ALU kernel, then the
// matrix-core kernel in each tuning configuration (kVariantMfma + kCfg*).
enum Variant { kVariantValu = 0, kVariantMfma = 1, kVariantCount = 8 };

struct KernelSet {
  RhsLauncher rhs = nullptr;  // writes rhs
  RhsLauncher rk = nullptr;   // fused Runge-Kutta stage (nullptr: rhs + update kernel)
  int tile = 0;               // elements per workgroup
  int frag_count = 0;         // scalars of the MFMA fragment array (0 if unused)
  int frag16_bytes = 0;       // bytes of the 16-bit split fragment array (0 if unused)
  BatchLauncher batch = nullptr;  // batched fused stage (matrix-core variant)
};

// Kernels for order N (1..9), precision (dg_precision), variant and flux
// form (material: per-element eps, mu); rhs == nullptr when the combination
// is not built.
KernelSet kernels(int N, int precision, int variant, bool material);

hipError_t launch_update(const UpdateArgs& a, int precision, hipStream_t s);

}  // namespace dgd
