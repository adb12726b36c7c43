// Fused DG Maxwell right-hand side on the matrix cores (FP64 / FP32 MFMA,
// and split 16-bit contractions with FP32 accumulation).
//
// The operator of Section 2 is, per element, one dense contraction:
//   rhs[c][i] = sum_d sum_j D_d[i][j] X_d[c][j] + sum_m LIFT[i][m] F[c][m]
// with X_d = (m_d x H, E x m_d) the fields pre-combined with the element's
// constant metric row m_d = (d_x, d_y, d_z), d in {r, s, t} (so the volume
// sum is the curl term of Section 2.1), and F the Fscale-scaled upwind flux
// at the 4 Nfp face nodes.  A workgroup of two waves owns a tile of 16
// elements: wave 0 produces the E equations, wave 1 the H equations, each as
// MFMAs with rows = nodes i (Np padded to 16), columns = the 16 elements,
// depth = [Dr | Ds | Dt | LIFT] columns (each padded to 4).  At high order
// (enough 16-row blocks) each role is split over two waves by row blocks,
// four waves per tile.
//
//  * The operator is pre-swizzled on the host into MFMA A-fragments
//    (row block ib, depth step kg, lane) and streamed through L1/L2 (one
//    coalesced load feeds three MFMAs, one per output component).
//  * The tile's fields sit in LDS as [c][j][e] (16 elements fastest), read in
//    B-fragment layout; X_d is formed in registers.
//  * The flux is evaluated once per (element, face node) by all lanes:
//    the neighbour trace comes through the orientation table (a boundary
//    face reads the own node and mirrors it), and the fluxes are staged in LDS in
//    B-fragment order over the field tile for the LIFT MFMAs -- the facial
//    buffer of the paper's split pipeline never reaches HBM.
//  * Epilogue: accumulators go through LDS to coalesced 16-byte stores; in
//    the Runge-Kutta mode the stage update res <- a res + dt rhs,
//    u_out <- u + b res is applied there (u_out is a second state buffer, as
//    neighbours still read u during the stage).  FP64 launches past the
//    last-level cache store through streaming stores.
//  * The split 16-bit forms (split_wave) contract the fields themselves on
//    16x16x32 MFMAs and apply the metric after each direction's contraction;
//    fields and fluxes are split into heads and tails once per tile, in LDS,
//    and each wave produces all six components of one row block.
//  * Tiles are mapped to workgroups so that each of the 8 XCDs gets a
//    contiguous range of elements (neighbours then share that XCD's L2).
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "rhs_valu.hpp"

namespace dgd {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16];
// accumulator register r of lane l holds D[row(l / 16, r)][l % 16].  The row
// map differs by type (measured on gfx950 with one-hot operands): FP32 keeps
// four consecutive rows per lane group, FP64 interleaves them.
template <typename T>
struct Mfma16;
template <>
struct Mfma16<float> {
  using acc = f32x4;
  __device__ static inline acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int q, int r) { return 4 * q + r; }
  // 4-row form (16 blocks of 4x4, depth 1 each): block l / 4 takes A row i
  // from lane 4 (l / 4) + i and B column j from lane 4 (l / 4) + j, which in
  // the 16x16x4 B layout is depth l / 16 of element l % 16; lane l register
  // r receives row r, element l % 16, summed over depth l / 16 only (the four
  // lane groups are added at the end).  Measured on gfx950 with one-hot
  // operands; same flop rate as the 16x16x4 form.
  __device__ static inline acc mac4(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma16<double> {
  using acc = f64x4;
  __device__ static inline acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int q, int r) { return q + 4 * r; }
  // 4-row form (4 blocks of 4x4x4): block b = (l % 16) / 4 takes A[i][k] from
  // lane 16 k + 4 b + i and B[k][j] from lane 16 k + 4 b + j -- the 16x16x4 B
  // layout again -- and lane l receives row l / 16 of element l % 16 in one
  // scalar, kept in component 0.  Measured on gfx950 with one-hot operands;
  // same flop rate as the 16x16x4 form.
  __device__ static inline acc mac4(double a, double b, acc c) {
    c[0] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[0], 0, 0, 0);
    return c;
  }
};

// x / D for 0 <= x < XMAX as (x R) >> S with a 24-bit multiply: full rate on
// the vector ALU, where a 32-bit division by a constant takes a quarter-rate
// multiply-high and a 32-bit multiply-add a quarter-rate 64-bit one.  S is the
// smallest shift that is exact over the range, checked at compile time.
template <int D, int XMAX>
struct SmallDiv {
  static constexpr bool exact(int s) {
    const unsigned long long r = ((1ull << s) + D - 1) / D;
    if (r >= (1u << 24) || (unsigned long long)XMAX * r >= (1ull << 32)) return false;
    for (int x = 0; x < XMAX; ++x)
      if (int((unsigned long long)x * r >> s) != x / D) return false;
    return true;
  }
  static constexpr int shift() {
    for (int s = 8; s <= 24; ++s)
      if (exact(s)) return s;
    return -1;
  }
  static constexpr int S = shift();
  static_assert(S > 0, "no exact 24-bit reciprocal for this range");
  static constexpr unsigned R = unsigned(((1ull << S) + D - 1) / D);
  __device__ static inline int div(int x) { return int(unsigned(__umul24(unsigned(x), R)) >> S); }
};

// 24-bit product (both factors below 2^24): one full-rate instruction.
__device__ inline int mul24(int a, int b) { return __umul24(unsigned(a), unsigned(b)); }

template <int N>
struct MfmaShape {
  static constexpr int Np = Order<N>::Np, Nfp = Order<N>::Nfp, NF = Order<N>::NF;
  static constexpr int Np4 = (Np + 3) & ~3;   // volume depth per direction, padded
  static constexpr int RB = (Np + 15) / 16;   // 16-row blocks
  static constexpr int KSV = Np4 / 4;         // depth steps per direction
  static constexpr int KSL = NF / 4;          // depth steps of LIFT (4 Nfp is a multiple of 4)
  static constexpr int KS = 3 * KSV + KSL;
  // LDS row strides: 16 elements + 1, so that the tile store and the flux
  // store, which walk consecutive rows of one element, spread over the banks.
  static constexpr int TS = 17, TQ = 17;
  static constexpr int frag_count = RB * KS * 64;
  // The LDS tile holds the fields [c][Np4][TS] first, then the fluxes
  // [c][NF][TQ], then the output staging [c][16][Np] and 4 discard slots per
  // lane.
  static constexpr int FIELDS = 6 * Np4 * TS, FLUXES = 6 * NF * TQ, STAGE = 6 * 16 * Np + 256;
  static constexpr int TILE = FIELDS > FLUXES ? (FIELDS > STAGE ? FIELDS : STAGE) : (FLUXES > STAGE ? FLUXES : STAGE);
  // Split lift: the fluxes go to LDS and are lifted in two halves of face
  // nodes, m < HB and m >= HB, through a region of 6 x HB rows.  The flux
  // phase covers 8 face-node rows per 128-lane iteration, so HB is a whole
  // number of iterations (and of 4-row depth steps).
  static constexpr int FLUX_ITERS = (16 * NF + 127) / 128;
  static constexpr int HALF_ITERS = (FLUX_ITERS + 1) / 2;
  static constexpr int HB = 8 * HALF_ITERS;
  static constexpr int tile(bool half) {
    const int f = half ? 6 * HB * TQ : FLUXES;
    return FIELDS > f ? (FIELDS > STAGE ? FIELDS : STAGE) : (f > STAGE ? f : STAGE);
  }
};

// LDS rows of the split forms: one row per (component, element) holding the
// row's values in 8-value records (a row of 8 J8 values, then a 16-byte pad
// so that the 16 elements of a lane group hit distinct banks).  A record is
// written in FP32 and then replaced, in place or in a second region, by its
// 8 heads (16 bytes) and 8 tails (16 bytes): one record is one B operand.
template <int N>
struct SplitShape {
  using S = MfmaShape<N>;
  static constexpr int KV = (S::Np + 31) / 32;  // volume depth steps per direction
  static constexpr int KL = (S::NF + 31) / 32;  // lift depth steps
  static constexpr int ST = 3 * KV + KL;        // operator steps (direction-major, then lift)
  static constexpr int J8 = (S::Np + 7) / 8;    // records per field row
  static constexpr int J8F = (S::NF + 7) / 8;   // records per flux row
  static constexpr int RSV = 8 * J8 + 4, RSF = 8 * J8F + 4;  // row strides (floats)
  // The flux reads its own traces from the FP32 field rows, which are kept
  // beside the split records where both fit in 80 KB (N <= 6); beyond that the
  // records replace them in place and the own traces come from global memory
  // with the neighbour traces.
  static constexpr bool INPLACE = 2 * 96 * RSV * 4 > 80 * 1024;
  static constexpr int SPLIT = INPLACE ? 0 : 96 * RSV;  // offset of the split field records
  static constexpr int max3(int a, int b, int c) { return a > b ? (a > c ? a : c) : (b > c ? b : c); }
  static constexpr int TILE = max3(SPLIT + 96 * RSV, 96 * RSF, S::STAGE);
  // operator fragments: [row block][step][head, tail][lane] x 16 bytes
  static constexpr int frag_bytes = S::RB * ST * 2 * 64 * 16;
};

// Tuning configurations of the matrix-core kernels: the autotuner's search
// space (the paper tunes its work decomposition by timing generated
// variants, Section 4).  kCfgDefault takes the heuristics below; every other
// configuration changes exactly one of them: the waves per tile, the
// operator-fragment prefetch depth, the occupancy the register allocation
// must allow, the flux interleave, the split lift, the 4-row tail block.
enum : int {
  kCfgDefault = 0,
  kCfgWaves = 1,
  kCfgPrefetch = 2,
  kCfgOccupancy = 3,
  kCfgInterleave = 4,
  kCfgLift = 5,
  kCfgTail = 6,
  kCfgCount = 7
};

// Waves per tile: 2 (wave 0 the E equations, wave 1 the H equations, all row
// blocks each) or 4 (the same two roles, each split over two waves by row
// blocks; with an odd number of blocks the first wave of a role takes one
// more).  Four halves the accumulators and operator-fragment traffic per
// wave, which at high order is what bounds the waves per SIMD, at the price
// of forming the volume operand twice (N = 7, FP32: 1 -> 2 waves per SIMD,
// 42% -> 55% of peak).  kCfgWaves takes the other choice (four waves need at
// least two row blocks).
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr int waves_per_tile() {
  constexpr int RB = MfmaShape<N>::RB;
  // The split forms' waves each produce all six components of their row
  // blocks (split_wave): one wave per block (up to 14 at N = 9), or with
  // kCfgWaves two blocks per wave.
  if constexpr (MIX != 0) return CFG == kCfgWaves && RB >= 2 ? (RB + 1) / 2 : RB;
  // Four waves from RB = 4 (N = 5) for FP64 / FP32 (measured on MI355X).
  constexpr int d = RB >= 4 ? 4 : 2;
  if constexpr (CFG == kCfgWaves) return d == 4 ? 2 : (RB >= 2 ? 4 : 2);
  return d;
}

// Row blocks of the first wave of a role (all of them with two waves per
// tile, the larger half with four) and of the second.
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr int row_blocks_first() {
  constexpr int RB = MfmaShape<N>::RB;
  constexpr int W = waves_per_tile<N, T, MIX, CFG>();
  if constexpr (MIX != 0) return (RB + W - 1) / W;
  return W == 2 ? RB : (RB + 1) / 2;
}
// (split forms: the waves past the first RB mod W take one block less)
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr int row_blocks_second() {
  constexpr int W = waves_per_tile<N, T, MIX, CFG>();
  if constexpr (MIX != 0) return MfmaShape<N>::RB / W;
  return W == 2 ? MfmaShape<N>::RB : MfmaShape<N>::RB - row_blocks_first<N, T, MIX, CFG>();
}

// Whether the last 16-row block, which holds at most 4 nodes (N = 1, 3, 4,
// 6), runs on the 4-row MFMA form: a quarter of a full block's matrix-core
// time.  With two waves per tile the block belongs to both role waves; with
// four, to the wave of each role that owns the upper row blocks, which then
// runs its own copy of the wave code -- in FP32 at N = 6 that copy would cost
// a wave per SIMD (168 -> 184 registers), so there only FP64 uses it.
// kCfgTail takes the other choice where the last block qualifies.
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr bool mfma_tail() {
  using S = MfmaShape<N>;
  constexpr bool fits = MIX == 0 && S::Np - 16 * (S::RB - 1) <= 4;
  constexpr bool d = fits && (waves_per_tile<N, T, MIX, CFG>() == 2 || sizeof(T) == 8);
  return CFG == kCfgTail ? (fits && !d) : d;
}

template <int N, typename T, int MIX = 0>
constexpr size_t mfma_lds_bytes() {
  return MIX ? size_t(SplitShape<N>::TILE) * 4 : size_t(MfmaShape<N>::TILE) * sizeof(T);
}

// Whether the MFMA variant is built for (N, T): the LDS tile and the
// accumulators must fit -- row blocks per wave x 3 x 4 scalars per lane (the
// split forms: x 6, plus one block's per-direction partial products), at
// most 144 registers.
template <int N, typename T, int MIX = 0, int CFG = kCfgDefault>
constexpr bool mfma_supported() {
  constexpr int RBW = row_blocks_first<N, T, MIX, CFG>();
  constexpr int acc = MIX ? RBW * 6 * 4 + 24 : RBW * 3 * 4 * int(sizeof(T)) / 4;
  return mfma_lds_bytes<N, T, MIX>() <= 160 * 1024 && acc <= 144;
}

// Raw buffer loads: a 128-bit resource (base, size) in SGPRs plus a 32-bit
// byte offset per lane and a wave-uniform byte offset, so gathers and operator
// fragments need no 64-bit address arithmetic on the vector ALU.  Offsets at
// or beyond the resource size read as zero instead of faulting.
__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ inline T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <>
__device__ inline float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ inline double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

// State shared by the waves of a workgroup.
template <int N, typename T, bool HALF = false, bool MAT = false, bool SPLIT = false>
struct MfmaTile {
  using S = MfmaShape<N>;
  static constexpr bool kHalf = HALF;
  // fields [c][j][e], then fluxes [c][m][e], then output [c][e][i]; the split
  // forms hold rows [c][e] of records (SplitShape) in place of the first two
  alignas(16) T su[SPLIT ? SplitShape<N>::TILE : S::tile(HALF)];
  // geometry records of the tile's elements (kGeoStride values each)
  alignas(16) T geo[(16 * kGeoStride * sizeof(T) + 15) / 16 * 16 / sizeof(T)];
  int16_t fmask[S::NF];
  alignas(16) uint8_t nbr[(4 * 24 * S::Nfp + 15) / 16 * 16];
  int32_t code[16 * 4];               // face codes of the tile's elements
  // per (element, face): s_E, s_H, a_E, a_H of the material record
  T face[MAT ? 16 * 4 * 4 : 1];
};

// Where the flux work of a tile runs relative to the contraction.  Flux
// (gathers, jumps, upwind formula) is vector-ALU and memory work; the volume
// loop keeps the matrix cores busy.  With IL the gathers are issued early in
// the volume loop (behind a few steps of operator fragments already in
// flight, since loads complete in issue order) and the flux iterations are
// spread over the later volume steps, so the vector ALU works while the
// matrix core does; without IL the flux phase runs between volume and lift.
template <int NV, int NFI, int PRE>
struct FluxSchedule {
  static constexpr int first = PRE + 1;  // first step whose frag wait follows the gathers
  // volume step after which flux iteration fi runs (NV: after the loop)
  __device__ static constexpr int at(int fi) {
    return first >= NV ? NV : first + (fi * (NV - first)) / NFI;
  }
};

// Contraction of one wave.  H = 0 produces the E equations (curl H + LIFT fE),
// H = 1 the H equations (-curl E + LIFT fH).  With V = H, (P, Q) = (dE, dH)
// for H = 0 and V = -E, (P, Q) = (dH, -dE) for H = 1, the volume operand is
// X_d = m_d x V and the flux f = 1/2 Fscale [ -n x Q + alpha (n (n.P) - P) ].
// Flux work comes in three parts: gather() issues the neighbour loads,
// flux_step(fi) evaluates flux iteration fi into registers, flux_store()
// waits for the tile's readers and writes the fluxes over the field tile.
// The wave produces row blocks rb0 .. rb0 + RBW - 1 of its three components
// (all RB blocks with two waves per tile, half of them with four).
template <int N, typename T, int H, bool IL, int NFI, int RBW, bool TW, bool PALT, typename Tile, typename Gather,
          typename FluxStep, typename FluxStore>
__device__ __attribute__((always_inline)) inline void mfma_wave(const RhsArgs& a, Tile& t, const T (&mr)[9], int lane, int rb0,
                                 typename Mfma16<T>::acc (&acc)[RBW][3], Gather&& gather,
                                 FluxStep&& flux_step, FluxStore&& flux_store) {
  using S = MfmaShape<N>;
  using M = Mfma16<T>;
  using acc_t = typename M::acc;
  constexpr int Np4 = S::Np4, NF = S::NF, RB = RBW, KSV = S::KSV, KSL = S::KSL;
  constexpr int KS = S::KS, TS = S::TS, TQ = S::TQ;
  constexpr uint32_t sz = sizeof(T);
  const int e = lane & 15, q = lane >> 4;
  // The fragment array holds the RB row blocks, then the last block again in
  // the 4-row layout (lane l: row 16 (RB - 1) + l % 4, depth l / 16).
  constexpr bool TAIL = TW;  // this wave's last row block is the 4-row one
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(a.ops_frag, uint32_t((S::RB + 1) * KS * 64) * sz);
  auto mac = [&](int ib, T av, T bv, acc_t c) -> acc_t {
    if constexpr (TAIL) {
      if (ib == RB - 1) return M::mac4(av, bv, c);
    }
    return M::mac(av, bv, c);
  };

#pragma unroll
  for (int ib = 0; ib < RB; ++ib)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[ib][c] = acc_t{0, 0, 0, 0};

  // Software pipeline: global loads are issued kPre depth steps before use
  // (one step when the accumulators already take most of the registers;
  // more when the gathers sit in the load queue behind them).  PALT takes
  // the alternative depth (1 <-> 2, 4 -> 2).
  constexpr int kPreD = IL ? (RB >= 4 ? 2 : 4) : (RB >= 6 ? 1 : 2);
  constexpr int kPre = PALT ? (kPreD == 2 ? 1 : 2) : kPreD;
  constexpr int NV = 3 * KSV;  // volume depth steps, ordered (ks, d)
  using FS = FluxSchedule<NV, NFI, kPre>;
  const uint32_t lane_off = uint32_t(lane + rb0 * KS * 64) * sz;
  auto frag_of = [&](int step, int ib) -> T {
    const int kg = step < NV ? (step % 3) * KSV + step / 3 : 3 * KSV + (step - NV);
    // lane_off already points at block rb0 = S::RB - RB for a tail wave, so
    // the 4-row block (absolute index S::RB) is block RB from there.
    const int blk = (TAIL && ib == RB - 1) ? RB : ib;
    return buf_load<T>(rf, lane_off, uint32_t((blk * KS + kg) * 64) * sz);
  };
  T Abuf[kPre + 1][RB];
#pragma unroll
  for (int s = 0; s < kPre; ++s)
#pragma unroll
    for (int ib = 0; ib < RB; ++ib) Abuf[s][ib] = frag_of(s, ib);

  // Volume: X_d = m_d x V at node j = 4 ks + q of element e.
  constexpr int vb = H ? 0 : 3;
  const T vs = H ? T(-1) : T(1);
#pragma unroll
  for (int ks = 0; ks < KSV; ++ks) {
    const int j = 4 * ks + q;
    T v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = vs * t.su[((vb + c) * Np4 + j) * TS + e];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int step = 3 * ks + d;
      if (step + kPre < KS) {
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) Abuf[(step + kPre) % (kPre + 1)][ib] = frag_of(step + kPre, ib);
      }
      if constexpr (IL) {
        if (step == 0) gather();
      }
      const T mx = mr[3 * d], my = mr[3 * d + 1], mz = mr[3 * d + 2];
      T X[3];
      X[0] = my * v[2] - mz * v[1];
      X[1] = mz * v[0] - mx * v[2];
      X[2] = mx * v[1] - my * v[0];
#pragma unroll
      for (int ib = 0; ib < RB; ++ib)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[ib][c] = mac(ib, Abuf[step % (kPre + 1)][ib], X[c], acc[ib][c]);
      if constexpr (IL) {
#pragma unroll
        for (int fi = 0; fi < NFI; ++fi)
          if (FS::at(fi) == step) flux_step(fi);
      }
    }
  }
  if constexpr (IL) {
#pragma unroll
    for (int fi = 0; fi < NFI; ++fi)
      if (FS::at(fi) >= NV) flux_step(fi);
  } else {
    gather();
#pragma unroll
    for (int fi = 0; fi < NFI; ++fi) flux_step(fi);
  }

  // Lifting: F (already scaled by Fscale / 2) comes from the LDS flux tile,
  // in one pass or, with the split lift, in two halves of face-node rows.
  constexpr int cb = H ? 3 : 0;
  constexpr bool HALF = Tile::kHalf;
  constexpr int FR = HALF ? S::HB : NF;  // rows per component in the flux region
  auto lift = [&](int ks0, int ks1, int base) {
#pragma unroll
    for (int ks = ks0; ks < ks1; ++ks) {
      const int step = NV + ks;
      if (step + kPre < KS) {
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) Abuf[(step + kPre) % (kPre + 1)][ib] = frag_of(step + kPre, ib);
      }
      const int m = 4 * ks + q - base;
      T F[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] = t.su[((cb + c) * FR + m) * TQ + e];
#pragma unroll
      for (int ib = 0; ib < RB; ++ib)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[ib][c] = mac(ib, Abuf[step % (kPre + 1)][ib], F[c], acc[ib][c]);
    }
  };
  if constexpr (!HALF) {
    flux_store(-1);
    __syncthreads();
    lift(0, KSL, 0);
  } else {
    flux_store(0);
    __syncthreads();
    lift(0, S::HB / 4, 0);
    __syncthreads();  // first half read before the second overwrites it
    flux_store(1);
    __syncthreads();
    lift(S::HB / 4, KSL, S::HB);
  }
  // FP32 4-row block: add the partial sums of the four depth lane groups.
  if constexpr (TAIL && sizeof(T) == 4) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        T v = acc[RB - 1][c][r];
        v += __shfl_xor(v, 16);
        v += __shfl_xor(v, 32);
        acc[RB - 1][c][r] = v;
      }
  }
}

// ---------------------------------------------------------------------------
// Split-precision contraction on 16-bit matrix cores.
//
// Same operator as mfma_wave, on 16x16x32 MFMAs in BF16 or FP16 with FP32
// accumulation.  Both operands are split into a 16-bit head and a 16-bit
// tail, a = a_hi + a_lo with a_hi = round(a), a_lo = round(a - a_hi): the
// operator once on the host, the fields and the fluxes once per tile in LDS.
// NPROD selects the products accumulated: 1: a_hi b_hi, 2: + a_lo b_hi,
// 3: + a_hi b_lo (the a_lo b_lo term is below FP32 rounding).
//
// The metric is applied after the contraction: per direction d the wave
// forms Y = D_d V for the three components of its source field V (H for the
// E equations, -E for the H equations) and folds m_d x Y into its output, so
// the operand of the volume MFMAs is the field itself -- split once per tile
// and shared by both roles -- instead of m_d x V split again per direction and
// role.  Depth: 32 nodes of one direction per step (each direction padded to
// a multiple of 32), then the lift's face nodes, padded to 32.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

// 16x16x32 MFMA: lane l supplies A[l % 16][8 (l / 16) + v] and
// B[8 (l / 16) + v][l % 16], v = 0..7; accumulator register r of lane l holds
// D[4 (l / 16) + r][l % 16] (checked on gfx950 against a host product).
template <typename H16>
struct Mfma32;
template <>
struct Mfma32<__bf16> {
  using v8 = bf16x8;
  __device__ static inline f32x4 mac(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma32<_Float16> {
  using v8 = f16x8;
  __device__ static inline f32x4 mac(v8 a, v8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <typename H16>
__device__ inline void split8(const float (&x)[8], typename Mfma32<H16>::v8& hi, typename Mfma32<H16>::v8& lo) {
  // Pairs: one packed conversion per head pair, widened back from the packed
  // value (elementwise, the compiler converts each head twice: once alone
  // for the tail, once packed for the store).
  typedef H16 h2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
#pragma unroll
  for (int v = 0; v < 8; v += 2) {
    const f2 xv = {x[v], x[v + 1]};
    const h2 h = __builtin_convertvector(xv, h2);
    const f2 b = __builtin_convertvector(h, f2);
    const h2 l = __builtin_convertvector(f2{xv[0] - b[0], xv[1] - b[1]}, h2);
    hi[v] = h[0];
    hi[v + 1] = h[1];
    lo[v] = l[0];
    lo[v + 1] = l[1];
  }
}

// Splits the FP32 records of ROWS rows of stride RS (J records each) at src
// into head/tail records at dst (dst == src: in place); run by NT lanes.
template <typename H16, int ROWS, int J, int RS, int NT>
__device__ __attribute__((always_inline)) inline void split_records(const float* src, float* dst, int tid) {
  using v8 = typename Mfma32<H16>::v8;
  constexpr int n = ROWS * J;
#pragma unroll
  for (int it = 0; it < (n + NT - 1) / NT; ++it) {
    const int r = tid + NT * it;
    if (r < n) {
      const int row = SmallDiv<J, NT * ((n + NT - 1) / NT)>::div(r), j8 = r - mul24(row, J);
      const int o = mul24(row, RS) + 8 * j8;
      const f32x4 a = *reinterpret_cast<const f32x4*>(src + o);
      const f32x4 b = *reinterpret_cast<const f32x4*>(src + o + 4);
      const float x[8] = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
      v8 hi, lo;
      split8<H16>(x, hi, lo);
      *reinterpret_cast<v8*>(dst + o) = hi;
      *reinterpret_cast<v8*>(dst + o + 4) = lo;
    }
  }
}

// Contraction of one wave of a split form: the wave produces all six
// components of row blocks rb0 .. rb0 + RBW - 1, one block at a time, so
// each operator fragment it loads feeds both equations (E: curl H + LIFT fE,
// H: -curl E + LIFT fH).  Per block and direction d, Y = D_d [H; E] (six
// partial products), folded as out_E += m_d x Y_H and out_H -= m_d x Y_E.
template <int N, typename H16, int NPROD, int NFI, int RBW, bool PALT, typename Tile, typename Gather,
          typename FluxStep, typename FluxPut, typename FluxStore>
__device__ __attribute__((always_inline)) inline void split_wave(const RhsArgs& a, Tile& t, const float (&mr)[9],
                                                                 int lane, int rb0, f32x4 (&out)[RBW][6],
                                                                 Gather&& gather, FluxStep&& flux_step,
                                                                 FluxPut&& flux_put, FluxStore&& flux_store) {
  using X = SplitShape<N>;
  using MM = Mfma32<H16>;
  using v8 = typename MM::v8;
  constexpr int KV = X::KV, KL = X::KL, ST = X::ST, J8 = X::J8, J8F = X::J8F, RSV = X::RSV, RSF = X::RSF;
  constexpr int NVS = RBW * 3 * KV;         // volume steps of this wave (block, direction, depth)
  constexpr int NS = NVS + RBW * KL;        // then the lift steps (block, depth)
  const int e = lane & 15, q = lane >> 4;
  const __amdgpu_buffer_rsrc_t rf = make_rsrc(a.ops_frag16, uint32_t(X::frag_bytes));

  // Operator fragments (head, tail) of step s, prefetched kPre steps ahead
  // (two; PALT: one).  The lift's first fragments are issued once the fluxes
  // are in registers and the gathered traces are dead, so that none is held
  // through the flux phase.
  constexpr int kPre = PALT ? 1 : 2;
  v8 Ahi[kPre + 1], Alo[kPre + 1];
  auto fetch = [&](int s) {
    if (s < NS) {
      const int ib = rb0 + (s < NVS ? s / (3 * KV) : (s - NVS) / KL);
      const int st = s < NVS ? s % (3 * KV) : 3 * KV + (s - NVS) % KL;
      const uint32_t off = uint32_t(((ib * ST + st) * 2 * 64 + lane) * 16);
      Ahi[s % (kPre + 1)] = __builtin_bit_cast(v8, __builtin_amdgcn_raw_buffer_load_b128(rf, (int)off, 0, 0));
      if constexpr (NPROD >= 2)
        Alo[s % (kPre + 1)] =
            __builtin_bit_cast(v8, __builtin_amdgcn_raw_buffer_load_b128(rf, (int)off, 64 * 16, 0));
    }
  };
#pragma unroll
  for (int s = 0; s < kPre; ++s) fetch(s);

  // B operands of one step for component c: the record of this lane's
  // element and depth group (records past the row's end are clamped: the
  // operator columns there are zero, and the clamped record is finite).
  auto b_of = [&](const float* row0, int rs, int rec, int c, v8& bh, v8& bl) {
    const float* p = row0 + (c * 16 + e) * rs + 8 * rec;
    bh = *reinterpret_cast<const v8*>(p);
    if constexpr (NPROD >= 3) bl = *reinterpret_cast<const v8*>(p + 4);
  };
  auto mac = [&](int slot, const v8& bh, const v8& bl, f32x4 c0) {
    f32x4 y = MM::mac(Ahi[slot], bh, c0);
    if constexpr (NPROD >= 2) y = MM::mac(Alo[slot], bh, y);
    if constexpr (NPROD >= 3) y = MM::mac(Ahi[slot], bl, y);
    return y;
  };

  // Volume: Y[c] = D_d of field (c + 3) mod 6, i.e. Y[0..2] from H, Y[3..5]
  // from E.
  const float* fv = t.su + X::SPLIT;
  f32x4 Y[6];
#pragma unroll
  for (int s = 0; s < NVS; ++s) {
    if (s + kPre < NVS) fetch(s + kPre);
    const int ib = s / (3 * KV), d = (s / KV) % 3, ks = s % KV;
    const int rec = 4 * ks + q < J8 ? 4 * ks + q : J8 - 1;
    // Each direction reads its operands afresh: shared with the other
    // directions they would keep all three directions' Y live at once.
    if (ks == 0 && s > 0) asm volatile("" ::: "memory");
    const int slot = s % (kPre + 1);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      v8 bh, bl;
      b_of(fv, RSV, rec, c < 3 ? c + 3 : c - 3, bh, bl);
      Y[c] = mac(slot, bh, bl, ks == 0 ? f32x4{0, 0, 0, 0} : Y[c]);
    }
    if (ks == KV - 1) {
      const float mx = mr[3 * d], my = mr[3 * d + 1], mz = mr[3 * d + 2];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
          const float sg = hh ? -1.f : 1.f;
          const f32x4* y = Y + 3 * hh;
          const float c0 = sg * (my * y[2][r] - mz * y[1][r]);
          const float c1 = sg * (mz * y[0][r] - mx * y[2][r]);
          const float c2 = sg * (mx * y[1][r] - my * y[0][r]);
          out[ib][3 * hh + 0][r] = d == 0 ? c0 : out[ib][3 * hh + 0][r] + c0;
          out[ib][3 * hh + 1][r] = d == 0 ? c1 : out[ib][3 * hh + 1][r] + c1;
          out[ib][3 * hh + 2][r] = d == 0 ? c2 : out[ib][3 * hh + 2][r] + c2;
        }
      }
      // The fold completes here, before the next direction's operands are
      // read, so that only one direction's partial products are live.
#pragma unroll
      for (int c = 0; c < 6; ++c) asm volatile("" : "+v"(out[ib][c]));
    }
  }
  if constexpr (X::INPLACE) {
    // The field records are the tile's only copy of the fields, and the
    // flux rows replace them: once every wave is done with them, the fluxes
    // go to LDS as they are computed, FCH iterations at a time, the traces of
    // the next FCH in flight meanwhile.
    constexpr int FCH = 2;
    gather(0, FCH);
    __syncthreads();
#pragma unroll
    for (int c0 = 0; c0 < NFI; c0 += FCH) {
      if (c0 + FCH < NFI) gather(c0 + FCH, c0 + 2 * FCH);
#pragma unroll
      for (int fi = c0; fi < c0 + FCH && fi < NFI; ++fi) {
        flux_step(fi);
        flux_put(fi);
      }
    }
#pragma unroll
    for (int s = NVS; s < NVS + kPre; ++s) fetch(s);
    flux_store(-2);
  } else {
    gather();
#pragma unroll
    for (int fi = 0; fi < NFI; ++fi) flux_step(fi);
#pragma unroll
    for (int s = NVS; s < NVS + kPre; ++s) fetch(s);
    flux_store(-1);
  }

  // Lifting: the fluxes' head/tail records written by the workgroup.
  __syncthreads();
#pragma unroll
  for (int s = NVS; s < NS; ++s) {
    fetch(s + kPre);
    const int ib = (s - NVS) / KL, ls = (s - NVS) % KL;
    const int rec = 4 * ls + q < J8F ? 4 * ls + q : J8F - 1;
    const int slot = s % (kPre + 1);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      v8 bh, bl;
      b_of(t.su, RSF, rec, c, bh, bl);
      out[ib][c] = mac(slot, bh, bl, out[ib][c]);
    }
  }
}

// Whether a tile's flux work is interleaved with its volume contraction (see
// FluxSchedule): the neighbour traces, then the fluxes computed from them
// (6 scalars per flux iteration), stay in registers through the volume loop.
// Measured on MI355X it pays in FP64 (7% at N = 3, the order where the
// registers allow it); in FP32 it costs a wave per SIMD and gains nothing
// (the FP32 matrix and vector pipes never co-issue: SQ_VALU_MFMA_COEXEC_CYCLES
// reads 0).  The split forms do not interleave: their fluxes go through LDS
// rows that replace the field tile.
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr bool flux_interleaved() {
  constexpr int iters = (16 * MfmaShape<N>::NF + 127) / 128;
  constexpr bool d = MIX == 0 && sizeof(T) == 8 && iters * 6 * sizeof(T) / 4 <= 72;
  return CFG == kCfgInterleave ? (MIX == 0 && !d) : d;
}

// Whether the lift runs in two halves (see MfmaShape::tile): it trades two
// barriers for a smaller flux region.  Used where the flux region sets the
// LDS size and the registers allow one more workgroup per CU once it
// shrinks: FP64 at N = 4 (3 -> 4 workgroups per CU).
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr bool lift_split() {
  constexpr bool d = MIX == 0 && sizeof(T) == 8 && N == 4;
  return CFG == kCfgLift ? (MIX == 0 && !d) : d;
}

// Workgroup = the waves sharing one tile of 16 elements: for FP64 / FP32 two
// or four, wave role h = 0 producing the E equations, h = 1 the H equations
// (see mfma_wave); for the split forms one per row block (see split_wave).
// MIX = 0: contraction in T on 16x16x4 MFMAs; MIX = 1..3: T = float with the
// contraction split in BF16 (NPROD = MIX) on 16x16x32 MFMAs (split_wave);
// MIX = 4..6: split in FP16 (NPROD = MIX - 3).
//
// MAT: per-element eps and mu (material record, see kMatStride): the metric
// of the volume operand is scaled by 1 / eps (E role) or 1 / mu (H role), and
// the flux takes the record's per-face scales and upwind weights.
//
// CFG: tuning configuration (kCfg*).
template <int N, typename T, bool RK, int MIX, bool MAT = false, int CFG = kCfgDefault>
__device__ __attribute__((always_inline)) inline void rhs_mfma_tile(const RhsArgs& a, int64_t tile) {
  using S = MfmaShape<N>;
  using M = Mfma16<T>;
  using acc_t = typename M::acc;
  constexpr int Np = S::Np, Nfp = S::Nfp, NF = S::NF, Np4 = S::Np4, RB = S::RB, TS = S::TS, TQ = S::TQ;
  constexpr bool LIFT_HALF = lift_split<N, T, MIX, CFG>();
  constexpr int WPT = waves_per_tile<N, T, MIX, CFG>();
  constexpr bool PALT = CFG == kCfgPrefetch;
  constexpr int NT = 64 * WPT;        // lanes per tile
  constexpr int RBW = row_blocks_first<N, T, MIX, CFG>();    // row blocks of a role's first wave
  constexpr int RBW1 = row_blocks_second<N, T, MIX, CFG>();  // and of its second (four waves per tile)
  // Split forms: the 16-bit type, the products, the LDS rows (SplitShape).
  constexpr bool SPL = MIX != 0;
  using H16 = typename std::conditional<(MIX <= 3), __bf16, _Float16>::type;
  constexpr int NPROD = MIX <= 3 ? MIX : MIX - 3;
  using X = SplitShape<N>;
  constexpr bool OWNG = SPL && X::INPLACE;  // own traces of the flux from global memory
  __shared__ MfmaTile<N, T, LIFT_HALF, MAT, SPL> t;

  const int64_t fs = a.fs;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int h = (tid >> 6) & 1;       // 0: E equations, 1: H equations
  const int rh = tid >> 7;            // row-block half (four waves per tile)
  // Split forms: wave w owns all six components of its row blocks, the
  // first RB mod W waves one block more than the others.
  constexpr int SRM = S::RB % WPT;
  const int sw = tid >> 6;
  const int rb0 = SPL ? (sw < SRM || SRM == 0 ? sw * RBW : SRM * RBW + (sw - SRM) * RBW1) : rh * RBW;
  const int e = lane & 15, q = lane >> 4;
  const int64_t k0 = tile * 16;
  const int ne = int((a.K - k0) < 16 ? (a.K - k0) : 16);
  const bool live = e < ne;
  const int64_t ke = k0 + (live ? e : 0);

  // All loads of the prologue are unconditional raw buffer loads: lanes past
  // the end of a ragged tile use an out-of-range offset and read zero, so no
  // load sits behind a branch and all of them are in flight together.
  constexpr uint32_t sz = sizeof(T);
  constexpr uint32_t kOob = 0x80000000u;
  const __amdgpu_buffer_rsrc_t rg = make_rsrc(a.geo, uint32_t(a.K) * kGeoStride * sz);
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.conn, uint32_t(a.K) * 4 * 4);
  const __amdgpu_buffer_rsrc_t ru = make_rsrc(a.u, 6u * uint32_t(fs) * sz);

  // Every global load of the prologue is issued before the first LDS write:
  // a write needs its data, and a load issued after such a wait (or in a
  // later branch) would add a full memory round trip to the prologue.
  // Geometry records of the tile (metric, then per face the normal and
  // Fscale): one contiguous block, loaded with 16-byte loads into LDS (past
  // the last element they read zero).
  constexpr int kGeoVec = (16 * kGeoStride * int(sz) + 15) / 16;
  constexpr int kGeoIters = (kGeoVec + NT - 1) / NT;
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  u32x4 gv[kGeoIters];
#pragma unroll
  for (int it = 0; it < kGeoIters; ++it) {
    const int i = tid + NT * it;
    const uint32_t go = i < kGeoVec ? uint32_t(k0 * kGeoStride) * sz + 16u * uint32_t(i) : kOob;
    gv[it] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rg, (int)go, 0, 0));
  }
  // Material: the role's 1 / eps or 1 / mu, and the face scales and weights.
  T mscale = T(1);
  T fmr[4] = {T(0), T(0), T(0), T(0)};
  const __amdgpu_buffer_rsrc_t rmat = make_rsrc(a.mat, MAT ? uint32_t(a.K) * kMatStride * sz : 0u);
  if constexpr (MAT) mscale = buf_load<T>(rmat, live ? uint32_t(ke * kMatStride + h) * sz : kOob, 0);
  // Connectivity codes and material face records (lanes 0..63: 16 elements
  // x 4 faces).
  int32_t cf;
  {
    const int ee = (tid >> 2) & 15, f = tid & 3;
    const bool lv = tid < 64 && ee < ne;
    cf = __builtin_bit_cast(int32_t, __builtin_amdgcn_raw_buffer_load_b32(
                                         rc, lv ? uint32_t((k0 + ee) * 4 + f) * 4 : kOob, 0, 0));
    cf = lv ? cf : -1;
    if constexpr (MAT) {
      const uint32_t mo = lv ? uint32_t((k0 + ee) * kMatStride + 2 + 4 * f) * sz : kOob;
#pragma unroll
      for (int i = 0; i < 4; ++i) fmr[i] = buf_load<T>(rmat, mo, i * sz);
    }
  }
  // Tables (indices clamped so the loads need no branch); 16-byte loads for
  // the orientation table (its device copy is padded to a multiple of 16 B).
  constexpr int kFmaskIters = (NF + NT - 1) / NT;
  int32_t fmv[kFmaskIters];
#pragma unroll
  for (int it = 0; it < kFmaskIters; ++it) {
    const int i = tid + NT * it;
    fmv[it] = a.fmask[i < NF ? i : NF - 1];
  }
  constexpr int kNbrVec = (4 * 24 * Nfp + 15) / 16;
  constexpr int kNbrIters = (kNbrVec + NT - 1) / NT;
  uint4 nbv[kNbrIters];
#pragma unroll
  for (int it = 0; it < kNbrIters; ++it) {
    const int i = tid + NT * it;
    nbv[it] = reinterpret_cast<const uint4*>(a.nbr)[i < kNbrVec ? i : kNbrVec - 1];
  }
  // Fields of the tile (global reads contiguous per field): one value per
  // lane and load, or for the split forms with Np a multiple of 4 four
  // consecutive values of one element per lane (16-byte loads: a quarter of
  // the load instructions, which bound the split forms' address unit).
  constexpr bool V4 = SPL && Np % 4 == 0;
  constexpr int kLoadIters = V4 ? 1 : (16 * Np + NT - 1) / NT;
  constexpr int kLoad4 = (4 * Np + NT - 1) / NT;
  T tv[kLoadIters][6];
  u32x4 tv4[V4 ? kLoad4 : 1][6];
  if constexpr (V4) {
#pragma unroll
    for (int it = 0; it < kLoad4; ++it) {
      const int i4 = 4 * (tid + NT * it);
      const uint32_t vo = i4 < ne * Np ? uint32_t(k0 * Np + i4) * sz : kOob;
#pragma unroll
      for (int c = 0; c < 6; ++c)
        tv4[it][c] = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(ru, (int)vo, (int)(uint32_t(c * fs) * sz), 0));
    }
  } else {
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
      const int idx = tid + NT * it;
      const bool in = idx < ne * Np;
      const uint32_t vo = in ? uint32_t(k0 * Np + idx) * sz : kOob;
#pragma unroll
      for (int c = 0; c < 6; ++c) tv[it][c] = buf_load<T>(ru, vo, uint32_t(c * fs) * sz);
    }
  }

  // LDS: geometry, codes, material face records, tables, then the fields.
#pragma unroll
  for (int it = 0; it < kGeoIters; ++it) {
    const int i = tid + NT * it;
    if (i < kGeoVec) reinterpret_cast<u32x4*>(t.geo)[i] = gv[it];
  }
  if (tid < 64) {
    t.code[tid] = cf;
    if constexpr (MAT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) t.face[4 * tid + i] = fmr[i];
    }
  }
#pragma unroll
  for (int it = 0; it < kFmaskIters; ++it) {
    const int i = tid + NT * it;
    if (i < NF) t.fmask[i] = int16_t(fmv[it]);
  }
#pragma unroll
  for (int it = 0; it < kNbrIters; ++it) {
    const int i = tid + NT * it;
    if (i < kNbrVec) reinterpret_cast<uint4*>(t.nbr)[i] = nbv[it];
  }
  if constexpr (SPL) {
    // FP32 rows [c][e] (records of 8 nodes, zero past Np), then their
    // head/tail records in the split region (or in place).
    if constexpr (V4) {
#pragma unroll
      for (int it = 0; it < kLoad4; ++it) {
        const int i4 = 4 * (tid + NT * it);
        const int ee = i4 / Np, j = i4 - ee * Np;
        if (i4 < 16 * Np) {
          int o = ee * X::RSV + j;
          asm("" : "+v"(o));  // one address, constant offsets per component
#pragma unroll
          for (int c = 0; c < 6; ++c) *reinterpret_cast<u32x4*>(&t.su[o + c * 16 * X::RSV]) = tv4[it][c];
        }
      }
    } else {
#pragma unroll
      for (int it = 0; it < kLoadIters; ++it) {
        const int idx = tid + NT * it;
        const int ee = idx / Np, j = idx - ee * Np;
        if (idx < 16 * Np) {
          int o = ee * X::RSV + j;
          asm("" : "+v"(o));
#pragma unroll
          for (int c = 0; c < 6; ++c) t.su[o + c * 16 * X::RSV] = tv[it][c];
        }
      }
    }
    constexpr int pad = 8 * X::J8 - Np;
    if constexpr (pad > 0) {
      for (int idx = tid; idx < 96 * pad; idx += NT) {
        const int row = idx / pad;
        t.su[row * X::RSV + Np + (idx - row * pad)] = T(0);
      }
    }
    __syncthreads();
    split_records<H16, 96, X::J8, X::RSV, NT>(t.su, t.su + X::SPLIT, tid);
  } else {
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
      const int idx = tid + NT * it;
      const int ee = idx / Np, j = idx - ee * Np;
      if (idx < 16 * Np) {
        int o = mul24(j, TS) + ee;
        asm("" : "+v"(o));  // one address, constant offsets per component
#pragma unroll
        for (int c = 0; c < 6; ++c) t.su[o + c * Np4 * TS] = tv[it][c];
      }
    }
    if constexpr (Np4 > Np) {
      for (int idx = tid; idx < 6 * (Np4 - Np) * 16; idx += NT) {
        const int c = idx / ((Np4 - Np) * 16), r = idx - c * ((Np4 - Np) * 16);
        t.su[(c * Np4 + Np + r / 16) * TS + (r & 15)] = T(0);
      }
    }
  }
  __syncthreads();
  // Metric of this lane's element, with a material the role's 1 / eps or 1 / mu.
  T mr[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) mr[i] = t.geo[e * kGeoStride + i];
  if constexpr (MAT) {
#pragma unroll
    for (int i = 0; i < 9; ++i) mr[i] *= mscale;
  }

  // Flux phase, run by all lanes of the tile between the volume and the lift phases:
  // one lane per (element, face node) pair, each flux evaluated once.  All
  // exterior traces of a lane are gathered at once; own traces are read from
  // the field tile, which is then overwritten by the fluxes [c][m][e].
  constexpr int kPairs = 16 * NF;
  constexpr int kFluxIters = (kPairs + NT - 1) / NT;
  // Pair pr of the tile: face-node-fastest, so that a gather instruction's
  // lanes walk the faces of few elements and touch few cache lines of their
  // neighbours (measured on MI355X: a fifth less time for the split forms at
  // N = 5); element-fastest with the split lift, whose halves are runs of
  // flux iterations over face-node rows.
  auto pair_of = [&](int pr, int& ee, int& m) {
    if constexpr (!LIFT_HALF) {
      ee = SmallDiv<NF, NT * kFluxIters>::div(pr);
      m = pr - mul24(ee, NF);
    } else {
      ee = pr & 15;
      m = pr >> 4;
    }
  };
  const T alpha = T(a.alpha);
  T gx[kFluxIters][6];
  T ox[OWNG ? kFluxIters : 1][6];
  // Gathers of traces that lie in the tile read LDS (measured on MI355X:
  // FP32 N = 5 stage -2.8%, FP64 N = 4 -8%, f16x3 N = 5 -1.3%; with the
  // LDS reads made at the flux step, FP64 N = 1-3 RHS -4 to -5% and FP32
  // N = 1, 3, 4 -2 to -4%, while the split forms at N <= 3 gain nothing).
  // Not with the split forms' in-place records, which replace the FP32 rows.
  constexpr bool LOCAL = !OWNG && (MIX == 0 || N >= 4);
  T fl[kFluxIters][6];
  // LDS index of a local trace (component 0), -1 for a gathered one.  The
  // LDS reads wait until flux_step: issued here they would overwrite
  // registers whose global loads are still in flight (the load of a local
  // lane is a null load), and the wait for those loads would serialise the
  // gather iterations.
  int loc[LOCAL ? kFluxIters : 1];
  auto gather = [&](int it0 = 0, int it1 = 1 << 20) {
#pragma unroll
    for (int it = 0; it < kFluxIters; ++it) {
      if (it < it0 || it >= it1) continue;
      const int pr = tid + NT * it;
      int ee, m;
      pair_of(pr, ee, m);
      const int f = SmallDiv<Nfp, NF>::div(m), jj = m - mul24(f, Nfp);
      const int32_t cf = (pr < kPairs) ? t.code[4 * ee + f] : -1;
      // interior: neighbour node; boundary: own node (mirror applied below); dead: zero.
      // With LOCAL a trace of an element of the tile (the own node on a
      // wall, or a neighbour inside the tile) comes from the field tile in
      // LDS, the others from global memory.
      uint32_t vo = kOob;
      bool local = false;
      int le = 0, ln = 0;   // element in the tile, node
      if (pr < kPairs && ee < ne) {
        // element relative to the tile (32-bit: element indices are below 2^26)
        const int dk = cf >= 0 ? int(int64_t(cf >> 5) - k0) : ee;
        const int nn = cf >= 0 ? int(t.nbr[mul24(f, 24 * Nfp) + mul24(cf & 31, Nfp) + jj]) : int(t.fmask[m]);
        local = LOCAL && unsigned(dk) < unsigned(ne);
        le = dk;
        ln = nn;
        if (!local) vo = ((uint32_t(k0) + uint32_t(dk)) * uint32_t(Np) + uint32_t(nn)) * sz;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) gx[it][c] = buf_load<T>(ru, vo, uint32_t(c * fs) * sz);
      if constexpr (LOCAL) loc[it] = local ? (SPL ? mul24(le, X::RSV) + ln : ln * TS + le) : -1;
      if constexpr (OWNG) {
        const uint32_t oo = (pr < kPairs && ee < ne) ? uint32_t((k0 + ee) * Np + t.fmask[m]) * sz : kOob;
#pragma unroll
        for (int c = 0; c < 6; ++c) ox[it][c] = buf_load<T>(ru, oo, uint32_t(c * fs) * sz);
      }
    }
  };
  // Own trace of component c at node own of element ee.
  auto own_at = [&](int it, int c, int ee, int own) -> T {
    if constexpr (OWNG) return ox[it][c];
    else if constexpr (SPL) return t.su[(c * 16 + ee) * X::RSV + own];
    else return t.su[(c * Np4 + own) * TS + ee];
  };
  auto flux_step = [&](int it) {
    const int pr = tid + NT * it;
    int ee, m;
    pair_of(pr, ee, m);
    if (pr < kPairs) {
      if constexpr (LOCAL) {
        if (loc[it] >= 0) {
#pragma unroll
          for (int c = 0; c < 6; ++c) gx[it][c] = t.su[loc[it] + c * (SPL ? 16 * X::RSV : Np4 * TS)];
        }
      }
      const int f = SmallDiv<Nfp, NF>::div(m);
      const int own = t.fmask[m];
      // exterior state E+ = se g, H+ = sh g with g the gathered trace
      // (interior: the neighbour's, se = sh = 1; boundary: the own one)
      const int32_t cd = t.code[4 * ee + f];
      T d[6];
      {
        const T se = cd >= 0 ? T(1) : (cd == -1 ? T(-1) : (cd == -2 ? T(1) : T(0)));
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] = own_at(it, c, ee, own) - se * gx[it][c];
      }
      {
        const T sh = cd >= -1 ? T(1) : (cd == -2 ? T(-1) : T(0));
#pragma unroll
        for (int c = 3; c < 6; ++c) d[c] = own_at(it, c, ee, own) - sh * gx[it][c];
      }
      const T* gr = &t.geo[ee * kGeoStride + 9 + 4 * f];
      const T nx = gr[0], ny = gr[1], nz = gr[2];
      T scE, scH, aE, aH;
      if constexpr (MAT) {
        const T* fr = &t.face[4 * (4 * ee + f)];
        scE = fr[0];
        scH = fr[1];
        aE = fr[2];
        aH = fr[3];
      } else {
        scE = scH = T(0.5) * gr[3];
        aE = aH = alpha;
      }
      const T ndE = nx * d[0] + ny * d[1] + nz * d[2];
      const T ndH = nx * d[3] + ny * d[4] + nz * d[5];
      fl[it][0] = scE * (-(ny * d[5] - nz * d[4]) + aE * (nx * ndE - d[0]));
      fl[it][1] = scE * (-(nz * d[3] - nx * d[5]) + aE * (ny * ndE - d[1]));
      fl[it][2] = scE * (-(nx * d[4] - ny * d[3]) + aE * (nz * ndE - d[2]));
      fl[it][3] = scH * ((ny * d[2] - nz * d[1]) + aH * (nx * ndH - d[3]));
      fl[it][4] = scH * ((nz * d[0] - nx * d[2]) + aH * (ny * ndH - d[4]));
      fl[it][5] = scH * ((nx * d[1] - ny * d[0]) + aH * (nz * ndH - d[5]));
    }
  };
  // part -1: all fluxes, rows c NF + m; part 0 / 1 (split lift): the flux
  // iterations of the first / second half of face-node rows, rows
  // c HB + m - part HB.  Parts -1 and 0 first wait until every read of the
  // field tile is done, since the fluxes overwrite it.
  // Split forms: flux iteration it into the FP32 rows [c][e] of face-node
  // records.
  auto flux_put = [&](int it) {
    if constexpr (SPL) {
      const int pr = tid + NT * it;
      int ee, m;
      pair_of(pr, ee, m);
      if (pr < kPairs) {
        int o = ee * X::RSF + m;
        asm("" : "+v"(o));  // one address, constant offsets (as in flux_store)
#pragma unroll
        for (int c = 0; c < 6; ++c) t.su[o + c * 16 * X::RSF] = fl[it][c];
      }
    }
  };
  auto flux_store = [&](int part) {
    if constexpr (SPL) {
      // The rows (part -1: after every read of the field tile is done; part
      // -2: already put), zero past NF, then split in place.
      if (part == -1) {
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kFluxIters; ++it) flux_put(it);
      }
      constexpr int pad = 8 * X::J8F - NF;
      if constexpr (pad > 0) {
        for (int idx = tid; idx < 96 * pad; idx += NT) {
          const int row = idx / pad;
          t.su[row * X::RSF + NF + (idx - row * pad)] = T(0);
        }
      }
      __syncthreads();
      split_records<H16, 96, X::J8F, X::RSF, NT>(t.su, t.su, tid);
      return;
    }
    constexpr int FR = LIFT_HALF ? S::HB : NF;
    if (part <= 0) __syncthreads();
    const int it0 = part == 1 ? S::HALF_ITERS : 0;
    const int it1 = part == 0 ? S::HALF_ITERS : kFluxIters;
    const int base = part == 1 ? S::HB : 0;
#pragma unroll
    for (int it = 0; it < kFluxIters; ++it) {
      const int pr = tid + NT * it;
      int ee, m;
      pair_of(pr, ee, m);
      if (it >= it0 && it < it1 && pr < kPairs) {
        // One address per pair, the components at constant offsets (left
        // to itself the compiler merges m = pr - NF ee into each component's
        // row index and spends three integer instructions per store).
        int o = mul24(m - base, TQ) + ee;
        asm("" : "+v"(o));
#pragma unroll
        for (int c = 0; c < 6; ++c) t.su[o + c * FR * TQ] = fl[it][c];
      }
    }
  };

  constexpr bool IL = flux_interleaved<N, T, MIX, CFG>();
  static_assert(WPT == 2 || (!IL && !LIFT_HALF), "interleaved flux and split lift assume 128 lanes per tile");
  // Output groups of the epilogue: the two roles with three components each,
  // or for the split forms one group of all six components.
  constexpr int CPG = SPL ? 6 : 3;
  acc_t acc[RBW][CPG];
  using B0 = std::integral_constant<int, RBW>;
  using B1 = std::integral_constant<int, RBW1>;
  // The waves of a role run one copy of the wave code when they own equal
  // numbers of row blocks and no 4-row tail, else one copy each.
  constexpr bool TAIL = mfma_tail<N, T, MIX, CFG>();
  constexpr bool ONE_COPY = SPL ? RBW1 == RBW : (WPT == 2 || (!TAIL && RBW1 == RBW));
  const bool first_blocks = SPL ? (sw < SRM || SRM == 0) : (WPT == 2 || rh == 0);
  const int nb = first_blocks ? RBW : RBW1;  // row blocks of this wave
  if constexpr (MIX == 0) {
    auto role = [&](auto tw, auto blocks) {
      constexpr bool TW = decltype(tw)::value;
      constexpr int NB = decltype(blocks)::value;
      auto& ac = reinterpret_cast<acc_t(&)[NB][3]>(acc);
      if (h == 0)
        mfma_wave<N, T, 0, IL, kFluxIters, NB, TW, PALT>(a, t, mr, lane, rb0, ac, gather, flux_step, flux_store);
      else
        mfma_wave<N, T, 1, IL, kFluxIters, NB, TW, PALT>(a, t, mr, lane, rb0, ac, gather, flux_step, flux_store);
    };
    if constexpr (ONE_COPY) {
      role(std::integral_constant<bool, TAIL>{}, B0{});
    } else {
      if (rh == 1)
        role(std::integral_constant<bool, TAIL>{}, B1{});
      else
        role(std::false_type{}, B0{});
    }
  } else {
    auto blocks = [&](auto nbk) {
      constexpr int NB = decltype(nbk)::value;
      auto& ac = reinterpret_cast<acc_t(&)[NB][6]>(acc);
      split_wave<N, H16, NPROD, kFluxIters, NB, PALT>(a, t, mr, lane, rb0, ac, gather, flux_step, flux_put,
                                                      flux_store);
    };
    if constexpr (ONE_COPY) {
      blocks(B0{});
    } else {
      if (first_blocks)
        blocks(B0{});
      else
        blocks(B1{});
    }
  }

  // Epilogue through LDS: [c][e][i] for the group's fields (the role's
  // three, or all six for the split forms; the waves of a group fill
  // disjoint row blocks), then contiguous stores per field, shared by the
  // group's waves.
  const int nv = ne * Np;
  constexpr int kRoleLanes = SPL ? NT : 64 * (WPT / 2);
  const int rl = SPL ? tid : lane + 64 * rh;   // lane within the group
  const int gf = SPL ? 0 : 3 * h;              // the group's first field
  // Output traffic in 16-byte accesses of V consecutive values per lane: a
  // tile's run of a field is 16 Np values, 16-byte aligned (fields start on
  // 256-byte boundaries and 16 Np sizeof(T) is a multiple of 16).
  constexpr int V = 16 / int(sizeof(T));
  using VT = T __attribute__((ext_vector_type(V)));
  constexpr int kOutIters = (16 * Np + V * kRoleLanes - 1) / (V * kRoleLanes);
  // Runge-Kutta stage: the residual and state loads of the update are issued
  // before the accumulators go through LDS, up to kAhead (component, slot)
  // items at a time, so their latency overlaps the exchange and the stores of
  // earlier items.  The field offset depends on the role (a per-lane value to
  // the compiler), so it goes into the vector offset: a per-lane scalar
  // offset would make every load a waterfall loop.
  constexpr int kItems = CPG * kOutIters;
  constexpr int kAheadRegs = sizeof(T) == 8 ? 112 : 40;  // VGPRs given to loads in flight
  constexpr int kAhead = RK ? (kItems * 8 <= kAheadRegs ? kItems : kAheadRegs / 8) : 0;
  VT rv[RK ? kItems : 1], uv[RK ? kItems : 1];
  // The first stage (rk_a = 0) reads no residual: an empty resource makes the
  // residual loads return zero without touching memory, so whatever res holds
  // on entry (NaN included) never enters the update.
  const __amdgpu_buffer_rsrc_t rr = make_rsrc(a.res, (RK && a.rk_a != 0.0) ? 6u * uint32_t(fs) * sz : 0u);
  auto vload = [&](__amdgpu_buffer_rsrc_t r, uint32_t vo) {
    return __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, 0, 0));
  };
  auto rk_load = [&](int j) {
    const int c = j / kOutIters, it = j % kOutIters;
    const int idx = V * (rl + kRoleLanes * it);
    const uint32_t vo = idx < nv ? uint32_t((gf + c) * fs + k0 * Np + idx) * sz : kOob;
    // the residual is read once per stage: a non-temporal load (cache policy
    // NT) keeps it from displacing neighbour traces in L2 (stage -1 to -2%)
    rv[j] = __builtin_bit_cast(VT, __builtin_amdgcn_raw_buffer_load_b128(rr, (int)vo, 0, 2));
    uv[j] = vload(ru, vo);
  };
#pragma unroll
  for (int j = 0; j < kAhead; ++j) rk_load(j);
  __syncthreads();
  T* so = t.su + gf * (16 * Np);
  T* discard = t.su + 6 * 16 * Np + 4 * lane;
  const bool tail_wave = TAIL && rb0 + nb == RB;
#pragma unroll
  for (int ib = 0; ib < RBW; ++ib)
#pragma unroll
    for (int c = 0; c < CPG; ++c) {
      if (ib >= nb) continue;
      if (ib == nb - 1 && tail_wave) {
        // 4-row block: FP64 row q in component 0; FP32 rows r, reduced over
        // the lane groups, written by group 0.
        if constexpr (sizeof(T) == 8) {
          const int i = 16 * (rb0 + ib) + q;
          if (i < Np) so[(c * 16 + e) * Np + i] = acc[ib][c][0];
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = 16 * (rb0 + ib) + r;
            if (q == 0 && i < Np) so[(c * 16 + e) * Np + i] = acc[ib][c][r];
          }
        }
        continue;
      }
      // Rows past Np go to a per-lane discard slot after the staging area:
      // an address select instead of a branch per row.
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * (rb0 + ib) + M::row(q, r);
        *(i < Np ? &so[(c * 16 + e) * Np + i] : discard + r) = acc[ib][c][r];
      }
    }
  __syncthreads();
  // Staged values (component c, slot it) of this lane, read without a branch
  // (the index is clamped into the component's rows) so that a component's
  // reads are issued together rather than one per store.
  auto so_at = [&](int c, int it) {
    const int idx = V * (rl + kRoleLanes * it);
    return *reinterpret_cast<const VT*>(&so[c * 16 * Np + (idx < 16 * Np ? idx : 16 * Np - V)]);
  };
  // Stores go through one buffer resource per output field that covers just
  // the field's K Np values: the 16-byte store that straddles the end of a
  // ragged last tile loses its out-of-range dwords (the range check is per
  // dword), so no store sits behind a per-value branch.  The group is
  // wave-uniform, which makes the resources scalar.
  const int gfu = __builtin_amdgcn_readfirstlane(gf);
  typedef uint32_t w32x4 __attribute__((ext_vector_type(4)));
  auto field_rsrc = [&](void* base, int c) {
    return make_rsrc(static_cast<T*>(base) + (gfu + c) * fs, uint32_t(a.K) * Np * sz);
  };
  auto put = [&](auto streaming, __amdgpu_buffer_rsrc_t r, int idx, VT v) {
    const uint32_t vo = idx < nv ? uint32_t(k0 * Np + idx) * sz : kOob;
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(w32x4, v), r, (int)vo, 0,
                                           decltype(streaming)::value ? 2 : 0);
  };
  auto out = [&](auto streaming) {
    if constexpr (!RK) {
#pragma unroll
      for (int c = 0; c < CPG; ++c) {
        VT ov[kOutIters];
#pragma unroll
        for (int it = 0; it < kOutIters; ++it) ov[it] = so_at(c, it);
        const __amdgpu_buffer_rsrc_t ro = field_rsrc(a.rhs, c);
#pragma unroll
        for (int it = 0; it < kOutIters; ++it) put(streaming, ro, V * (rl + kRoleLanes * it), ov[it]);
      }
    } else {
      const T ra = T(a.rk_a), rb = T(a.rk_b), dt = T(a.rk_dt);
#pragma unroll
      for (int c = 0; c < CPG; ++c) {
        VT ov[kOutIters];
#pragma unroll
        for (int it = 0; it < kOutIters; ++it) ov[it] = so_at(c, it);
        const __amdgpu_buffer_rsrc_t rs = field_rsrc(a.res, c), rn = field_rsrc(a.u_out, c);
#pragma unroll
        for (int it = 0; it < kOutIters; ++it) {
          const int j = c * kOutIters + it;
          if (j + kAhead < kItems) rk_load(j + kAhead);
          const VT r = ra * rv[j] + dt * ov[it];
          const int idx = V * (rl + kRoleLanes * it);
          put(streaming, rs, idx, r);
          put(streaming, rn, idx, uv[j] + rb * r);
        }
      }
    }
  };
  // Outputs go through streaming (non-temporal) stores when the host says
  // the arrays a launch touches exceed the last-level cache: there they
  // cannot stay resident for the next launch anyway, such stores retire
  // sooner, and they leave the L2 to the neighbour traces (measured on
  // MI355X: FP64 2-4%; K = 663,552, N = 5: FP32 stage -1.4%, split -3%).
  if (a.stream_out) {
    out(std::true_type{});
    return;
  }
  out(std::false_type{});
}

// Minimum waves per SIMD the register allocation must allow (1: no
// constraint).  Set where the unconstrained allocation lands one or two
// registers past the 168 that three waves per SIMD allow (512 / 3, in
// granules of 8), which the allocator then meets without spilling.
// kCfgOccupancy asks for what the tile's LDS allows (workgroups per CU x
// waves per workgroup over the 4 SIMDs, at most 8).
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr int lds_waves_per_simd() {
  constexpr size_t tile_bytes = sizeof(MfmaTile<N, T, lift_split<N, T, MIX, CFG>(), false, (MIX != 0)>);
  constexpr int wg = int((160 * 1024) / tile_bytes);
  constexpr int w = wg * waves_per_tile<N, T, MIX, CFG>() / 4;
  return w > 8 ? 8 : (w < 1 ? 1 : w);
}
template <int N, typename T, int MIX, int CFG = kCfgDefault>
constexpr int min_waves_per_simd() {
  // At least two waves per SIMD where the LDS allows them (the allocation
  // lands just past 256 registers at some orders: FP32 N = 7 takes 269
  // unconstrained and 233 without spilling when asked), except with two
  // waves per tile at high order, where four-wave tiles are the default.
  constexpr int ls = lds_waves_per_simd<N, T, MIX, CFG>();
  constexpr int two = CFG == kCfgWaves ? 1 : (ls < 2 ? ls : 2);
  constexpr int d = (sizeof(T) == 4 && MIX == 0 && N == 6) ? 3 : two;
  return CFG == kCfgOccupancy ? lds_waves_per_simd<N, T, MIX, CFG>() : d;
}

// Whether tuning configuration CFG is built for (N, T, MIX): the default
// wherever the kernel is; another only where it changes the kernel and the
// resulting combination is one the kernel supports (the interleaved flux and
// the split lift need two waves per tile and exclude each other).
template <int N, typename T, int MIX, int CFG>
constexpr bool config_built() {
  if constexpr (!mfma_supported<N, T, MIX, kCfgDefault>() || !mfma_supported<N, T, MIX, CFG>()) {
    return false;
  } else {
    constexpr int W = waves_per_tile<N, T, MIX, CFG>();
    constexpr bool IL = flux_interleaved<N, T, MIX, CFG>(), LH = lift_split<N, T, MIX, CFG>();
    constexpr bool ok = (W == 2 || (!IL && !LH)) && !(IL && LH);
    if constexpr (CFG == kCfgDefault) return ok;
    if constexpr (CFG == kCfgWaves) return ok && W != waves_per_tile<N, T, MIX>();
    if constexpr (CFG == kCfgPrefetch) return ok;
    if constexpr (CFG == kCfgOccupancy)
      return ok && lds_waves_per_simd<N, T, MIX, CFG>() > min_waves_per_simd<N, T, MIX>() &&
             lds_waves_per_simd<N, T, MIX, CFG>() >= 2;
    if constexpr (CFG == kCfgInterleave) return ok && MIX == 0 && IL != flux_interleaved<N, T, MIX>();
    if constexpr (CFG == kCfgLift) return ok && MIX == 0 && LH != lift_split<N, T, MIX>();
    if constexpr (CFG == kCfgTail) return ok && MIX == 0 && mfma_tail<N, T, MIX, CFG>() != mfma_tail<N, T, MIX>();
    return false;
  }
}

// Workgroup b runs on XCD b % 8; give each XCD a contiguous range of the
// n tiles (launch 8 * ceil(n / 8) workgroups; the surplus returns).
__device__ inline int64_t xcd_tile(int64_t n) {
  const int64_t per = (n + 7) / 8;
  return int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
}

// With a tile order (a space-filling-curve order of the tiles' centroids),
// the XCD-contiguous slots walk it instead of the element numbering, so the
// tiles resident on one XCD at a time are spatial neighbours and their
// neighbour-trace gathers hit that XCD's L2.
template <int N, typename T, bool RK, int MIX, bool MAT = false, int CFG = kCfgDefault>
__global__ __launch_bounds__((64 * waves_per_tile<N, T, MIX, CFG>()),
                             (min_waves_per_simd<N, T, MIX, CFG>())) void rhs_mfma_kernel(RhsArgs a) {
  int64_t tile = xcd_tile((a.K + 15) / 16);
  if (tile >= (a.K + 15) / 16) return;
  if (a.tile_order) tile = a.tile_order[tile];
  rhs_mfma_tile<N, T, RK, MIX, MAT, CFG>(a, tile);
}

// One Runge-Kutta stage for every problem of a batch that has order N: the
// work list holds (problem, tile) pairs, problem by problem; per-problem
// pointers come from the descriptor table.  parity 0 reads u and writes the
// second state buffer, parity 1 the reverse.
template <int N, typename T, int MIX>
__global__ __launch_bounds__((64 * waves_per_tile<N, T, MIX>()), (min_waves_per_simd<N, T, MIX>())) void rk_mfma_batch_kernel(
    BatchArgs b) {
  const int64_t item = xcd_tile(b.n_items);
  if (item >= b.n_items) return;
  const int2 w = b.items[item];
  const BatchProblem& P = b.probs[w.x];
  RhsArgs a;
  a.u = b.parity ? P.u2 : P.u;
  a.u_out = b.parity ? P.u : P.u2;
  a.res = P.res;
  a.rhs = nullptr;
  a.geo = P.geo;
  a.conn = P.conn;
  a.mat = nullptr;
  a.tile_order = nullptr;
  a.ops = nullptr;
  a.ops_frag = b.ops_frag;
  a.ops_frag16 = b.ops_frag16;
  a.nbr = b.nbr;
  a.fmask = b.fmask;
  a.K = P.K;
  a.fs = P.fs;
  a.alpha = P.alpha;
  a.rk_a = b.rk_a;
  a.rk_b = b.rk_b;
  a.rk_dt = P.dt;
  a.stream_out = b.stream_out;
  rhs_mfma_tile<N, T, true, MIX>(a, w.y);
}

template <int N, typename T, int MIX = 0>
hipError_t launch_rk_mfma_batch(const BatchArgs& b, hipStream_t s) {
  const unsigned grid = unsigned(8 * ((b.n_items + 7) / 8));
  hipLaunchKernelGGL((rk_mfma_batch_kernel<N, T, MIX>), dim3(grid), dim3(64 * waves_per_tile<N, T, MIX>()), 0, s, b);
  return hipGetLastError();
}

template <int N, typename T, int MIX = 0, bool MAT = false, int CFG = kCfgDefault>
hipError_t launch_rhs_mfma(const RhsArgs& a, hipStream_t s) {
  const int64_t nt = (a.K + 15) / 16;
  const unsigned grid = unsigned(8 * ((nt + 7) / 8));
  hipLaunchKernelGGL((rhs_mfma_kernel<N, T, false, MIX, MAT, CFG>), dim3(grid),
                     dim3(64 * waves_per_tile<N, T, MIX, CFG>()), 0, s, a);
  return hipGetLastError();
}

template <int N, typename T, int MIX = 0, bool MAT = false, int CFG = kCfgDefault>
hipError_t launch_rk_mfma(const RhsArgs& a, hipStream_t s) {
  const int64_t nt = (a.K + 15) / 16;
  const unsigned grid = unsigned(8 * ((nt + 7) / 8));
  hipLaunchKernelGGL((rhs_mfma_kernel<N, T, true, MIX, MAT, CFG>), dim3(grid),
                     dim3(64 * waves_per_tile<N, T, MIX, CFG>()), 0, s, a);
  return hipGetLastError();
}

}  // namespace dgd
