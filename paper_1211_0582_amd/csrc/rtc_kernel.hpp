// Right-hand side of a general hyperbolic system in nodal DG form, compiled
// at run time (hipRTC) for one system, order and precision -- the run-time
// code generation of Section 4: the system's volume flux, numerical flux and
// boundary states arrive as generated source, so every constant of the
// system (which flux-matrix entries are zero, which fields a boundary state
// touches) is known to the compiler, as are N, Np and Nfp.
//
// This text is compiled by hipRTC only (no HIP runtime header: hipRTC
// provides the device builtins).  The generated source in front of it
// defines
//   #define DG_ORDER <N>
//   typedef <float|double> dg_real;
//   struct System {
//     static constexpr int M;                 // fields
//     template <typename T> static void volume(const T (&m)[3], const T (&u)[M], T (&x)[M]);
//         // x = -sum_d m_d F_d(u): the volume flux along the metric row m
//     template <typename T> static void exterior(int code, T nx, T ny, T nz, const T (&um)[M], T (&up)[M]);
//         // exterior state of a boundary face with condition code `code`
//     template <typename T> static void flux(T nx, T ny, T nz, T alpha, const T (&um)[M], const T (&up)[M],
//                                            T (&f)[M]);  // f = n.F - (n.F)*
//   };
// (all __device__).  The kernel is the matrix-core contraction of the
// library's Maxwell kernels (Section 2.1's local differentiation and
// lifting as one product with [Dr|Ds|Dt|LIFT], operator fragments prepared
// by the library on the host, 16 elements per workgroup, the volume operand
// X_d formed in registers, the fluxes staged in LDS), with the field count
// and the flux arithmetic taken from System: wave w of the workgroup
// produces fields w*FPW .. w*FPW + FPW - 1, at most three per wave.
#include <cstdint>
#include <type_traits>

namespace dgrtc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
template <>
struct Mfma<float> {
  using acc = f32x4;
  __device__ static inline acc mac(float a, float b, acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static constexpr int row(int q, int r) { return 4 * q + r; }
};
template <>
struct Mfma<double> {
  using acc = f64x4;
  __device__ static inline acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int q, int r) { return q + 4 * r; }
};

__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename T>
__device__ inline T load(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, 0, 0));
}

// Kernel arguments; layout shared with the library's host code.
struct Args {
  const void* u;           // state [M][fs], element-major inside a field
  void* rhs;               // output, same layout
  const void* geo;         // K x 25: metric (9), then per face nx, ny, nz, Fscale
  const int32_t* conn;     // K x 4: nbr*32 + nbr_face*6 + orient, or -1 - bc
  const void* frag;        // [Dr|Ds|Dt|LIFT] 16x4 MFMA A-fragments [block][depth step][lane]
  const uint8_t* nbr;      // 4 x 24 x Nfp neighbour node per (face, code, face node)
  const int32_t* fmask;    // 4 x Nfp
  int64_t K, fs;
  double alpha;
};

constexpr int kGeo = 25;
constexpr uint32_t kOob = 0x80000000u;

template <int N>
struct Shape {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2, NF = 4 * Nfp;
  static constexpr int Np4 = (Np + 3) & ~3, RB = (Np + 15) / 16, KSV = Np4 / 4, KSL = NF / 4, KS = 3 * KSV + KSL;
  static constexpr int TS = 17, TQ = 16;
};

template <int M>
struct Waves {
  static constexpr int W = (M + 2) / 3;            // waves per workgroup
  static constexpr int FPW = (M + W - 1) / W;      // fields per wave
};

template <int N, typename T, typename Sys>
__device__ inline void tile_rhs(const Args& a, int64_t tile) {
  using S = Shape<N>;
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc;
  constexpr int M = Sys::M, W = Waves<M>::W, FPW = Waves<M>::FPW, NT = 64 * W;
  constexpr int Np = S::Np, Nfp = S::Nfp, NF = S::NF, Np4 = S::Np4, RB = S::RB, KSV = S::KSV, KSL = S::KSL;
  constexpr int KS = S::KS, TS = S::TS, TQ = S::TQ;
  constexpr int FIELDS = M * Np4 * TS, FLUXES = M * NF * TQ, STAGE = M * 16 * Np;
  constexpr int TILE = FIELDS > FLUXES ? (FIELDS > STAGE ? FIELDS : STAGE) : (FLUXES > STAGE ? FLUXES : STAGE);
  constexpr uint32_t sz = sizeof(T);
  __shared__ T su[TILE];
  __shared__ int16_t s_fmask[NF];
  __shared__ uint8_t s_nbr[4 * 24 * Nfp];
  __shared__ int32_t s_code[64];
  __shared__ T s_face[64 * 4];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int e = lane & 15, q = lane >> 4;
  const int64_t fs = a.fs, k0 = tile * 16;
  const int ne = int((a.K - k0) < 16 ? (a.K - k0) : 16);
  const bool live = e < ne;
  const __amdgpu_buffer_rsrc_t rg = rsrc(a.geo, uint32_t(a.K) * kGeo * sz);
  const __amdgpu_buffer_rsrc_t ru = rsrc(a.u, uint32_t(M) * uint32_t(fs) * sz);
  const __amdgpu_buffer_rsrc_t rf = rsrc(a.frag, uint32_t((RB + 1) * KS * 64) * sz);

  // Prologue: metric of this lane's element, face records, tables, fields.
  T mr[9];
  {
    const uint32_t go = live ? uint32_t((k0 + e) * kGeo) * sz : kOob;
#pragma unroll
    for (int i = 0; i < 9; ++i) mr[i] = load<T>(rg, go + i * sz);
  }
  if (tid < 64) {
    const int ee = tid >> 2, f = tid & 3;
    const bool lv = ee < ne;
    s_code[tid] = lv ? a.conn[(k0 + ee) * 4 + f] : -1;
    const uint32_t go = lv ? uint32_t((k0 + ee) * kGeo + 9 + 4 * f) * sz : kOob;
#pragma unroll
    for (int i = 0; i < 4; ++i) s_face[4 * tid + i] = load<T>(rg, go + i * sz);
  }
  for (int i = tid; i < NF; i += NT) s_fmask[i] = int16_t(a.fmask[i]);
  for (int i = tid; i < 4 * 24 * Nfp; i += NT) s_nbr[i] = a.nbr[i];
  for (int idx = tid; idx < 16 * Np4; idx += NT) {
    const int ee = idx / Np4, j = idx - ee * Np4;
    const bool in = ee < ne && j < Np;
    const uint32_t vo = in ? uint32_t(k0 * Np + ee * Np + j) * sz : kOob;
#pragma unroll
    for (int c = 0; c < M; ++c) su[(c * Np4 + j) * TS + ee] = load<T>(ru, vo + uint32_t(c * fs) * sz);
  }
  __syncthreads();

  // Wave w produces fields C0 .. C0 + FPW - 1 (C0 = w FPW); the wave index is
  // made a compile-time constant so that every field index is one.
  auto body = [&](auto wi) {
    constexpr int C0 = decltype(wi)::value * FPW;
    constexpr int NC = (M - C0) < FPW ? (M - C0) : FPW;  // fields of this wave
    acc_t acc[RB][NC];
#pragma unroll
    for (int ib = 0; ib < RB; ++ib)
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[ib][c] = acc_t{0, 0, 0, 0};
    auto frag = [&](int kg, int ib) { return load<T>(rf, uint32_t(((ib * KS + kg) * 64) + lane) * sz); };

    // Volume: X_d = -sum_x m_{d,x} F_x(u) at node j = 4 ks + q of element e.
    // Padded depth rows j >= Np meet zero operator columns, but a nonlinear
    // flux of their zero fields need not be finite (0 / 0), and 0 x NaN is
    // NaN in the product: their operand is set to zero.
#pragma unroll
    for (int ks = 0; ks < KSV; ++ks) {
      const int j = 4 * ks + q;
      T uv[M];
#pragma unroll
      for (int c = 0; c < M; ++c) uv[c] = su[(c * Np4 + j) * TS + e];
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const T md[3] = {mr[3 * d], mr[3 * d + 1], mr[3 * d + 2]};
        T x[M];
        Sys::template volume<T>(md, uv, x);
        if (j >= Np) {
#pragma unroll
          for (int c = 0; c < M; ++c) x[c] = T(0);
        }
        T av[RB];
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) av[ib] = frag(d * KSV + ks, ib);
#pragma unroll
        for (int ib = 0; ib < RB; ++ib)
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[ib][c] = Mf::mac(av[ib], x[C0 + c], acc[ib][c]);
      }
    }

    // Flux: one lane per (element, face node) pair, all lanes of the tile.
    constexpr int kPairs = 16 * NF, kIters = (kPairs + NT - 1) / NT;
    const T alpha = T(a.alpha);
    T fl[kIters][M];
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
      const int pr = tid + NT * it;
      const int ee = pr & 15, m = pr >> 4;
      if (pr < kPairs) {
        const int f = m / Nfp, jj = m - f * Nfp;
        const int32_t cf = s_code[4 * ee + f];
        const int own = s_fmask[m];
        T um[M], up[M];
#pragma unroll
        for (int c = 0; c < M; ++c) um[c] = su[(c * Np4 + own) * TS + ee];
        const T* fr = &s_face[4 * (4 * ee + f)];
        if (cf >= 0) {
          const uint32_t vo =
              ee < ne ? uint32_t(int64_t(cf >> 5) * Np + s_nbr[(f * 24 + (cf & 31)) * Nfp + jj]) * sz : kOob;
#pragma unroll
          for (int c = 0; c < M; ++c) up[c] = load<T>(ru, vo + uint32_t(c * fs) * sz);
        } else {
          Sys::template exterior<T>(-1 - cf, fr[0], fr[1], fr[2], um, up);
        }
        T fv[M];
        Sys::template flux<T>(fr[0], fr[1], fr[2], alpha, um, up, fv);
#pragma unroll
        for (int c = 0; c < M; ++c) fl[it][c] = fr[3] * fv[c];
      }
    }
    __syncthreads();  // every read of the field tile is done: the fluxes overwrite it
#pragma unroll
    for (int it = 0; it < kIters; ++it) {
      const int pr = tid + NT * it;
      const int ee = pr & 15, m = pr >> 4;
      if (pr < kPairs) {
#pragma unroll
        for (int c = 0; c < M; ++c) su[(c * NF + m) * TQ + ee] = fl[it][c];
      }
    }
    __syncthreads();

    // Lift: F (already scaled by Fscale) from the LDS flux tile.
#pragma unroll
    for (int ks = 0; ks < KSL; ++ks) {
      const int m = 4 * ks + q;
      T av[RB];
#pragma unroll
      for (int ib = 0; ib < RB; ++ib) av[ib] = frag(3 * KSV + ks, ib);
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T fv = su[((C0 + c) * NF + m) * TQ + e];
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) acc[ib][c] = Mf::mac(av[ib], fv, acc[ib][c]);
      }
    }
    __syncthreads();  // flux tile read: the staging overwrites it

    // Epilogue: stage [c][e][i] in LDS, then contiguous stores per field.
#pragma unroll
    for (int ib = 0; ib < RB; ++ib)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * ib + Mf::row(q, r);
          if (i < Np) su[((C0 + c) * 16 + e) * Np + i] = acc[ib][c][r];
        }
    __syncthreads();
    T* out = static_cast<T*>(a.rhs);
    const int nv = ne * Np;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T* base = out + (C0 + c) * fs + k0 * Np;
      for (int idx = lane; idx < nv; idx += 64) base[idx] = su[(C0 + c) * 16 * Np + idx];
    }
  };
  static_assert(W <= 4, "at most 12 fields");
  if (w == 0) body(std::integral_constant<int, 0>{});
  if constexpr (W > 1) if (w == 1) body(std::integral_constant<int, 1>{});
  if constexpr (W > 2) if (w == 2) body(std::integral_constant<int, 2>{});
  if constexpr (W > 3) if (w == 3) body(std::integral_constant<int, 3>{});
}

}  // namespace dgrtc

extern "C" __global__ void __launch_bounds__(64 * dgrtc::Waves<System::M>::W) dg_rtc_rhs(dgrtc::Args a) {
  const int64_t nt = (a.K + 15) / 16;
  // workgroup b on XCD b % 8: each XCD takes a contiguous range of tiles
  const int64_t per = (nt + 7) / 8;
  const int64_t tile = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= nt) return;
  dgrtc::tile_rhs<DG_ORDER, dg_real, System>(a, tile);
}
