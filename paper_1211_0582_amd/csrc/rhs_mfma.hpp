// Fused DG Maxwell right-hand side on the matrix cores (FP64 / FP32 MFMA).
//
// The operator of Section 2 is, per element, one dense contraction:
//   rhs[c][i] = sum_d sum_j D_d[i][j] X_d[c][j] + sum_m LIFT[i][m] F[c][m]
// with X_d = (m_d x H, E x m_d) the fields pre-combined with the element's
// constant metric row m_d = (d_x, d_y, d_z), d in {r, s, t} (so the volume
// sum is the curl term of Section 2.1), and F the Fscale-scaled upwind flux
// at the 4 Nfp face nodes.  One wave owns 16 elements and runs that
// contraction as 16x16x4 MFMAs: rows = nodes i (Np padded to 16), columns =
// the 16 elements, depth = [Dr | Ds | Dt | LIFT] columns (each padded to 4).
//
//  * The operator is pre-swizzled on the host into MFMA A-fragments
//    (row block ib, depth step kg, lane) and streamed through L1/L2 (one
//    coalesced load feeds six MFMAs, one per output component).
//  * The tile's fields sit in LDS as [c][j][e] (16 elements fastest), read in
//    B-fragment layout; X_d is formed in registers.
//  * The flux gather happens directly in B-fragment layout: lane (e, m)
//    gathers the neighbour trace through the orientation table, evaluates the
//    flux and feeds it to the LIFT MFMAs -- the facial buffer of the paper's
//    split pipeline never exists.
//  * Epilogue: accumulators go through LDS to coalesced stores; in the
//    Runge-Kutta mode the stage update res <- a res + dt rhs,
//    u_out <- u + b res is applied there (u_out is a second state buffer, as
//    neighbours still read u during the stage).
//  * Tiles are mapped to workgroups so that each of the 8 XCDs gets a
//    contiguous range of elements (neighbours then share that XCD's L2).
#pragma once

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
};
template <>
struct Mfma16<double> {
  using acc = f64x4;
  __device__ static inline acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static constexpr int row(int q, int r) { return q + 4 * r; }
};

template <int N>
struct MfmaShape {
  static constexpr int Np = Order<N>::Np, Nfp = Order<N>::Nfp, NF = Order<N>::NF;
  static constexpr int Np4 = (Np + 3) & ~3;   // volume depth per direction, padded
  static constexpr int RB = (Np + 15) / 16;   // 16-row blocks
  static constexpr int KSV = Np4 / 4;         // depth steps per direction
  static constexpr int KSL = NF / 4;          // depth steps of LIFT (4 Nfp is a multiple of 4)
  static constexpr int KS = 3 * KSV + KSL;
  static constexpr int TS = 17;               // LDS row stride (16 elements + 1)
  static constexpr int frag_count = RB * KS * 64;
};

template <int N, typename T>
constexpr size_t mfma_lds_bytes() {
  return size_t(6) * MfmaShape<N>::Np4 * MfmaShape<N>::TS * sizeof(T);
}

// Whether the MFMA variant is built for (N, T): the LDS tile and the
// accumulators (RB * 3 * 4 scalars per lane) must fit.
template <int N, typename T>
constexpr bool mfma_supported() {
  return mfma_lds_bytes<N, T>() <= 65536 && MfmaShape<N>::RB * 3 * 4 * sizeof(T) / 4 <= 128;
}

// Workgroup = two waves sharing one tile of 16 elements.  Wave h = 0 produces
// the E equations (curl H + LIFT fE), wave h = 1 the H equations
// (-curl E + LIFT fH).  Both run the same code with the field roles swapped:
// with V = H, (P, Q) = (dE, dH) for h = 0 and V = -E, (P, Q) = (dH, -dE) for
// h = 1, the volume operand is X_d = m_d x V and the flux is
// f = 1/2 Fscale [ -n x Q + alpha (n (n.P) - P) ].
template <int N, typename T, bool RK>
__global__ __launch_bounds__(128) void rhs_mfma_kernel(RhsArgs a) {
  using S = MfmaShape<N>;
  using M = Mfma16<T>;
  using acc_t = typename M::acc;
  constexpr int Np = S::Np, Nfp = S::Nfp, NF = S::NF, Np4 = S::Np4, RB = S::RB, KSV = S::KSV, KSL = S::KSL;
  constexpr int KS = S::KS, TS = S::TS;
  __shared__ T su[6 * Np4 * TS];
  __shared__ int16_t s_fmask[NF];
  __shared__ uint8_t s_nbr[4 * 24 * Nfp];
  __shared__ int32_t s_code[16 * 4];   // face codes of the tile's elements
  __shared__ T s_face[16 * 4 * 4];     // nx, ny, nz, Fscale / 2 per (element, face)

  const T* __restrict__ u = static_cast<const T*>(a.u);
  const T* __restrict__ geo = static_cast<const T*>(a.geo);
  const T* __restrict__ frag = static_cast<const T*>(a.ops_frag);
  const int64_t fs = a.fs;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int h = tid >> 6;             // 0: E equations, 1: H equations
  const int e = lane & 15, q = lane >> 4;

  // XCD-aware tile: workgroup b runs on XCD b % 8; give each XCD a contiguous range.
  const int64_t nt = (a.K + 15) / 16;
  const int64_t per = (nt + 7) / 8;
  const int64_t tile = int64_t(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (tile >= nt) return;
  const int64_t k0 = tile * 16;
  const int ne = int((a.K - k0) < 16 ? (a.K - k0) : 16);
  const bool live = e < ne;
  const int64_t ke = k0 + (live ? e : 0);

  // Metric of this lane's element in registers; face records and tables in LDS.
  T mr[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) mr[i] = live ? geo[ke * kGeoStride + i] : T(0);
  if (tid < 64) {
    const int ee = tid >> 2, f = tid & 3;  // 16 elements x 4 faces
    const bool lv = ee < ne;
    const int64_t kk = k0 + (lv ? ee : 0);
    s_code[tid] = lv ? a.conn[kk * 4 + f] : -1;
    const T* gf = geo + kk * kGeoStride + 9 + 4 * f;
    s_face[4 * tid + 0] = lv ? gf[0] : T(0);
    s_face[4 * tid + 1] = lv ? gf[1] : T(0);
    s_face[4 * tid + 2] = lv ? gf[2] : T(0);
    s_face[4 * tid + 3] = lv ? T(0.5) * gf[3] : T(0);
  }
  for (int i = tid; i < NF; i += 128) s_fmask[i] = int16_t(a.fmask[i]);
  for (int i = tid; i < 4 * 24 * Nfp; i += 128) s_nbr[i] = a.nbr[i];

  // 1. fields of the tile -> LDS [c][j][e] (global reads contiguous per field)
  constexpr int kLoadIters = (16 * Np + 127) / 128;
#pragma unroll
  for (int c = 0; c < 6; ++c) {
    const T* src = u + c * fs + k0 * Np;
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
      const int idx = tid + 128 * it;
      if (idx < 16 * Np) {
        const int ee = idx / Np, j = idx - ee * Np;
        su[(c * Np4 + j) * TS + ee] = (ee < ne) ? src[idx] : T(0);
      }
    }
    if constexpr (Np4 > Np) {
      for (int idx = tid; idx < (Np4 - Np) * 16; idx += 128)
        su[(c * Np4 + Np + idx / 16) * TS + (idx & 15)] = T(0);
    }
  }
  __syncthreads();

  acc_t acc[RB][3];
#pragma unroll
  for (int ib = 0; ib < RB; ++ib)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[ib][c] = acc_t{0, 0, 0, 0};

  // Field roles of this wave: V (volume) = fields vb.. with sign vs; own
  // outputs are fields 3h .. 3h+2.
  const int vb = h ? 0 : 3;           // V = H (h = 0) or -E (h = 1)
  const T vs = h ? T(-1) : T(1);

  // Software pipeline: every global load is issued kPre depth steps before its
  // use (operator fragments over the whole depth, neighbour traces).
  constexpr int kPre = 2;
  constexpr int NV = 3 * KSV;  // volume depth steps, ordered (ks, d)
  auto frag_of = [&](int step, int ib) -> T {
    const int kg = step < NV ? (step % 3) * KSV + step / 3 : 3 * KSV + (step - NV);
    return frag[(ib * KS + kg) * 64 + lane];
  };
  T Abuf[kPre + 1][RB];
#pragma unroll
  for (int s = 0; s < kPre; ++s)
#pragma unroll
    for (int ib = 0; ib < RB; ++ib) Abuf[s][ib] = frag_of(s, ib);

  // 2. volume: X_d = m_d x V at node j = 4 ks + q of element e
#pragma unroll
  for (int ks = 0; ks < KSV; ++ks) {
    const int j = 4 * ks + q;
    T v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = vs * su[((vb + c) * Np4 + j) * TS + e];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int step = 3 * ks + d;
      if (step + kPre < KS) {
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) Abuf[(step + kPre) % (kPre + 1)][ib] = frag_of(step + kPre, ib);
      }
      const T mx = mr[3 * d], my = mr[3 * d + 1], mz = mr[3 * d + 2];
      T X[3];
      X[0] = my * v[2] - mz * v[1];
      X[1] = mz * v[0] - mx * v[2];
      X[2] = mx * v[1] - my * v[0];
#pragma unroll
      for (int ib = 0; ib < RB; ++ib)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[ib][c] = M::mac(Abuf[step % (kPre + 1)][ib], X[c], acc[ib][c]);
    }
  }

  // 3. lifting, flux evaluated in B-fragment layout at face node m = 4 ks + q.
  auto gather = [&](int ks, T (&out)[6]) {
    const int m = 4 * ks + q;
    const int f = m / Nfp;
    const int jj = m - f * Nfp;
    const int32_t cf = s_code[4 * e + f];
    const int64_t g = cf >= 0 ? int64_t(cf >> 5) * Np + s_nbr[(f * 24 + (cf & 31)) * Nfp + jj] : ke * Np;
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = u[c * fs + g];
  };
  T Pbuf[kPre + 1][6];
#pragma unroll
  for (int s = 0; s < kPre; ++s) gather(s, Pbuf[s]);

  const T alpha = T(a.alpha);
  const int pb = h ? 3 : 0;            // P = jump of fields pb..pb+2
  const int qb = h ? 0 : 3;            // Q = qs * jump of fields qb..qb+2
  const T qs = h ? T(-1) : T(1);
#pragma unroll
  for (int ks = 0; ks < KSL; ++ks) {
    const int step = NV + ks;
    if (step + kPre < KS) {
#pragma unroll
      for (int ib = 0; ib < RB; ++ib) Abuf[(step + kPre) % (kPre + 1)][ib] = frag_of(step + kPre, ib);
    }
    if (ks + kPre < KSL) gather(ks + kPre, Pbuf[(ks + kPre) % (kPre + 1)]);
    const int m = 4 * ks + q;
    const int f = m / Nfp;
    const int own = s_fmask[m];
    const bool wall = s_code[4 * e + f] < 0;
    T d[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const T em = su[(c * Np4 + own) * TS + e];
      // wall: E+ = -E-, H+ = H-  =>  dE = 2 E-, dH = 0
      const T ep = wall ? (c < 3 ? -em : em) : Pbuf[ks % (kPre + 1)][c];
      d[c] = em - ep;
    }
    T P[3], Q[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P[c] = h ? d[3 + c] : d[c];
      Q[c] = qs * (h ? d[c] : d[3 + c]);
    }
    (void)pb;
    (void)qb;
    const T* fr = &s_face[4 * (4 * e + f)];
    const T nx = fr[0], ny = fr[1], nz = fr[2], sc = fr[3];
    const T nP = nx * P[0] + ny * P[1] + nz * P[2];
    T F[3];
    F[0] = sc * (-(ny * Q[2] - nz * Q[1]) + alpha * (nx * nP - P[0]));
    F[1] = sc * (-(nz * Q[0] - nx * Q[2]) + alpha * (ny * nP - P[1]));
    F[2] = sc * (-(nx * Q[1] - ny * Q[0]) + alpha * (nz * nP - P[2]));
#pragma unroll
    for (int ib = 0; ib < RB; ++ib)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[ib][c] = M::mac(Abuf[step % (kPre + 1)][ib], F[c], acc[ib][c]);
  }

  // 4. epilogue through LDS: [c][e][i] for this wave's three fields, then
  // contiguous stores per field.
  __syncthreads();
  T* so = su + h * (3 * 16 * Np);
#pragma unroll
  for (int ib = 0; ib < RB; ++ib)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * ib + M::row(q, r);
        if (i < Np) so[(c * 16 + e) * Np + i] = acc[ib][c][r];
      }
  __syncthreads();
  const int nv = ne * Np;
  constexpr int kOutIters = (16 * Np + 63) / 64;
  if constexpr (!RK) {
    T* __restrict__ rhs = static_cast<T*>(a.rhs);
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int it = 0; it < kOutIters; ++it) {
        const int idx = lane + 64 * it;
        if (idx < nv) rhs[(3 * h + c) * fs + k0 * Np + idx] = so[c * 16 * Np + idx];
      }
  } else {
    T* __restrict__ res = static_cast<T*>(a.res);
    T* __restrict__ uo = static_cast<T*>(a.u_out);
    const T ra = T(a.rk_a), rb = T(a.rk_b), dt = T(a.rk_dt);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T rv[kOutIters], uv[kOutIters];
#pragma unroll
      for (int it = 0; it < kOutIters; ++it) {
        const int idx = lane + 64 * it;
        const int64_t g = (3 * h + c) * fs + k0 * Np + idx;
        rv[it] = idx < nv ? res[g] : T(0);
        uv[it] = idx < nv ? u[g] : T(0);
      }
#pragma unroll
      for (int it = 0; it < kOutIters; ++it) {
        const int idx = lane + 64 * it;
        if (idx < nv) {
          const int64_t g = (3 * h + c) * fs + k0 * Np + idx;
          const T r = ra * rv[it] + dt * so[c * 16 * Np + idx];
          res[g] = r;
          uo[g] = uv[it] + rb * r;
        }
      }
    }
  }
}

template <int N, typename T>
hipError_t launch_rhs_mfma(const RhsArgs& a, hipStream_t s) {
  const int64_t nt = (a.K + 15) / 16;
  const unsigned grid = unsigned(8 * ((nt + 7) / 8));
  hipLaunchKernelGGL((rhs_mfma_kernel<N, T, false>), dim3(grid), dim3(128), 0, s, a);
  return hipGetLastError();
}

template <int N, typename T>
hipError_t launch_rk_mfma(const RhsArgs& a, hipStream_t s) {
  const int64_t nt = (a.K + 15) / 16;
  const unsigned grid = unsigned(8 * ((nt + 7) / 8));
  hipLaunchKernelGGL((rhs_mfma_kernel<N, T, true>), dim3(grid), dim3(128), 0, s, a);
  return hipGetLastError();
}

}  // namespace dgd
