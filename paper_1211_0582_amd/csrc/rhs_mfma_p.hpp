// Persistent matrix-core variant of the fused right-hand side ("mfma_p").
//
// Same arithmetic as rhs_mfma.hpp (one 16-element tile per pair of waves,
// E equations on one wave and H equations on the other, the contraction
// [Dr|Ds|Dt|LIFT] x [X; F] on MFMAs, the flux evaluated once per face node and
// staged in LDS), organised so that memory traffic overlaps the contraction:
//
//  * one workgroup per CU holds TPW tile slots (2 waves each) and walks a
//    range of tiles of its XCD, one tile per slot and iteration;
//  * the operator's MFMA fragments are copied to LDS once per workgroup, so
//    the volume and lift loops issue no global loads;
//  * at the start of the volume loop each slot issues the neighbour traces of
//    its current tile and then the fields of its next tile; the traces are
//    consumed by the flux phase, the fields are written to LDS at the top of
//    the next iteration.  Loads complete in issue order, so neither wait
//    blocks on anything issued later.
// MIX selects the contraction as in rhs_mfma.hpp: 0 native 16x16x4 MFMAs in
// T; 1..3 BF16 and 4..6 FP16 split products (T = float).
#pragma once

#include "rhs_mfma.hpp"

namespace dgd {

template <int N, typename T, int MIX>
struct PersistFrag {
  // native: [row block][depth step][lane] scalars; split: 16 bytes per lane
  static constexpr int bytes = MIX == 0 ? MfmaShape<N>::frag_count * int(sizeof(T)) : MixedShape<N>::frag_bytes;
};

template <int N, typename T, int MIX, int TPW>
struct PersistShared {
  using S = MfmaShape<N>;
  alignas(16) uint8_t frag[PersistFrag<N, T, MIX>::bytes];
  int16_t fmask[S::NF];
  alignas(16) uint8_t nbr[(4 * 24 * S::Nfp + 15) / 16 * 16];
  struct Slot {
    T su[S::TILE];                       // fields, then fluxes, then output staging
    int32_t code[16 * 4];
    T face[16 * 4 * 4];
  } slot[TPW];
};

// Tile slots per workgroup: 4, else 2 (an even number of waves per SIMD),
// whichever the LDS of one CU holds; 0 when neither fits or the
// accumulators do not fit the registers.
template <int N, typename T, int MIX>
constexpr int persist_tpw() {
  if (MfmaShape<N>::RB * 3 * 4 * sizeof(T) / 4 > 96) return 0;
  if (sizeof(PersistShared<N, T, MIX, 4>) <= 160 * 1024) return 4;
  if (sizeof(PersistShared<N, T, MIX, 2>) <= 160 * 1024) return 2;
  return 0;
}

template <int N, typename T, bool RK, int MIX, int TPW>
__global__ __launch_bounds__(128 * TPW) void rhs_mfma_p_kernel(RhsArgs a, int per_xcd_wgs) {
  using S = MfmaShape<N>;
  using M = Mfma16<T>;
  using acc_t = typename M::acc;
  constexpr int Np = S::Np, Nfp = S::Nfp, NF = S::NF, Np4 = S::Np4, RB = S::RB, KSV = S::KSV, KSL = S::KSL;
  constexpr int KS = S::KS, TS = S::TS, TQ = S::TQ;
  constexpr uint32_t sz = sizeof(T);
  constexpr uint32_t kOob = 0x80000000u;
  __shared__ PersistShared<N, T, MIX, TPW> sh;

  const int tid = threadIdx.x;
  const int sidx = tid >> 7;  // tile slot
  // Thread within the slot.  Made opaque at the top of every tile iteration
  // so that index arithmetic derived from it is recomputed per tile instead
  // of being hoisted out of the loop and held in (spilled) registers.
  int stid = tid & 127;
  auto& sl = sh.slot[sidx];
  const int64_t fs = a.fs;

  const __amdgpu_buffer_rsrc_t ru = make_rsrc(a.u, 6u * uint32_t(fs) * sz);
  const __amdgpu_buffer_rsrc_t rg = make_rsrc(a.geo, uint32_t(a.K) * kGeoStride * sz);
  const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.conn, uint32_t(a.K) * 16u);

  // Operator fragments and tables -> LDS, once.
  {
    constexpr int nvec = PersistFrag<N, T, MIX>::bytes / 16;
    const uint4* src = reinterpret_cast<const uint4*>(MIX == 0 ? a.ops_frag : a.ops_frag16);
    uint4* dst = reinterpret_cast<uint4*>(sh.frag);
    for (int i = tid; i < nvec; i += 128 * TPW) dst[i] = src[i];
    for (int i = tid; i < NF; i += 128 * TPW) sh.fmask[i] = int16_t(a.fmask[i]);
    constexpr int kNbrVec = (4 * 24 * Nfp + 15) / 16;
    for (int i = tid; i < kNbrVec; i += 128 * TPW)
      reinterpret_cast<uint4*>(sh.nbr)[i] = reinterpret_cast<const uint4*>(a.nbr)[i];
  }

  // Tile sequence: XCD x = b % 8 owns tiles [x per, (x+1) per); its
  // per_xcd_wgs workgroups interleave their slots over that range.  Every
  // slot runs the same number of iterations (the workgroup's barriers need
  // it); a slot past the end works on an empty tile (no loads, no stores).
  const int64_t nt = (a.K + 15) / 16;
  const int64_t per = (nt + 7) / 8;
  const int xcd = blockIdx.x % 8, wj = blockIdx.x / 8;
  const int64_t lstride = int64_t(per_xcd_wgs) * TPW;
  const int64_t iters = (per + lstride - 1) / lstride;
  auto tile_of = [&](int64_t it) -> int64_t {
    const int64_t lt = int64_t(wj) * TPW + sidx + it * lstride;
    const int64_t t = int64_t(xcd) * per + lt;
    return (lt < per && t < nt) ? t : -1;
  };
  auto live_of = [&](int64_t t) -> int { return t < 0 ? 0 : int((a.K - t * 16) < 16 ? (a.K - t * 16) : 16); };

  constexpr int kLoadIters = (16 * Np + 127) / 128;
  constexpr int kPairs = 16 * NF;
  constexpr int kFluxIters = (kPairs + 127) / 128;
  constexpr int kOutIters = (16 * Np + 63) / 64;

  // Registers carried across iterations: the next tile's fields and metadata.
  T tv[kLoadIters][6];
  T mr_next[9];
  int32_t code_next = -1;
  T face_next[4];
  auto load_tile = [&](int64_t t) {
    const int ne = live_of(t);
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
      const int idx = stid + 128 * it;
      const uint32_t vo = idx < ne * Np ? uint32_t(t * 16 * Np + idx) * sz : kOob;
#pragma unroll
      for (int c = 0; c < 6; ++c) tv[it][c] = buf_load<T>(ru, vo, uint32_t(c * fs) * sz);
    }
    const int el = stid & 15;
    const uint32_t go = el < ne ? uint32_t((t * 16 + el) * kGeoStride) * sz : kOob;
#pragma unroll
    for (int i = 0; i < 9; ++i) mr_next[i] = buf_load<T>(rg, go, i * sz);
    if (stid < 64) {
      const int ee = stid >> 2, f = stid & 3;
      const bool lv = ee < ne;
      const uint32_t fo = lv ? uint32_t((t * 16 + ee) * kGeoStride + 9 + 4 * f) * sz : kOob;
      const int32_t cf = __builtin_bit_cast(
          int32_t, __builtin_amdgcn_raw_buffer_load_b32(rc, lv ? uint32_t((t * 16 + ee) * 4 + f) * 4 : kOob, 0, 0));
      code_next = lv ? cf : -1;
#pragma unroll
      for (int i = 0; i < 4; ++i) face_next[i] = buf_load<T>(rg, fo, i * sz);
    }
  };
  auto store_tile = [&]() {  // registers -> LDS of this slot
#pragma unroll
    for (int it = 0; it < kLoadIters; ++it) {
      const int idx = stid + 128 * it;
      const int ee = idx / Np, jj = idx - ee * Np;
      if (idx < 16 * Np) {
#pragma unroll
        for (int c = 0; c < 6; ++c) sl.su[(c * Np4 + jj) * TS + ee] = tv[it][c];
      }
    }
    if constexpr (Np4 > Np) {
      for (int idx = stid; idx < 6 * (Np4 - Np) * 16; idx += 128) {
        const int c = idx / ((Np4 - Np) * 16), r = idx - c * ((Np4 - Np) * 16);
        sl.su[(c * Np4 + Np + r / 16) * TS + (r & 15)] = T(0);
      }
    }
    if (stid < 64) {
      sl.code[stid] = code_next;
      sl.face[4 * stid + 0] = face_next[0];
      sl.face[4 * stid + 1] = face_next[1];
      sl.face[4 * stid + 2] = face_next[2];
      sl.face[4 * stid + 3] = T(0.5) * face_next[3];
    }
  };

  load_tile(tile_of(0));
  const T alpha = T(a.alpha);
  for (int64_t it = 0; it < iters; ++it) {
    asm volatile("" : "+v"(stid));
    const int lane = stid & 63;
    const int h = stid >> 6;  // 0: E equations, 1: H equations
    const int e = lane & 15, q = lane >> 4;
    const int64_t t = tile_of(it);
    const int ne = live_of(t);
    const int64_t k0 = t < 0 ? 0 : t * 16;
    store_tile();
    T mr[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) mr[i] = mr_next[i];
    __syncthreads();

    // Issue: neighbour traces of this tile (interior: neighbour node; wall:
    // own node, mirrored below; dead lane: zero), then the next tile.
    T gx[kFluxIters][6];
#pragma unroll
    for (int fi = 0; fi < kFluxIters; ++fi) {
      const int pr = stid + 128 * fi;
      const int ee = pr & 15, m = pr >> 4;
      const int f = m / Nfp, jj = m - f * Nfp;
      uint32_t vo = kOob;
      if (pr < kPairs && ee < ne) {
        const int32_t cf = sl.code[4 * ee + f];
        vo = uint32_t(cf >= 0 ? int64_t(cf >> 5) * Np + sh.nbr[(f * 24 + (cf & 31)) * Nfp + jj]
                              : (k0 + ee) * Np + sh.fmask[m]) * sz;
      }
#pragma unroll
      for (int c = 0; c < 6; ++c) gx[fi][c] = buf_load<T>(ru, vo, uint32_t(c * fs) * sz);
    }
    load_tile(tile_of(it + 1));

    // Volume: operand X_d = m_d x V, V = H (h = 0) or -E (h = 1).
    acc_t acc[RB][3];
#pragma unroll
    for (int ib = 0; ib < RB; ++ib)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[ib][c] = acc_t{0, 0, 0, 0};
    const int vb = h ? 0 : 3;
    const T vs = h ? T(-1) : T(1);
    const int cb = h ? 3 : 0;
    if constexpr (MIX == 0) {
      const T* fr = reinterpret_cast<const T*>(sh.frag);
#pragma unroll
      for (int ks = 0; ks < KSV; ++ks) {
        const int jn = 4 * ks + q;
        T v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = vs * sl.su[((vb + c) * Np4 + jn) * TS + e];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          const int kg = d * KSV + ks;
          const T mx = mr[3 * d], my = mr[3 * d + 1], mz = mr[3 * d + 2];
          T X[3];
          X[0] = my * v[2] - mz * v[1];
          X[1] = mz * v[0] - mx * v[2];
          X[2] = mx * v[1] - my * v[0];
#pragma unroll
          for (int ib = 0; ib < RB; ++ib) {
            const T A = fr[(ib * KS + kg) * 64 + lane];
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[ib][c] = M::mac(A, X[c], acc[ib][c]);
          }
        }
      }
    } else {
      using X = MixedShape<N>;
      using H16 = typename std::conditional<(MIX <= 3), __bf16, _Float16>::type;
      using MM = Mfma16x16<H16>;
      using v4 = typename MM::v4;
      typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
      constexpr int NPROD = MIX <= 3 ? MIX : MIX - 3;
      constexpr int SV = X::SV, ST = X::ST;
      const uint4* fr = reinterpret_cast<const uint4*>(sh.frag);
#pragma unroll
      for (int s = 0; s < SV; ++s) {
        const int kap = 16 * s + 4 * q;
        float xv[3][4];
        if (kap < 3 * Np4) {
          const int d = kap / Np4, jn = kap - d * Np4;
          const float mx = mr[3 * d], my = mr[3 * d + 1], mz = mr[3 * d + 2];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const float v0 = vs * sl.su[((vb + 0) * Np4 + jn + v) * TS + e];
            const float v1 = vs * sl.su[((vb + 1) * Np4 + jn + v) * TS + e];
            const float v2 = vs * sl.su[((vb + 2) * Np4 + jn + v) * TS + e];
            xv[0][v] = my * v2 - mz * v1;
            xv[1][v] = mz * v0 - mx * v2;
            xv[2][v] = mx * v1 - my * v0;
          }
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v) xv[c][v] = 0.f;
        }
        v4 bh[3], bl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) split4<H16>(xv[c], bh[c], bl[c]);
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) {
          const uint4 w = fr[(ib * ST + s) * 64 + lane];
          const v4 ahi = __builtin_bit_cast(v4, u32x2{w.x, w.y});
          const v4 alo = __builtin_bit_cast(v4, u32x2{w.z, w.w});
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            acc[ib][c] = MM::mac(ahi, bh[c], acc[ib][c]);
            if constexpr (NPROD >= 2) acc[ib][c] = MM::mac(alo, bh[c], acc[ib][c]);
            if constexpr (NPROD >= 3) acc[ib][c] = MM::mac(ahi, bl[c], acc[ib][c]);
          }
        }
      }
    }

    // Flux of every (element, face node) pair once, into the LDS tile.
    T fl[kFluxIters][6];
#pragma unroll
    for (int fi = 0; fi < kFluxIters; ++fi) {
      const int pr = stid + 128 * fi;
      const int ee = pr & 15, m = pr >> 4;
      if (pr < kPairs) {
        const int f = m / Nfp;
        const int own = sh.fmask[m];
        const T se = sl.code[4 * ee + f] < 0 ? T(-1) : T(1);  // wall: E+ = -E-, H+ = H-
        T d[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
          const T em = sl.su[(c * Np4 + own) * TS + ee];
          d[c] = c < 3 ? em - se * gx[fi][c] : em - gx[fi][c];
        }
        const T* fr = &sl.face[4 * (4 * ee + f)];
        const T nx = fr[0], ny = fr[1], nz = fr[2], sc = fr[3];
        const T ndE = nx * d[0] + ny * d[1] + nz * d[2];
        const T ndH = nx * d[3] + ny * d[4] + nz * d[5];
        fl[fi][0] = sc * (-(ny * d[5] - nz * d[4]) + alpha * (nx * ndE - d[0]));
        fl[fi][1] = sc * (-(nz * d[3] - nx * d[5]) + alpha * (ny * ndE - d[1]));
        fl[fi][2] = sc * (-(nx * d[4] - ny * d[3]) + alpha * (nz * ndE - d[2]));
        fl[fi][3] = sc * ((ny * d[2] - nz * d[1]) + alpha * (nx * ndH - d[3]));
        fl[fi][4] = sc * ((nz * d[0] - nx * d[2]) + alpha * (ny * ndH - d[4]));
        fl[fi][5] = sc * ((nx * d[1] - ny * d[0]) + alpha * (nz * ndH - d[5]));
      }
    }
    __syncthreads();  // own-trace and volume reads of the tile are done
#pragma unroll
    for (int fi = 0; fi < kFluxIters; ++fi) {
      const int pr = stid + 128 * fi;
      const int ee = pr & 15, m = pr >> 4;
      if (pr < kPairs) {
#pragma unroll
        for (int c = 0; c < 6; ++c) sl.su[(c * NF + m) * TQ + ee] = fl[fi][c];
      }
    }
    __syncthreads();

    // Lifting: F (scaled by Fscale / 2) from the LDS flux tile.
    if constexpr (MIX == 0) {
      const T* fr = reinterpret_cast<const T*>(sh.frag);
#pragma unroll
      for (int ks = 0; ks < KSL; ++ks) {
        const int m = 4 * ks + q;
        const int kg = 3 * KSV + ks;
        T F[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) F[c] = sl.su[((cb + c) * NF + m) * TQ + e];
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) {
          const T A = fr[(ib * KS + kg) * 64 + lane];
#pragma unroll
          for (int c = 0; c < 3; ++c) acc[ib][c] = M::mac(A, F[c], acc[ib][c]);
        }
      }
    } else {
      using X = MixedShape<N>;
      using H16 = typename std::conditional<(MIX <= 3), __bf16, _Float16>::type;
      using MM = Mfma16x16<H16>;
      using v4 = typename MM::v4;
      typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
      constexpr int NPROD = MIX <= 3 ? MIX : MIX - 3;
      constexpr int SV = X::SV, SL = X::SL, ST = X::ST;
      const uint4* fr = reinterpret_cast<const uint4*>(sh.frag);
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int m = 16 * s + 4 * q;
        float fv[3][4];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v) fv[c][v] = (m + v < NF) ? sl.su[((cb + c) * NF + m + v) * TQ + e] : 0.f;
        v4 bh[3], bl[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) split4<H16>(fv[c], bh[c], bl[c]);
#pragma unroll
        for (int ib = 0; ib < RB; ++ib) {
          const uint4 w = fr[(ib * ST + SV + s) * 64 + lane];
          const v4 ahi = __builtin_bit_cast(v4, u32x2{w.x, w.y});
          const v4 alo = __builtin_bit_cast(v4, u32x2{w.z, w.w});
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            acc[ib][c] = MM::mac(ahi, bh[c], acc[ib][c]);
            if constexpr (NPROD >= 2) acc[ib][c] = MM::mac(alo, bh[c], acc[ib][c]);
            if constexpr (NPROD >= 3) acc[ib][c] = MM::mac(ahi, bl[c], acc[ib][c]);
          }
        }
      }
    }
    __syncthreads();  // flux reads done before the tile becomes output staging

    // Epilogue: accumulators -> LDS [c][e][i] -> contiguous stores per field.
    T* so = sl.su + h * (3 * 16 * Np);
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
    if constexpr (!RK) {
      T* __restrict__ rhs = static_cast<T*>(a.rhs);
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int oi = 0; oi < kOutIters; ++oi) {
          const int idx = lane + 64 * oi;
          if (idx < nv) rhs[(3 * h + c) * fs + k0 * Np + idx] = so[c * 16 * Np + idx];
        }
    } else {
      T* __restrict__ res = static_cast<T*>(a.res);
      T* __restrict__ uo = static_cast<T*>(a.u_out);
      const __amdgpu_buffer_rsrc_t rr = make_rsrc(a.res, 6u * uint32_t(fs) * sz);
      const T ra = T(a.rk_a), rb = T(a.rk_b), dt = T(a.rk_dt);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T rv[kOutIters], uv[kOutIters];
#pragma unroll
        for (int oi = 0; oi < kOutIters; ++oi) {
          const int idx = lane + 64 * oi;
          // The field offset depends on the role (a per-lane value to the
          // compiler), so it goes into the vector offset: a per-lane scalar
          // offset would make every load a waterfall loop.
          const uint32_t vo = idx < nv ? uint32_t((3 * h + c) * fs + k0 * Np + idx) * sz : kOob;
          rv[oi] = buf_load<T>(rr, vo, 0);
          uv[oi] = buf_load<T>(ru, vo, 0);
        }
#pragma unroll
        for (int oi = 0; oi < kOutIters; ++oi) {
          const int idx = lane + 64 * oi;
          if (idx < nv) {
            const int64_t g = (3 * h + c) * fs + k0 * Np + idx;
            const T r = ra * rv[oi] + dt * so[c * 16 * Np + idx];
            res[g] = r;
            uo[g] = uv[oi] + rb * r;
          }
        }
      }
    }
    __syncthreads();  // staging reads done before the next tile is stored
  }
}

// Persistent grid: as many workgroups as the CUs hold at once (one per CU for
// the shapes built here), a multiple of 8 so that each XCD gets the same
// number, and no more than the tiles need.
template <int N, typename T, bool RK, int MIX>
hipError_t launch_mfma_p(const RhsArgs& a, hipStream_t s) {
  constexpr int TPW = persist_tpw<N, T, MIX>();
  static int wgs_of[16] = {};
  int dev = 0;
  hipGetDevice(&dev);
  int& wgs = wgs_of[dev & 15];
  if (wgs == 0) {
    int cus = 0, occ = 0;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, rhs_mfma_p_kernel<N, T, RK, MIX, TPW>, 128 * TPW, 0);
    wgs = ((cus > 0 ? cus : 256) * (occ > 0 ? occ : 1) + 7) / 8 * 8;
  }
  const int64_t nt = (a.K + 15) / 16;
  const int64_t per = (nt + 7) / 8;
  const int64_t need = (per + TPW - 1) / TPW;  // workgroups per XCD that have a tile
  int per_xcd = wgs / 8;
  if (need < per_xcd) per_xcd = int(need > 0 ? need : 1);
  hipLaunchKernelGGL((rhs_mfma_p_kernel<N, T, RK, MIX, TPW>), dim3(8 * per_xcd), dim3(128 * TPW), 0, s, a, per_xcd);
  return hipGetLastError();
}

template <int N, typename T, int MIX = 0>
hipError_t launch_rhs_mfma_p(const RhsArgs& a, hipStream_t s) {
  return launch_mfma_p<N, T, false, MIX>(a, s);
}

template <int N, typename T, int MIX = 0>
hipError_t launch_rk_mfma_p(const RhsArgs& a, hipStream_t s) {
  return launch_mfma_p<N, T, true, MIX>(a, s);
}

}  // namespace dgd
