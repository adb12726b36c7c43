// C ABI of the DG library: setup, right-hand side, LSERK stepping, layout
// conversion.  Host setup (reference element, geometry, connectivity) is in
// host_refelem.cpp / host_mesh.cpp; the kernels are in rhs_valu.hpp and
// lserk.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "dg.h"
#include "dg_host.h"
#include "device_common.hpp"
#include "host_common.hpp"
#include "problem.hpp"
#include "tuning_table.hpp"

using namespace dgh;



namespace {

// Coefficients of the five-stage, fourth-order 2N-storage Runge-Kutta scheme
// of Carpenter and Kennedy (1994).
}  // namespace

const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

namespace {

// Round-to-nearest-even conversions to the 16-bit formats (host side).
uint16_t float_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);  // inf / nan (not produced here)
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
float bf16_to_float(uint16_t h) {
  const uint32_t u = uint32_t(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t float_to_f16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const float a = std::fabs(f);
  if (a >= 65520.0f) return uint16_t(sign | 0x7c00u);         // overflow -> inf
  if (a < 5.9604645e-8f * 0.5f) return uint16_t(sign);        // rounds to zero
  int ex;
  const double m = std::frexp(double(a), &ex);               // a = m 2^ex, m in [0.5, 1)
  int e16 = ex - 1 + 15;                                       // biased exponent of 1.x form
  double q;
  if (e16 <= 0) {                                              // subnormal: units of 2^-24
    q = std::nearbyint(double(a) * 16777216.0);
    return uint16_t(sign | uint32_t(q));                       // q may reach 1024 = smallest normal
  }
  q = std::nearbyint((m * 2.0 - 1.0) * 1024.0);                // 10-bit fraction, ties to even
  if (q >= 1024.0) {
    q = 0.0;
    ++e16;
  }
  if (e16 >= 31) return uint16_t(sign | 0x7c00u);
  return uint16_t(sign | (uint32_t(e16) << 10) | uint32_t(q));
}
float f16_to_float(uint16_t h) {
  const uint32_t e = (h >> 10) & 0x1fu, fr = h & 0x3ffu;
  float v;
  if (e == 0)
    v = std::ldexp(float(fr), -24);
  else if (e == 31)
    v = fr ? NAN : INFINITY;
  else
    v = std::ldexp(float(fr + 1024u), int(e) - 25);
  return (h & 0x8000u) ? -v : v;
}

dg_status hip_fail(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define DG_HIP(call, what)                       \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename T>
std::vector<T> cast_vec(const std::vector<double>& v) {
  return std::vector<T>(v.begin(), v.end());
}

void free_problem(dg_problem p) {
  if (!p) return;
  DeviceGuard guard(p->device);
  hipFree(p->d_geo);
  hipFree(p->d_conn);
  hipFree(p->d_ops);
  hipFree(p->d_nbr);
  hipFree(p->d_fmask);
  hipFree(p->d_frag);
  hipFree(p->d_frag16);
  hipFree(p->d_scratch);
  hipFree(p->d_mat);
  hipFree(p->d_mass);
  hipFree(p->d_weight);
  hipFree(p->d_partial);
  hipFree(p->d_tile_order);
  delete p;
}

// Material records (see kMatStride) from per-element eps and mu (NULL: 1).
std::vector<double> material_records(const HostMesh& hm, const double* eps, const double* mu, double alpha) {
  const int64_t K = hm.K;
  auto e_of = [&](int64_t k) { return eps ? eps[k] : 1.0; };
  auto m_of = [&](int64_t k) { return mu ? mu[k] : 1.0; };
  std::vector<double> rec(size_t(K) * dgd::kMatStride);
  for (int64_t k = 0; k < K; ++k) {
    double* r = &rec[size_t(k) * dgd::kMatStride];
    const double ek = e_of(k), mk = m_of(k), zm = std::sqrt(mk / ek);
    r[0] = 1.0 / ek;
    r[1] = 1.0 / mk;
    for (int f = 0; f < 4; ++f) {
      const int32_t c = hm.conn[size_t(k) * 4 + f];
      const double zp = c >= 0 ? std::sqrt(m_of(c >> 5) / e_of(c >> 5)) : zm;
      const double fsc = hm.face[(size_t(k) * 4 + f) * 4 + 3];
      r[2 + 4 * f] = fsc * zp / (zm + zp) / ek;
      r[3 + 4 * f] = fsc * (1.0 / zp) / (1.0 / zm + 1.0 / zp) / mk;
      r[4 + 4 * f] = alpha / zp;
      r[5 + 4 * f] = alpha * zp;
    }
  }
  return rec;
}

// Tile order: the 16-element tiles sorted by the Morton code of their
// centroids (bounding box quantised to 2^10 cells per axis), so that tiles
// processed at the same time are spatial neighbours.
dg_status upload_tile_order(dg_problem p) {
  const int64_t nt = (p->K + 15) / 16;
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  std::vector<double> cen(static_cast<size_t>(nt) * 3, 0.0);
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t k0 = t * 16, k1 = std::min<int64_t>(p->K, k0 + 16);
    for (int64_t k = k0; k < k1; ++k)
      for (int v = 0; v < 4; ++v)
        for (int d = 0; d < 3; ++d) cen[size_t(t) * 3 + d] += p->verts[size_t(k) * 12 + v * 3 + d];
    for (int d = 0; d < 3; ++d) {
      double& c = cen[size_t(t) * 3 + d];
      c /= double(4 * (k1 - k0));
      lo[d] = std::min(lo[d], c);
      hi[d] = std::max(hi[d], c);
    }
  }
  auto spread = [](uint64_t x) {  // 10 bits -> every third bit of 30
    x &= 0x3ff;
    x = (x | (x << 16)) & 0x30000ff;
    x = (x | (x << 8)) & 0x300f00f;
    x = (x | (x << 4)) & 0x30c30c3;
    x = (x | (x << 2)) & 0x9249249;
    return x;
  };
  std::vector<std::pair<uint64_t, int32_t>> key(static_cast<size_t>(nt));
  for (int64_t t = 0; t < nt; ++t) {
    uint64_t m = 0;
    for (int d = 0; d < 3; ++d) {
      const double w = hi[d] > lo[d] ? (cen[size_t(t) * 3 + d] - lo[d]) / (hi[d] - lo[d]) : 0.0;
      m |= spread(uint64_t(std::min(1023.0, std::max(0.0, w * 1024.0)))) << d;
    }
    key[size_t(t)] = {m, int32_t(t)};
  }
  std::stable_sort(key.begin(), key.end());
  std::vector<int32_t> order(static_cast<size_t>(nt));
  for (int64_t t = 0; t < nt; ++t) order[size_t(t)] = key[size_t(t)].second;
  DG_HIP(hipMalloc(&p->d_tile_order, order.size() * sizeof(int32_t)), "hipMalloc(tile order)");
  DG_HIP(hipMemcpy(p->d_tile_order, order.data(), order.size() * sizeof(int32_t), hipMemcpyHostToDevice),
         "upload tile order");
  return DG_OK;
}

// Diagnostics data: M = (V V^T)^-1, J eps and J mu per element, partial sums.
dg_status upload_diag(dg_problem p, const RefElement& re, const HostMesh& hm, const double* eps, const double* mu) {
  Mat M;
  if (!invert(matmul(re.V, transpose(re.V)), M)) return fail(DG_EUNSUPPORTED, "singular Vandermonde");
  std::vector<double> w(size_t(hm.K) * 2);
  for (int64_t k = 0; k < hm.K; ++k) {
    w[2 * k] = hm.J[k] * (eps ? eps[k] : 1.0);
    w[2 * k + 1] = hm.J[k] * (mu ? mu[k] : 1.0);
  }
  const int E = dgd::energy_tile(re.Np);
  const int64_t blocks = (hm.K + E - 1) / E;
  DG_HIP(hipMalloc(&p->d_mass, M.a.size() * sizeof(double)), "hipMalloc(mass matrix)");
  DG_HIP(hipMalloc(&p->d_weight, w.size() * sizeof(double)), "hipMalloc(element weights)");
  DG_HIP(hipMalloc(&p->d_partial, size_t(blocks) * sizeof(double)), "hipMalloc(partial sums)");
  DG_HIP(hipMemcpy(p->d_mass, M.a.data(), M.a.size() * sizeof(double), hipMemcpyHostToDevice), "upload mass");
  DG_HIP(hipMemcpy(p->d_weight, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice), "upload weights");
  return DG_OK;
}

template <typename T>
dg_status upload(dg_problem p, const RefElement& re, const HostMesh& hm, const std::vector<double>& mat) {
  const int Np = re.Np, NF = 4 * re.Nfp;
  const int64_t K = hm.K;
  // Geometry records.
  std::vector<T> geo(size_t(K) * dgd::kGeoStride);
  for (int64_t k = 0; k < K; ++k) {
    T* g = &geo[size_t(k) * dgd::kGeoStride];
    for (int i = 0; i < 9; ++i) g[i] = T(hm.metric[size_t(k) * 9 + i]);
    for (int i = 0; i < 16; ++i) g[9 + i] = T(hm.face[size_t(k) * 16 + i]);
  }
  // Operators, transposed so that lanes holding consecutive output rows read
  // consecutive addresses.
  std::vector<T> ops(size_t(3) * Np * Np + size_t(NF) * Np);
  const Mat* D[3] = {&re.Dr, &re.Ds, &re.Dt};
  for (int d = 0; d < 3; ++d)
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) ops[size_t(d) * Np * Np + size_t(j) * Np + i] = T((*D[d])(i, j));
  for (int i = 0; i < Np; ++i)
    for (int m = 0; m < NF; ++m) ops[size_t(3) * Np * Np + size_t(m) * Np + i] = T(re.LIFT(i, m));

  DG_HIP(hipMalloc(&p->d_geo, geo.size() * sizeof(T)), "hipMalloc(geometry)");
  DG_HIP(hipMalloc(&p->d_conn, hm.conn.size() * sizeof(int32_t)), "hipMalloc(connectivity)");
  DG_HIP(hipMalloc(&p->d_ops, ops.size() * sizeof(T)), "hipMalloc(operators)");
  // The orientation table is padded to a multiple of 16 bytes (kernels copy
  // it with 16-byte loads).
  std::vector<uint8_t> nbr(re.nbr_node);
  nbr.resize((nbr.size() + 15) / 16 * 16, 0);
  DG_HIP(hipMalloc(&p->d_nbr, nbr.size()), "hipMalloc(neighbour table)");
  DG_HIP(hipMalloc(&p->d_fmask, re.fmask.size() * sizeof(int32_t)), "hipMalloc(fmask)");
  DG_HIP(hipMalloc(&p->d_scratch, size_t(p->state_elems) * sizeof(T)), "hipMalloc(scratch)");
  DG_HIP(hipMemcpy(p->d_geo, geo.data(), geo.size() * sizeof(T), hipMemcpyHostToDevice), "upload geometry");
  DG_HIP(hipMemcpy(p->d_conn, hm.conn.data(), hm.conn.size() * sizeof(int32_t), hipMemcpyHostToDevice),
         "upload connectivity");
  DG_HIP(hipMemcpy(p->d_ops, ops.data(), ops.size() * sizeof(T), hipMemcpyHostToDevice), "upload operators");
  DG_HIP(hipMemcpy(p->d_nbr, nbr.data(), nbr.size(), hipMemcpyHostToDevice), "upload table");
  std::vector<int32_t> fm(re.fmask.begin(), re.fmask.end());
  DG_HIP(hipMemcpy(p->d_fmask, fm.data(), fm.size() * sizeof(int32_t), hipMemcpyHostToDevice), "upload fmask");
  DG_HIP(hipMemset(p->d_scratch, 0, size_t(p->state_elems) * sizeof(T)), "clear scratch");
  if (!mat.empty()) {
    const std::vector<T> mt = cast_vec<T>(mat);
    DG_HIP(hipMalloc(&p->d_mat, mt.size() * sizeof(T)), "hipMalloc(material)");
    DG_HIP(hipMemcpy(p->d_mat, mt.data(), mt.size() * sizeof(T), hipMemcpyHostToDevice), "upload material");
  }

  // MFMA A-fragments: row block ib, depth step kg, lane l holds
  // Op[16 ib + l % 16][depth column of (kg, l / 16)] with Op = [Dr|Ds|Dt|LIFT],
  // each direction's depth padded from Np to a multiple of 4 with zeros.  An
  // extra block RB repeats the last block in the 4-row MFMA layout, lane l
  // holding Op[16 (RB - 1) + l % 4][depth column of (kg, l / 16)].
  const int Np4 = (Np + 3) & ~3, RB = (Np + 15) / 16, KSV = Np4 / 4, KSL = NF / 4, KS = 3 * KSV + KSL;
  std::vector<T> frag(size_t(RB + 1) * KS * 64, T(0));
  for (int ib = 0; ib <= RB; ++ib)
    for (int kg = 0; kg < KS; ++kg)
      for (int l = 0; l < 64; ++l) {
        const int row = ib < RB ? 16 * ib + (l & 15) : 16 * (RB - 1) + (l & 3), q = l >> 4;
        double v = 0.0;
        if (row < Np) {
          if (kg < 3 * KSV) {
            const int j = 4 * (kg % KSV) + q;
            if (j < Np) v = (*D[kg / KSV])(row, j);
          } else {
            v = re.LIFT(row, 4 * (kg - 3 * KSV) + q);
          }
        }
        frag[(size_t(ib) * KS + kg) * 64 + l] = T(v);
      }
  DG_HIP(hipMalloc(&p->d_frag, frag.size() * sizeof(T)), "hipMalloc(fragments)");
  DG_HIP(hipMemcpy(p->d_frag, frag.data(), frag.size() * sizeof(T), hipMemcpyHostToDevice), "upload fragments");

  // 16x16x32 fragments of the split precisions: row block ib, step st, lane
  // l holds for v = 0..7 the heads (16 bytes) and, 1 KB further on, the tails
  // of Op[16 ib + l % 16][k], k = 8 (l / 16) + v within the step.  Steps
  // st = d KV + ks cover nodes 32 ks + k of direction d, steps 3 KV + ls the
  // lift's face nodes 32 ls + k; rows and columns past Np or NF are zero.
  if (p->precision >= DG_BF16X3) {
    const bool bf = p->precision == DG_BF16X3 || p->precision == DG_BF16 || p->precision == DG_BF16X2;
    const int KV = (Np + 31) / 32, KL = (NF + 31) / 32, ST = 3 * KV + KL;
    std::vector<uint16_t> f16(size_t(RB) * ST * 2 * 64 * 8, 0);
    for (int ib = 0; ib < RB; ++ib)
      for (int st = 0; st < ST; ++st)
        for (int l = 0; l < 64; ++l)
          for (int v = 0; v < 8; ++v) {
            const int row = 16 * ib + (l & 15), k = 8 * (l >> 4) + v;
            double val = 0.0;
            if (row < Np) {
              if (st < 3 * KV) {
                const int j = 32 * (st % KV) + k;
                if (j < Np) val = (*D[st / KV])(row, j);
              } else {
                const int m = 32 * (st - 3 * KV) + k;
                if (m < NF) val = re.LIFT(row, m);
              }
            }
            const uint16_t hi = bf ? float_to_bf16(float(val)) : float_to_f16(float(val));
            const float hv = bf ? bf16_to_float(hi) : f16_to_float(hi);
            const uint16_t lo = bf ? float_to_bf16(float(val - double(hv))) : float_to_f16(float(val - double(hv)));
            const size_t base = ((size_t(ib) * ST + st) * 2 * 64 + l) * 8;
            f16[base + v] = hi;
            f16[base + 64 * 8 + v] = lo;
          }
    DG_HIP(hipMalloc(&p->d_frag16, f16.size() * 2), "hipMalloc(16-bit fragments)");
    DG_HIP(hipMemcpy(p->d_frag16, f16.data(), f16.size() * 2, hipMemcpyHostToDevice), "upload 16-bit fragments");
  }
  return DG_OK;
}

}  // namespace

dgd::RhsArgs rhs_args(dg_problem p, const void* u, void* rhs) {
  dgd::RhsArgs a;
  a.u = u;
  a.rhs = rhs;
  a.geo = p->d_geo;
  a.conn = p->d_conn;
  a.mat = p->d_mat;
  a.ops = p->d_ops;
  a.ops_frag = p->d_frag;
  a.ops_frag16 = p->d_frag16;
  a.nbr = p->d_nbr;
  a.fmask = p->d_fmask;
  a.K = p->K;
  a.fs = p->fs;
  a.alpha = p->alpha;
  a.res = nullptr;
  a.u_out = nullptr;
  a.rk_a = a.rk_b = a.rk_dt = 0.0;
  // u read, rhs written.
  a.stream_out = 2 * p->state_elems * p->elem_bytes > kLastLevelCacheBytes;
  a.tile_order = p->use_tile_order ? p->d_tile_order : nullptr;
  return a;
}

dg_status check_rk_args(dg_problem p, const void* u, const void* res, double dt, int32_t nsteps) {
  if (!p || !u || !res) return fail(DG_EINVAL, "null argument");
  if (u == res) return fail(DG_EINVAL, "u and res must not alias");
  if (!aligned16(u) || !aligned16(res)) return fail(DG_EINVAL, "state arrays must be 16-byte aligned");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (!std::isfinite(dt)) return fail(DG_EINVAL, "dt must be finite");
  return DG_OK;
}

hipError_t launch_rhs(dg_problem p, const dgd::RhsArgs& a, hipStream_t s) {
  return p->rtc_fn ? launch_rtc(p, a, s) : p->ks.rhs(a, s);
}

dg_status rk_steps(dg_problem p, void* u, void* res, double dt, int32_t nsteps, void* buf, hipStream_t s) {
  const size_t bytes = size_t(p->state_elems) * p->elem_bytes;
  if (p->ks.rk && !p->rtc_fn) {
    // Fused stages: each stage reads one state buffer and writes the other
    // (neighbours still read the input during the stage), res in place.
    dgd::RhsArgs ra = rhs_args(p, u, nullptr);
    void* cur = u;
    void* nxt = buf;
    ra.res = res;
    ra.rk_dt = dt;
    // u and res read, res and the other state buffer written.
    ra.stream_out = 3 * p->state_elems * p->elem_bytes > kLastLevelCacheBytes;
    for (int32_t n = 0; n < nsteps; ++n)
      for (int st = 0; st < 5; ++st) {
        ra.u = cur;
        ra.u_out = nxt;
        ra.rk_a = kRkA[st];
        ra.rk_b = kRkB[st];
        hipError_t e = p->ks.rk(ra, s);
        if (e != hipSuccess) return hip_fail(e, "fused stage kernel launch");
        std::swap(cur, nxt);
      }
    if (cur != u) DG_HIP(hipMemcpyAsync(u, cur, bytes, hipMemcpyDeviceToDevice, s), "state copy");
    return DG_OK;
  }
  const dgd::RhsArgs ra = rhs_args(p, u, buf);
  for (int32_t n = 0; n < nsteps; ++n)
    for (int st = 0; st < 5; ++st) {
      hipError_t e = launch_rhs(p, ra, s);
      if (e != hipSuccess) return hip_fail(e, "rhs kernel launch");
      dgd::UpdateArgs ua;
      ua.u = u;
      ua.res = res;
      ua.rhs = buf;
      ua.n = p->K * p->Np;
      ua.fs = p->fs;
      ua.nfields = p->nfields;
      ua.a = kRkA[st];
      ua.b = kRkB[st];
      ua.dt = dt;
      e = dgd::launch_update(ua, p->precision, s);
      if (e != hipSuccess) return hip_fail(e, "update kernel launch");
    }
  return DG_OK;
}

namespace {
const char* const kVariantNames[dgd::kVariantCount] = {
    "valu", "mfma", "mfma_waves", "mfma_prefetch", "mfma_occupancy", "mfma_interleave", "mfma_lift", "mfma_tail"};
}  // namespace

extern "C" {

const char* dg_last_error(void) { return error_text(); }

dg_status dg_host_ref_nodes(int32_t N, double* r, double* s, double* t) {
  clear_error();
  if (!r || !s || !t) return fail(DG_EINVAL, "null output");
  const RefElement* re = ref_element(N);
  if (!re) return fail(DG_EUNSUPPORTED, "order N must be in 1..9");
  std::memcpy(r, re->r.data(), sizeof(double) * re->Np);
  std::memcpy(s, re->s.data(), sizeof(double) * re->Np);
  std::memcpy(t, re->t.data(), sizeof(double) * re->Np);
  return DG_OK;
}

dg_status dg_host_ref_operators(int32_t N, double* Dr, double* Ds, double* Dt, double* LIFT, int32_t* Fmask,
                                double* Mf) {
  clear_error();
  const RefElement* re = ref_element(N);
  if (!re) return fail(DG_EUNSUPPORTED, "order N must be in 1..9");
  const size_t nn = size_t(re->Np) * re->Np;
  if (Dr) std::memcpy(Dr, re->Dr.a.data(), nn * sizeof(double));
  if (Ds) std::memcpy(Ds, re->Ds.a.data(), nn * sizeof(double));
  if (Dt) std::memcpy(Dt, re->Dt.a.data(), nn * sizeof(double));
  if (LIFT) std::memcpy(LIFT, re->LIFT.a.data(), re->LIFT.a.size() * sizeof(double));
  if (Fmask)
    for (size_t i = 0; i < re->fmask.size(); ++i) Fmask[i] = re->fmask[i];
  if (Mf) std::memcpy(Mf, re->Mf.data(), re->Mf.size() * sizeof(double));
  return DG_OK;
}

dg_status dg_host_mesh(int32_t N, int64_t Nv, const double* VX, int64_t K, const int32_t* EToV,
                       const int8_t* face_bc, double* metric, double* J, double* face, double* sJ, int64_t* vmapP,
                       int32_t* conn) {
  clear_error();
  HostMesh hm;
  dg_status st = build_mesh(N, Nv, VX, K, EToV, face_bc, hm);
  if (st != DG_OK) return st;
  const RefElement* re = ref_element(N);
  if (!re) return fail(DG_EUNSUPPORTED, "reference element construction failed");
  if (metric) std::memcpy(metric, hm.metric.data(), hm.metric.size() * sizeof(double));
  if (J) std::memcpy(J, hm.J.data(), hm.J.size() * sizeof(double));
  if (face) std::memcpy(face, hm.face.data(), hm.face.size() * sizeof(double));
  if (sJ) std::memcpy(sJ, hm.sJ.data(), hm.sJ.size() * sizeof(double));
  if (conn) std::memcpy(conn, hm.conn.data(), hm.conn.size() * sizeof(int32_t));
  if (vmapP) {
    const int Np = re->Np, Nfp = re->Nfp;
    for (int64_t k = 0; k < K; ++k)
      for (int f = 0; f < 4; ++f) {
        const int32_t c = hm.conn[size_t(k) * 4 + f];
        for (int j = 0; j < Nfp; ++j) {
          int64_t v = -1;
          if (c >= 0) v = int64_t(c >> 5) * Np + re->nbr_node[(f * 24 + (c & 31)) * Nfp + j];
          vmapP[(size_t(k) * 4 + f) * Nfp + j] = v;
        }
      }
  }
  return DG_OK;
}

}  // extern "C"

dg_status setup_problem_impl(const dg_mesh_desc* desc, int nfields, bool system, dg_problem* out) {
  if (!desc || !out) return fail(DG_EINVAL, "null argument");
  if (desc->precision < DG_FP64 || desc->precision > DG_F16X2) return fail(DG_EINVAL, "precision out of range");
  if (!std::isfinite(desc->alpha)) return fail(DG_EINVAL, "alpha must be finite");
  if (desc->N < 1 || desc->N > kMaxOrder) return fail(DG_EUNSUPPORTED, "order N must be in 1..9");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) ndev = 0;
  if (desc->device < -1 || desc->device >= ndev) return fail(DG_EINVAL, "device out of range");
  bool material = false;
  if (desc->K >= 1)
    for (const double* v : {desc->eps, desc->mu})
      if (v)
        for (int64_t k = 0; k < desc->K; ++k) {
          if (!(std::isfinite(v[k]) && v[k] > 0.0))
            return fail(DG_EINVAL, "eps and mu must be finite and positive (element " + std::to_string(k) + ")");
          if (v[k] != 1.0) material = true;
        }
  if (material && desc->precision != DG_FP64 && desc->precision != DG_FP32)
    return fail(DG_EUNSUPPORTED, "eps or mu other than 1 needs precision FP64 or FP32");
  if (material && system) return fail(DG_EUNSUPPORTED, "a compiled system takes no eps or mu");
  HostMesh hm;
  dg_status st = build_mesh(desc->N, desc->Nv, desc->VX, desc->K, desc->EToV, desc->face_bc, hm);
  if (st != DG_OK) return st;
  const RefElement* re = ref_element(desc->N);
  if (!re) return fail(DG_EUNSUPPORTED, "reference element construction failed");
  {
    // The kernels address a state array with 32-bit buffer offsets and use
    // offset 2^31 as the "reads zero" sentinel, so an array must stay below it.
    const int64_t eb = desc->precision == DG_FP64 ? 8 : 4;
    const int64_t fs = ((desc->K * re->Np + 256 / eb - 1) / (256 / eb)) * (256 / eb);
    if (nfields * fs * eb >= (int64_t(1) << 31))
      return fail(DG_EUNSUPPORTED, "state array of 2 GiB or more (K * Np too large for this precision)");
  }

  // Validation is done: from here on the problem's device is current.
  int dev = desc->device;
  if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return fail(DG_EHIP, "hipGetDevice failed");
  DeviceGuard guard(dev);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  auto p = new dg_problem_s();
  p->N = desc->N;
  p->Np = re->Np;
  p->Nfp = re->Nfp;
  p->precision = desc->precision;
  p->elem_bytes = desc->precision == DG_FP64 ? 8 : 4;
  p->K = desc->K;
  p->alpha = desc->alpha;
  // Each field starts on a 256-byte boundary.
  const int64_t align = 256 / p->elem_bytes;
  p->fs = ((p->K * p->Np + align - 1) / align) * align;
  p->nfields = nfields;
  p->state_elems = int64_t(nfields) * p->fs;
  p->n_boundary = hm.n_boundary;
  p->material = material;
  // dt ~ dx / N^2 (Section 3's time-step restriction): 2 / ((N+1)^2 max Fscale)
  // for eps = mu = 1; with materials the wave speed 1 / sqrt(eps mu) of the
  // fastest element scales it.
  double cmax = 1.0;
  if (material) {
    cmax = 0.0;
    for (int64_t k = 0; k < desc->K; ++k)
      cmax = std::max(cmax, 1.0 / std::sqrt((desc->eps ? desc->eps[k] : 1.0) * (desc->mu ? desc->mu[k] : 1.0)));
  }
  p->dt_cfl1 = 2.0 / ((desc->N + 1.0) * (desc->N + 1.0) * hm.max_fscale * cmax);
  // Default kernel: the matrix-core variant where it is built, else the vector
  // one (a compiled system brings its own kernel).
  if (system) {
    p->variant = dgd::kVariantCount;  // "system"
    p->tile = 16;
  } else {
    p->variant = dgd::kVariantMfma;
    p->ks = dgd::kernels(desc->N, desc->precision, p->variant, material);
    if (!p->ks.rhs) {
      p->variant = dgd::kVariantValu;
      p->ks = dgd::kernels(desc->N, desc->precision, p->variant, material);
    }
    if (!p->ks.rhs) {
      delete p;
      return fail(DG_EUNSUPPORTED, "no kernel for this order and precision");
    }
    // The autotuner's winner for (precision, N, size bucket), where built.
    const int tv = material ? -1 : dgd::tuned_variant(desc->precision, desc->N, desc->K);
    if (tv >= 0) {
      const dgd::KernelSet k = dgd::kernels(desc->N, desc->precision, tv, false);
      if (k.rhs) {
        p->variant = tv;
        p->ks = k;
      }
    }
    p->tile = p->ks.tile;
  }
  p->device = dev;
  p->verts.resize(size_t(p->K) * 12);
  for (int64_t k = 0; k < p->K; ++k)
    for (int v = 0; v < 4; ++v)
      for (int d = 0; d < 3; ++d) p->verts[size_t(k) * 12 + v * 3 + d] = desc->VX[3 * int64_t(desc->EToV[4 * k + v]) + d];
  const std::vector<double> mat = material ? material_records(hm, desc->eps, desc->mu, desc->alpha) : std::vector<double>();
  st = (p->precision == DG_FP64) ? upload<double>(p, *re, hm, mat) : upload<float>(p, *re, hm, mat);
  if (st == DG_OK) st = upload_diag(p, *re, hm, desc->eps, desc->mu);
  if (st == DG_OK) st = upload_tile_order(p);
  if (st != DG_OK) {
    free_problem(p);
    return st;
  }
  *out = p;
  return DG_OK;
}

dg_status setup_problem(const dg_mesh_desc* desc, int nfields, bool system, dg_problem* out) {
  return setup_problem_impl(desc, nfields, system, out);
}

extern "C" dg_status dg_setup_mesh(const dg_mesh_desc* desc, dg_problem* out) {
  clear_error();
  return setup_problem_impl(desc, 6, false, out);
}

extern "C" {

dg_status dg_info_get(dg_problem p, dg_info* info) {
  clear_error();
  if (!p || !info) return fail(DG_EINVAL, "null argument");
  info->N = p->N;
  info->Np = p->Np;
  info->Nfp = p->Nfp;
  info->precision = p->precision;
  info->K = p->K;
  info->field_stride = p->fs;
  info->state_elems = p->state_elems;
  info->elem_bytes = p->elem_bytes;
  info->tile_elems = p->tile;
  info->dt_cfl1 = p->dt_cfl1;
  info->alpha = p->alpha;
  info->n_boundary_faces = p->n_boundary;
  info->variant = p->variant;
  info->nfields = p->nfields;
  return DG_OK;
}

int32_t dg_variant_count(void) { return dgd::kVariantCount; }

const char* dg_variant_name(int32_t v) { return (v >= 0 && v < dgd::kVariantCount) ? kVariantNames[v] : nullptr; }

dg_status dg_set_variant(dg_problem p, int32_t v) {
  clear_error();
  if (!p) return fail(DG_EINVAL, "null problem");
  if (p->rtc_fn) return fail(DG_EUNSUPPORTED, "a compiled system has exactly one kernel");
  if (v < 0 || v >= dgd::kVariantCount) return fail(DG_EINVAL, "variant out of range");
  dgd::KernelSet k = dgd::kernels(p->N, p->precision, v, p->material);
  if (!k.rhs) return fail(DG_EUNSUPPORTED, "variant not built for this order/precision");
  p->variant = v;
  p->ks = k;
  p->tile = k.tile;
  return DG_OK;
}

dg_status dg_set_tile_order(dg_problem p, int32_t enable) {
  clear_error();
  if (!p) return fail(DG_EINVAL, "null problem");
  p->use_tile_order = enable != 0;
  return DG_OK;
}

dg_status dg_rhs(dg_problem p, const void* u, void* rhs, void* stream) {
  clear_error();
  if (!p || !u || !rhs) return fail(DG_EINVAL, "null argument");
  if (u == rhs) return fail(DG_EINVAL, "u and rhs must not alias");
  if (!aligned16(u) || !aligned16(rhs)) return fail(DG_EINVAL, "state arrays must be 16-byte aligned");
  if (!p->ks.rhs && !p->rtc_fn) return fail(DG_EUNSUPPORTED, "no kernel for this order/precision");
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  hipError_t e = launch_rhs(p, rhs_args(p, u, rhs), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "rhs kernel launch");
  return DG_OK;
}

dg_status dg_time_rhs(dg_problem p, const void* u, void* rhs, int32_t warmup, int32_t reps, void* stream,
                      double* ms) {
  clear_error();
  if (!p || !u || !rhs || !ms) return fail(DG_EINVAL, "null argument");
  if (reps < 1 || warmup < 0) return fail(DG_EINVAL, "need reps >= 1 and warmup >= 0");
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int32_t i = 0; i < warmup; ++i) {
    dg_status st = dg_rhs(p, u, rhs, stream);
    if (st != DG_OK) return st;
  }
  hipEvent_t e0, e1;
  DG_HIP(hipEventCreate(&e0), "event create");
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    hipEventDestroy(e0);
    return hip_fail(e, "event create");
  }
  dg_status st = DG_OK;
  e = hipEventRecord(e0, s);
  for (int32_t i = 0; i < reps && st == DG_OK && e == hipSuccess; ++i) st = dg_rhs(p, u, rhs, stream);
  if (st == DG_OK && e == hipSuccess) e = hipEventRecord(e1, s);
  if (st == DG_OK && e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.f;
  if (st == DG_OK && e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != DG_OK) return st;
  if (e != hipSuccess) return hip_fail(e, "event timing");
  *ms = double(t) / reps;
  return DG_OK;
}

dg_status dg_rk_step(dg_problem p, void* u, void* res, double t, double dt, int32_t nsteps, void* stream) {
  clear_error();
  (void)t;
  dg_status st = check_rk_args(p, u, res, dt, nsteps);
  if (st != DG_OK) return st;
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  return rk_steps(p, u, res, dt, nsteps, p->d_scratch, static_cast<hipStream_t>(stream));
}

dg_status dg_energy(dg_problem p, const void* u, const void* ref, double* dev_out, void* stream) {
  clear_error();
  if (!p || !u || !dev_out) return fail(DG_EINVAL, "null argument");
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  hipError_t e = dgd::launch_energy(u, ref, p->d_mass, p->d_weight, p->K, p->fs, p->Np, p->nfields,
                                    p->precision == DG_FP64, p->d_partial, dev_out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "energy kernel launch");
  return DG_OK;
}

dg_status dg_pack(dg_problem p, const double* host_u, void* dev_u, void* stream) {
  clear_error();
  if (!p || !host_u || !dev_u) return fail(DG_EINVAL, "null argument");
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = p->K * p->Np;
  if (p->precision == DG_FP64) {
    std::vector<double> st(size_t(p->state_elems), 0.0);
    for (int c = 0; c < p->nfields; ++c) std::memcpy(&st[size_t(c * p->fs)], host_u + c * n, size_t(n) * sizeof(double));
    DG_HIP(hipMemcpyAsync(dev_u, st.data(), st.size() * sizeof(double), hipMemcpyHostToDevice, s), "pack copy");
    DG_HIP(hipStreamSynchronize(s), "pack sync");
  } else {
    std::vector<float> st(size_t(p->state_elems), 0.0f);
    for (int c = 0; c < p->nfields; ++c)
      for (int64_t i = 0; i < n; ++i) st[size_t(c * p->fs + i)] = float(host_u[c * n + i]);
    DG_HIP(hipMemcpyAsync(dev_u, st.data(), st.size() * sizeof(float), hipMemcpyHostToDevice, s), "pack copy");
    DG_HIP(hipStreamSynchronize(s), "pack sync");
  }
  return DG_OK;
}

dg_status dg_unpack(dg_problem p, const void* dev_u, double* host_u, void* stream) {
  clear_error();
  if (!p || !host_u || !dev_u) return fail(DG_EINVAL, "null argument");
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return hip_fail(guard.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = p->K * p->Np;
  if (p->precision == DG_FP64) {
    std::vector<double> st(size_t(p->state_elems));
    DG_HIP(hipMemcpyAsync(st.data(), dev_u, st.size() * sizeof(double), hipMemcpyDeviceToHost, s), "unpack copy");
    DG_HIP(hipStreamSynchronize(s), "unpack sync");
    for (int c = 0; c < p->nfields; ++c) std::memcpy(host_u + c * n, &st[size_t(c * p->fs)], size_t(n) * sizeof(double));
  } else {
    std::vector<float> st(size_t(p->state_elems));
    DG_HIP(hipMemcpyAsync(st.data(), dev_u, st.size() * sizeof(float), hipMemcpyDeviceToHost, s), "unpack copy");
    DG_HIP(hipStreamSynchronize(s), "unpack sync");
    for (int c = 0; c < p->nfields; ++c)
      for (int64_t i = 0; i < n; ++i) host_u[c * n + i] = double(st[size_t(c * p->fs + i)]);
  }
  return DG_OK;
}

dg_status dg_nodes(dg_problem p, double* host_xyz) {
  clear_error();
  if (!p || !host_xyz) return fail(DG_EINVAL, "null argument");
  const RefElement* re = ref_element(p->N);
  for (int64_t k = 0; k < p->K; ++k) {
    const double* X = &p->verts[size_t(k) * 12];
    for (int i = 0; i < p->Np; ++i) {
      const double l0 = -0.5 * (1.0 + re->r[i] + re->s[i] + re->t[i]);
      const double l1 = 0.5 * (1.0 + re->r[i]), l2 = 0.5 * (1.0 + re->s[i]), l3 = 0.5 * (1.0 + re->t[i]);
      for (int d = 0; d < 3; ++d)
        host_xyz[(size_t(k) * p->Np + i) * 3 + d] = l0 * X[d] + l1 * X[3 + d] + l2 * X[6 + d] + l3 * X[9 + d];
    }
  }
  return DG_OK;
}

void dg_destroy(dg_problem p) { free_problem(p); }

}  // extern "C"
