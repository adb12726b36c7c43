// LSERK stage update and the per-order kernel table.
//
// Stage s of the five-stage low-storage RK4 scheme (Carpenter & Kennedy):
//   res <- A_s res + dt rhs;  u <- u + B_s res.
// A pure streaming kernel (three reads, two writes per scalar): one thread
// per scalar, the fields on the grid's y axis so no division is needed to
// skip the padding between fields.
#include "device_common.hpp"

namespace dgd {

#define DG_DECL(n)                                             \
  KernelSet kernels_n##n##_g0(int precision, int variant, bool material); \
  KernelSet kernels_n##n##_g1(int precision, int variant, bool material); \
  KernelSet kernels_n##n##_g2(int precision, int variant, bool material);
DG_DECL(1)
DG_DECL(2)
DG_DECL(3)
DG_DECL(4)
DG_DECL(5)
DG_DECL(6)
DG_DECL(7)
DG_DECL(8)
DG_DECL(9)
#undef DG_DECL

KernelSet kernels(int N, int p, int v, bool m) {
  if (v < 0 || v >= kVariantCount) return KernelSet{};
#define DG_CASE(n)                                                     \
  case n:                                                              \
    return p == 0 ? kernels_n##n##_g0(p, v, m) : p == 1 ? kernels_n##n##_g1(p, v, m) : kernels_n##n##_g2(p, v, m);
  switch (N) {
    DG_CASE(1)
    DG_CASE(2)
    DG_CASE(3)
    DG_CASE(4)
    DG_CASE(5)
    DG_CASE(6)
    DG_CASE(7)
    DG_CASE(8)
    DG_CASE(9)
    default: return KernelSet{};
  }
#undef DG_CASE
}

template <typename T>
__global__ __launch_bounds__(256) void lserk_update_kernel(T* __restrict__ u, T* __restrict__ res,
                                                           const T* __restrict__ rhs, int64_t n, int64_t fs,
                                                           T a, T b, T dt) {
  const int64_t off = int64_t(blockIdx.y) * fs;
  const bool first = a == T(0);
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const T r = first ? dt * rhs[off + i] : a * res[off + i] + dt * rhs[off + i];
    res[off + i] = r;
    u[off + i] += b * r;
  }
}

hipError_t launch_update(const UpdateArgs& a, int precision, hipStream_t s) {
  int64_t blocks = (a.n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  const dim3 grid(unsigned(blocks), unsigned(a.nfields));
  if (precision == 0)
    hipLaunchKernelGGL(lserk_update_kernel<double>, grid, dim3(256), 0, s, static_cast<double*>(a.u),
                       static_cast<double*>(a.res), static_cast<const double*>(a.rhs), a.n, a.fs, a.a, a.b,
                       a.dt);
  else
    hipLaunchKernelGGL(lserk_update_kernel<float>, grid, dim3(256), 0, s, static_cast<float*>(a.u),
                       static_cast<float*>(a.res), static_cast<const float*>(a.rhs), a.n, a.fs, float(a.a),
                       float(a.b), float(a.dt));
  return hipGetLastError();
}

}  // namespace dgd
