// LSERK stage update and the per-order kernel table.
//
// Stage s of the five-stage low-storage RK4 scheme (Carpenter & Kennedy):
//   res <- A_s res + dt rhs;  u <- u + B_s res.
// A pure streaming kernel (three reads, two writes per scalar): one thread
// per scalar, the six fields on the grid's y axis so no division is needed
// to skip the padding between fields.
#include "device_common.hpp"

namespace dgd {

#define DG_DECL(n) KernelSet kernels_n##n(int precision, int variant, bool material);
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
  switch (N) {
    case 1: return kernels_n1(p, v, m);
    case 2: return kernels_n2(p, v, m);
    case 3: return kernels_n3(p, v, m);
    case 4: return kernels_n4(p, v, m);
    case 5: return kernels_n5(p, v, m);
    case 6: return kernels_n6(p, v, m);
    case 7: return kernels_n7(p, v, m);
    case 8: return kernels_n8(p, v, m);
    case 9: return kernels_n9(p, v, m);
    default: return KernelSet{};
  }
}

// a = 0 (the first stage) does not read res, so its contents on entry never
// enter the update.
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
  const dim3 grid(unsigned(blocks), 6);
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
