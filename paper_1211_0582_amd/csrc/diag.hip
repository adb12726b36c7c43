// On-device diagnostics: the discrete energy of a state, or of its difference
// from a reference state, in the mass-matrix norm of Section 2 (M^k = J_k M
// on affine elements, Section 2.1), weighted by the material:
//   E(u - ref) = 1/2 sum_k J_k [ eps_k (E - E_ref)^T M (E - E_ref)
//                               + mu_k  (H - H_ref)^T M (H - H_ref) ].
// With ref = the interpolated exact solution, sqrt(2 E) is the L2 error of
// the discrete solution; with ref = NULL it is the energy that the upwind
// flux never increases, so long runs can check themselves on the device.
//
// The weights of fields 0..2 are J eps, of the others J mu (eps = mu = 1 for
// compiled systems, whose fields all take J).
//
// Two launches: blocks of 256 lanes each take a tile of E = 256 / Np whole
// elements (one element at N = 9), stage the fields of the tile in LDS
// and form, per (element, node i), (M v)_i v_i with M symmetric read as
// M[j][i] (consecutive lanes read consecutive addresses), all in binary64;
// each block writes its partial sum, and one block adds the partials in a
// fixed order, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "problem.hpp"

namespace dgd {

namespace {

constexpr int kDiagLanes = 256;

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kDiagLanes / 64; ++i) s += red[i];
  return s;
}

// Partial energy of the elements of block b (E elements per block).
template <typename T>
__global__ __launch_bounds__(kDiagLanes) void energy_partial_kernel(const T* __restrict__ u, const T* __restrict__ ref,
                                                                    const double* __restrict__ M,
                                                                    const double* __restrict__ w, int64_t K,
                                                                    int64_t fs, int Np, int E, int nfields,
                                                                    double* __restrict__ partial) {
  extern __shared__ double sv[];  // E * Np values of one field
  __shared__ double red[kDiagLanes / 64];
  const int tid = threadIdx.x;
  const int64_t k0 = int64_t(blockIdx.x) * E;
  const int ne = int((K - k0) < E ? (K - k0) : E);
  const int e = tid / Np, i = tid - e * Np;
  const bool live = e < ne;
  double acc = 0.0;
  for (int c = 0; c < nfields; ++c) {
    __syncthreads();
    for (int x = tid; x < ne * Np; x += kDiagLanes) {
      const int64_t g = c * fs + k0 * Np + x;
      sv[x] = double(u[g]) - (ref ? double(ref[g]) : 0.0);
    }
    __syncthreads();
    if (live) {
      const double* ve = sv + e * Np;
      double q = 0.0;
      for (int j = 0; j < Np; ++j) q += M[j * Np + i] * ve[j];
      acc += w[2 * (k0 + e) + (c < 3 ? 0 : 1)] * q * ve[i];
    }
  }
  const double s = block_sum(acc, red);
  if (tid == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kDiagLanes) void energy_final_kernel(const double* __restrict__ partial, int64_t n,
                                                                  double* __restrict__ out) {
  __shared__ double red[kDiagLanes / 64];
  double acc = 0.0;
  for (int64_t x = threadIdx.x; x < n; x += kDiagLanes) acc += partial[x];
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) *out = 0.5 * s;
}

}  // namespace

int energy_tile(int Np) { return Np >= kDiagLanes ? 1 : kDiagLanes / Np; }

hipError_t launch_energy(const void* u, const void* ref, const double* M, const double* w, int64_t K, int64_t fs,
                         int Np, int nfields, bool fp64, double* partial, double* out, hipStream_t s) {
  const int E = energy_tile(Np);
  const int64_t blocks = (K + E - 1) / E;
  const size_t lds = size_t(E) * Np * sizeof(double);
  if (fp64)
    hipLaunchKernelGGL(energy_partial_kernel<double>, dim3(unsigned(blocks)), dim3(kDiagLanes), lds, s,
                       static_cast<const double*>(u), static_cast<const double*>(ref), M, w, K, fs, Np, E, nfields,
                       partial);
  else
    hipLaunchKernelGGL(energy_partial_kernel<float>, dim3(unsigned(blocks)), dim3(kDiagLanes), lds, s,
                       static_cast<const float*>(u), static_cast<const float*>(ref), M, w, K, fs, Np, E, nfields,
                       partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(energy_final_kernel, dim3(1), dim3(kDiagLanes), 0, s, partial, blocks, out);
  return hipGetLastError();
}

}  // namespace dgd
