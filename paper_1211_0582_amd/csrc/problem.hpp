// Internal definition of a problem handle, shared by the C ABI sources.
#pragma once

#include <cstdint>
#include <vector>

#include "dg.h"
#include "device_common.hpp"

struct dg_problem_s {
  int N = 0, Np = 0, Nfp = 0, precision = 0, elem_bytes = 8, tile = 1, device = 0;
  int64_t K = 0, fs = 0, state_elems = 0, n_boundary = 0;
  double alpha = 1.0, dt_cfl1 = 0.0;
  void* d_geo = nullptr;
  int32_t* d_conn = nullptr;
  void* d_ops = nullptr;
  uint8_t* d_nbr = nullptr;
  int32_t* d_fmask = nullptr;
  void* d_frag = nullptr;     // MFMA A-fragments of [Dr|Ds|Dt|LIFT]
  void* d_frag16 = nullptr;   // the same split into 16-bit heads and tails (split precisions)
  void* d_scratch = nullptr;  // rhs buffer (unfused stepping) / second state buffer (fused)
  void* d_mat = nullptr;      // material records (K x kMatStride), nullptr for eps = mu = 1
  bool material = false;
  std::vector<double> verts;  // K x 4 x 3 vertex coordinates (for dg_nodes)
  int variant = 0;
  dgd::KernelSet ks;
};

// Coefficients of the five-stage, fourth-order 2N-storage Runge-Kutta scheme
// of Carpenter and Kennedy (1994).
extern const double kRkA[5];
extern const double kRkB[5];

// Last-level cache of the device (MI355X: 256 MB Infinity Cache).  An FP64
// launch whose arrays exceed it writes its outputs with streaming stores: they
// could not stay resident for the next launch, and such stores retire sooner.
constexpr int64_t kLastLevelCacheBytes = int64_t(256) << 20;

// The kernels write state arrays with 16-byte stores.
inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Makes `device` current for the guard's lifetime and restores the caller's
// current device afterwards (every call on a problem runs on its device).
struct DeviceGuard {
  int prev = -1, dev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int d) : dev(d) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  }
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
};

// Kernel arguments of a right-hand-side evaluation of p.
dgd::RhsArgs rhs_args(dg_problem p, const void* u, void* rhs);
