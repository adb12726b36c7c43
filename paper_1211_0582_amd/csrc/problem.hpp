// Internal definition of a problem handle, shared by the C ABI sources.
#pragma once

#include <cstdint>
#include <vector>

#include "dg.h"
#include "device_common.hpp"

struct dg_problem_s {
  int N = 0, Np = 0, Nfp = 0, precision = 0, elem_bytes = 8, tile = 1, device = 0;
  int nfields = 6;                // fields per state array (6 for Maxwell; a compiled system's M)
  void* rtc_fn = nullptr;         // hipFunction_t of a run-time compiled system, else nullptr
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
  double* d_mass = nullptr;     // reference mass matrix M (Np x Np, binary64) for the diagnostics
  double* d_weight = nullptr;   // K x 2: J eps, J mu per element
  double* d_partial = nullptr;  // per-block partial sums of the diagnostics
  int32_t* d_tile_order = nullptr;  // Morton order of the 16-element tiles' centroids
  bool use_tile_order = true;
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

namespace dgd {
// Energy of u - ref (ref may be nullptr) into *out (device), see diag.hip.
int energy_tile(int Np);
hipError_t launch_energy(const void* u, const void* ref, const double* M, const double* w, int64_t K, int64_t fs,
                         int Np, int nfields, bool fp64, double* partial, double* out, hipStream_t s);
}  // namespace dgd

// Problem setup shared by dg_setup_mesh (Maxwell, 6 fields) and
// dg_setup_system (a compiled system of nfields fields, no built-in kernel).
dg_status setup_problem(const dg_mesh_desc* desc, int nfields, bool system, dg_problem* out);
// Right-hand side launch of p (built-in kernel or compiled system).
hipError_t launch_rhs(dg_problem p, const dgd::RhsArgs& a, hipStream_t s);
// Launch of a compiled system's kernel (rtc.cpp).
hipError_t launch_rtc(dg_problem p, const dgd::RhsArgs& a, hipStream_t s);

// Argument checks of dg_rk_step (sets the error text).
dg_status check_rk_args(dg_problem p, const void* u, const void* res, double dt, int32_t nsteps);
// nsteps LSERK steps of p with `buf` (one state array of device memory) as the
// second state buffer of the fused stages or the right-hand side of the
// unfused ones; the problem's device must be current.
dg_status rk_steps(dg_problem p, void* u, void* res, double dt, int32_t nsteps, void* buf, hipStream_t s);
