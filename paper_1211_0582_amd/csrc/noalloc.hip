// dg_rk_step_noalloc: LSERK stepping that allocates nothing, for callers that
// cannot call hipMalloc (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).  The second state buffer of the fused
// stages (or the right-hand side of the unfused ones), which dg_rk_step takes
// from the problem's own scratch, comes from a file-scope device array of
// DG_NOALLOC_SCRATCH_BYTES instead.
//
// The array's name is a host-side stand-in in host code: its device address
// is looked up once per device with hipGetSymbolAddress (on the entry point's
// first call on that device, with the device current) and only that address
// is passed to kernels and copies.  Each device holds its own copy until the
// process ends; every call on a device shares it and leaves its contents
// behind, so calls that overlap on one device race.  No kernel reads a part of
// it that the same call has not written (the stages write every node value
// before the next stage reads it; padding is never read), so nothing needs
// clearing between calls.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "dg.h"
#include "host_common.hpp"
#include "problem.hpp"

using namespace dgh;

static __device__ __align__(256) unsigned char scratch[DG_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device `dev`.
dg_status scratch_on(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DG_EUNSUPPORTED, "device ordinal beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(DG_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DG_OK;
}

}  // namespace

extern "C" dg_status dg_rk_step_noalloc(dg_problem p, void* u, void* res, double t, double dt, int32_t nsteps,
                                        void* stream) {
  clear_error();
  (void)t;
  dg_status st = check_rk_args(p, u, res, dt, nsteps);
  if (st != DG_OK) return st;
  const int64_t need = p->state_elems * p->elem_bytes;
  if (need > int64_t(DG_NOALLOC_SCRATCH_BYTES))
    return fail(DG_EUNSUPPORTED, "one state array takes " + std::to_string(need) + " bytes, more than the " +
                                     std::to_string(int64_t(DG_NOALLOC_SCRATCH_BYTES)) +
                                     "-byte static scratch of dg_rk_step_noalloc");
  DeviceGuard guard(p->device);
  if (guard.err != hipSuccess) return fail(DG_EHIP, std::string("hipSetDevice: ") + hipGetErrorString(guard.err));
  void* buf = nullptr;
  st = scratch_on(p->device, &buf);
  if (st != DG_OK) return st;
  return rk_steps(p, u, res, dt, nsteps, buf, static_cast<hipStream_t>(stream));
}
