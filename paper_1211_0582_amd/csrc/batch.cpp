// Batched time stepping of many independent problems (C ABI).
//
// Problems are grouped by order N.  A Runge-Kutta stage is one launch per
// group of the fused matrix-core stage kernel over a work list of (problem,
// tile) pairs; per-problem pointers, sizes and time steps live in a device
// descriptor table that each call refreshes.  A whole step (5 stages x
// groups) is captured once into a graph per buffer parity and replayed, so
// the host issues one graph launch per step however many problems there
// are -- the regime where the paper notes that the host's submission rate
// (about 1000 Hz) stops being enough for small per-problem work.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "dg.h"
#include "device_common.hpp"
#include "host_common.hpp"
#include "problem.hpp"

using namespace dgh;

struct dg_batch_s {
  std::vector<dg_problem> problems;
  struct Group {
    int N = 0;
    int2* d_items = nullptr;
    int64_t n_items = 0;
    dgd::BatchLauncher launch = nullptr;
    const void* frag = nullptr;
    const void* frag16 = nullptr;
    const uint8_t* nbr = nullptr;
    const int32_t* fmask = nullptr;
  };
  std::vector<Group> groups;
  dgd::BatchProblem* d_table = nullptr;
  std::vector<dgd::BatchProblem> table;
  bool table_valid = false;
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // step starting at parity 0 / 1
  int precision = 0, device = 0;
  int stream_out = 0;  // streaming stores: the step's state arrays exceed the last-level cache
};

namespace {

dg_status hip_err(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define DG_HIP(call, what)                             \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_err(e_, what);    \
  } while (0)

void free_batch(dg_batch b) {
  if (!b) return;
  DeviceGuard guard(b->problems.empty() ? b->device : b->problems[0]->device);
  for (int i = 0; i < 2; ++i)
    if (b->graph[i]) hipGraphExecDestroy(b->graph[i]);
  for (auto& g : b->groups) hipFree(g.d_items);
  hipFree(b->d_table);
  for (dg_problem p : b->problems) dg_destroy(p);
  delete b;
}

// Stage s of a step whose first stage reads buffer `parity0`.
dg_status launch_step(dg_batch b, int parity0, hipStream_t s) {
  for (int st = 0; st < 5; ++st)
    for (auto& g : b->groups) {
      dgd::BatchArgs a;
      a.probs = b->d_table;
      a.items = g.d_items;
      a.n_items = g.n_items;
      a.ops_frag = g.frag;
      a.ops_frag16 = g.frag16;
      a.nbr = g.nbr;
      a.fmask = g.fmask;
      a.parity = (parity0 + st) & 1;
      a.rk_a = kRkA[st];
      a.rk_b = kRkB[st];
      a.stream_out = b->stream_out;
      hipError_t e = g.launch(a, s);
      if (e != hipSuccess) return hip_err(e, "batched stage launch");
    }
  return DG_OK;
}

dg_status build_graphs(dg_batch b) {
  hipStream_t cs;
  DG_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  dg_status st = DG_OK;
  for (int par = 0; par < 2 && st == DG_OK; ++par) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      st = hip_err(e, "begin capture");
      break;
    }
    dg_status ls = launch_step(b, par, cs);
    e = hipStreamEndCapture(cs, &g);
    if (ls != DG_OK) {
      st = ls;
    } else if (e != hipSuccess) {
      st = hip_err(e, "end capture");
    } else {
      e = hipGraphInstantiate(&b->graph[par], g, nullptr, nullptr, 0);
      if (e != hipSuccess) st = hip_err(e, "graph instantiate");
    }
    if (g) hipGraphDestroy(g);
  }
  hipStreamDestroy(cs);
  return st;
}

}  // namespace

extern "C" {

dg_status dg_setup_batch(int32_t n, const dg_mesh_desc* descs, dg_batch* out) {
  clear_error();
  if (n < 1 || !descs || !out) return fail(DG_EINVAL, "need n >= 1 and non-null descs/out");
  for (int32_t i = 1; i < n; ++i) {
    if (descs[i].precision != descs[0].precision) return fail(DG_EINVAL, "all problems of a batch share one precision");
    if (descs[i].device != descs[0].device) return fail(DG_EINVAL, "all problems of a batch share one device");
  }
  auto b = new dg_batch_s();
  b->precision = descs[0].precision;
  for (int32_t i = 0; i < n; ++i) {
    dg_problem p = nullptr;
    dg_status st = dg_setup_mesh(&descs[i], &p);
    if (st == DG_OK && p->material) {
      dg_destroy(p);
      st = fail(DG_EUNSUPPORTED, "batched problems must have eps = mu = 1");
    } else if (st == DG_OK && !p->ks.batch) {
      // the batched stage exists for the matrix-core kernel only
      if (dg_set_variant(p, dgd::kVariantMfma) != DG_OK || !p->ks.batch) {
        dg_destroy(p);
        st = fail(DG_EUNSUPPORTED, "problem " + std::to_string(i) + ": no batched kernel for its order and precision");
      }
    }
    if (st != DG_OK) {
      std::string msg = std::string("problem ") + std::to_string(i) + ": " + error_text();
      free_batch(b);
      return fail(st, msg);
    }
    b->problems.push_back(p);
  }
  b->device = b->problems[0]->device;
  DeviceGuard guard(b->device);
  // One step cycles through every problem's u, res and second state buffer.
  int64_t step_bytes = 0;
  for (dg_problem p : b->problems) step_bytes += 3 * p->state_elems * p->elem_bytes;
  b->stream_out = step_bytes > kLastLevelCacheBytes;
  std::map<int, std::vector<int2>> items;
  for (int32_t i = 0; i < n; ++i) {
    dg_problem p = b->problems[i];
    const int64_t nt = (p->K + 15) / 16;
    for (int64_t t = 0; t < nt; ++t) items[p->N].push_back(make_int2(i, int(t)));
  }
  for (auto& kv : items) {
    dg_batch_s::Group g;
    g.N = kv.first;
    g.n_items = int64_t(kv.second.size());
    dg_problem first = nullptr;
    for (dg_problem p : b->problems)
      if (p->N == g.N) {
        first = p;
        break;
      }
    g.launch = first->ks.batch;
    g.frag = first->d_frag;
    g.frag16 = first->d_frag16;
    g.nbr = first->d_nbr;
    g.fmask = first->d_fmask;
    hipError_t e = hipMalloc(&g.d_items, kv.second.size() * sizeof(int2));
    if (e == hipSuccess)
      e = hipMemcpy(g.d_items, kv.second.data(), kv.second.size() * sizeof(int2), hipMemcpyHostToDevice);
    b->groups.push_back(g);
    if (e != hipSuccess) {
      dg_status st = hip_err(e, "batch work list");
      free_batch(b);
      return st;
    }
  }
  b->table.resize(size_t(n));
  hipError_t e = hipMalloc(&b->d_table, sizeof(dgd::BatchProblem) * size_t(n));
  if (e != hipSuccess) {
    dg_status st = hip_err(e, "batch table");
    free_batch(b);
    return st;
  }
  *out = b;
  return DG_OK;
}

dg_status dg_batch_problem(dg_batch b, int32_t i, dg_problem* p) {
  clear_error();
  if (!b || !p) return fail(DG_EINVAL, "null argument");
  if (i < 0 || i >= int32_t(b->problems.size())) return fail(DG_EINVAL, "problem index out of range");
  *p = b->problems[size_t(i)];
  return DG_OK;
}

dg_status dg_rk_step_batch(dg_batch b, void* const* u, void* const* res, const double* dt, int32_t nsteps,
                           int32_t mode, void* stream) {
  clear_error();
  if (!b || !u || !res || !dt) return fail(DG_EINVAL, "null argument");
  if (nsteps < 0) return fail(DG_EINVAL, "nsteps must be >= 0");
  if (mode < 0 || mode > 2) return fail(DG_EINVAL, "mode must be 0, 1 or 2");
  const size_t n = b->problems.size();
  for (size_t i = 0; i < n; ++i) {
    if (!u[i] || !res[i] || u[i] == res[i]) return fail(DG_EINVAL, "problem " + std::to_string(i) + ": bad u/res");
    if (!aligned16(u[i]) || !aligned16(res[i]))
      return fail(DG_EINVAL, "problem " + std::to_string(i) + ": state arrays must be 16-byte aligned");
    if (!std::isfinite(dt[i])) return fail(DG_EINVAL, "problem " + std::to_string(i) + ": dt not finite");
  }
  DeviceGuard guard(b->device);
  if (guard.err != hipSuccess) return hip_err(guard.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (mode == 2) {  // one launch per problem and stage
    for (size_t i = 0; i < n; ++i) {
      dg_status st = dg_rk_step(b->problems[i], u[i], res[i], 0.0, dt[i], nsteps, stream);
      if (st != DG_OK) return st;
    }
    return DG_OK;
  }
  std::vector<dgd::BatchProblem> table(n);
  for (size_t i = 0; i < n; ++i) {
    dg_problem p = b->problems[i];
    dgd::BatchProblem& d = table[i];
    d.u = u[i];
    d.res = res[i];
    d.u2 = p->d_scratch;
    d.geo = p->d_geo;
    d.conn = p->d_conn;
    d.K = p->K;
    d.fs = p->fs;
    d.dt = dt[i];
    d.alpha = p->alpha;
  }
  // Upload only when pointers or time steps changed.  The source is pageable
  // host memory owned by the batch: the runtime stages such a copy before
  // hipMemcpyAsync returns, so the next call may overwrite it.
  if (!b->table_valid || std::memcmp(table.data(), b->table.data(), sizeof(dgd::BatchProblem) * n) != 0) {
    b->table = table;
    DG_HIP(hipMemcpyAsync(b->d_table, b->table.data(), sizeof(dgd::BatchProblem) * n, hipMemcpyHostToDevice, s),
           "batch table upload");
    b->table_valid = true;
  }
  if (mode == 0 && !b->graph[0]) {
    dg_status st = build_graphs(b);
    if (st != DG_OK) return st;
  }
  int parity = 0;
  for (int32_t k = 0; k < nsteps; ++k) {
    if (mode == 0) {
      DG_HIP(hipGraphLaunch(b->graph[parity], s), "graph launch");
    } else {
      dg_status st = launch_step(b, parity, s);
      if (st != DG_OK) return st;
    }
    parity ^= 1;  // five stages: the state ends in the other buffer
  }
  if (parity)
    for (size_t i = 0; i < n; ++i) {
      dg_problem p = b->problems[i];
      DG_HIP(hipMemcpyAsync(u[i], p->d_scratch, size_t(p->state_elems) * p->elem_bytes, hipMemcpyDeviceToDevice, s),
             "state copy");
    }
  return DG_OK;
}

void dg_destroy_batch(dg_batch b) { free_batch(b); }

}  // extern "C"
