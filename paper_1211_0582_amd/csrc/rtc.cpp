// Run-time compiled systems (C ABI): the run-time code generation of
// Section 4.  A system's generated source (volume flux, numerical flux,
// boundary states; see rtc_kernel.hpp) is put in front of the kernel
// template, compiled with hipRTC for the problem's order, precision and the
// device's architecture, and loaded as a module; the kernel is then launched
// like the built-in ones.  Compiled modules are cached per (device,
// architecture, order, precision, source) for the life of the process.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "dg.h"
#include "host_common.hpp"
#include "problem.hpp"

using namespace dgh;

// Text of rtc_kernel.hpp, embedded at build time.
extern const char kRtcKernelSource[];

namespace {

// Host copy of dgrtc::Args (same layout on the host and the device: LP64).
struct RtcArgs {
  const void* u;
  void* rhs;
  const void* geo;
  const int32_t* conn;
  const void* frag;
  const uint8_t* nbr;
  const int32_t* fmask;
  int64_t K, fs;
  double alpha;
};

constexpr int kMaxFields = 12;

std::string full_source(const char* system_source, int N, int precision, int nfields) {
  std::string s = "#define DG_ORDER " + std::to_string(N) + "\n";
  s += precision == DG_FP64 ? "typedef double dg_real;\n" : "typedef float dg_real;\n";
  s += "#line 1 \"system\"\n";
  s += system_source;
  s += "\nstatic_assert(System::M == " + std::to_string(nfields) + ", \"System::M differs from nfields\");\n";
  s += "#line 1 \"rtc_kernel.hpp\"\n";
  s += kRtcKernelSource;
  return s;
}

// Compiles `src` for `arch`; on failure returns DG_EINVAL with the log.
dg_status compile(const std::string& src, const std::string& arch, std::vector<char>& code, std::string& log) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "dg_system.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS)
    return fail(DG_EHIP, "hiprtcCreateProgram failed");
  const std::string arch_opt = "--offload-arch=" + arch;
  // Packed FP32 instructions are switched off, as for every device compile.
  const char* opts[] = {arch_opt.c_str(), "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops"};
  const hiprtcResult r = hiprtcCompileProgram(prog, int(sizeof(opts) / sizeof(opts[0])), opts);
  size_t n = 0;
  hiprtcGetProgramLogSize(prog, &n);
  log.assign(n, '\0');
  if (n) hiprtcGetProgramLog(prog, &log[0]);
  while (!log.empty() && log.back() == '\0') log.pop_back();
  if (r != HIPRTC_SUCCESS) {
    hiprtcDestroyProgram(&prog);
    return fail(DG_EINVAL, "system source does not compile: " + log);
  }
  hiprtcGetCodeSize(prog, &n);
  code.assign(n, 0);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return DG_OK;
}

struct Module {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
};
std::mutex g_mutex;
std::map<std::tuple<int, std::string, int, int, std::string>, Module> g_modules;

dg_status module_for(int device, const char* system_source, int N, int precision, int nfields, hipFunction_t* fn) {
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return fail(DG_EHIP, std::string("hipGetDeviceProperties: ") + hipGetErrorString(e));
  const std::string arch = prop.gcnArchName;
  const auto key = std::make_tuple(device, arch, N, precision, std::string(system_source));
  std::lock_guard<std::mutex> lock(g_mutex);
  auto it = g_modules.find(key);
  if (it == g_modules.end()) {
    std::vector<char> code;
    std::string log;
    dg_status st = compile(full_source(system_source, N, precision, nfields), arch, code, log);
    if (st != DG_OK) return st;
    Module m;
    e = hipModuleLoadData(&m.mod, code.data());
    if (e != hipSuccess) return fail(DG_EHIP, std::string("hipModuleLoadData: ") + hipGetErrorString(e));
    e = hipModuleGetFunction(&m.fn, m.mod, "dg_rtc_rhs");
    if (e != hipSuccess) {
      hipModuleUnload(m.mod);
      return fail(DG_EHIP, std::string("hipModuleGetFunction: ") + hipGetErrorString(e));
    }
    it = g_modules.emplace(key, m).first;
  }
  *fn = it->second.fn;
  return DG_OK;
}

}  // namespace

hipError_t launch_rtc(dg_problem p, const dgd::RhsArgs& a, hipStream_t s) {
  RtcArgs r;
  r.u = a.u;
  r.rhs = a.rhs;
  r.geo = a.geo;
  r.conn = a.conn;
  r.frag = a.ops_frag;
  r.nbr = a.nbr;
  r.fmask = a.fmask;
  r.K = a.K;
  r.fs = a.fs;
  r.alpha = a.alpha;
  const int64_t nt = (a.K + 15) / 16;
  const unsigned grid = unsigned(8 * ((nt + 7) / 8));
  const unsigned waves = unsigned((p->nfields + 2) / 3);
  void* params[] = {&r};
  return hipModuleLaunchKernel(static_cast<hipFunction_t>(p->rtc_fn), grid, 1, 1, 64 * waves, 1, 1, 0, s, params,
                               nullptr);
}

extern "C" {

dg_status dg_system_compile(const char* system_source, int32_t nfields, int32_t N, int32_t precision,
                            const char* arch, char* log, int64_t log_size) {
  clear_error();
  if (!system_source || !arch) return fail(DG_EINVAL, "null argument");
  if (nfields < 1 || nfields > kMaxFields) return fail(DG_EINVAL, "nfields must be in 1..12");
  if (N < 1 || N > kMaxOrder) return fail(DG_EUNSUPPORTED, "order N must be in 1..9");
  if (precision != DG_FP64 && precision != DG_FP32) return fail(DG_EUNSUPPORTED, "compiled systems are FP64 or FP32");
  std::vector<char> code;
  std::string text;
  dg_status st = compile(full_source(system_source, N, precision, nfields), arch, code, text);
  if (log && log_size > 0) {
    const size_t n = std::min<size_t>(text.size(), size_t(log_size - 1));
    std::memcpy(log, text.data(), n);
    log[n] = '\0';
  }
  return st;
}

dg_status dg_setup_system(const dg_mesh_desc* desc, const char* system_source, int32_t nfields, dg_problem* out) {
  clear_error();
  if (!desc || !system_source || !out) return fail(DG_EINVAL, "null argument");
  if (nfields < 1 || nfields > kMaxFields) return fail(DG_EINVAL, "nfields must be in 1..12");
  if (desc->precision != DG_FP64 && desc->precision != DG_FP32)
    return fail(DG_EUNSUPPORTED, "compiled systems are FP64 or FP32");
  dg_problem p = nullptr;
  dg_status st = setup_problem(desc, nfields, true, &p);
  if (st != DG_OK) return st;
  DeviceGuard guard(p->device);
  hipFunction_t fn = nullptr;
  st = module_for(p->device, system_source, p->N, p->precision, nfields, &fn);
  if (st != DG_OK) {
    const std::string msg = error_text();
    dg_destroy(p);
    return fail(st, msg);
  }
  p->rtc_fn = fn;
  *out = p;
  return DG_OK;
}

}  // extern "C"
