// Exact-size kernels: the paper generates one routine per input size (its
// generated code is specific to each n, where the library it compares with is
// generic in size: Preliminary performance results paragraph).  Here the
// in-place FP64 kernel of the plan in use (variant, waves) is compiled at run
// time with hiprtc for the call's n_max as a compile-time constant, so that
// the tile loops, the padding masks and the tile count fold away; the code
// object is cached per (op, n, variant, waves) on the handle.  Instances of a
// call whose n differs from n_max take the generic branch compiled into the
// same kernel, so any batch stays correct.
//
// The kernel source is this library's own headers, found in the csrc
// directory next to the built library (../csrc relative to the .so) or in
// TLA_KERNEL_DIR.  Without them, or if compilation fails, the call uses the
// ahead-of-time generic kernel.
#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "tla_host.h"

namespace tla {

struct JitEntry {
  hipModule_t mod = nullptr;
  hipFunction_t fn = nullptr;
  bool failed = false;
};

struct JitState {
  std::map<long long, JitEntry> cache;
  std::string dir;
  int compiled = 0, failed = 0;
};

namespace {

long long jit_key(int op, int n, int var, int nw) { return (((long long)op * 4096 + n) * 16 + var) * 64 + nw; }

// directory of the kernel headers: TLA_KERNEL_DIR, else ../csrc next to this library
std::string kernel_dir() {
  if (const char* e = getenv("TLA_KERNEL_DIR")) return e;
  Dl_info info;
  if (dladdr(reinterpret_cast<const void*>(&kernel_dir), &info) && info.dli_fname) {
    std::string p = info.dli_fname;
    const size_t s = p.rfind('/');
    if (s != std::string::npos) return p.substr(0, s) + "/../csrc";
  }
  return "";
}

const char* body_name(int op) {
  return op == TLA_POTRF ? "potrf_inplace_body" : (op == TLA_TRSYL ? "trsyl_inplace_body" : "trlyap_inplace_body");
}

// Register budget (resident waves per SIMD) of the ahead-of-time kernel of
// the same plan (tla_large.hip): 4 for the one-wave Cholesky, 5 for the
// one-wave tile-wavefront Sylvester and Lyapunov, the compiler's choice else.
int waves_per_eu(int op, int var, int nw) {
  if (nw != 1) return 1;
  if (op == TLA_POTRF) return 4;
  return var == 0 ? 5 : 1;
}

std::string source(int op) {
  std::string s =
      "#include \"tla_inplace.hpp\"\n"
      "namespace tla {\n"
      "extern \"C\" __global__ __launch_bounds__(TLA_NW * 64) __attribute__((amdgpu_waves_per_eu(TLA_WPE)))\n"
      "void tla_exact(KArgs g) {\n"
      "  extern __shared__ __align__(16) unsigned char smem[];\n"
      "  Inst in = fetch_uniform(g, blockIdx.x);\n"
      "  if (in.n == TLA_N) {\n"
      "    in.n = TLA_N;  // the instance's order as a compile-time constant\n"
      "    BODY<TLA_NW, TLA_VAR>(g, in, smem);\n"
      "  } else {\n"
      "    BODY<TLA_NW, TLA_VAR>(g, in, smem);\n"
      "  }\n"
      "}\n"
      "}  // namespace tla\n";
  const std::string b = body_name(op);
  for (size_t p; (p = s.find("BODY")) != std::string::npos;) s.replace(p, 4, b);
  return s;
}

bool compile(JitState* js, int op, int n, int var, int nw, JitEntry& e) {
  if (js->dir.empty()) return false;
  const std::string src = source(op);
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "tla_exact.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) return false;
  const std::string inc = "-I" + js->dir;
  const std::string dn = "-DTLA_N=" + std::to_string(n), dv = "-DTLA_VAR=" + std::to_string(var),
                    dw = "-DTLA_NW=" + std::to_string(nw), de = "-DTLA_WPE=" + std::to_string(waves_per_eu(op, var, nw));
  // the same code generation switches as the library's own build
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", inc.c_str(), dn.c_str(), dv.c_str(), dw.c_str(), de.c_str()};
  const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    if (getenv("TLA_LOG")) {
      size_t ls = 0;
      hiprtcGetProgramLogSize(prog, &ls);
      std::vector<char> log(ls + 1, 0);
      hiprtcGetProgramLog(prog, log.data());
      fprintf(stderr, "tla: exact-size kernel (op %d, n %d) did not compile:\n%s\n", op, n, log.data());
    }
    hiprtcDestroyProgram(&prog);
    return false;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  std::vector<char> code(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  if (hipModuleLoadData(&e.mod, code.data()) != hipSuccess) return false;
  if (hipModuleGetFunction(&e.fn, e.mod, "tla_exact") != hipSuccess) {
    hipModuleUnload(e.mod);
    e.mod = nullptr;
    return false;
  }
  return true;
}

}  // namespace

void jit_release(tla_ctx* h) {
  JitState* js = h->jit;
  if (!js) return;
  for (auto& kv : js->cache)
    if (kv.second.mod) hipModuleUnload(kv.second.mod);
  delete js;
  h->jit = nullptr;
}

// Launches the exact-size kernel of (op, n_max, variant, waves) for the
// in-place FP64 plan; returns TLA_E_UNSUPPORTED (nothing launched) when no
// such kernel can be had, so that the caller takes the generic one.
tla_status jit_launch(tla_ctx* h, int op, int var, int nw, size_t lds, const KArgs& a) {
  if (!h->jit) {
    h->jit = new (std::nothrow) JitState();
    if (!h->jit) return TLA_E_NOMEM;
    h->jit->dir = kernel_dir();
  }
  JitState* js = h->jit;
  JitEntry& e = js->cache[jit_key(op, a.n_max, var, nw)];
  if (!e.fn) {
    if (e.failed) return TLA_E_UNSUPPORTED;
    if (!compile(js, op, a.n_max, var, nw, e)) {
      e.failed = true;
      ++js->failed;
      return TLA_E_UNSUPPORTED;
    }
    ++js->compiled;
  }
  KArgs args = a;
  void* params[] = {&args};
  if (hipModuleLaunchKernel(e.fn, a.batch, 1, 1, 64 * nw, 1, 1, (unsigned)lds, h->stream, params, nullptr) !=
      hipSuccess)
    return TLA_E_HIP;
  return TLA_OK;
}

}  // namespace tla

using namespace tla;

extern "C" tla_status tla_set_exact_size(tla_handle h, int mode) {
  if (!h || mode < 0 || mode > 2) return TLA_E_ARG;
  h->exact_size = mode;
  return TLA_OK;
}

extern "C" tla_status tla_exact_size_stats(tla_handle h, int* compiled, int* failed) {
  if (!h || !compiled || !failed) return TLA_E_ARG;
  *compiled = h->jit ? h->jit->compiled : 0;
  *failed = h->jit ? h->jit->failed : 0;
  return TLA_OK;
}
