// C ABI of libtla: handles, argument checks, plan selection and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tla.h"
#include "tla_host.h"

using namespace tla;

// ------------------------------------------------------------------ plans
namespace tla {

static const char* kVarNames[3][5] = {
    {"right-looking", "left-looking", "bordered", nullptr, nullptr},
    {"tile-wavefront", "rows-lazy", "rows-eager", "cols-lazy", "cols-eager"},
    {"tile-wavefront", "rows-lazy", "right-looking", nullptr, nullptr}};
static const int kNumVar[3] = {3, 5, 3};

int num_variants(int op) { return (op >= 0 && op < 3) ? kNumVar[op] : 0; }

bool plan_valid(int op, const tla_plan& p) {
  if (op < 0 || op > 2) return false;
  if (p.variant < 0 || p.variant >= kNumVar[op]) return false;
  if (p.tile != 8 && p.tile != 16) return false;
  if (p.engine != 0 && p.engine != 1) return false;
  if (p.tile == 8 && p.engine == 1) return false;
  if (p.waves != 1 && p.waves != 2 && p.waves != 4) return false;
  return true;
}

// candidates: variant x (tile, engine) x waves
int num_candidates(int op) { return num_variants(op) * kNumTE * kNumNW; }
bool candidate(int op, int i, tla_plan* p) {
  if (i < 0 || i >= num_candidates(op)) return false;
  const int nwi = i % kNumNW, te = (i / kNumNW) % kNumTE, var = i / (kNumNW * kNumTE);
  p->variant = var;
  p->tile = te_tile(te);
  p->engine = te == 2 ? 1 : 0;
  p->waves = nwi == 0 ? 1 : (nwi == 1 ? 2 : 4);
  return true;
}

tla_plan default_plan(int op, int n, int prec) {
  (void)prec;
  tla_plan p;
  p.variant = 0;
  p.tile = 16;
  p.engine = 1;
  p.waves = n <= 16 ? 1 : (n <= 32 ? 2 : 4);
  (void)op;
  return p;
}

}  // namespace tla

// ----------------------------------------------------------- utilities
#define TLA_HIP(x)                                   \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) {                          \
      if (getenv("TLA_LOG"))                         \
        fprintf(stderr, "tla: %s failed: %s\n", #x, hipGetErrorString(e_)); \
      return TLA_E_HIP;                              \
    }                                                \
  } while (0)

static int g_lds_limit = 160 * 1024;

extern "C" const char* tla_status_string(tla_status s) {
  switch (s) {
    case TLA_OK: return "ok";
    case TLA_E_ARG: return "invalid argument";
    case TLA_E_HIP: return "HIP runtime error";
    case TLA_E_NOMEM: return "out of memory";
    case TLA_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

extern "C" tla_status tla_create(tla_handle* h, int device) {
  if (!h) return TLA_E_ARG;
  *h = nullptr;
  int count = 0;
  TLA_HIP(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(device));
  hipDeviceProp_t prop;
  TLA_HIP(hipGetDeviceProperties(&prop, device));
  g_lds_limit = (int)prop.sharedMemPerBlock;
  tla_ctx* c = new (std::nothrow) tla_ctx();
  if (!c) return TLA_E_NOMEM;
  c->device = device;
  c->stream = nullptr;
  c->lds_limit = (int)prop.sharedMemPerBlock;
  c->num_cu = prop.multiProcessorCount;
  *h = c;
  return TLA_OK;
}

extern "C" tla_status tla_destroy(tla_handle h) {
  if (!h) return TLA_E_ARG;
  hipSetDevice(h->device);
  h->release();
  delete h;
  return TLA_OK;
}

extern "C" tla_status tla_set_stream(tla_handle h, void* stream) {
  if (!h) return TLA_E_ARG;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  return TLA_OK;
}

extern "C" tla_status tla_sync(tla_handle h) {
  if (!h) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(h->device));
  TLA_HIP(hipStreamSynchronize(h->stream));
  return TLA_OK;
}

extern "C" tla_status tla_set_refine(tla_handle h, double tau, int max_iter) {
  if (!h || !(tau >= 0.0) || max_iter < 0) return TLA_E_ARG;
  h->tau = tau;
  h->max_iter = max_iter;
  return TLA_OK;
}

// ------------------------------------------------------------- launching
namespace tla {

// LDS bytes for one instance of `op` with ntmax tiles per dimension.
size_t lds_bytes(int op, int prec, int tb, int nw, int ntmax, bool lu_lds) {
  const size_t np = (size_t)ntmax * tb;
  const size_t mat8 = np * (np + 1) * 8, mat4 = np * (np + 1) * 4;
  const size_t scr = (size_t)nw * 4 * tb * 8 + 16;
  if (prec == TLA_F64) {
    if (op == TLA_POTRF) return mat8 + scr;
    if (op == TLA_TRSYL) return mat8 * (lu_lds ? 3 : 1) + scr;
    return mat8 * (lu_lds ? 2 : 1) + scr;
  }
  // mixed: FP32 work matrix + FP64 solution + FP32 coefficients (if staged)
  if (op == TLA_POTRF) return mat8 + 2 * mat4 + scr;
  if (op == TLA_TRSYL) return mat8 + mat4 * (lu_lds ? 3 : 1) + scr;
  return mat8 + mat4 * (lu_lds ? 2 : 1) + scr;
}

tla_status launch(tla_ctx* h, int op, int prec, const tla_plan& p, const KArgs& a0) {
  KArgs a = a0;
  const int tb = p.tile, te = te_index(p.tile, p.engine), nwi = nw_index(p.waves);
  a.ntmax = (a.n_max + tb - 1) / tb;
  if (a.ntmax < 1) a.ntmax = 1;
  a.tau = h->tau;
  a.max_iter = h->max_iter;
  bool lu = true;
  size_t lds = lds_bytes(op, prec, tb, p.waves, a.ntmax, true);
  if (op != TLA_POTRF && lds > (size_t)h->lds_limit) {
    lu = false;
    lds = lds_bytes(op, prec, tb, p.waves, a.ntmax, false);
  }
  if (lds > (size_t)h->lds_limit) return TLA_E_UNSUPPORTED;
  KFn fn = nullptr;
  if (prec == TLA_F64) {
    if (op == TLA_POTRF) fn = potrf_f64_kernel(p.variant, te, nwi);
    else if (op == TLA_TRSYL) fn = trsyl_f64_kernel(p.variant, te, nwi, lu);
    else fn = trlyap_f64_kernel(p.variant, te, nwi, lu);
  } else {
    if (op == TLA_POTRF) fn = potrf_mixed_kernel(prec, p.variant, te, nwi);
    else if (op == TLA_TRSYL) fn = trsyl_mixed_kernel(prec, p.variant, te, nwi, lu);
    else fn = trlyap_mixed_kernel(prec, p.variant, te, nwi, lu);
  }
  if (!fn) return TLA_E_UNSUPPORTED;
  if (getenv("TLA_LOG"))
    fprintf(stderr, "tla: op %d prec %d batch %d n_max %d plan(v%d t%d e%d w%d) lds %zu lu_lds %d\n", op, prec,
            a.batch, a.n_max, p.variant, p.tile, p.engine, p.waves, lds, (int)lu);
  TLA_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  hipLaunchKernelGGL(fn, dim3(a.batch), dim3(64 * p.waves), lds, h->stream, a);
  TLA_HIP(hipGetLastError());
  return TLA_OK;
}

tla_plan pick_plan(tla_ctx* h, int op, int n, int prec, int batch) {
  auto f = h->forced.find(op * 8 + prec);
  if (f != h->forced.end()) return f->second;
  tla_plan p;
  if (h->picker == TLA_PICK_MLP && mlp_pick(h, op, n, prec, batch, &p)) return p;
  if (h->picker != TLA_PICK_DEFAULT && table_pick(h, op, n, prec, batch, &p)) return p;
  return default_plan(op, n, prec);
}

}  // namespace tla

static tla_status common_checks(tla_handle h, tla_prec prec, int batch, int n_max) {
  if (!h) return TLA_E_ARG;
  if (batch < 0 || n_max < 0) return TLA_E_ARG;
  if (prec < TLA_F64 || prec > TLA_MIXED_BF16) return TLA_E_ARG;
  if (n_max > tla::kMaxN) return TLA_E_UNSUPPORTED;
  return TLA_OK;
}

extern "C" tla_status tla_potrf_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int* n,
                                        double* const* A, const int* lda, int* info, tla_stat* stat) {
  tla_status s = common_checks(h, prec, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !A || !lda || !info) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(h->device));
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.c = A;
  a.ldc = lda;
  a.info = info;
  a.stat = stat;
  return launch(h, TLA_POTRF, prec, pick_plan(h, TLA_POTRF, n_max, prec, batch), a);
}

extern "C" tla_status tla_trsyl_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int* n,
                                        const double* const* L, const int* ldl, const double* const* U,
                                        const int* ldu, double* const* C, const int* ldc, int* info,
                                        tla_stat* stat) {
  tla_status s = common_checks(h, prec, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !L || !ldl || !U || !ldu || !C || !ldc || !info) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(h->device));
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.a = L;
  a.lda = ldl;
  a.b = U;
  a.ldb = ldu;
  a.c = C;
  a.ldc = ldc;
  a.info = info;
  a.stat = stat;
  return launch(h, TLA_TRSYL, prec, pick_plan(h, TLA_TRSYL, n_max, prec, batch), a);
}

extern "C" tla_status tla_trlyap_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int* n,
                                         const double* const* L, const int* ldl, double* const* S,
                                         const int* lds, int* info, tla_stat* stat) {
  tla_status s = common_checks(h, prec, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !L || !ldl || !S || !lds || !info) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(h->device));
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.a = L;
  a.lda = ldl;
  a.c = S;
  a.ldc = lds;
  a.info = info;
  a.stat = stat;
  return launch(h, TLA_TRLYAP, prec, pick_plan(h, TLA_TRLYAP, n_max, prec, batch), a);
}

// --------------------------------------------------------- plan control
extern "C" tla_status tla_set_plan(tla_handle h, tla_op op, tla_prec prec, const tla_plan* plan) {
  if (!h || op < 0 || op > 2 || prec < 0 || prec > 3) return TLA_E_ARG;
  if (!plan || plan->variant < 0) {
    h->forced.erase(op * 8 + prec);
    return TLA_OK;
  }
  if (!plan_valid(op, *plan)) return TLA_E_ARG;
  if (prec != TLA_F64 && plan->engine == 1 && plan->tile != 16) return TLA_E_ARG;
  h->forced[op * 8 + prec] = *plan;
  return TLA_OK;
}

extern "C" tla_status tla_get_plan(tla_handle h, tla_op op, int n, tla_prec prec, int batch, tla_plan* plan) {
  if (!h || !plan || op < 0 || op > 2) return TLA_E_ARG;
  *plan = pick_plan(h, op, n, prec, batch);
  return TLA_OK;
}

extern "C" int tla_num_candidates(tla_op op) { return num_candidates(op); }

extern "C" tla_status tla_candidate(tla_op op, int i, tla_plan* plan) {
  if (!plan) return TLA_E_ARG;
  return candidate(op, i, plan) ? TLA_OK : TLA_E_ARG;
}

extern "C" const char* tla_variant_name(tla_op op, int variant) {
  if (op < 0 || op > 2 || variant < 0 || variant >= kNumVar[op]) return "invalid";
  return kVarNames[op][variant];
}

extern "C" tla_status tla_set_picker(tla_handle h, tla_picker mode) {
  if (!h || mode < TLA_PICK_DEFAULT || mode > TLA_PICK_MLP) return TLA_E_ARG;
  h->picker = mode;
  return TLA_OK;
}
