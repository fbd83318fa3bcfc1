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

static const char* kVarNames[3][9] = {
    {"right-looking", "left-looking", "bordered", nullptr, nullptr, nullptr, nullptr, nullptr, nullptr},
    {"tile-wavefront", "rows-lazy", "rows-eager", "cols-lazy", "cols-eager", "2d-bordered", "2d-border-lazy",
     "2d-border-eager", "jacobi-sweeps"},
    {"tile-wavefront", "rows-lazy", "right-looking", "cols-lazy", "jacobi-sweeps", nullptr, nullptr, nullptr, nullptr}};
// blocked-algorithm variants (CHOL_NVAR, SYL_NVAR, LYA_NVAR, checked where the
// kernels are listed), then the splitting-iteration solve of the mixed
// precisions for the Sylvester and Lyapunov equations
static const int kNumBlocked[3] = {3, 8, 4};
static const int kNumVar[3] = {3, 9, 5};

int num_variants(int op) { return (op >= 0 && op < 3) ? kNumVar[op] : 0; }

bool is_jacobi(int op, int variant) {
  return (op == TLA_TRSYL || op == TLA_TRLYAP) && variant == kNumBlocked[op];
}

bool plan_valid(int op, const tla_plan& p) {
  if (op < 0 || op > 2) return false;
  if (p.variant < 0 || p.variant >= kNumVar[op]) return false;
  if (p.tile != 8 && p.tile != 16) return false;
  if (p.engine != 0 && p.engine != 1) return false;
  if (p.tile == 8 && p.engine == 1) return false;
  if (p.waves != 1 && p.waves != 2 && p.waves != 4) return false;
  // place 2 (FP64 solution in the workspace) only exists for the mixed kernels
  // and place 3 (in place in global memory) only for FP64; the launcher
  // reports the other precision unsupported
  if (p.place < 0 || p.place > 3) return false;
  if (op == TLA_POTRF && p.place == 1) return false;
  if (p.place == 3 && !(p.tile == 16 && p.engine == 1)) return false;
  // the splitting-iteration solve: 16 x 16 matrix-core tiles, registers, one
  // wave per tile column (waves is not a choice there)
  if (is_jacobi(op, p.variant) && !(p.tile == 16 && p.engine == 1 && p.waves == 1 && p.place == 3)) return false;
  return true;
}

// candidates: variant x (tile, engine) x waves x coefficient placement 0..2,
// then variant x waves with placement 3 (16 x 16 matrix-core tiles only)
static int num_places(int op) { return op == TLA_POTRF ? 2 : 3; }
static int num_candidates_lds(int op) { return kNumBlocked[op] * kNumTE * kNumNW * num_places(op); }
static int num_candidates_blocked(int op) { return num_candidates_lds(op) + kNumBlocked[op] * kNumNW; }
int num_candidates(int op) {
  if (op < 0 || op > 2) return 0;
  return num_candidates_blocked(op) + (kNumVar[op] - kNumBlocked[op]);
}
bool candidate(int op, int i, tla_plan* p) {
  if (i < 0 || i >= num_candidates(op)) return false;
  if (i >= num_candidates_blocked(op)) {  // the splitting-iteration solve (mixed precisions only)
    p->variant = kNumBlocked[op];
    p->tile = 16;
    p->engine = 1;
    p->waves = 1;
    p->place = 3;
    return true;
  }
  if (i >= num_candidates_lds(op)) {
    i -= num_candidates_lds(op);
    const int nwi = i % kNumNW;
    p->variant = i / kNumNW;
    p->tile = 16;
    p->engine = 1;
    p->waves = nwi == 0 ? 1 : (nwi == 1 ? 2 : 4);
    p->place = 3;
    return true;
  }
  const int np = num_places(op);
  p->place = i % np;
  if (op == TLA_POTRF && p->place == 1) p->place = 2;  // potrf: 0 or 2
  i /= np;
  const int nwi = i % kNumNW, te = (i / kNumNW) % kNumTE, var = i / (kNumNW * kNumTE);
  p->variant = var;
  p->tile = te_tile(te);
  p->engine = te == 2 ? 1 : 0;
  p->waves = nwi == 0 ? 1 : (nwi == 1 ? 2 : 4);
  return true;
}

// The plan used without a tuning table: 16 x 16 matrix-core tiles, the
// tile-wavefront variant for the Sylvester and Lyapunov equations, and what
// measured best at n = 32, 64 and 128 otherwise.  FP64: in place in global
// memory, one wave per instance up to n = 64 (two or four above), bordered
// Cholesky (left-looking for the large sizes, where it measured 1.4x faster
// than right-looking).  Mixed: above n = 32 with the FP64 solution in the
// workspace.
tla_plan default_plan(int op, int n, int prec) {
  tla_plan p;
  // Sylvester and Lyapunov, mixed: the splitting-iteration solve where it
  // measured faster than the blocked mixed kernels (BF16 products up to
  // n = 64, FP32 products up to n = 32)
  if ((op == TLA_TRSYL || op == TLA_TRLYAP) &&
      ((prec == TLA_MIXED_BF16 && n <= kJacobiMaxN) || (prec == TLA_MIXED_F32 && n <= 32))) {
    p.variant = op == TLA_TRSYL ? 8 : 4;
    p.tile = 16;
    p.engine = 1;
    p.waves = 1;
    p.place = 3;
    return p;
  }
  p.variant = (op == TLA_POTRF && n > kMaxN) ? 1 : 0;
  p.tile = 16;
  p.engine = 1;
  if (prec == TLA_F64) {
    // in place, one wave per instance up to n = 64 (bordered Cholesky)
    if (op == TLA_POTRF && n <= kMaxN) p.variant = 2;
    p.waves = (op == TLA_POTRF || n <= 64) ? 1 : (op == TLA_TRSYL ? 4 : 2);
    p.place = 3;
  } else if (n <= 32) {
    p.waves = n <= 16 ? 1 : 2;
    p.place = 0;
  } else {
    p.waves = op == TLA_POTRF ? 4 : 2;
    p.place = 2;
  }
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
  // the allocation-free entry point's scratch array on this device
  const tla_status ns = noalloc_init(device);
  if (ns != TLA_OK) return ns;
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
  ++h->gen;
  return TLA_OK;
}

// ------------------------------------------------------------- launching
namespace tla {

// LDS bytes for one instance of `op` with ntmax tiles per dimension.
// FP64 kernels, placement 0: coefficients and X in LDS, 1: X only, 3: the
// tile solvers' scratch only (X in place in global memory).
// Mixed kernels: FP32 work matrix W (+ FP32 coefficients / factor copy) and
// the FP64 solution (placements 0, 1) in LDS; placement 2 moves the solution
// to the workspace, placement 3 the work matrices too; see tla_registry.h.
size_t lds_bytes(int op, int prec, int tb, int nw, int ntmax, int pl) {
  const size_t np = (size_t)ntmax * tb;
  const size_t mat8 = np * (np + 1) * 8, mat4 = np * (np + 1) * 4;
  // tile solvers' scratch (FP32 elements for the mixed kernels whose FP64
  // fallback is a second launch), alignment, reduction cells
  const size_t scr_elem = (prec != TLA_F64 && pl >= 2) ? 4 : 8;
  const size_t scr = (size_t)nw * wave_scratch(tb) * scr_elem + 16 + 8 * (nw + 4);
  if (prec == TLA_F64) {
    if (pl == 3) return inplace_lds_bytes(nw);
    if (op == TLA_POTRF) return mat8 + scr;
    if (op == TLA_TRSYL) return mat8 * (pl == 0 ? 3 : 1) + scr;
    return mat8 * (pl == 0 ? 2 : 1) + scr;
  }
  if (pl == 3) return scr;
  if (op == TLA_POTRF) return (pl == 0 ? mat8 + 2 * mat4 : mat4) + scr;  // place 2: factor copy in the workspace
  const size_t coef = pl == 0 ? (op == TLA_TRSYL ? 2 : 1) * mat4 : 0;
  return (pl == 2 ? 0 : mat8) + mat4 + coef + scr;
}

// Grows the handle's workspace and refinement-record buffers.  A buffer is
// freed only after the whole device has finished (work on an earlier stream
// of the handle may still use it), and every reallocation bumps the handle's
// generation so that no cached ragged graph replays with the old address.
static tla_status ensure_buffers(tla_ctx* h, size_t work_bytes, int batch) {
  if (work_bytes > h->work_bytes) {
    ++h->gen;
    if (h->work) {
      hipDeviceSynchronize();
      hipFree(h->work);
      h->work = nullptr;
      h->work_bytes = 0;
    }
    if (hipMalloc(&h->work, work_bytes) != hipSuccess) return TLA_E_NOMEM;
    h->work_bytes = work_bytes;
  }
  if ((size_t)batch > h->stat_cap) {
    ++h->gen;
    if (h->stat_buf) {
      hipDeviceSynchronize();
      hipFree(h->stat_buf);
      h->stat_buf = nullptr;
      h->stat_cap = 0;
    }
    if (hipMalloc(&h->stat_buf, (size_t)batch * sizeof(tla_stat)) != hipSuccess) return TLA_E_NOMEM;
    h->stat_cap = batch;
  }
  return TLA_OK;
}

static KFn kernel_for(int op, int prec, const tla_plan& p, int pl) {
  const int te = te_index(p.tile, p.engine), nwi = nw_index(p.waves);
  if (prec == TLA_F64) {
    if (pl == 3) return inplace_kernel(op, p.variant, nwi);
    if (op == TLA_POTRF) return potrf_f64_kernel(p.variant, te, nwi);
    if (op == TLA_TRSYL) return trsyl_f64_kernel(p.variant, te, nwi, pl == 0);
    return trlyap_f64_kernel(p.variant, te, nwi, pl == 0);
  }
  if (pl == 3) {
    if (op == TLA_POTRF) return potrf_mixed_ws_kernel(prec, p.variant, nwi);
    if (op == TLA_TRSYL) return trsyl_mixed_ws_kernel(prec, p.variant, nwi);
    return trlyap_mixed_ws_kernel(prec, p.variant, nwi);
  }
  if (op == TLA_POTRF) return potrf_mixed_kernel(prec, p.variant, te, nwi, pl == 0 ? 0 : 1);
  if (op == TLA_TRSYL) return trsyl_mixed_kernel(prec, p.variant, te, nwi, pl);
  return trlyap_mixed_kernel(prec, p.variant, te, nwi, pl);
}

// First placement whose LDS fits: returns -1 when none does.  FP64 runs
// placements 0 / 1 (potrf 0) and 3, the mixed precisions 0 / 1 / 2 / 3
// (potrf 0 / 2 / 3); the search moves to larger placements of the same family.
int choose_placement(tla_ctx* h, int op, int prec, const tla_plan& p, int ntmax, size_t* lds) {
  const int last = 3;
  if (p.place > last) return -1;
  for (int pl = p.place; pl <= last; ++pl) {
    if (op == TLA_POTRF && pl == 1) continue;
    if (prec == TLA_F64 && pl == 2) continue;
    if (pl == 3 && !(p.tile == 16 && p.engine == 1)) continue;
    const size_t b = lds_bytes(op, prec, p.tile, p.waves, ntmax, pl);
    if (b <= (size_t)h->lds_limit) { *lds = b; return pl; }
  }
  return -1;
}

static tla_status launch_one(tla_ctx* h, KFn fn, size_t lds, int grid, int waves, const KArgs& a) {
  TLA_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds));
  hipLaunchKernelGGL(fn, dim3(grid), dim3(64 * waves), lds, h->stream, a);
  TLA_HIP(hipGetLastError());
  return TLA_OK;
}

// Workspace doubles per instance for the mixed kernels with the FP64 solution
// there (placement 2), or the FP32 work matrices too (placement 3, large n).
static long long work_stride(int pl, int ntmax) {
  const long long np = (long long)ntmax * 16, mat = np * (np + 1);
  return pl == 3 ? 2 * mat : (3 * mat + 1) / 2;  // place 2: solution + an FP32 matrix
}

static tla_status ensure_work(tla_ctx* h, KArgs& a, int pl) {
  a.work_stride = work_stride(pl, a.ntmax);
  tla_status s = ensure_buffers(h, (size_t)a.batch * a.work_stride * sizeof(double), a.batch);
  if (s != TLA_OK) return s;
  a.work = h->work;
  if (!a.stat) a.stat = h->stat_buf;
  return TLA_OK;
}

// The splitting-iteration mixed solve, then the FP64 pass over the instances
// it left unconverged (the in-place FP64 tile-wavefront kernel, one wave).
static tla_status launch_jacobi(tla_ctx* h, int op, int prec, KArgs a) {
  size_t lds = 0;
  int waves = 1;
  KFn fn = jacobi_kernel(op, prec, a.n_max, &lds, &waves);
  if (!fn || lds > (size_t)h->lds_limit) return TLA_E_UNSUPPORTED;
  if (!a.stat) {
    // the FP64 pass reads the refinement records
    tla_status s = ensure_buffers(h, 0, a.batch);
    if (s != TLA_OK) return s;
    a.stat = h->stat_buf;
  }
  a.ntmax = (a.n_max + 15) / 16;
  if (getenv("TLA_LOG"))
    fprintf(stderr, "tla: op %d prec %d batch %d n_max %d jacobi-sweeps waves %d lds %zu\n", op, prec, a.batch,
            a.n_max, waves, lds);
  tla_status s = launch_one(h, fn, lds, a.batch, waves, a);
  if (s != TLA_OK) return s;
  KFn fb = inplace_kernel(op, 0, 0);
  if (!fb) return TLA_E_UNSUPPORTED;
  a.only_flagged = 1;
  return launch_one(h, fb, inplace_lds_bytes(1), a.batch, 1, a);
}

tla_status launch(tla_ctx* h, int op, int prec, const tla_plan& p, const KArgs& a0) {
  KArgs a = a0;
  a.tau = h->tau;
  a.max_iter = h->max_iter;
  a.only_flagged = 0;
  if (is_jacobi(op, p.variant)) {
    if (prec == TLA_F64 || a.n_max > kJacobiMaxN) return TLA_E_UNSUPPORTED;
    return launch_jacobi(h, op, prec, a);
  }
  if (a.n_max > kMaxN) {
    // large sizes: FP64 in place over global memory, variant from the plan.
    // (The mixed precisions are not offered here: their 16-wave kernels with
    // the work matrices in the workspace faulted the GPU on their first
    // Lyapunov run, cause not found; the code path is switched off.)
    if (prec != TLA_F64) return TLA_E_UNSUPPORTED;
    // left-looking Cholesky: block panels, each update one batched product
    // (from n = 384; at n = 256 the one-workgroup kernel measured faster)
    if (op == TLA_POTRF && p.variant == 1 && a.n_max >= 384) return potrf_panel(h, a);
    // tile-wavefront Sylvester: the same wavefront over 128 x 128 blocks
    if (op == TLA_TRSYL && p.variant == 0 && a.n_max >= 384) return trsyl_blocks(h, a);
    a.ntmax = (a.n_max + 15) / 16;
    KFn fn64 = large_kernel(op, p.variant);
    if (!fn64) return TLA_E_UNSUPPORTED;
    return launch_one(h, fn64, large_lds_bytes(), a.batch, large_waves(), a);
  }
  a.ntmax = (a.n_max + p.tile - 1) / p.tile;
  if (a.ntmax < 1) a.ntmax = 1;
  size_t lds = 0;
  const int pl = choose_placement(h, op, prec, p, a.ntmax, &lds);
  if (pl < 0) return TLA_E_UNSUPPORTED;
  const bool xg = prec != TLA_F64 && pl >= 2;
  KFn fn = kernel_for(op, prec, p, pl);
  if (!fn) return TLA_E_UNSUPPORTED;
  if (xg) {
    tla_status s = ensure_work(h, a, pl);
    if (s != TLA_OK) return s;
  }
  if (getenv("TLA_LOG"))
    fprintf(stderr, "tla: op %d prec %d batch %d n_max %d plan(v%d t%d e%d w%d) lds %zu placement %d\n", op, prec,
            a.batch, a.n_max, p.variant, p.tile, p.engine, p.waves, lds, pl);
  if (prec == TLA_F64 && pl == 3 && h->exact_size) {
    // the same in-place kernel compiled for this n (falls through when
    // unavailable); in the measured mode only where it timed faster
    bool use = h->exact_size == 1;
    if (h->exact_size == 2) {
      const long long key = ((long long)(op * 256 + a.n_max) * 16 + p.variant) * 8 + p.waves;
      auto it = h->exact_choice.find(key);
      if (it == h->exact_choice.end()) {
        bool faster = false;
        tla_status ds = exact_size_decide(h, op, a.n_max, std::min(a.batch, 4096), p, &faster);
        if (ds != TLA_OK) return ds;
        it = h->exact_choice.emplace(key, faster).first;
      }
      use = it->second;
    }
    if (use) {
      const tla_status js = jit_launch(h, op, p.variant, p.waves, lds, a);
      if (js != TLA_E_UNSUPPORTED) return js;
    }
  }
  tla_status s = launch_one(h, fn, lds, a.batch, p.waves, a);
  if (s != TLA_OK || !xg) return s;
  // second pass: FP64 solve of the instances the mixed kernel left
  // unconverged, by the LDS-resident FP64 kernel of the same variant
  size_t lds64 = 0;
  tla_plan p64 = p;
  p64.place = op == TLA_POTRF ? 0 : 1;
  const int pl64 = choose_placement(h, op, TLA_F64, p64, a.ntmax, &lds64);
  if (pl64 < 0) return TLA_E_UNSUPPORTED;
  KFn fb = kernel_for(op, TLA_F64, p64, pl64);
  if (!fb) return TLA_E_UNSUPPORTED;
  a.only_flagged = 1;
  return launch_one(h, fb, lds64, a.batch, p.waves, a);
}

// Whether a plan exists for (op, prec, n): the splitting-iteration solve has
// BF16 and FP32 products and n <= kJacobiMaxN only (the blocked plans run
// everywhere; placements that do not fit move to a larger one at launch).
bool plan_runs(int op, int prec, int n, const tla_plan& p) {
  if (is_jacobi(op, p.variant)) return (prec == TLA_MIXED_F32 || prec == TLA_MIXED_BF16) && n <= kJacobiMaxN;
  return true;
}

tla_plan pick_plan(tla_ctx* h, int op, int n, int prec, int batch) {
  auto f = h->forced.find(op * 8 + prec);
  if (f != h->forced.end()) return f->second;
  tla_plan p;
  if (h->picker == TLA_PICK_MLP && mlp_pick(h, op, n, prec, batch, &p)) return p;
  // a table entry of a nearby size may name a plan that does not exist at n
  if (h->picker != TLA_PICK_DEFAULT && table_pick(h, op, n, prec, batch, &p) && plan_runs(op, prec, n, p)) return p;
  return default_plan(op, n, prec);
}

}  // namespace tla

static tla_status common_checks(tla_handle h, tla_prec prec, int batch, int n_max) {
  if (!h) return TLA_E_ARG;
  if (batch < 0 || n_max < 0) return TLA_E_ARG;
  if (prec < TLA_F64 || prec > TLA_MIXED_BF16) return TLA_E_ARG;
  if (n_max > tla::kMaxLargeN) return TLA_E_UNSUPPORTED;
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

extern "C" tla_status tla_potrs_batched(tla_handle h, int batch, int n_max, const int* n, int nrhs_max,
                                        const int* nrhs, const double* const* X, const int* ldx, double* const* B,
                                        const int* ldb, int* info) {
  tla_status s = common_checks(h, TLA_F64, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (nrhs_max < 0) return TLA_E_ARG;
  if (!n || !nrhs || !X || !ldx || !B || !ldb || !info) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(h->device));
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.a = X;
  a.lda = ldx;
  a.c = B;
  a.ldc = ldb;
  a.info = info;
  a.m = nrhs;
  a.m_max = nrhs_max;
  // one wave per 16-column tile of right-hand sides, up to 4
  const int tiles = (nrhs_max + 15) / 16;
  const int nwi = tiles <= 1 ? 0 : (tiles == 2 ? 1 : 2);
  const int nw = 1 << nwi;
  return launch_one(h, potrs_kernel(nwi), potrs_lds_bytes(nw), batch, nw, a);
}

extern "C" tla_status tla_potri_batched(tla_handle h, int batch, int n_max, const int* n, const double* const* X,
                                        const int* ldx, double* const* Y, const int* ldy, int* info) {
  tla_status s = common_checks(h, TLA_F64, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !X || !ldx || !Y || !ldy || !info) return TLA_E_ARG;
  TLA_HIP(hipSetDevice(h->device));
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.a = X;
  a.lda = ldx;
  a.c = Y;
  a.ldc = ldy;
  a.info = info;
  a.m = n;  // n right-hand sides: the columns of the identity
  a.m_max = n_max;
  hipLaunchKernelGGL(potri_eye_kernel(), dim3(batch), dim3(256), 0, h->stream, a);
  TLA_HIP(hipGetLastError());
  const int tiles = (n_max + 15) / 16;
  const int nwi = tiles <= 1 ? 0 : (tiles == 2 ? 1 : 2);
  const int nw = 1 << nwi;
  return launch_one(h, potrs_kernel(nwi), potrs_lds_bytes(nw), batch, nw, a);
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
  ++h->gen;
  return TLA_OK;
}
