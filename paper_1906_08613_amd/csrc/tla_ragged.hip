// Ragged batches: instances of all three operations with uneven n in one
// call.  The work list is ordered on the device (counting sort by a cost
// rank, longest first, within three size classes), then one persistent
// kernel per size class pulls instances from its queue with an atomic
// counter and runs the same per-instance bodies as the uniform kernels.
// The whole sequence is captured once as a HIP graph and replayed when the
// same descriptor array, batch, n_max, precision and result arrays come again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "tla_host.h"
#include "tla_inplace.hpp"
#include "tla_mixed.hpp"

namespace tla {

constexpr int kRagClasses = 3;                // n <= 32, n <= 64, n <= 128
constexpr int kRagClassMax[kRagClasses] = {32, 64, 128};
constexpr int kRagKeysPerClass = 3 * (kMaxN + 1);
constexpr int kRagKeys = kRagClasses * kRagKeysPerClass;

__host__ __device__ inline int rag_class(int n) { return n <= 32 ? 0 : (n <= 64 ? 1 : 2); }

struct RagArgs {
  const tla_desc* d;
  int batch, n_max;
  int* info;
  tla_stat* stat;
  const int* rank;   // [3][kMaxN+1]: position of (op, n) in decreasing cost order
  int* keycount;     // [kRagKeys]
  int* keyoff;       // [kRagKeys]
  int* queue;        // [batch]
  int* cls;          // [3 start | 3 count | 3 counter | 3 second-pass counter]
};

__global__ void k_rag_zero(RagArgs r) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kRagKeys; i += gridDim.x * blockDim.x) r.keycount[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x < 12) r.cls[threadIdx.x] = 0;
}

// Validates each descriptor; invalid ones get their info here (-1 bad n,
// -2 bad leading dimension, -3 unknown operation), n = 0 gets info 0.
__device__ inline bool rag_valid(const tla_desc& d, int n_max, int* info, tla_stat* st) {
  int bad = 0;
  if (d.op < 0 || d.op > 2) bad = -3;
  else if (d.n < 0 || d.n > n_max) bad = -1;
  else {
    const int m = d.n > 1 ? d.n : 1;
    if (d.op == TLA_POTRF && d.lda < m) bad = -2;
    if (d.op == TLA_TRSYL && (d.lda < m || d.ldb < m || d.ldc < m)) bad = -2;
    if (d.op == TLA_TRLYAP && (d.lda < m || d.ldc < m)) bad = -2;
  }
  if (bad != 0 || d.n == 0) {
    *info = bad;
    if (st) { st->iters = 0; st->flags = 0; st->eta = 0.0; }
    return false;
  }
  return true;
}

__device__ inline int rag_key(const RagArgs& r, const tla_desc& d) {
  return rag_class(d.n) * kRagKeysPerClass + r.rank[d.op * (kMaxN + 1) + d.n];
}

__global__ void k_rag_hist(RagArgs r) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= r.batch) return;
  const tla_desc d = r.d[b];
  if (!rag_valid(d, r.n_max, r.info + b, r.stat ? r.stat + b : nullptr)) return;
  atomicAdd(&r.keycount[rag_key(r, d)], 1);
}

// single workgroup: exclusive scan of the key histogram, class ranges
__global__ void k_rag_scan(RagArgs r) {
  __shared__ int part[256];
  const int t = threadIdx.x;
  constexpr int per = (kRagKeys + 255) / 256;
  int s = 0;
  for (int k = 0; k < per; ++k) {
    const int i = t * per + k;
    if (i < kRagKeys) s += r.keycount[i];
  }
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int i = 0; i < 256; ++i) { const int v = part[i]; part[i] = acc; acc += v; }
  }
  __syncthreads();
  int acc = part[t];
  for (int k = 0; k < per; ++k) {
    const int i = t * per + k;
    if (i < kRagKeys) { const int v = r.keycount[i]; r.keyoff[i] = acc; acc += v; }
  }
  __syncthreads();
  if (t < kRagClasses) {
    const int first = t * kRagKeysPerClass, last = first + kRagKeysPerClass - 1;
    r.cls[t] = r.keyoff[first];
    r.cls[3 + t] = r.keyoff[last] + r.keycount[last] - r.keyoff[first];
  }
}

__global__ void k_rag_scatter(RagArgs r) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= r.batch) return;
  const tla_desc d = r.d[b];
  if (d.op < 0 || d.op > 2 || d.n <= 0 || d.n > r.n_max) return;
  const int m = d.n;
  if ((d.op == TLA_POTRF && d.lda < m) || (d.op == TLA_TRSYL && (d.lda < m || d.ldb < m || d.ldc < m)) ||
      (d.op == TLA_TRLYAP && (d.lda < m || d.ldc < m)))
    return;
  const int pos = atomicAdd(&r.keyoff[rag_key(r, d)], 1);
  r.queue[pos] = b;
}

// the descriptor's roles mapped onto the uniform kernels' operand slots
__device__ inline Inst rag_inst(const tla_desc& d, int* info, tla_stat* st) {
  Inst in;
  in.n = d.n;
  in.info = info;
  in.stat = st;
  if (d.op == TLA_POTRF) {
    in.a = nullptr; in.lda = 1; in.b = nullptr; in.ldb = 1; in.c = d.a; in.ldc = d.lda;
  } else if (d.op == TLA_TRSYL) {
    in.a = d.a; in.lda = d.lda; in.b = d.b; in.ldb = d.ldb; in.c = d.c; in.ldc = d.ldc;
  } else {
    in.a = d.a; in.lda = d.lda; in.b = nullptr; in.ldb = 1; in.c = d.c; in.ldc = d.ldc;
  }
  return in;
}

struct RagVariants { int v[3]; };

// MIXED: 0 = FP64 solve, 1 = FP32 + FP64 refinement.  PL: placement of the
// Sylvester/Lyapunov operands (and, for the mixed kernels, PL == 2 puts the
// FP64 solution of all three operations in the workspace; for FP64, PL == 3
// solves all three in place in global memory).
// Variants compiled into the ragged workers: Cholesky all three, Sylvester
// the 1-D ones and the tile wavefront (0..4), Lyapunov 0..2.  One worker holds
// every operation's bodies, so each further variant raises its register use;
// with the 2-D Sylvester and the lazy-column Lyapunov variants the mixed
// workers fell to one wave per SIMD.  The planner maps a tuned variant outside
// these to the tile wavefront.
constexpr int kRagVars[3] = {CHOL_NVAR, 5, 3};

// Calls f(std::integral_constant<int, V>) for the variant V == v (v is
// uniform over the workgroup; out-of-range values take the last variant).
template <int V, int NV, class F>
__device__ __forceinline__ void with_variant(int v, const F& f) {
  if constexpr (V + 1 >= NV) {
    f(std::integral_constant<int, V>{});
  } else {
    if (v == V) f(std::integral_constant<int, V>{});
    else with_variant<V + 1, NV>(v, f);
  }
}

template <int TB, int ENG, int NW, int MIXED, int PL>
__device__ void rag_run(const KArgs& g, const Inst& in, int op, const RagVariants& rv, unsigned char* smem) {
  if constexpr (MIXED == 0 && PL == 3) {
    static_assert(TB == 16 && ENG == ENG_MFMA, "in-place workers use 16 x 16 matrix-core tiles");
    if (op == TLA_POTRF) with_variant<0, kRagVars[0]>(rv.v[0], [&](auto vc) { constexpr int V = decltype(vc)::value; potrf_inplace_body<NW, V>(g, in, smem); });
    else if (op == TLA_TRSYL) with_variant<0, kRagVars[1]>(rv.v[1], [&](auto vc) { constexpr int V = decltype(vc)::value; trsyl_inplace_body<NW, V>(g, in, smem); });
    else with_variant<0, kRagVars[2]>(rv.v[2], [&](auto vc) { constexpr int V = decltype(vc)::value; trlyap_inplace_body<NW, V>(g, in, smem); });
  } else if constexpr (MIXED == 0) {
    if (op == TLA_POTRF)
      with_variant<0, kRagVars[0]>(rv.v[0], [&](auto vc) { constexpr int V = decltype(vc)::value; potrf_f64_body<TB, ENG, NW, V>(g, in, smem); });
    else if (op == TLA_TRSYL)
      with_variant<0, kRagVars[1]>(rv.v[1], [&](auto vc) { constexpr int V = decltype(vc)::value; trsyl_f64_body<TB, ENG, NW, V, PL == 0>(g, in, smem); });
    else
      with_variant<0, kRagVars[2]>(rv.v[2], [&](auto vc) { constexpr int V = decltype(vc)::value; trlyap_f64_body<TB, ENG, NW, V, PL == 0>(g, in, smem); });
  } else {
    if (op == TLA_POTRF)
      with_variant<0, kRagVars[0]>(rv.v[0], [&](auto vc) { constexpr int V = decltype(vc)::value; potrf_mixed_body<TB, ENG, NW, V, PL == 2>(g, in, smem); });
    else if (op == TLA_TRSYL)
      with_variant<0, kRagVars[1]>(rv.v[1], [&](auto vc) { constexpr int V = decltype(vc)::value; trsyl_mixed_body<TB, ENG, NW, V, PL == 0, PL == 2>(g, in, smem); });
    else
      with_variant<0, kRagVars[2]>(rv.v[2], [&](auto vc) { constexpr int V = decltype(vc)::value; trlyap_mixed_body<TB, ENG, NW, V, PL == 0, PL == 2>(g, in, smem); });
  }
}

// Register budget of the FP64 class workers, in resident waves per SIMD.  A
// worker holds the bodies of all three operations and the compiler alone
// gives it up to 256 registers (one or two waves); these budgets cost at most
// a few spilled registers and made the FP64 ragged batch 6% faster.  The
// mixed workers measured 12% slower with the same budgets and keep the
// compiler's choice.
template <int MIXED, int PL>
constexpr int kRagWaves = MIXED != 0 ? 1 : (PL == 3 ? 4 : (PL == 0 ? 3 : 1));

// Persistent worker for one size class.  counter_slot selects the atomic
// counter (first pass or FP64 second pass).
template <int TB, int ENG, int NW, int MIXED, int PL>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(kRagWaves<MIXED, PL>))) void k_ragged(RagArgs r, KArgs g, RagVariants rv, int cls, int counter_slot) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_item;
  const int start = r.cls[cls], count = r.cls[3 + cls];
  int* ctr = r.cls + counter_slot * 3 + cls;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) {
      const int i = atomicAdd(ctr, 1);
      s_item = i < count ? r.queue[start + i] : -1;
    }
    __syncthreads();
    const int b = s_item;
    if (b < 0) break;
    const tla_desc d = r.d[b];
    const Inst in = rag_inst(d, r.info + b, g.stat ? g.stat + b : nullptr);
    rag_run<TB, ENG, NW, MIXED, PL>(g, in, d.op, rv, smem);
  }
}

typedef void (*RagFn)(RagArgs, KArgs, RagVariants, int, int);

// class configuration: waves, placement, kernel
struct RagClassCfg {
  int waves, pl;
  RagFn fn;
};

static RagClassCfg rag_cfg(int prec, int cls, bool second_pass) {
  // FP64: class 0 keeps the operands in LDS; the larger classes solve in
  // place in global memory so that many instances share a compute unit.
  // The FP64 second pass of the mixed path keeps the LDS-resident workers.
  if (second_pass) {
    if (cls == 0) return {2, 0, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 2, 0, 0>)};
    return {4, 1, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 4, 0, 1>)};
  }
  if (prec == TLA_F64) {
    if (cls == 0) return {2, 0, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 2, 0, 0>)};
    if (cls == 1) return {1, 3, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 1, 0, 3>)};
    return {2, 3, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 2, 0, 3>)};
  }
  if (cls == 0) return {2, 0, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 2, 1, 0>)};
  if (cls == 1) return {4, 1, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 4, 1, 1>)};
  return {4, 2, reinterpret_cast<RagFn>(&k_ragged<16, ENG_MFMA, 4, 1, 2>)};
}

// decreasing-cost rank of (op, n): nominal flops plus a per-entry term for
// the data movement
static std::vector<int> cost_rank() {
  std::vector<std::pair<double, int>> v;
  for (int op = 0; op < 3; ++op)
    for (int n = 0; n <= kMaxN; ++n) {
      const double f = op == 0 ? n * (double)n * n / 3.0 : (op == 1 ? 2.0 : 1.0) * n * (double)n * n;
      const double bytes = (op == 1 ? 3.0 : (op == 2 ? 2.0 : 1.0)) * n * (double)n * 8.0;
      v.push_back({f + 20.0 * bytes, op * (kMaxN + 1) + n});
    }
  std::stable_sort(v.begin(), v.end(), [](auto& a, auto& b) { return a.first > b.first; });
  std::vector<int> rank(3 * (kMaxN + 1));
  for (size_t i = 0; i < v.size(); ++i) rank[v[i].second] = (int)i;
  return rank;
}

}  // namespace tla

using namespace tla;

struct RagBuffers {
  int* rank = nullptr;
  int* keycount = nullptr;
  int* keyoff = nullptr;
  int* queue = nullptr;
  int* cls = nullptr;
  int cap = 0;
};

namespace tla {
struct RagState {
  RagBuffers buf;
  hipStream_t cap_stream = nullptr;
  unsigned long long gen = 0;  // handle generation the cached graphs were captured in
  struct Entry {
    const void* d;
    int batch, n_max, prec;
    void *info, *stat, *stream;
    hipGraphExec_t exec;
    hipGraph_t graph;
  };
  std::vector<Entry> graphs;
};

void ragged_release(tla_ctx* h) {
  RagState* s = h->rag;
  if (!s) return;
  for (auto& e : s->graphs) { hipGraphExecDestroy(e.exec); hipGraphDestroy(e.graph); }
  hipFree(s->buf.rank); hipFree(s->buf.keycount); hipFree(s->buf.keyoff); hipFree(s->buf.queue); hipFree(s->buf.cls);
  if (s->cap_stream) hipStreamDestroy(s->cap_stream);
  delete s;
  h->rag = nullptr;
}
}  // namespace tla

struct RagLaunch {
  RagFn fn;
  int grid, waves;
  size_t lds;
  KArgs g;
  RagVariants rv;
  int cls, slot;
};

// Host-side part: per class and pass, the kernel, grid and LDS (queries that
// must not run while a stream is being captured).
static void rag_drop_graphs(RagState* s) {
  for (auto& e : s->graphs) { hipGraphExecDestroy(e.exec); hipGraphDestroy(e.graph); }
  s->graphs.clear();
}

constexpr int kRagMaxLaunches = 2 * kRagClasses;  // class workers of the first pass and the FP64 second pass

static tla_status rag_plan(tla_ctx* h, int prec, int batch, int n_max, tla_stat* stat, RagLaunch* out, int* nout) {
  *nout = 0;
  for (int pass = 0; pass < (prec == TLA_F64 ? 1 : 2); ++pass) {
    for (int cls = kRagClasses - 1; cls >= 0; --cls) {
      if (n_max <= (cls == 0 ? 0 : kRagClassMax[cls - 1])) continue;  // class cannot occur
      // the FP64 second pass is only for classes whose FP64 solutions live
      // in the workspace (elsewhere the fallback runs inside the kernel)
      if (pass == 1 && rag_cfg(prec, cls, false).pl != 2) continue;
      const RagClassCfg cfg = rag_cfg(prec, cls, pass == 1);
      const int cmax = std::min(n_max, kRagClassMax[cls]);
      RagLaunch L{};
      L.fn = cfg.fn;
      L.waves = cfg.waves;
      L.cls = cls;
      L.slot = pass == 0 ? 2 : 3;
      KArgs& g = L.g;
      g.batch = batch;
      g.n_max = n_max;
      g.ntmax = (cmax + 15) / 16;
      g.tau = h->tau;
      g.max_iter = h->max_iter;
      g.stat = stat;
      g.only_flagged = pass == 1;
      for (int op = 0; op < 3; ++op) {
        tla_plan p;
        const int rep = std::min(cls == 0 ? 24 : (cls == 1 ? 48 : 96), n_max);
        const bool ok = h->picker != TLA_PICK_DEFAULT && table_pick(h, op, rep, prec, batch, &p) && p.tile == 16 &&
                        p.engine == 1;
        L.rv.v[op] = ok && p.variant < kRagVars[op] ? p.variant : 0;
      }
      const int eff_prec = pass == 1 ? TLA_F64 : prec;
      for (int op = 0; op < 3; ++op) {
        int pl = cfg.pl;
        if (op == TLA_POTRF && pl != 3) pl = (eff_prec != TLA_F64 && cfg.pl == 2) ? 2 : 0;
        L.lds = std::max(L.lds, lds_bytes(op, eff_prec, 16, cfg.waves, g.ntmax, pl));
      }
      if (L.lds > (size_t)h->lds_limit) return TLA_E_UNSUPPORTED;
      if (hipFuncSetAttribute(reinterpret_cast<const void*>(cfg.fn), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)L.lds) != hipSuccess)
        return TLA_E_HIP;
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void*>(cfg.fn), 64 * cfg.waves,
                                                       L.lds) != hipSuccess || occ < 1)
        occ = 1;
      L.grid = std::min(h->num_cu * occ, batch);
      if (eff_prec != TLA_F64 && cfg.pl == 2) {
        const size_t np = (size_t)g.ntmax * 16;
        g.work_stride = (long long)((3 * np * (np + 1) + 1) / 2);
        if ((size_t)L.grid * g.work_stride * sizeof(double) > h->work_bytes) return TLA_E_NOMEM;
        g.work = h->work;
      }
      out[(*nout)++] = L;
    }
  }
  return TLA_OK;
}

// Enqueues the work-list preparation and the class workers; r holds the
// work-list buffers (the handle's, or the allocation-free entry point's).
static tla_status rag_enqueue(hipStream_t st, const RagArgs& r, const RagLaunch* plan, int nplan) {
  const int tpb = 256, blocks = (r.batch + tpb - 1) / tpb;
  hipLaunchKernelGGL(k_rag_zero, dim3(8), dim3(256), 0, st, r);
  hipLaunchKernelGGL(k_rag_hist, dim3(blocks), dim3(tpb), 0, st, r);
  hipLaunchKernelGGL(k_rag_scan, dim3(1), dim3(256), 0, st, r);
  hipLaunchKernelGGL(k_rag_scatter, dim3(blocks), dim3(tpb), 0, st, r);
  for (int i = 0; i < nplan; ++i) {
    const RagLaunch& L = plan[i];
    hipLaunchKernelGGL(L.fn, dim3(L.grid), dim3(64 * L.waves), L.lds, st, r, L.g, L.rv, L.cls, L.slot);
  }
  return hipGetLastError() == hipSuccess ? TLA_OK : TLA_E_HIP;
}

extern "C" tla_status tla_ragged_batched(tla_handle h, tla_prec prec, int batch, int n_max, const tla_desc* d,
                                         int* info, tla_stat* stat) {
  if (!h || batch < 0 || n_max < 0 || prec < TLA_F64 || prec > TLA_MIXED_BF16) return TLA_E_ARG;
  if (batch == 0) return TLA_OK;
  if (!d || !info) return TLA_E_ARG;
  if (n_max > kMaxN) return TLA_E_UNSUPPORTED;
  if (prec == TLA_MIXED_F16 || prec == TLA_MIXED_BF16) return TLA_E_UNSUPPORTED;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  if (!h->rag) {
    h->rag = new (std::nothrow) RagState();
    if (!h->rag) return TLA_E_NOMEM;
    if (hipStreamCreateWithFlags(&h->rag->cap_stream, hipStreamNonBlocking) != hipSuccess) return TLA_E_HIP;
  }
  RagState* s = h->rag;
  if (batch > s->buf.cap) {
    hipDeviceSynchronize();
    rag_drop_graphs(s);
    hipFree(s->buf.queue);
    if (hipMalloc(&s->buf.queue, (size_t)batch * sizeof(int)) != hipSuccess) return TLA_E_NOMEM;
    s->buf.cap = batch;
  }
  if (!s->buf.rank) {
    std::vector<int> rank = cost_rank();
    if (hipMalloc(&s->buf.rank, rank.size() * sizeof(int)) != hipSuccess ||
        hipMalloc(&s->buf.keycount, kRagKeys * sizeof(int)) != hipSuccess ||
        hipMalloc(&s->buf.keyoff, kRagKeys * sizeof(int)) != hipSuccess ||
        hipMalloc(&s->buf.cls, 16 * sizeof(int)) != hipSuccess)
      return TLA_E_NOMEM;
    if (hipMemcpy(s->buf.rank, rank.data(), rank.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
      return TLA_E_HIP;
  }
  // the mixed second pass reads refinement records: use the handle's when none given
  tla_stat* st = stat;
  if (prec != TLA_F64) {
    // workspace for the FP64 solutions of the largest class (one slot per persistent workgroup)
    const size_t np = 128, slot = (3 * np * (np + 1) + 1) / 2 * sizeof(double);  // solution + an FP32 matrix
    const size_t need = (size_t)h->num_cu * 8 * slot;
    if (need > h->work_bytes || (!stat && (size_t)batch > h->stat_cap)) {
      hipDeviceSynchronize();
      ++h->gen;
      if (need > h->work_bytes) {
        hipFree(h->work);
        h->work = nullptr;
        h->work_bytes = 0;
        if (hipMalloc(&h->work, need) != hipSuccess) return TLA_E_NOMEM;
        h->work_bytes = need;
      }
      if (!stat && (size_t)batch > h->stat_cap) {
        hipFree(h->stat_buf);
        h->stat_buf = nullptr;
        h->stat_cap = 0;
        if (hipMalloc(&h->stat_buf, (size_t)batch * sizeof(tla_stat)) != hipSuccess) return TLA_E_NOMEM;
        h->stat_cap = batch;
      }
    }
    if (!st) st = h->stat_buf;
  }
  // graphs captured before a workspace reallocation, a refinement-setting
  // change or a tuning-table change hold stale pointers or parameters
  if (s->gen != h->gen) {
    rag_drop_graphs(s);
    s->gen = h->gen;
  }
  for (auto& e : s->graphs) {
    if (e.d == d && e.batch == batch && e.n_max == n_max && e.prec == prec && e.info == info && e.stat == st &&
        e.stream == (void*)h->stream) {
      return hipGraphLaunch(e.exec, h->stream) == hipSuccess ? TLA_OK : TLA_E_HIP;
    }
  }
  RagLaunch plan[kRagMaxLaunches];
  int nplan = 0;
  tla_status ps = rag_plan(h, prec, batch, n_max, st, plan, &nplan);
  if (ps != TLA_OK) return ps;
  const RagArgs r{d, batch, n_max, info, st, s->buf.rank, s->buf.keycount, s->buf.keyoff, s->buf.queue, s->buf.cls};
  if (getenv("TLA_NO_GRAPH")) return rag_enqueue(h->stream, r, plan, nplan);
  // capture the whole sequence once; later calls replay it
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(s->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return TLA_E_HIP;
  tla_status rs = rag_enqueue(s->cap_stream, r, plan, nplan);
  hipError_t ce = hipStreamEndCapture(s->cap_stream, &graph);
  if (rs != TLA_OK) { if (graph) hipGraphDestroy(graph); return rs; }
  if (ce != hipSuccess) return TLA_E_HIP;
  hipGraphExec_t exec = nullptr;
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) { hipGraphDestroy(graph); return TLA_E_HIP; }
  s->graphs.push_back({d, batch, n_max, prec, info, st, (void*)h->stream, exec, graph});
  return hipGraphLaunch(exec, h->stream) == hipSuccess ? TLA_OK : TLA_E_HIP;
}

// ----------------------------------------------------- allocation-free path
// For callers that cannot allocate (code under HIP graph capture, serving
// loops): the work-list buffers live in one file-scope device array instead of
// handle-owned allocations.  Layout in ints: the cost-rank table, the key
// histogram and offsets, the class ranges and counters, then the queue of up
// to kNoAllocMaxBatch instances (4 MiB in all).
namespace tla {
constexpr int kNoAllocMaxBatch = 1 << 20;
constexpr int kNaRank = 0, kNaKeyCount = 512, kNaKeyOff = kNaKeyCount + 1280, kNaCls = kNaKeyOff + 1280,
              kNaQueue = 4096;
static_assert(3 * (kMaxN + 1) <= kNaKeyCount - kNaRank && kRagKeys <= 1280 && kNaCls + 16 <= kNaQueue,
              "scratch layout");
constexpr int kNaInts = kNaQueue + kNoAllocMaxBatch;
constexpr int kNaMaxDevices = 64;
}  // namespace tla

// Each GPU holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns for that device (never through this name).
static __device__ __align__(256) int scratch[tla::kNaInts];

namespace tla {
static int* g_na_ptr[kNaMaxDevices] = {};

// Called once per device by tla_create with that device current: looks up
// this device's copy of the scratch array and writes the cost-rank table
// into it (the table never changes afterwards).
tla_status noalloc_init(int device) {
  if (device < 0 || device >= kNaMaxDevices) return TLA_E_UNSUPPORTED;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (g_na_ptr[device]) return TLA_OK;
  int* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return TLA_E_HIP;
  const std::vector<int> rank = cost_rank();
  if (hipMemcpy(ptr + kNaRank, rank.data(), rank.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return TLA_E_HIP;
  g_na_ptr[device] = ptr;
  return TLA_OK;
}
}  // namespace tla

// Same work and results as tla_ragged_batched for FP64 (the same class
// workers and per-instance bodies), enqueued directly on the handle's stream:
// no allocation, no graph capture.  Every call on a GPU shares that GPU's
// scratch array, so calls that overlap on one GPU race.
extern "C" tla_status tla_ragged_batched_noalloc(tla_handle h, tla_prec prec, int batch, int n_max,
                                                 const tla_desc* d, int* info, tla_stat* stat) {
  if (!h || batch < 0 || n_max < 0 || prec < TLA_F64 || prec > TLA_MIXED_BF16) return TLA_E_ARG;
  if (batch > kNoAllocMaxBatch) return TLA_E_ARG;
  if (batch == 0) return TLA_OK;
  if (!d || !info) return TLA_E_ARG;
  if (n_max > kMaxN) return TLA_E_UNSUPPORTED;
  if (prec != TLA_F64) return TLA_E_UNSUPPORTED;
  if (h->device < 0 || h->device >= kNaMaxDevices || !g_na_ptr[h->device]) return TLA_E_HIP;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  RagLaunch plan[kRagMaxLaunches];
  int nplan = 0;
  tla_status ps = rag_plan(h, prec, batch, n_max, stat, plan, &nplan);
  if (ps != TLA_OK) return ps;
  int* p = g_na_ptr[h->device];
  const RagArgs r{d, batch, n_max, info, stat, p + kNaRank, p + kNaKeyCount, p + kNaKeyOff, p + kNaQueue, p + kNaCls};
  return rag_enqueue(h->stream, r, plan, nplan);
}
