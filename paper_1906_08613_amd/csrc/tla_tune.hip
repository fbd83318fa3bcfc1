// Autotuner: times every candidate plan on synthetic device inputs and keeps
// the fastest per (op, n, precision), as the paper's generator does with its
// alternative algorithms and implementation parameters (Generator structure
// paragraph, autotuning).  Timing uses HIP events around single launches;
// in-place inputs are restored from pristine copies between launches,
// outside the timed interval.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tla_host.h"

using namespace tla;

namespace {

// counter-based 64-bit mixer (SplitMix64 finaliser) for device-side inputs
__device__ inline unsigned long long mix64(unsigned long long z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ inline double u01(unsigned long long s) { return (double)(mix64(s) >> 11) * 0x1.0p-53; }

// kind 0: SPD by diagonal dominance (n + U[0,1] on the diagonal, U[-1,1] off);
// kind 1: lower triangular, off-diagonal U[-1,1]/n, diagonal U[1,2];
// kind 2: upper triangular, same; kind 3: dense U[-1,1].
__global__ void k_fill(double* M, int n, int batch, int kind, unsigned long long seed) {
  const long long per = (long long)n * n;
  const long long total = per * batch;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long t = e % per;
    const int i = (int)(t % n), j = (int)(t / n);
    const long long b = e / per;
    double v;
    if (kind == 0) {
      const int r = i < j ? i : j, c = i < j ? j : i;
      const double x = u01(seed ^ (unsigned long long)(b * per + r + (long long)c * n));
      v = (i == j) ? n + x : 2.0 * x - 1.0;
    } else {
      const double x = u01(seed ^ (unsigned long long)e);
      if (kind == 3) v = 2.0 * x - 1.0;
      else if (i == j) v = 1.0 + x;
      else if ((kind == 1 && i > j) || (kind == 2 && i < j)) v = (2.0 * x - 1.0) / n;
      else v = 0.0;
    }
    M[e] = v;
  }
}

__global__ void k_setup(int* nv, int* ld, double** pa, double** pb, double** pc, double* a, double* b,
                        double* c, int n, int batch) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < batch) {
    nv[i] = n;
    ld[i] = n;
    const long long off = (long long)i * n * n;
    pa[i] = a + off;
    pb[i] = b + off;
    pc[i] = c + off;
  }
}

struct Bench {
  int n = 0, batch = 0;
  int *nv = nullptr, *ld = nullptr, *info = nullptr;
  double **pa = nullptr, **pb = nullptr, **pc = nullptr;
  double *a = nullptr, *b = nullptr, *c = nullptr, *c0 = nullptr;
  tla_stat* stat = nullptr;
  ~Bench() {
    hipFree(nv); hipFree(ld); hipFree(info); hipFree(pa); hipFree(pb); hipFree(pc);
    hipFree(a); hipFree(b); hipFree(c); hipFree(c0); hipFree(stat);
  }
};

tla_status make_bench(Bench& B, int op, int n, int batch, hipStream_t s) {
  B.n = n;
  B.batch = batch;
  const size_t m = (size_t)n * n * batch * sizeof(double);
  if (hipMalloc(&B.nv, batch * sizeof(int)) != hipSuccess || hipMalloc(&B.ld, batch * sizeof(int)) != hipSuccess ||
      hipMalloc(&B.info, batch * sizeof(int)) != hipSuccess || hipMalloc(&B.pa, batch * sizeof(double*)) != hipSuccess ||
      hipMalloc(&B.pb, batch * sizeof(double*)) != hipSuccess || hipMalloc(&B.pc, batch * sizeof(double*)) != hipSuccess ||
      hipMalloc(&B.a, m) != hipSuccess || hipMalloc(&B.b, m) != hipSuccess || hipMalloc(&B.c, m) != hipSuccess ||
      hipMalloc(&B.c0, m) != hipSuccess || hipMalloc(&B.stat, batch * sizeof(tla_stat)) != hipSuccess)
    return TLA_E_NOMEM;
  const int blocks = 1024;
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, B.a, n, batch, 1, 0x1234ull);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, B.b, n, batch, 2, 0x5678ull);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, B.c0, n, batch, op == TLA_POTRF ? 0 : 3, 0x9abcull);
  hipLaunchKernelGGL(k_setup, dim3((batch + 255) / 256), dim3(256), 0, s, B.nv, B.ld, B.pa, B.pb, B.pc, B.a, B.b,
                     B.c, n, batch);
  if (hipGetLastError() != hipSuccess) return TLA_E_HIP;
  return TLA_OK;
}

tla_status time_plan(tla_ctx* h, Bench& B, int op, int prec, const tla_plan& p, int reps, double* sec) {
  KArgs a{};
  a.batch = B.batch;
  a.n_max = B.n;
  a.n = B.nv;
  a.a = B.pa;
  a.lda = B.ld;
  a.b = B.pb;
  a.ldb = B.ld;
  a.c = B.pc;
  a.ldc = B.ld;
  a.info = B.info;
  a.stat = B.stat;
  const size_t m = (size_t)B.n * B.n * B.batch * sizeof(double);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TLA_E_HIP;
  std::vector<float> t;
  tla_status st = TLA_OK;
  for (int r = -1; r < reps && st == TLA_OK; ++r) {  // r = -1 is a warm-up
    if (hipMemcpyAsync(B.c, B.c0, m, hipMemcpyDeviceToDevice, h->stream) != hipSuccess) { st = TLA_E_HIP; break; }
    hipEventRecord(e0, h->stream);
    st = launch(h, op, prec, p, a);
    hipEventRecord(e1, h->stream);
    if (hipEventSynchronize(e1) != hipSuccess) { st = TLA_E_HIP; break; }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    if (r >= 0) t.push_back(ms);
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (st != TLA_OK) return st;
  std::sort(t.begin(), t.end());
  *sec = t.empty() ? 0.0 : 1e-3 * t[t.size() / 2];
  return TLA_OK;
}

}  // namespace

namespace tla {
tla_status exact_size_decide(tla_ctx* h, int op, int n, int batch, const tla_plan& p, bool* use_exact) {
  *use_exact = false;
  Bench B;
  tla_status st = make_bench(B, op, n, batch, h->stream);
  if (st != TLA_OK) return st;
  const int saved = h->exact_size;
  double tg = 0.0, te = 0.0;
  h->exact_size = 0;
  st = time_plan(h, B, op, TLA_F64, p, 3, &tg);
  if (st == TLA_OK) {
    h->exact_size = 1;
    st = time_plan(h, B, op, TLA_F64, p, 3, &te);
  }
  h->exact_size = saved;
  if (st == TLA_OK) *use_exact = te < 0.98 * tg;
  return st;
}

tla_status judge_time(tla_ctx* h, int op, int n, int prec, int batch, const tla_plan* plans, int count, double* sec) {
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  Bench B;
  tla_status st = make_bench(B, op, n, batch, h->stream);
  if (st != TLA_OK) return st;
  for (int i = 0; i < count; ++i) {
    sec[i] = INFINITY;
    double t = 0.0;
    const tla_status s = time_plan(h, B, op, prec, plans[i], 2, &t);
    if (s == TLA_OK) {
      sec[i] = t;
      h->records.push_back({op, n, prec, batch, plans[i], t});
    } else if (s != TLA_E_UNSUPPORTED) {
      return s;
    }
  }
  return TLA_OK;
}
}  // namespace tla

extern "C" tla_status tla_time_plan(tla_handle h, tla_op op, int n, tla_prec prec, int batch, const tla_plan* plan,
                                    int reps, double* seconds) {
  if (!h || !plan || !seconds || n < 1 || n > kMaxLargeN || batch < 1 || reps < 1 || op < 0 || op > 2) return TLA_E_ARG;
  if (!plan_valid(op, *plan)) return TLA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  Bench B;
  tla_status st = make_bench(B, op, n, batch, h->stream);
  if (st != TLA_OK) return st;
  return time_plan(h, B, op, prec, *plan, reps, seconds);
}

extern "C" tla_status tla_tune(tla_handle h, int n_ops, const int* ops, int n_ns, const int* ns, int n_precs,
                               const int* precs, int batch, int reps) {
  if (!h || n_ops < 1 || !ops || n_ns < 1 || !ns || n_precs < 1 || !precs || batch < 1 || reps < 1)
    return TLA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  for (int io = 0; io < n_ops; ++io) {
    const int op = ops[io];
    if (op < 0 || op > 2) return TLA_E_ARG;
    for (int in = 0; in < n_ns; ++in) {
      const int n = ns[in];
      if (n < 1 || n > kMaxLargeN) return TLA_E_ARG;
      Bench B;
      tla_status st = make_bench(B, op, n, batch, h->stream);
      if (st != TLA_OK) return st;
      for (int ip = 0; ip < n_precs; ++ip) {
        const int prec = precs[ip];
        double best = INFINITY;
        tla_plan bp{};
        bool seen[16] = {};  // by variant index (at most 9 variants)
        for (int c = 0; c < num_candidates(op); ++c) {
          tla_plan p;
          candidate(op, c, &p);
          // above the LDS-resident sizes only the variant selects a kernel
          if (n > kMaxN) {
            if (seen[p.variant]) continue;
            seen[p.variant] = true;
          }
          double sec = 0;
          st = time_plan(h, B, op, prec, p, reps, &sec);
          if (st == TLA_E_UNSUPPORTED) continue;
          if (st != TLA_OK) return st;
          h->records.push_back(TuneRecord{op, n, prec, batch, p, sec});
          if (sec < best) { best = sec; bp = p; }
        }
        if (best < INFINITY) h->best[table_key(op, n, prec)] = bp;
      }
    }
  }
  ++h->gen;  // the table changed: cached ragged graphs hold the old variants
  return TLA_OK;
}

namespace tla {
bool table_pick(tla_ctx* h, int op, int n, int prec, int batch, tla_plan* p) {
  (void)batch;
  if (h->best.empty()) return false;
  // exact n, else the tuned n of the same (op, prec) nearest in log scale
  auto it = h->best.find(table_key(op, n, prec));
  if (it != h->best.end()) { *p = it->second; return true; }
  double bestd = INFINITY;
  bool found = false;
  for (auto& kv : h->best) {
    const long long k = kv.first;
    const int kn = (int)(k % 100000), kop = (int)(k / 100000 / 16), kprec = (int)(k / 100000 % 16);
    if (kop != op || kprec != prec) continue;
    const double d = std::fabs(std::log((double)kn / (double)(n > 0 ? n : 1)));
    if (d < bestd) { bestd = d; *p = kv.second; found = true; }
  }
  return found;
}
}  // namespace tla

extern "C" tla_status tla_save_table(tla_handle h, const char* path) {
  if (!h || !path) return TLA_E_ARG;
  FILE* f = fopen(path, "w");
  if (!f) return TLA_E_ARG;
  fprintf(f, "# op n prec batch variant tile engine waves place seconds\n");
  for (auto& r : h->records)
    fprintf(f, "%d %d %d %d %d %d %d %d %d %.9e\n", r.op, r.n, r.prec, r.batch, r.plan.variant, r.plan.tile,
            r.plan.engine, r.plan.waves, r.plan.place, r.seconds);
  fclose(f);
  return TLA_OK;
}

extern "C" tla_status tla_load_table(tla_handle h, const char* path) {
  if (!h || !path) return TLA_E_ARG;
  FILE* f = fopen(path, "r");
  if (!f) return TLA_E_ARG;
  char line[512];
  std::map<long long, double> bt;
  for (auto& kv : h->best) bt[kv.first] = INFINITY;
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    TuneRecord r;
    if (sscanf(line, "%d %d %d %d %d %d %d %d %d %lf", &r.op, &r.n, &r.prec, &r.batch, &r.plan.variant,
               &r.plan.tile, &r.plan.engine, &r.plan.waves, &r.plan.place, &r.seconds) != 10)
      continue;
    if (!plan_valid(r.op, r.plan)) continue;
    h->records.push_back(r);
    const long long k = table_key(r.op, r.n, r.prec);
    auto it = bt.find(k);
    if (it == bt.end() || r.seconds < it->second) { bt[k] = r.seconds; h->best[k] = r.plan; }
  }
  fclose(f);
  ++h->gen;
  return TLA_OK;
}

void tla_ctx::release() {
  tla::mlp_release(this);
  tla::ragged_release(this);
  tla::jit_release(this);
  if (work) hipFree(work);
  if (ge_work) hipFree(ge_work);
  if (panel_work) hipFree(panel_work);
  panel_work = nullptr;
  if (stat_buf) hipFree(stat_buf);
  work = nullptr;
  ge_work = nullptr;
  stat_buf = nullptr;
}
