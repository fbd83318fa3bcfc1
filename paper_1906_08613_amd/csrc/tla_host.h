// Host-side state of a libtla handle.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "../../include/tla.h"
#include "tla_registry.h"

namespace tla {

constexpr int kMaxN = 128;        // largest n of the LDS-resident kernels (and of ragged batches)
constexpr int kMaxLargeN = 4096;  // largest n of the in-place global-memory kernels

struct TuneRecord {
  int op, n, prec, batch;
  tla_plan plan;
  double seconds;
};

struct MlpState;  // learned cost model (tla_mlp.hip)
struct JitState;  // exact-size kernels compiled at run time (tla_jit.hip)
struct RagState;  // ragged batches: work-list buffers and captured graphs (tla_ragged.hip)

}  // namespace tla

struct tla_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int lds_limit = 160 * 1024;
  int num_cu = 256;
  double tau = 1e-13;
  int max_iter = 8;
  int picker = TLA_PICK_TABLE;
  std::map<int, tla_plan> forced;                 // key op*8 + prec
  std::vector<tla::TuneRecord> records;           // every measurement
  std::map<long long, tla_plan> best;             // key (op, n, prec) -> fastest plan
  tla::MlpState* mlp = nullptr;
  tla::RagState* rag = nullptr;
  tla::JitState* jit = nullptr;
  int exact_size = 0;                             // exact-size kernels: 0 off, 1 on, 2 where measured faster
  std::map<long long, bool> exact_choice;         // mode 2: key (op, n, variant, waves) -> measured verdict
  double* work = nullptr;                         // FP64 workspace of the mixed kernels
  size_t work_bytes = 0;
  double* ge_work = nullptr;                      // general-equation front end: Schur factors, pointer arrays
  size_t ge_bytes = 0;
  void* panel_work = nullptr;                     // large Cholesky by block panels: per-instance arrays
  size_t panel_bytes = 0;
  tla_stat* stat_buf = nullptr;                   // refinement records when the caller passes none
  size_t stat_cap = 0;
  // Bumped whenever something a captured ragged graph has baked in changes:
  // the workspace or refinement-record buffers are reallocated, the
  // refinement settings change, or the tuning table / picker changes.
  // Cached graphs from an older generation are dropped before any replay.
  unsigned long long gen = 0;
  // The measured autotuner as the judge of the learned picker: predictions
  // within a factor (1 + judge_margin) of the best one are timed (at most
  // judge_max of them) and the measured winner is kept per (op, n, prec).
  double judge_margin = 0.10;
  int judge_max = 4;
  int judged = 0, mispredicted = 0;
  std::map<long long, tla_plan> judged_plans;     // key (op, n, prec) -> measured winner
  void release();
};

namespace tla {
inline long long table_key(int op, int n, int prec) { return ((long long)op * 16 + prec) * 100000 + n; }
bool table_pick(tla_ctx* h, int op, int n, int prec, int batch, tla_plan* p);
bool mlp_pick(tla_ctx* h, int op, int n, int prec, int batch, tla_plan* p);
// Times `count` plans of (op, n, prec) on synthetic inputs of `batch`
// instances (the autotuner's timer, synchronous) into sec[]; an unsupported
// plan gets +infinity.
tla_status judge_time(tla_ctx* h, int op, int n, int prec, int batch, const tla_plan* plans, int count, double* sec);
void mlp_release(tla_ctx* h);
void ragged_release(tla_ctx* h);
void jit_release(tla_ctx* h);
// Exact-size in-place FP64 kernel of (op, n_max, variant, waves): TLA_OK when
// launched, TLA_E_UNSUPPORTED (nothing launched) when none can be had.
tla_status jit_launch(tla_ctx* h, int op, int var, int nw, size_t lds, const KArgs& a);
// Times plan p of (op, n, FP64) with the exact-size kernels off and on (the
// autotuner's timer, synthetic inputs); *use_exact when on measured at least
// 2% faster.
tla_status exact_size_decide(tla_ctx* h, int op, int n, int batch, const tla_plan& p, bool* use_exact);
// Per-device set-up of the allocation-free ragged path (tla_ragged.hip).
tla_status noalloc_init(int device);
tla_status launch(tla_ctx* h, int op, int prec, const tla_plan& p, const KArgs& a);
// Large FP64 Cholesky, left-looking by block panels (tla_panel.hip).
tla_status potrf_panel(tla_ctx* h, const KArgs& a);
// Large FP64 Sylvester by a wavefront over 128 x 128 blocks (tla_panel.hip).
tla_status trsyl_blocks(tla_ctx* h, const KArgs& a);
size_t lds_bytes(int op, int prec, int tb, int nw, int ntmax, int placement);
int choose_placement(tla_ctx* h, int op, int prec, const tla_plan& p, int ntmax, size_t* lds);
bool plan_valid(int op, const tla_plan& p);
bool is_jacobi(int op, int variant);
bool plan_runs(int op, int prec, int n, const tla_plan& p);
int num_candidates(int op);
bool candidate(int op, int i, tla_plan* p);
tla_plan default_plan(int op, int n, int prec);
}  // namespace tla
