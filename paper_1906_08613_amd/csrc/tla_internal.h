// Internal types shared by the host library and its kernels.
#pragma once
#include "../../include/tla.h"

namespace tla {

// Per-wave LDS scratch of the tile solvers, in elements: two broadcast
// vectors of TB plus two staged TB x TB coefficient tiles (ld TB + 1).
__host__ __device__ constexpr int wave_scratch(int tb) { return 2 * tb + 2 * tb * (tb + 1); }

// Arguments of every batched kernel (device pointers, passed by value).
//   potrf : c = A (in/out), ldc
//   trsyl : a = L, b = U, c = C -> X
//   trlyap: a = L, c = S -> X
struct KArgs {
  int batch, n_max;
  int ntmax;             // tiles per dimension the LDS was sized for
  int max_iter;          // refinement: maximum number of corrections
  double tau;            // refinement: target backward error
  const int* n;
  const double* const* a;
  const int* lda;
  const double* const* b;
  const int* ldb;
  double* const* c;
  const int* ldc;
  int* info;
  tla_stat* stat;
  double* work;          // FP64 workspace, one slot per workgroup (mixed path), may be null
  long long work_stride; // doubles per slot in `work`
  int only_flagged;      // FP64 kernels: solve only instances whose stat asks for the FP64 path
  const int* m;          // solve with the factor: right-hand sides per instance
  int m_max;             // ... and their largest count
};

}  // namespace tla
