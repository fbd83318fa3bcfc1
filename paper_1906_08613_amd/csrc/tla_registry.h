// Kernel lookup by plan.  Each operation/precision family exports one lookup
// function; `te` encodes (tile, engine): 0 = (8, vector ALU), 1 = (16, vector
// ALU), 2 = (16, matrix cores); `nwi` encodes waves per instance 1 / 2 / 4.
#pragma once
#include "tla_internal.h"

namespace tla {
typedef void (*KFn)(KArgs);
constexpr int kNumTE = 3, kNumNW = 3;
inline int te_index(int tile, int engine) { return tile == 8 ? 0 : (engine ? 2 : 1); }
inline int nw_index(int waves) { return waves == 1 ? 0 : (waves == 2 ? 1 : 2); }
inline int te_tile(int te) { return te == 0 ? 8 : 16; }

KFn potrf_f64_kernel(int var, int te, int nwi);
KFn trsyl_f64_kernel(int var, int te, int nwi, bool lu_lds);
KFn trlyap_f64_kernel(int var, int te, int nwi, bool lu_lds);
}  // namespace tla

namespace tla {
// Mixed-precision kernels.  te 0/1 run FP32 vector-ALU tile updates; te 2
// runs them on the matrix cores in the input type named by prec
// (TLA_MIXED_F32: FP32, TLA_MIXED_F16: FP16, TLA_MIXED_BF16: BF16).
// placement: potrf 0 = FP64 solution in LDS, 1 = in the global workspace;
// trsyl/trlyap 0 = coefficients and solution in LDS, 1 = coefficients read
// through the caches, 2 = solution in the global workspace as well.
KFn potrf_mixed_kernel(int prec, int var, int te, int nwi, int placement);
// FP32 work matrices and the FP64 solution in the workspace (placement 3, n up
// to 128); 16 x 16 matrix-core tiles in the type named by prec;
// nwi 0..2 = 1, 2, 4 waves.
KFn potrf_mixed_ws_kernel(int prec, int var, int nwi);
KFn trsyl_mixed_ws_kernel(int prec, int var, int nwi);
KFn trlyap_mixed_ws_kernel(int prec, int var, int nwi);
KFn trsyl_mixed_kernel(int prec, int var, int te, int nwi, int placement);
KFn trlyap_mixed_kernel(int prec, int var, int te, int nwi, int placement);
}  // namespace tla

namespace tla {
// In-place kernels over global memory, FP64, 16 x 16 matrix-core tiles.
// Large sizes (n above the LDS-resident maximum): one per variant, 16 waves
// per instance.  Placement 3 of the smaller sizes: nwi as above.
KFn large_kernel(int op, int var);
size_t large_lds_bytes();
int large_waves();
KFn inplace_kernel(int op, int var, int nwi);
size_t inplace_lds_bytes(int nw);
// Solve with the upper Cholesky factor (FP64, in place on B); nwi as above.
// KArgs: a = factor, lda, c = B, ldc, m / m_max = right-hand sides.
KFn potrs_kernel(int nwi);
size_t potrs_lds_bytes(int nw);
// Identity into c (n x n, ldc) of every valid instance; 256 threads.
KFn potri_eye_kernel();
}  // namespace tla

namespace tla {
// Mixed precision with the splitting-iteration low-precision solve
// (tla_jacobi.hip): Sylvester and Lyapunov, n <= kJacobiMaxN, products on the
// BF16 (split into head and tail) or FP32 matrix cores.  Returns null when not
// built for (op, prec, n_max); *lds / *waves receive the launch shape.
constexpr int kJacobiMaxN = 64;
KFn jacobi_kernel(int op, int prec, int n_max, size_t* lds, int* waves);
}  // namespace tla

