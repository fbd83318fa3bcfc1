// FP32-I/O entry points: the three operations of the paper's Fig. 2 on
// single-precision matrices, solved in single precision.  They run the same
// in-place blocked bodies as the FP64 kernels with float elements: 16 x 16
// tiles in the FP32 matrix-core layout (v_mfma_f32_16x16x4f32 for the tile
// updates), the register-blocked diagonal-tile solvers in FP32, and the
// caller's matrices solved in place in global memory with only the tile
// solvers' scratch in LDS.  The plan is the FP64 default of the same size:
// bordered Cholesky up to n = 128 and left-looking above, the tile wavefront
// for the Sylvester and Lyapunov equations; one wavefront per instance up to
// n = 64, two or four up to 128, sixteen above.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#include "tla_host.h"
#include "tla_inplace.hpp"

namespace tla {
namespace {

template <int NW, int VAR>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW == 1 ? 4 : 1))) void k_spotrf(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  potrf_inplace_body<NW, VAR, float>(g, fetch_uniform(g, blockIdx.x), smem);
}
template <int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW == 1 ? 5 : 1))) void k_strsyl(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trsyl_inplace_body<NW, SYL_WF, float>(g, fetch_uniform(g, blockIdx.x), smem);
}
template <int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW == 1 ? 5 : 1))) void k_strlyap(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trlyap_inplace_body<NW, LYA_WF, float>(g, fetch_uniform(g, blockIdx.x), smem);
}

// waves per instance for (op, n_max): the FP64 default plan's choice
int single_waves(int op, int n_max) {
  if (n_max > kMaxN) return kLargeNW;
  if (op == TLA_POTRF || n_max <= 64) return 1;
  return op == TLA_TRSYL ? 4 : 2;
}

KFn single_kernel(int op, int nw) {
  if (op == TLA_POTRF) {
    if (nw == 1) return reinterpret_cast<KFn>(&k_spotrf<1, CHOL_BD>);
    if (nw == kLargeNW) return reinterpret_cast<KFn>(&k_spotrf<kLargeNW, CHOL_LL>);
  } else if (op == TLA_TRSYL) {
    switch (nw) {
      case 1: return reinterpret_cast<KFn>(&k_strsyl<1>);
      case 4: return reinterpret_cast<KFn>(&k_strsyl<4>);
      case kLargeNW: return reinterpret_cast<KFn>(&k_strsyl<kLargeNW>);
    }
  } else if (op == TLA_TRLYAP) {
    switch (nw) {
      case 1: return reinterpret_cast<KFn>(&k_strlyap<1>);
      case 2: return reinterpret_cast<KFn>(&k_strlyap<2>);
      case kLargeNW: return reinterpret_cast<KFn>(&k_strlyap<kLargeNW>);
    }
  }
  return nullptr;
}

tla_status launch_single(tla_ctx* h, int op, KArgs a) {
  const int nw = single_waves(op, a.n_max);
  KFn fn = single_kernel(op, nw);
  if (!fn) return TLA_E_UNSUPPORTED;
  a.ntmax = (a.n_max + 15) / 16;
  a.tau = h->tau;
  a.max_iter = h->max_iter;
  const size_t lds = (size_t)nw * wave_scratch(kLargeTB) * sizeof(float) + 16;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
      hipSuccess)
    return TLA_E_HIP;
  hipLaunchKernelGGL(fn, dim3(a.batch), dim3(64 * nw), lds, h->stream, a);
  return hipGetLastError() == hipSuccess ? TLA_OK : TLA_E_HIP;
}

tla_status single_checks(tla_handle h, int batch, int n_max) {
  if (!h || batch < 0 || n_max < 0) return TLA_E_ARG;
  if (n_max > kMaxLargeN) return TLA_E_UNSUPPORTED;
  return TLA_OK;
}

}  // namespace
}  // namespace tla

using namespace tla;

// The pointer arrays hold float addresses; KArgs carries every matrix pointer
// untyped (the in-place bodies read them as float for these entry points).
extern "C" tla_status tla_spotrf_batched(tla_handle h, int batch, int n_max, const int* n, float* const* A,
                                         const int* lda, int* info) {
  tla_status s = single_checks(h, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !A || !lda || !info) return TLA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.c = reinterpret_cast<double* const*>(A);
  a.ldc = lda;
  a.info = info;
  return launch_single(h, TLA_POTRF, a);
}

extern "C" tla_status tla_strsyl_batched(tla_handle h, int batch, int n_max, const int* n, const float* const* L,
                                         const int* ldl, const float* const* U, const int* ldu, float* const* C,
                                         const int* ldc, int* info) {
  tla_status s = single_checks(h, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !L || !ldl || !U || !ldu || !C || !ldc || !info) return TLA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.a = reinterpret_cast<const double* const*>(L);
  a.lda = ldl;
  a.b = reinterpret_cast<const double* const*>(U);
  a.ldb = ldu;
  a.c = reinterpret_cast<double* const*>(C);
  a.ldc = ldc;
  a.info = info;
  return launch_single(h, TLA_TRSYL, a);
}

extern "C" tla_status tla_strlyap_batched(tla_handle h, int batch, int n_max, const int* n, const float* const* L,
                                          const int* ldl, float* const* S, const int* lds, int* info) {
  tla_status s = single_checks(h, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !L || !ldl || !S || !lds || !info) return TLA_E_ARG;
  if (hipSetDevice(h->device) != hipSuccess) return TLA_E_HIP;
  KArgs a{};
  a.batch = batch;
  a.n_max = n_max;
  a.n = n;
  a.a = reinterpret_cast<const double* const*>(L);
  a.lda = ldl;
  a.c = reinterpret_cast<double* const*>(S);
  a.ldc = lds;
  a.info = info;
  return launch_single(h, TLA_TRLYAP, a);
}
