// In-place kernels over global memory (FP64): the large sizes and placement 3.
#include "tla_inplace.hpp"
#include "tla_registry.h"

namespace tla {

// One-wave in-place kernels (placement 3 of the sizes up to 128) are held to
// the register budget of 4 (Cholesky) or 5 (tile-wavefront Sylvester and
// Lyapunov) resident waves per SIMD: at n = 64 that measured 10% (Cholesky)
// and 2-3% (Sylvester) faster than the compiler's own choice of 3 or 4.  The
// other Sylvester and Lyapunov variants would spill at that budget.
template <int NW>
constexpr int kInplaceWavesChol = NW == 1 ? 4 : 1;
template <int NW, int VAR>
constexpr int kInplaceWaves = NW == 1 && VAR == 0 ? 5 : 1;

template <int NW, int VAR>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(kInplaceWavesChol<NW>))) void k_potrf_large(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  potrf_inplace_body<NW, VAR>(g, fetch_uniform(g, blockIdx.x), smem);
}
template <int NW, int VAR>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(kInplaceWaves<NW, VAR>))) void k_trsyl_large(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trsyl_inplace_body<NW, VAR>(g, fetch_uniform(g, blockIdx.x), smem);
}
template <int NW, int VAR>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(kInplaceWaves<NW, VAR>))) void k_trlyap_large(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trlyap_inplace_body<NW, VAR>(g, fetch_uniform(g, blockIdx.x), smem);
}

template <int NW>
static KFn inplace_kernel_nw(int op, int var) {
  static_assert(CHOL_NVAR == 3 && SYL_NVAR == 8 && LYA_NVAR == 4, "one case per variant below");
  if (op == TLA_POTRF) {
    switch (var) {
      case 0: return reinterpret_cast<KFn>(&k_potrf_large<NW, 0>);
      case 1: return reinterpret_cast<KFn>(&k_potrf_large<NW, 1>);
      case 2: return reinterpret_cast<KFn>(&k_potrf_large<NW, 2>);
    }
  } else if (op == TLA_TRSYL) {
    switch (var) {
      case 0: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 0>);
      case 1: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 1>);
      case 2: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 2>);
      case 3: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 3>);
      case 4: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 4>);
      case 5: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 5>);
      case 6: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 6>);
      case 7: return reinterpret_cast<KFn>(&k_trsyl_large<NW, 7>);
    }
  } else if (op == TLA_TRLYAP) {
    switch (var) {
      case 0: return reinterpret_cast<KFn>(&k_trlyap_large<NW, 0>);
      case 1: return reinterpret_cast<KFn>(&k_trlyap_large<NW, 1>);
      case 2: return reinterpret_cast<KFn>(&k_trlyap_large<NW, 2>);
      case 3: return reinterpret_cast<KFn>(&k_trlyap_large<NW, 3>);
    }
  }
  return nullptr;
}

KFn large_kernel(int op, int var) { return inplace_kernel_nw<kLargeNW>(op, var); }
size_t large_lds_bytes() { return inplace_lds_bytes(kLargeNW); }
int large_waves() { return kLargeNW; }

KFn inplace_kernel(int op, int var, int nwi) {
  switch (nwi) {
    case 0: return inplace_kernel_nw<1>(op, var);
    case 1: return inplace_kernel_nw<2>(op, var);
    case 2: return inplace_kernel_nw<4>(op, var);
  }
  return nullptr;
}
size_t inplace_lds_bytes(int nw) { return (size_t)nw * wave_scratch(kLargeTB) * sizeof(double) + 16; }

}  // namespace tla
