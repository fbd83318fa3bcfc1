// FP64 Cholesky kernels: every (variant, tile/engine, waves) combination.
#include "tla_kernels.hpp"
#include "tla_registry.h"

namespace tla {
namespace {
template <int VAR, int TE, int NWI>
void fill(KFn* tab) {
  constexpr int TB = TE == 0 ? 8 : 16;
  constexpr int ENG = TE == 2 ? ENG_MFMA : ENG_VALU;
  constexpr int NW = NWI == 0 ? 1 : (NWI == 1 ? 2 : 4);
  tab[(VAR * kNumTE + TE) * kNumNW + NWI] = reinterpret_cast<KFn>(&k_potrf_f64<TB, ENG, NW, VAR>);
  if constexpr (NWI + 1 < kNumNW) fill<VAR, TE, NWI + 1>(tab);
  else if constexpr (TE + 1 < kNumTE) fill<VAR, TE + 1, 0>(tab);
  else if constexpr (VAR + 1 < CHOL_NVAR) fill<VAR + 1, 0, 0>(tab);
}
}  // namespace

KFn potrf_f64_kernel(int var, int te, int nwi) {
  static KFn tab[CHOL_NVAR * kNumTE * kNumNW] = {};
  static bool init = false;
  if (!init) { fill<0, 0, 0>(tab); init = true; }
  if (var < 0 || var >= CHOL_NVAR || te < 0 || te >= kNumTE || nwi < 0 || nwi >= kNumNW) return nullptr;
  return tab[(var * kNumTE + te) * kNumNW + nwi];
}
}  // namespace tla
