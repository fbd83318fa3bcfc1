// FP64 Sylvester kernels: every (variant, tile/engine, waves, L/U placement).
#include "tla_kernels.hpp"
#include "tla_registry.h"

namespace tla {
namespace {
template <int VAR, int TE, int NWI, int LU>
void fill(KFn* tab) {
  constexpr int TB = TE == 0 ? 8 : 16;
  constexpr int ENG = TE == 2 ? ENG_MFMA : ENG_VALU;
  constexpr int NW = NWI == 0 ? 1 : (NWI == 1 ? 2 : 4);
  tab[((VAR * kNumTE + TE) * kNumNW + NWI) * 2 + LU] = reinterpret_cast<KFn>(&k_trsyl_f64<TB, ENG, NW, VAR, LU == 1>);
  if constexpr (LU == 0) fill<VAR, TE, NWI, 1>(tab);
  else if constexpr (NWI + 1 < kNumNW) fill<VAR, TE, NWI + 1, 0>(tab);
  else if constexpr (TE + 1 < kNumTE) fill<VAR, TE + 1, 0, 0>(tab);
  else if constexpr (VAR + 1 < SYL_NVAR) fill<VAR + 1, 0, 0, 0>(tab);
}
}  // namespace

KFn trsyl_f64_kernel(int var, int te, int nwi, bool lu_lds) {
  static KFn tab[SYL_NVAR * kNumTE * kNumNW * 2] = {};
  static bool init = false;
  if (!init) { fill<0, 0, 0, 0>(tab); init = true; }
  if (var < 0 || var >= SYL_NVAR || te < 0 || te >= kNumTE || nwi < 0 || nwi >= kNumNW) return nullptr;
  return tab[((var * kNumTE + te) * kNumNW + nwi) * 2 + (lu_lds ? 1 : 0)];
}
}  // namespace tla
