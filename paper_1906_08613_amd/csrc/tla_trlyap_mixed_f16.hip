// Mixed-precision trlyap kernels with f16 tile updates on the matrix cores.
// Index: (variant, tile/engine, waves, placement); placement 0: coefficients and FP64 solution in LDS; 1: coefficients read through the caches; 2: FP64 solution in the global workspace too.
#include "tla_mixed.hpp"
#include "tla_registry.h"

namespace tla {
namespace {
constexpr int kPL = 3;
template <int VAR, int TE, int NWI, int PL>
void fill(KFn* tab) {
  constexpr int TB = TE == 0 ? 8 : 16;
  constexpr int ENG = TE == 2 ? ENG_MFMA_F16 : ENG_VALU;
  constexpr int NW = NWI == 0 ? 1 : (NWI == 1 ? 2 : 4);
  tab[((VAR * kNumTE + TE) * kNumNW + NWI) * kPL + PL] = reinterpret_cast<KFn>(&k_trlyap_mixed<TB, ENG, NW, VAR, PL == 0, PL == 2>);
  if constexpr (PL + 1 < kPL) fill<VAR, TE, NWI, PL + 1>(tab);
  else if constexpr (NWI + 1 < kNumNW) fill<VAR, TE, NWI + 1, 0>(tab);
  else if constexpr (TE + 1 < kNumTE) fill<VAR, TE + 1, 0, 0>(tab);
  else if constexpr (VAR + 1 < LYA_NVAR) fill<VAR + 1, 2, 0, 0>(tab);
}
}  // namespace

KFn trlyap_mixed_kernel_f16(int var, int te, int nwi, int pl) {
  static KFn tab[LYA_NVAR * kNumTE * kNumNW * kPL] = {};
  static bool init = false;
  if (!init) { fill<0, 2, 0, 0>(tab); init = true; }
  if (var < 0 || var >= LYA_NVAR || te < 2 || te >= kNumTE || nwi < 0 || nwi >= kNumNW || pl < 0 || pl >= kPL)
    return nullptr;
  return tab[((var * kNumTE + te) * kNumNW + nwi) * kPL + pl];
}
// Work matrices in the workspace (placement 3, sizes up to the
// LDS-resident ones): 16 x 16 tiles on the matrix cores, waves 1 / 2 / 4.
namespace {
template <int VAR, int NWI>
void fill_ws(KFn* tab) {
  constexpr int NW = NWI == 0 ? 1 : (NWI == 1 ? 2 : 4);
  tab[VAR * 3 + NWI] = reinterpret_cast<KFn>(&k_trlyap_mixed<16, ENG_MFMA_F16, NW, VAR, false, true, true>);
  if constexpr (NWI + 1 < 3) fill_ws<VAR, NWI + 1>(tab);
  else if constexpr (VAR + 1 < LYA_NVAR) fill_ws<VAR + 1, 0>(tab);
}
}  // namespace

KFn trlyap_mixed_ws_kernel_f16(int var, int nwi) {
  static KFn tab[LYA_NVAR * 3] = {};
  static bool init = false;
  if (!init) { fill_ws<0, 0>(tab); init = true; }
  if (var < 0 || var >= LYA_NVAR || nwi < 0 || nwi >= 3) return nullptr;
  return tab[var * 3 + nwi];
}
}  // namespace tla
