// Mixed-precision trsyl kernels with FP32 tile updates on the vector ALU
// (tile/engine index 0: 8 x 8 tiles, 1: 16 x 16 tiles); the matrix-core ones
// and the registry entry point are in tla_trsyl_mixed_f32.hip.
#include "tla_mixed.hpp"
#include "tla_registry.h"

namespace tla {
namespace {
constexpr int kPL = 3, kTE = 2;
template <int VAR, int TE, int NWI, int PL>
void fill(KFn* tab) {
  constexpr int TB = TE == 0 ? 8 : 16;
  constexpr int NW = NWI == 0 ? 1 : (NWI == 1 ? 2 : 4);
  tab[((VAR * kTE + TE) * kNumNW + NWI) * kPL + PL] = reinterpret_cast<KFn>(&k_trsyl_mixed<TB, ENG_VALU, NW, VAR, PL == 0, PL == 2>);
  if constexpr (PL + 1 < kPL) fill<VAR, TE, NWI, PL + 1>(tab);
  else if constexpr (NWI + 1 < kNumNW) fill<VAR, TE, NWI + 1, 0>(tab);
  else if constexpr (TE + 1 < kTE) fill<VAR, TE + 1, 0, 0>(tab);
  else if constexpr (VAR + 1 < SYL_NVAR) fill<VAR + 1, 0, 0, 0>(tab);
}
}  // namespace

KFn trsyl_mixed_kernel_f32_valu(int var, int te, int nwi, int pl) {
  static KFn tab[SYL_NVAR * kTE * kNumNW * kPL] = {};
  static bool init = false;
  if (!init) { fill<0, 0, 0, 0>(tab); init = true; }
  if (var < 0 || var >= SYL_NVAR || te < 0 || te >= kTE || nwi < 0 || nwi >= kNumNW || pl < 0 || pl >= kPL)
    return nullptr;
  return tab[((var * kTE + te) * kNumNW + nwi) * kPL + pl];
}
}  // namespace tla
