// Dispatch of the mixed-precision kernels by precision of the tile updates.
#include "tla_registry.h"

namespace tla {
KFn potrf_mixed_kernel_f32(int, int, int, int);
KFn potrf_mixed_kernel_f16(int, int, int, int);
KFn potrf_mixed_kernel_bf16(int, int, int, int);
KFn trsyl_mixed_kernel_f32(int, int, int, int);
KFn trsyl_mixed_kernel_f16(int, int, int, int);
KFn trsyl_mixed_kernel_bf16(int, int, int, int);
KFn trlyap_mixed_kernel_f32(int, int, int, int);
KFn trlyap_mixed_kernel_f16(int, int, int, int);
KFn trlyap_mixed_kernel_bf16(int, int, int, int);

KFn potrf_mixed_ws_kernel_f32(int, int);
KFn potrf_mixed_ws_kernel_f16(int, int);
KFn potrf_mixed_ws_kernel_bf16(int, int);
KFn trsyl_mixed_ws_kernel_f32(int, int);
KFn trsyl_mixed_ws_kernel_f16(int, int);
KFn trsyl_mixed_ws_kernel_bf16(int, int);
KFn trlyap_mixed_ws_kernel_f32(int, int);
KFn trlyap_mixed_ws_kernel_f16(int, int);
KFn trlyap_mixed_ws_kernel_bf16(int, int);

// FP32 vector-ALU engines (te 0, 1) do not depend on the 16-bit type
static int eff_prec(int prec, int te) { return te < 2 ? TLA_MIXED_F32 : prec; }

KFn potrf_mixed_kernel(int prec, int var, int te, int nwi, int pl) {
  switch (eff_prec(prec, te)) {
    case TLA_MIXED_F32: return potrf_mixed_kernel_f32(var, te, nwi, pl);
    case TLA_MIXED_F16: return potrf_mixed_kernel_f16(var, te, nwi, pl);
    case TLA_MIXED_BF16: return potrf_mixed_kernel_bf16(var, te, nwi, pl);
  }
  return nullptr;
}
KFn trsyl_mixed_kernel(int prec, int var, int te, int nwi, int lu) {
  switch (eff_prec(prec, te)) {
    case TLA_MIXED_F32: return trsyl_mixed_kernel_f32(var, te, nwi, lu);
    case TLA_MIXED_F16: return trsyl_mixed_kernel_f16(var, te, nwi, lu);
    case TLA_MIXED_BF16: return trsyl_mixed_kernel_bf16(var, te, nwi, lu);
  }
  return nullptr;
}
KFn trlyap_mixed_kernel(int prec, int var, int te, int nwi, int lu) {
  switch (eff_prec(prec, te)) {
    case TLA_MIXED_F32: return trlyap_mixed_kernel_f32(var, te, nwi, lu);
    case TLA_MIXED_F16: return trlyap_mixed_kernel_f16(var, te, nwi, lu);
    case TLA_MIXED_BF16: return trlyap_mixed_kernel_bf16(var, te, nwi, lu);
  }
  return nullptr;
}
KFn potrf_mixed_ws_kernel(int prec, int var, int nwi) {
  switch (prec) {
    case TLA_MIXED_F32: return potrf_mixed_ws_kernel_f32(var, nwi);
    case TLA_MIXED_F16: return potrf_mixed_ws_kernel_f16(var, nwi);
    case TLA_MIXED_BF16: return potrf_mixed_ws_kernel_bf16(var, nwi);
  }
  return nullptr;
}
KFn trsyl_mixed_ws_kernel(int prec, int var, int nwi) {
  switch (prec) {
    case TLA_MIXED_F32: return trsyl_mixed_ws_kernel_f32(var, nwi);
    case TLA_MIXED_F16: return trsyl_mixed_ws_kernel_f16(var, nwi);
    case TLA_MIXED_BF16: return trsyl_mixed_ws_kernel_bf16(var, nwi);
  }
  return nullptr;
}
KFn trlyap_mixed_ws_kernel(int prec, int var, int nwi) {
  switch (prec) {
    case TLA_MIXED_F32: return trlyap_mixed_ws_kernel_f32(var, nwi);
    case TLA_MIXED_F16: return trlyap_mixed_ws_kernel_f16(var, nwi);
    case TLA_MIXED_BF16: return trlyap_mixed_ws_kernel_bf16(var, nwi);
  }
  return nullptr;
}
}  // namespace tla
