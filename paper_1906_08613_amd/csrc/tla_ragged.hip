// Ragged batches (placeholder until the persistent kernel lands).
#include "tla_host.h"
extern "C" tla_status tla_ragged_batched(tla_handle h, tla_prec prec, int batch, int n_max, const tla_desc* d,
                                         int* info, tla_stat* stat) {
  (void)prec; (void)n_max; (void)d; (void)info; (void)stat;
  if (!h || batch < 0) return TLA_E_ARG;
  return TLA_E_UNSUPPORTED;
}
