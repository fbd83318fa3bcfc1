// Learned cost model (placeholder until the MLP kernels land).
#include "tla_host.h"
namespace tla {
bool mlp_pick(tla_ctx*, int, int, int, int, tla_plan*) { return false; }
void mlp_release(tla_ctx*) {}
}  // namespace tla
