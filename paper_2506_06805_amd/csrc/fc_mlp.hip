// Learned amplitude update (placeholder until the MLP kernels land).
#include "fc_state.hpp"
namespace fc {
int learned_step(fc_ctx, fc_ints, const void*, const z*, const z*, const z*, const z*, z*, z*) {
  throw Error(FC_EUNSUPPORTED, "learned update not available");
}
}  // namespace fc
