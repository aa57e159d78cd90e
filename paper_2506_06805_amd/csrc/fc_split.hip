// Split-precision complex GEMM (placeholder until the MFMA split kernels land).
#include "fc_internal.hpp"
namespace fc {
void zgemm_split(fc_ctx, int, char, char, long, long, long, z, const z*, long, const z*, long, z, z*, long) {
  throw Error(FC_EUNSUPPORTED, "split-precision GEMM not available");
}
}  // namespace fc
