// GEMM variants used by the particle-particle ladder.
#pragma once
#include "fc_internal.hpp"

namespace fc {

// Output layout of the ladder assembly product: row m = (a - a0) v + e, column n = (b - b0) v + f
// is written to W[((m / v) nB + n / v) v^2 + (m % v) v + n % v], i.e. [(a, b)][e][f].  With
// `triangular` (a diagonal block pair, a0 == b0) output tiles whose smallest a exceeds their
// largest b are not computed.
struct LadderEpilogue {
  long v = 1, nB = 1;
  int triangular = 0;
};

// W = A B^T in the ladder layout, FP64 (A[m * lda + k], B[n * ldb + k]).
void zgemm_ladder(fc_ctx ctx, long M, long N, long K, const z* A, long lda, const z* B, long ldb, z* W,
                  const LadderEpilogue& lep);

}  // namespace fc
