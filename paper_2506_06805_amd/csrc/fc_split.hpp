// Split-precision operands (hi/lo 16-bit planes) and the NT product on them.
#pragma once
#include "fc_gemm.hpp"
#include "fc_internal.hpp"

namespace fc {

// staging choices of the 128-wide split tiles (fc_set_split_config): 0 register-staged 8 waves,
// 1 four waves, 2 direct-to-LDS 8 waves
constexpr int FC_SPLIT_NUM_CONFIGS = 3;
constexpr int FC_SPLIT_DEFAULT_CONFIG = 2;

struct SplitOp {
  DBuf buf;            // planes re_hi, re_lo, im_hi, im_lo, each [rows_pad][kp] (16-bit)
  long rows = 0, rows_pad = 0, kp = 0;
  double scale = 1.0;  // values stored as scale * x (a power of two; 1 when kb > 0)
  // kb > 0: column k stored as 2^bexp[k / kb] x instead (int per K batch, device) -- FP16 operands
  // whose contraction index is the Cholesky index, over which the vectors decay
  DBuf bexp;
  long kb = 0;
  int prec = FC_SPLIT_BF16;
};

// Split X[r * ldx + k] (r < rows, k < K), conjugated when conj.
SplitOp split_operand(fc_ctx ctx, int prec, const z* X, long rows, long K, long ldx, bool conj = false);
// Split X[r * ldx + colmap[k]] (colmap: device, K entries; negative entries give zero columns).
SplitOp split_operand_cols(fc_ctx ctx, int prec, const z* X, long rows, long K, long ldx, const int* colmap);
// The ladder's assembly operand: rows a v + e, columns P of s (L_ae^P - sum_m t_m^a L_me^P), from L_vv
// [a][e][P] in complex64 (l_c64) or complex128 and L_ov [m][e][P]; t1 (o x v) may be NULL (no
// dressing; with dressing o <= 64).  FP16 takes one power-of-two scale per batch of P from a bound on
// the dressed entries of that batch.
SplitOp split_lvv_dressed(fc_ctx ctx, int prec, const void* L, bool l_c64, const z* Lov, const z* t1, long o, long v,
                          long N);
// Zero the contraction columns [k0, kp) of every (padded) row of the four planes.
void split_zero_kpad(fc_ctx ctx, SplitOp& S, long k0);
// C[m][n] = alpha sum_k A[a_row0 + m][k] B[b_row0 + n][k] + beta C[m][n]
void gemm_split_nt(fc_ctx ctx, const SplitOp& A, long a_row0, long M, const SplitOp& B, long b_row0, long N, z alpha,
                   z beta, z* C, long ldc);

// Ladder assembly in split precision: FP32 complex W in the ladder layout (see LadderEpilogue).
void gemm_split_ladder(fc_ctx ctx, const SplitOp& A, long a_row0, long M, const SplitOp& B, long b_row0, long N,
                       float2* W, const LadderEpilogue& lep);

}  // namespace fc
