// Device-resident state behind the opaque handles of the C ABI.
#pragma once
#include "fc_internal.hpp"

// Integrals in the (possibly natural-spinor) basis.  Cholesky vectors are stored per block with
// the Cholesky index P fastest ([p][q][P]), the contraction dimension of every GEMM over P.
struct fc_ints_s {
  fc_ctx ctx = nullptr;
  int o = 0, v = 0, ncd = 0, precision = FC_FP64;
  std::vector<double> eps;        // host copy, n entries
  fc::DBuf eps_d;                 // device copy
  fc::ZTensor Loo, Lov, Lvo, Lvv; // L^P_ij, L^P_ia, L^P_ai, L^P_ab as [p][q][P]
  // complex64 vectors keep L^P_ab in complex64 ([a][b][P], float2); the complex128 copy in Lvv is
  // made on first use by a complex128 product (fc::lvv), so a ladder-only handle never holds it
  fc::DBuf Lvv64;
  // the stored integrals below are assembled on first use (fc::ensure_integrals)
  bool assembled = false;
  // stored antisymmetrised integrals with <= 2 virtual indices (Sec. 3)
  fc::ZTensor oooo, ooov, oovv, ovvo;  // <mn||ij>, <mn||ie>, <mn||ef>, <mb||ej>
  // the same integrals re-indexed (symmetry copies kept for contiguous GEMM operands)
  fc::ZTensor oovo, ovov, ovoo, vvoo;  // <mn||ej>, <ma||if> as [m][f][a][i], <mb||ij>, <ab||ij> as [i][j][a][b]
  fc::ZTensor oovv_r;                  // <mn||ef> as [m][e][n][f]: (n, f) contiguous for the ring terms
};

// H-bar blocks with at most two virtual indices, built once from converged amplitudes.
struct HbarBlocks {
  fc::ZTensor Fmi, Fae, Fme;           // F-bar_mi, F-bar_ae, F-bar_me
  fc::ZTensor Wmnij, Wmnie, Wmbej, Wmbij;
  bool ready = false;
};

// The sigma products rewritten as matrices over the packed 1h + 2h1p layout (r_i, then r_ij^a for
// i < j with a fastest), formed once from the H-bar blocks.  p = (i, j) and q = (m, n) run over
// occupied pairs with first < second, in lexicographic order.
struct SigmaOps {
  fc::ZTensor B1;    // [dim][o]: sigma_i = sum_x R[x] B1[x][i]  (F_mi, F_me and W_mnie terms)
  fc::ZTensor Xop;   // [(q, f)][e] = <mn||ef>: X_e = sum R[(q, f)] Xop[(q, f)][e]
  fc::ZTensor Wt;    // [(m, e)][(j, a)] = W_maej: the ring term over the unpacked r_im^e
  fc::ZTensor Mp;    // [p][q]: W_mnij and the P(ij) F_mi term, both mixing occupied pairs only
  fc::ZTensor B2;    // [o + v][(p, a)]: rows m: -W_maij; rows o + e: t_ij^ae
  fc::DBuf pairs;    // int2 (i, j) of each pair index
  bool ready = false;
  // left sigma (row vector times H-bar), formed on first use:
  fc::ZTensor BL1;   // [dim][o]: rows i < o: B1[m][i]; rows o + c: B2[m][c]   (t_m = sum_x Y[x] BL1[x][m])
  fc::ZTensor BL2;   // [o + v][(q, f)]: rows i: B1[o + (q, f)][i]; rows o + e: Xop[(q, f)][e]
  bool left_ready = false;
};

struct fc_amps_s {
  fc_ctx ctx = nullptr;
  fc_ints ints = nullptr;
  fc::ZTensor t1, t2;   // [i][a], [i][j][a][b]
  HbarBlocks hb;
  SigmaOps so;
};

namespace fc {
// fc_ccsd.hip
// fdiag (optional, o + v entries): diagonals of the F_mi and F_ae intermediates that multiply
// t_ij^ab in the T2 residual (F_mi + 1/2 t_j^e F_me and F_ae - 1/2 t_m^b F_me).
void ccsd_residual_dev(fc_ctx ctx, fc_ints I, const z* t1, const z* t2, z* r1, z* r2, int precision,
                       z* fdiag = nullptr);
// accumulate: R += the ladder term (no clear of R first)
void ladder_dev(fc_ctx ctx, fc_ints I, const z* tau, const z* t1dress, z* R, int precision, bool accumulate = false);
z ccsd_energy_dev(fc_ctx ctx, fc_ints I, const z* t1, const z* t2);
void assemble_integrals(fc_ctx ctx, fc_ints I);
// fc_integrals.hip: the stored integrals, assembled once on first use
void ensure_integrals(fc_ctx ctx, fc_ints I);
// L^P_ab in complex128 ([a][b][P]), widened once from the complex64 copy when that is all there is
const ZTensor& lvv(fc_ctx ctx, fc_ints I);
// the ladder with packed amplitudes: taup [i<j][e<f] and Rp [i<j][a<b] (complex128)
void ladder_packed_dev(fc_ctx ctx, fc_ints I, const z* taup, const z* t1dress, z* Rp, int precision);
// fc_mlp.hip
int learned_step(fc_ctx ctx, fc_ints I, const void* mlp, const z* t1, const z* t2, const z* r1, const z* r2,
                 const z* r2prev, const z* fdiag, z* o1, z* o2);
void learn_samples(fc_ctx ctx, fc_ints I, const z* t2, const z* r2, const z* r2prev, const z* t2s, const z* fdiag,
                   long nsamp, unsigned long long seed, float* X, float* q, float* r);
// fc_eom.hip
void build_hbar(fc_ctx ctx, fc_ints I, fc_amps T);
// left: S = R H-bar (rows of R are left vectors) instead of S = H-bar R
void sigma_dev(fc_ctx ctx, fc_ints I, fc_amps T, int nvec, const z* R, z* S, bool left = false);
// fc_aocd.hip
int cd_pivoted_dev(fc_ctx ctx, long m, const double* M, double tau, int max_vec, double* L, int* nvec,
                   int* piv_host);
void ao_to_spinor_dev(fc_ctx ctx, long nvec, long nao, long n, const double* Lao, const z* C, z* Lmo);
// fc_linalg.cpp (host FP64)
void herm_eig(int n, std::vector<z>& A, std::vector<double>& w);           // A -> eigenvectors (columns)
void gen_eig(int n, const std::vector<z>& A, std::vector<z>& w, std::vector<z>& VR);
bool lin_solve(int n, std::vector<z> A, std::vector<z>& b);                  // partial pivoting
double cond_herm(int n, const std::vector<z>& A);
}  // namespace fc
