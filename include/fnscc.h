/* fnscc.h - C ABI of libfnscc, the MI355X (gfx950) hot path of Cholesky-decomposed,
 * frozen-natural-spinor IP-EOM-CCSD (Chamoli, Nayak, Dutta, "A Reduced Cost Two-component
 * Relativistic Equation-of-Motion Coupled Cluster Method for Ionization Potential").
 *
 * Conventions shared by every call
 * --------------------------------
 * Spinors: p = 0..o-1 occupied, o..n-1 virtual (n = o + v); the occupied count excludes frozen
 *   core spinors. Energies eps_p are canonical (Fock matrix diagonal), FP64.
 * Complex numbers: interleaved (re, im) pairs. complex128 = two doubles, complex64 = two floats.
 * Cholesky vectors (Eq. 21-22): L[P][p][q] = L^P_pq, P = 0..ncd-1, row index p is the bra
 *   (conjugated) spinor. Each L^P is Hermitian because the AO vectors are real (Eq. 8).
 * Amplitudes: t1[i][a], t2[i][j][a][b] (full, antisymmetric in ij and in ab), complex128.
 * IP vectors (Eq. 17): r_i for i = 0..o-1, then r_ij^b for i<j in lexicographic order with b
 *   fastest; dim = o + o(o-1)/2 * v, complex128.
 * Pointers: "host" arguments are CPU memory; "device" arguments are device memory on the
 *   context's device. The caller owns every array it passes; the library copies what it keeps.
 * Errors: every call returns FC_OK or an FC_E* code and never throws; fc_last_error() returns the
 *   text of the last failure on that context. Calls are ordered on the context's stream and are
 *   not thread-safe for one context.
 * Memory: all device memory comes from the allocator callbacks given to fc_create (or hipMalloc
 *   when they are NULL); freed blocks are cached inside the context until fc_destroy.
 */
#ifndef FNSCC_H
#define FNSCC_H
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fc_ctx_s* fc_ctx;
typedef struct fc_ints_s* fc_ints;
typedef struct fc_amps_s* fc_amps;

typedef void* (*fc_alloc_fn)(size_t bytes, void* stream, void* user);
typedef void (*fc_free_fn)(void* ptr, size_t bytes, void* stream, void* user);

enum { FC_OK = 0, FC_EARG = 1, FC_EHIP = 2, FC_ENOMEM = 3, FC_ENOCONV = 4, FC_ENUMERIC = 5,
       FC_EUNSUPPORTED = 6 };
enum { FC_C128 = 0, FC_C64 = 1 };
/* Precision of the ladder and of the Cholesky assembly GEMMs. FC_FP64: FP64 MFMA throughout.
 * FC_SPLIT_BF16 / FC_SPLIT_FP16: each FP64 operand is split into a hi and a lo part of the
 * 16-bit type, the three products hi*hi + hi*lo + lo*hi run on MFMA with FP32 accumulation; all
 * other products of the CCSD residual then run in FP32 arithmetic (FP64 storage).
 * FC_FP32 is accepted by fc_zgemm only: FP32 arithmetic on FP64 operands and result.
 * FP32-arithmetic complex products use three real products (Are Bre, Aim Bim and
 * (Are + Aim)(Bre + Bim)); FP64 ones use four. */
enum { FC_FP64 = 0, FC_SPLIT_BF16 = 1, FC_SPLIT_FP16 = 2, FC_FP32 = 3 };

/* Create a context on `device`, ordering all work on `hip_stream` (a hipStream_t; NULL = the
 * default stream). alloc/release may be NULL (then hipMalloc/hipFree are used). */
int fc_create(fc_ctx* ctx, int device, void* hip_stream, fc_alloc_fn alloc, fc_free_fn release,
              void* user);
void fc_destroy(fc_ctx ctx);
const char* fc_last_error(fc_ctx ctx);
/* Timing flags: bit 0 = per-stage stream timers (each stage synchronises the stream);
 * bit 1 = hipEvents around every ladder evaluation on the context stream (no synchronisation). */
int fc_set_timing(fc_ctx ctx, int flags);
/* Writes "name=ms;...;ladder_events=n;ladder_event_ms=ms;calls_name=n;..." into buf (truncated
 * to len) and clears the timers. */
int fc_take_timings(fc_ctx ctx, char* buf, size_t len);
/* GEMM tile autotuning. When on, the first complex GEMM of each shape bucket (operand layouts,
 * sizes rounded up to powers of two, batching, epilogue) times every tile configuration once on a
 * scratch output and keeps the fastest for the bucket; later calls reuse the choice. The table can
 * be saved to and loaded from a text file (one "bucket config ms" line per bucket). Off by
 * default (a size heuristic is used). fc_autotune_size returns the number of tuned buckets. */
int fc_set_autotune(fc_ctx ctx, int on);
int fc_autotune_save(fc_ctx ctx, const char* path);
int fc_autotune_load(fc_ctx ctx, const char* path);
int fc_autotune_size(fc_ctx ctx);

/* fc_set_gemm_config - forces tile configuration cfg (0 <= cfg < fc_gemm_num_configs()) on every
 * single complex product of this context whose output it fits, in place of the size heuristic and
 * the autotuner; cfg = -1 restores them.  Results of a product do not depend on the configuration
 * beyond rounding order.  FC_EARG for a cfg outside [-1, fc_gemm_num_configs()). */
int fc_set_gemm_config(fc_ctx ctx, int cfg);
int fc_gemm_num_configs(void);

/* fc_set_split_config - forces the staging of the 128-wide tiles of the split-precision products
 * (FC_SPLIT_BF16 / FC_SPLIT_FP16 products and the ladder on them) of this context: 0 operands
 * staged through registers, 8 waves; 1 the same with 4 waves; 2 operands loaded straight into LDS,
 * 8 waves (0 <= cfg < fc_split_num_configs()); cfg = -1 restores the default (2).  0 and 2 give
 * the same bits; 1 differs in rounding order only.  FC_EARG for a cfg outside
 * [-1, fc_split_num_configs()). */
int fc_set_split_config(fc_ctx ctx, int cfg);
int fc_split_num_configs(void);

/* cd_ao_pivoted - single-step pivoted Cholesky of the AO two-electron supermatrix (Eq. 21):
 * M ~= sum_P l_P l_P^T.  Each step takes as pivot the largest remaining diagonal entry (the lowest
 * index among equal ones), forms l = (M[p, :] - sum_{earlier P} l_P[p] l_P) / sqrt(d_p) and
 * lowers the diagonal by l^2; the loop stops before the step whose pivot is < tau.
 * M: device, m x m doubles, row-major, symmetric positive semi-definite (the supermatrix
 * (mu nu|ka la) over any composite index of AO pairs; read only).  tau > 0.  L: device,
 * max_vec x m doubles, row P = vector P.  nvec: host, vectors formed.  piv: host, max_vec ints
 * (the pivot of each vector) or NULL.  FC_ENOCONV when max_vec < m vectors were formed while the
 * largest diagonal is still >= tau (L then holds those vectors); FC_EARG for bad sizes. */
int cd_ao_pivoted(fc_ctx ctx, long m, const double* M, double tau, int max_vec, double* L, int* nvec, int* piv);
/* ao_to_spinor - the two-component transform of Eq. 22:
 * L^P_pq = sum_{s = alpha, beta} sum_{mu nu} conj(C[s nao + mu][p]) L^P_{mu nu} C[s nao + nu][q].
 * Lao: device, nvec x nao x nao doubles (the real AO vectors, full square, as cd_ao_pivoted
 * returns them for the composite index mu nao + nu).  C: device, 2 nao x n complex128 spinor
 * coefficients (rows: alpha AOs, then beta AOs).  Lmo: device, nvec x n x n complex128, the
 * layout cd_integrals takes (select columns of C to transform a subset of spinors). */
int ao_to_spinor(fc_ctx ctx, int nvec, int nao, int n, const double* Lao, const void* C, void* Lmo);

/* cd_integrals - stage the Cholesky vectors (Eq. 22) and assemble the stored antisymmetrised
 * integrals with at most two virtual indices (Eq. 23 and the storage rule of Sec. 3:
 * <mn||ij>, <mn||ie>, <mn||ef>, <mb||ej> and the blocks derived from them by index symmetry).
 * eps: host, n doubles. L: ncd*n*n complex of `l_dtype`, host (l_on_device = 0) or device (1).
 * precision: FC_FP64 / FC_SPLIT_BF16 / FC_SPLIT_FP16, used by the assembly GEMMs and kept as the
 * default of the ladder. Returns FC_EARG for o < 1, v < 1, ncd < 1 or NULL pointers and
 * FC_EUNSUPPORTED for o == 1 or v == 1 (no doubles amplitudes, no 2h1p space). */
int cd_integrals(fc_ctx ctx, int o, int v, int ncd, const double* eps, const void* L, int l_dtype,
                 int l_on_device, int precision, fc_ints* out);
int fc_ints_info(fc_ints ints, int* o, int* v, int* ncd);
void fc_free_ints(fc_ints ints);

/* fns_truncate - frozen natural spinors (Eq. 24-28): MP2 virtual density
 * D_ab = 1/2 sum_ijc t_ij^ac conj(t_ij^bc), t = <ab||ij>/(eps_i+eps_j-eps_a-eps_b) on the device;
 * FP64 eigen-decomposition on the host (occupations descending); keep occupations > occ_thresh;
 * semicanonicalise F_vv in the kept space; U = V~ Z~ (v x v'); rotate the virtual Cholesky
 * vectors and rebuild the stored integrals. Occupied spinors are untouched.
 * occ: host, v doubles (all occupations, descending) or NULL. U: host, v*v' complex128 row-major
 * or NULL. *out is a new handle; `in` stays valid. FC_EUNSUPPORTED when fewer than two virtual
 * spinors pass the threshold. */
int fns_truncate(fc_ctx ctx, fc_ints in, double occ_thresh, fc_ints* out, int* v_kept, double* occ,
                 void* U);

/* Learned T2 update network (4 -> 64 -> 64 -> 2, tanh). Not part of the paper's method: a
 * per-amplitude gain g with t_ij^ab += q_ij^ab (1 + g), q the dressed Jacobi step
 * Omega / (D - (F_aa + F_bb - F_ii - F_jj)) (Omega / D where the dressing would bring the
 * denominator below half of D; the learned step keeps this base whatever precond says), features
 * built from the dressed diagonal u = (F_aa + F_bb - F_ii - F_jj) / D and the residual ratio
 * rho = Omega_k / Omega_{k-1} of the amplitude; Omega = 0 gives a zero step. */
typedef struct fc_mlp_s* fc_mlp;

/* Options of ccsd_solve. Jacobi update t += Omega/D (D dressed or bare, see precond) with complex
 * DIIS (FP64) over the last
 * diis_dim iterates (default 10, at most 16; <= 1 turns DIIS off). Converged when
 * |dE| < e_tol and RMS(Omega over unique amplitudes) < r_tol; e_tol, r_tol <= 0 (the defaults)
 * select 1e-10 and 1e-9 for FC_FP64 and 1e-8 and 1e-7 for the split precisions, whose product
 * errors move the IPs by ~1e-7 Eh anyway. learned = 1 with mlp != NULL uses
 * the learned T2 step (DIIS on top) until the residual fails to decrease for stall_window
 * iterations, then plain Jacobi + DIIS. t1_init/t2_init: device, full layout, or NULL for t = 0.
 * on_iter (may be NULL): called with the current iterate (device pointers, valid during the call)
 * before each residual evaluation; precision: FC_* or -1 to inherit from the integral handle. */
typedef struct {
  double e_tol, r_tol;
  int max_iter, diis_dim, learned, precision;
  const void* t1_init;
  const void* t2_init;
  const void* mlp;  /* fc_mlp handle or NULL */
  int stall_window; /* iterations without residual decrease before falling back (learned) */
  void (*on_iter)(int iter, const void* t1, const void* t2, void* user);
  void* user;
  int diis_start;   /* first iteration whose iterate enters the DIIS history (earlier: plain steps) */
  int precond;      /* 1 (default): Jacobi denominators dressed by the diagonals of the residual's
                       one-particle intermediates (a diagonal Newton step); 0: bare orbital-energy
                       denominators */
} fc_ccsd_opts;
void fc_ccsd_default_opts(fc_ccsd_opts* opts);

/* ccsd_solve - CCSD amplitude equations (Eq. 13-14) and energy (Eq. 15) for nb independent
 * instances. e_corr: host, nb x 2 doubles (re, im). iters: host, nb ints. Returns FC_ENOCONV
 * (outputs still filled with the last iterate) if any instance did not converge. */
int ccsd_solve(fc_ctx ctx, int nb, const fc_ints* ints, const fc_ccsd_opts* opts, fc_amps* t,
               double* e_corr, int* iters);
/* Residuals Omega1 = <Phi_i^a|e^-T H e^T|Phi0>, Omega2 = <Phi_ij^ab|...|Phi0> at the given
 * amplitudes (device, full layout); r1/r2 device outputs of the same layout. precision as above. */
int ccsd_residual(fc_ctx ctx, fc_ints ints, const void* t1, const void* t2, void* r1, void* r2,
                  int precision);
/* The particle-particle ladder alone: R_ij^ab = sum_ef tau_ij^ef (ae|bf), (ae|bf) = sum_P
 * L^P_ae L^P_bf rebuilt from the Cholesky vectors (Eq. 21, 23). tau: device o*o*v*v antisymmetric;
 * R: device o*o*v*v output (overwritten). dress_t1: device o*v or NULL; when given, L_ae is
 * replaced by L_ae - sum_m t_m^a L_me on both factors. */
int fc_ladder(fc_ctx ctx, fc_ints ints, const void* tau, const void* dress_t1, void* R,
              int precision);
/* fc_ladder_packed - the same ladder on the unique amplitudes only, for shapes whose full o^2 v^2
 * arrays do not fit (o = 40, v = 1698: 74 GB per full complex128 tensor, 18 GB packed).
 * taup: device, C(o,2) x C(v,2) complex128, taup[pij][pef] = tau_ij^ef for i < j, e < f, pairs in
 * lexicographic order (p = i (2n - i - 1) / 2 + j - i - 1).  Rp: device, C(o,2) x C(v,2)
 * complex128, Rp[pij][pab] = R_ij^ab for i < j, a < b (overwritten).  dress_t1 as fc_ladder.
 * precision: FC_FP64 / FC_SPLIT_BF16 / FC_SPLIT_FP16, or -1 for the handle's.  Synchronises the
 * context stream before returning. */
int fc_ladder_packed(fc_ctx ctx, fc_ints ints, const void* taup, const void* dress_t1, void* Rp, int precision);
/* fc_zgemm - the library's complex FP64 matrix product on the matrix cores (every contraction of
 * Eq. 12-18 and 23 reduces to it): C = alpha op(A) op(B) + beta C, row-major, device pointers to
 * interleaved complex128. opA: 'N' A[m*lda+k], 'T' A[k*lda+m], 'C' conj(A[k*lda+m]),
 * 'R' conj(A[m*lda+k]); opB: 'N' B[k*ldb+n], 'T' B[n*ldb+k], 'C' conj(B[n*ldb+k]),
 * 'R' conj(B[k*ldb+n]). alpha, beta: host (re, im). precision: FC_FP64, FC_FP32 (FP32 products
 * and sums), or FC_SPLIT_BF16 / FC_SPLIT_FP16 (hi/lo split products with FP32 sums, as in the
 * ladder; opA 'N' or 'R' with opB 'T' or 'C' only, other layouts FC_EUNSUPPORTED; an FP16 operand
 * takes one power-of-two scale per 128 columns of K). Stream-ordered; returns before completion
 * (the split precisions synchronise the context stream while choosing their FP16 scales). */
int fc_zgemm(fc_ctx ctx, char opA, char opB, long M, long N, long K, const double* alpha, const void* A,
             long lda, const void* B, long ldb, const double* beta, void* C, long ldc, int precision);
/* fc_zgemm_noalloc - fc_zgemm for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments, layouts
 * and result as fc_zgemm; it calls no allocator: the split-K partial sums of products with few
 * output tiles and long K live in a fixed workspace of 128 MiB per device (a static device array
 * set up by fc_create, held by every device the library runs on until the process ends).  The
 * tile configuration is always the size heuristic's (or the FNSCC_GEMM_CFG override), never an
 * autotuned one, so with autotuning off the result equals fc_zgemm's bit for bit.  A product whose
 * partial sums would exceed the workspace (only possible with a forced large tile) is refused
 * with FC_EARG before any launch.  Every partial sum is written before it is read, so nothing
 * needs clearing between calls; all calls on one GPU share the one workspace, so calls that
 * overlap in time on one GPU (several streams or threads) race. */
int fc_zgemm_noalloc(fc_ctx ctx, char opA, char opB, long M, long N, long K, const double* alpha, const void* A,
                     long lda, const void* B, long ldb, const double* beta, void* C, long ldc, int precision);
/* Amplitude handles: create from device arrays (copied), read back into device arrays. */
int fc_amps_create(fc_ctx ctx, fc_ints ints, const void* t1, const void* t2, fc_amps* out);
int fc_amps_read(fc_amps t, void* t1, void* t2);
void fc_free_amps(fc_amps t);

/* ipeom_sigma - sigma = H-bar R on the 1h + 2h1p space (Eq. 17-18) for nvec vectors.
 * R, S: device, nvec x dim complex128 (layout above). The H-bar blocks with at most two virtual
 * indices are built from `t` on first use and cached in the amplitude handle (Sec. 3); with a
 * split-precision integral handle their products run in FP32 arithmetic (FP64 storage), as do
 * the mixed-precision residual's products outside the ladder.  The sigma products are FP64.
 * nvec = 0 returns FC_OK without touching the device (R and S may be NULL); nvec < 0, or `t`
 * made from another integral handle: FC_EARG. */
int ipeom_sigma(fc_ctx ctx, fc_ints ints, fc_amps t, int nvec, const void* R, void* S);

/* ipeom_sigma_left - the left product S = Y H-bar (Eq. 19-20): each row of Y holds the
 * amplitudes l^i and l_b^ij (i < j) of one left vector in the layout of R above, and the matching
 * row of S is that row vector times the IP-EOM-CCSD matrix, so that for any R
 * sum_x S[x] R[x] = sum_x Y[x] (H-bar R)[x] (a bilinear product, no conjugation).
 * Y, S: device, nvec x dim complex128.  Errors as ipeom_sigma. */
int ipeom_sigma_left(fc_ctx ctx, fc_ints ints, fc_amps t, int nvec, const void* Y, void* S);

/* max_subspace: trial vectors kept before a restart collapses the subspace (0, the default:
 * 10 x nroots; the host eigenproblem of the projected matrix grows as its cube).
 * graph: 1 (default) captures the sigma launches of all instances once into a HIP graph and
 * replays it for every Davidson iteration; 0 launches them directly (same results bit for bit). */
typedef struct {
  double r_tol, w_tol;
  int max_iter, max_subspace, guess_per_root;
  int graph;
} fc_eom_opts;
void fc_eom_default_opts(fc_eom_opts* opts);
/* ipeom_davidson - lowest-nroots (by real part) eigenvalues omega_k of the IP-EOM-CCSD matrix
 * (Eq. 18) by non-Hermitian Davidson; subspace eigenproblem in FP64 on the host.
 * nb > 1 solves uneven instances together: every Davidson step is one launch for the whole
 * batch and the sigma products of all new trial vectors of all instances are one graph replay.
 * omega: host, sum(nroots) x 2 doubles (re, im), ascending real part per instance.
 * R_out: device, sum(nroots) x dim_b right eigenvectors (or NULL). iters: host, nb ints. */
int ipeom_davidson(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* t, const int* nroots,
                   const fc_eom_opts* opts, double* omega, void* R_out, int* iters);

/* ipeom_left - left eigenvectors L_k (Eq. 20) dual to the right eigenvectors R of ipeom_davidson,
 * normalised by the biorthogonality condition of Eq. 19: sum_x L_k[x] R_l[x] = delta_kl over the
 * packed layout (a bilinear product, no conjugation).  The lowest nroots left roots are solved by
 * the same batched Davidson on the transposed problem; L is then replaced by O^-1 L with
 * O = L R^T, which also handles degenerate roots.
 * R: device, sum(nroots) x dim_b right eigenvectors as returned by ipeom_davidson (same nb,
 * ints, t and nroots; read only).  omega: host, sum(nroots) x 2 doubles: for right root k, the
 * eigenvalue of the left root that overlaps it most (equal to the right eigenvalue within the
 * solver tolerance).  L_out: device, sum(nroots) x dim_b, row k dual to right root k.
 * weight: host, sum(nroots) x 2 doubles, the one-hole part sum_i l^i_k r_{k,i} of the
 * normalisation (the ionisation strength of root k when ground-state relaxation is neglected).
 * iters: host, nb ints, or NULL.  FC_ENUMERIC when the left and right roots do not pair up
 * (O near singular); FC_ENOCONV as ipeom_davidson. */
int ipeom_left(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* t, const int* nroots,
               const fc_eom_opts* opts, const void* R, double* omega, void* L_out, double* weight, int* iters);

/* Learned update network. Parameters: one FP32 vector W1 (64x4), b1, W2 (64x64), b2, W3 (2x64),
 * b3 (fc_mlp_num_params() entries). fc_mlp_create: params_host (host) or NULL for a seeded
 * initialisation. Training minimises sum_s |r_s - q_s g_s|^2 / sum_s |q_s|^2 over a minibatch of
 * B samples: X (device, B x 4 FP32 features), q (device, B complex64: the dressed Jacobi step),
 * r (device, B complex64: (t* - t) - q); fc_mlp_train_step does one Adam step (lr > 0) on FP32
 * master weights and refreshes the BF16 copy used by the solver; fc_mlp_grad returns the
 * gradient (host, FP32) without updating; fc_mlp_forward evaluates Y (device, B x 2) with the FP32
 * (bf16_weights = 0) or BF16-rounded weights. loss: host float or NULL. */
int fc_mlp_create(fc_ctx ctx, const float* params_host, unsigned long long seed, fc_mlp* out);
void fc_mlp_free(fc_mlp mlp);
long fc_mlp_num_params(void);
int fc_mlp_get_params(fc_mlp mlp, float* host, int bf16_rounded);
int fc_mlp_grad(fc_mlp mlp, const float* X, const float* q, const float* r, long B, float* grad_host, float* loss);
int fc_mlp_train_step(fc_mlp mlp, const float* X, const float* q, const float* r, long B, float lr, float* loss);
int fc_mlp_forward(fc_mlp mlp, const float* X, long B, float* Y, int bf16_weights);
/* fc_learned_step - one learned amplitude update as the solver applies it (test and measurement
 * helper): t1_out = t1 + q1 (the dressed Jacobi step of the singles); for every i < j, a < b, with
 * the features above built from fdiag and the residual ratio r2 / r2prev (r2prev NULL: ratio 0)
 * and g the network output with BF16-rounded weights, t2_out_ij^ab = t2_ij^ab + q (1 + g) with q
 * the dressed Jacobi step of the amplitude, written to all four antisymmetric images, and zero
 * where i == j or a == b.  t1, r1, t1_out: device o x v;
 * t2, r2, r2prev, t2_out: device o x o x v x v; fdiag: device o + v complex128 (F_mi then F_ae
 * diagonals).  All complex128. */
int fc_learned_step(fc_ctx ctx, fc_ints ints, fc_mlp mlp, const void* t1, const void* t2, const void* r1,
                    const void* r2, const void* r2prev, const void* fdiag, void* t1_out, void* t2_out);
/* Training samples at the iterate (t1, t2) (device, full layout) of a solve whose converged
 * doubles are t2_star, the previous iterate (t1prev, t2prev) giving the residual ratio (NULL: 0):
 * nsamp unique amplitudes (i<j, a<b) drawn by a counter-based hash of seed; writes X (B x 4),
 * q (B complex64) and r (B complex64) as defined above (device). */
int fc_learn_samples(fc_ctx ctx, fc_ints ints, const void* t1, const void* t2, const void* t1prev,
                     const void* t2prev, const void* t2_star, long nsamp, unsigned long long seed, float* X,
                     float* q, float* r);

/* Host FP64 dense eigensolvers used by the library (exported for testing; no GPU needed).
 * fc_host_zheev: Hermitian A (n x n complex128, row-major, host) -> ascending eigenvalues w and
 *   eigenvectors stored as the columns of A. fc_host_zgeev: general A -> eigenvalues w (n complex)
 *   and right eigenvectors as columns of VR (unit norm), unsorted. */
int fc_host_zheev(int n, double* A, double* w);
int fc_host_zgeev(int n, const double* A, double* w, double* VR);

#ifdef __cplusplus
}
#endif
#endif
