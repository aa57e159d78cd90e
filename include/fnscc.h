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
 * 16-bit type, the three products hi*hi + hi*lo + lo*hi run on MFMA with FP32 accumulation. */
enum { FC_FP64 = 0, FC_SPLIT_BF16 = 1, FC_SPLIT_FP16 = 2 };

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

/* cd_integrals - stage the Cholesky vectors (Eq. 22) and assemble the stored antisymmetrised
 * integrals with at most two virtual indices (Eq. 23 and the storage rule of Sec. 3:
 * <mn||ij>, <mn||ie>, <mn||ef>, <mb||ej> and the blocks derived from them by index symmetry).
 * eps: host, n doubles. L: ncd*n*n complex of `l_dtype`, host (l_on_device = 0) or device (1).
 * precision: FC_FP64 / FC_SPLIT_BF16 / FC_SPLIT_FP16, used by the assembly GEMMs and kept as the
 * default of the ladder. Returns FC_EARG for o < 1, v < 1, ncd < 1 or NULL pointers. */
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
 * or NULL. *out is a new handle; `in` stays valid. */
int fns_truncate(fc_ctx ctx, fc_ints in, double occ_thresh, fc_ints* out, int* v_kept, double* occ,
                 void* U);

/* Options of ccsd_solve. Jacobi update t += Omega/D with complex DIIS (FP64). Converged when
 * |dE| < e_tol and RMS(Omega over unique amplitudes) < r_tol. learned = 1 uses the learned
 * preconditioned T2 step (weights from fc_mlp_*), falling back to Jacobi+DIIS when the residual
 * stalls. t1_init/t2_init: device, full layout, or NULL for t = 0. */
typedef struct {
  double e_tol, r_tol;
  int max_iter, diis_dim, learned, precision;
  const void* t1_init;
  const void* t2_init;
  const void* mlp;  /* fc_mlp handle or NULL */
  int stall_window; /* iterations without residual decrease before falling back (learned) */
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
/* Amplitude handles: create from device arrays (copied), read back into device arrays. */
int fc_amps_create(fc_ctx ctx, fc_ints ints, const void* t1, const void* t2, fc_amps* out);
int fc_amps_read(fc_amps t, void* t1, void* t2);
void fc_free_amps(fc_amps t);

/* ipeom_sigma - sigma = H-bar R on the 1h + 2h1p space (Eq. 17-18) for nvec vectors.
 * R, S: device, nvec x dim complex128 (layout above). The H-bar blocks with at most two virtual
 * indices are built from `t` on first use and cached in the amplitude handle (Sec. 3). */
int ipeom_sigma(fc_ctx ctx, fc_ints ints, fc_amps t, int nvec, const void* R, void* S);

typedef struct {
  double r_tol, w_tol;
  int max_iter, max_subspace, guess_per_root;
} fc_eom_opts;
void fc_eom_default_opts(fc_eom_opts* opts);
/* ipeom_davidson - lowest-nroots (by real part) eigenvalues omega_k of the IP-EOM-CCSD matrix
 * (Eq. 18) by non-Hermitian Davidson; subspace eigenproblem in FP64 on the host.
 * omega: host, sum(nroots) x 2 doubles (re, im), ascending real part per instance.
 * R_out: device, sum(nroots) x dim_b right eigenvectors (or NULL). iters: host, nb ints. */
int ipeom_davidson(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* t, const int* nroots,
                   const fc_eom_opts* opts, double* omega, void* R_out, int* iters);

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
