// CCSD residuals (Eq. 13-14), energy (Eq. 15) and the particle-particle ladder.
//
// Working equations: spin-orbital Stanton-Gauss intermediates in complex-correct index order
// (creation-side indices in the bra).  Integrals with three virtual indices are never formed:
// each such contraction is factorised through the Cholesky vectors, and the four-virtual
// ladder sum_ef tau_ij^ef <ab||ef>/2 (plus the T1 part of W_abef) is evaluated as
//   sum_ef tau_ij^ef sum_P Lb^P_ae Lb^P_bf,   Lb^P_ae = L^P_ae - sum_m t_m^a L^P_me,
// with (ae|bf) rebuilt tile by tile from the Cholesky vectors (Eq. 21, 23).  The remaining
// pieces of the same terms are folded into
//   1/2 sum_mn tau_mn^ab W0_mnij + 1/4 sum_mn t_mn^ab X_ijmn,
//   W0_mnij = <mn||ij> + P(ij) sum_e t_j^e <mn||ie>,  X_ijmn = sum_ef tau_ij^ef <mn||ef>.
#include <algorithm>
#include <cmath>

#include "fc_state.hpp"

namespace fc {
namespace {
constexpr int TPB = 256;
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(1048576L, (n + TPB * 4 - 1) / (TPB * 4))); }
#define GRID_STRIDE(i, n) for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

__device__ inline z cmul(z a, z b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// tau~ = t2 + 1/2 (t_i^a t_j^b - t_i^b t_j^a), tau = t2 + t_i^a t_j^b - t_i^b t_j^a
__global__ void k_tau(const z* t1, const z* t2, z* tau, z* taut, long o, long v) {
  GRID_STRIDE(t, o * o * v * v) {
    long b = t % v, a = (t / v) % v, j = (t / (v * v)) % o, i = t / (v * v * o);
    z x = cmul(t1[i * v + a], t1[j * v + b]), y = cmul(t1[i * v + b], t1[j * v + a]);
    z d = make_double2(x.x - y.x, x.y - y.y);
    z s = t2[t];
    if (tau) tau[t] = make_double2(s.x + d.x, s.y + d.y);
    if (taut) taut[t] = make_double2(s.x + 0.5 * d.x, s.y + 0.5 * d.y);
  }
}
// Z_jn^fb = scale_t2 t2[j,n,f,b] + t1[j,f] t1[n,b] (scale_t2 = 1/2 for W_mbej) written as
// Zr[b][j][n][f], the order in which the ring product reads it: per (j, n) plane a 32 x 32 (f, b)
// tile is formed from coalesced reads along b and written through LDS along f.
// Grid: x = (f, b) tile, y = (j, n).
__global__ __launch_bounds__(256) void k_ring_amp_t(const z* __restrict__ t1, const z* __restrict__ t2,
                                                    z* __restrict__ Zr, long o, long v, double scale_t2) {
  __shared__ z T[32][33];
  const long nb = (v + 31) / 32;
  const long F0 = (blockIdx.x / nb) * 32, B0 = (blockIdx.x % nb) * 32;
  const long j = blockIdx.y / o, n = blockIdx.y % o;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const z* src = t2 + (j * o + n) * v * v;
  for (int r = ty; r < 32; r += 8) {
    const long f = F0 + r, b = B0 + tx;
    if (f < v && b < v) {
      const z p = cmul(t1[j * v + f], t1[n * v + b]), t = src[f * v + b];
      T[r][tx] = make_double2(scale_t2 * t.x + p.x, scale_t2 * t.y + p.y);
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const long b = B0 + r, f = F0 + tx;
    if (f < v && b < v) Zr[((b * o + j) * o + n) * v + f] = T[tx][r];
  }
}
// r -= D t with D_i^a = e_i - e_a, D_ij^ab = e_i + e_j - e_a - e_b
__global__ void k_sub_denom1(z* r, const z* t, const double* eps, long o, long v) {
  GRID_STRIDE(x, o * v) {
    long a = x % v, i = x / v;
    double d = eps[i] - eps[o + a];
    r[x].x -= d * t[x].x; r[x].y -= d * t[x].y;
  }
}
// out = t + r / D   (Jacobi step); diagonal (i==j or a==b) entries of t2 stay zero
__global__ void k_jacobi1(const z* t, const z* r, z* out, const double* eps, long o, long v) {
  GRID_STRIDE(x, o * v) {
    long a = x % v, i = x / v;
    double d = eps[i] - eps[o + a];
    out[x] = make_double2(t[x].x + r[x].x / d, t[x].y + r[x].y / d);
  }
}
__global__ void k_jacobi2(const z* t, const z* r, z* out, const double* eps, long o, long v) {
  GRID_STRIDE(x, o * o * v * v) {
    long b = x % v, a = (x / v) % v, j = (x / (v * v)) % o, i = x / (v * v * o);
    if (i == j || a == b) { out[x] = make_double2(0, 0); continue; }
    double d = eps[i] + eps[j] - eps[o + a] - eps[o + b];
    out[x] = make_double2(t[x].x + r[x].x / d, t[x].y + r[x].y / d);
  }
}
// The same step with the dressed diagonal of the T2 (T1) equation's one-particle operators,
// d - (F_aa + F_bb - F_ii - F_jj) with F = fd (complex; fd[0..o) occupied, fd[o..o+v) virtual):
// the diagonal of the residual's Jacobian, so the step is a diagonal Newton step.  Where the
// dressing would bring the denominator below half the bare one's size, the bare one is used.
__device__ inline z dressed_div(z r, double d, z df) {
  const double dr = d - df.x, di = -df.y;
  const double n2 = dr * dr + di * di;
  if (!(n2 >= 0.25 * d * d)) return make_double2(r.x / d, r.y / d);
  return make_double2((r.x * dr + r.y * di) / n2, (r.y * dr - r.x * di) / n2);
}
__global__ void k_jacobi1_dressed(const z* t, const z* r, z* out, const double* eps, const z* fd, long o, long v) {
  GRID_STRIDE(x, o * v) {
    long a = x % v, i = x / v;
    const double d = eps[i] - eps[o + a];
    const z df = make_double2(fd[o + a].x - fd[i].x, fd[o + a].y - fd[i].y);
    const z q = dressed_div(r[x], d, df);
    out[x] = make_double2(t[x].x + q.x, t[x].y + q.y);
  }
}
__global__ void k_jacobi2_dressed(const z* t, const z* r, z* out, const double* eps, const z* fd, long o, long v) {
  GRID_STRIDE(x, o * o * v * v) {
    long b = x % v, a = (x / v) % v, j = (x / (v * v)) % o, i = x / (v * v * o);
    if (i == j || a == b) { out[x] = make_double2(0, 0); continue; }
    const double d = eps[i] + eps[j] - eps[o + a] - eps[o + b];
    const z df = make_double2(fd[o + a].x + fd[o + b].x - fd[i].x - fd[j].x,
                              fd[o + a].y + fd[o + b].y - fd[i].y - fd[j].y);
    const z q = dressed_div(r[x], d, df);
    out[x] = make_double2(t[x].x + q.x, t[x].y + q.y);
  }
}
// X[m,n,i,j] -> X - X^(i<->j) added into W (o^4)
// out[k] = F[k * n + k]
__global__ void k_diag_copy(const z* F, long n, z* out) {
  GRID_STRIDE(k, n) { out[k] = F[k * n + k]; }
}
__global__ void k_antisym_oooo(z* W, const z* X, long o) {
  GRID_STRIDE(t, o * o * o * o) {
    long j = t % o, i = (t / o) % o, mn = t / (o * o);
    z a = X[t], b = X[(mn * o + j) * o + i];
    W[t].x += a.x - b.x; W[t].y += a.y - b.y;
  }
}

}  // namespace

z ccsd_energy_dev(fc_ctx ctx, fc_ints I, const z* t1, const z* t2) {
  ensure_integrals(ctx, I);
  const long o = I->o, v = I->v;
  ZTensor tau(ctx, {o, o, v, v});
  hipLaunchKernelGGL(k_tau, dim3(nblk(tau.size())), dim3(TPB), 0, ctx->stream, t1, t2, tau.p(), (z*)nullptr, o, v);
  z e = dotu(ctx, tau.size(), I->oovv.p(), tau.p());
  return make_double2(0.25 * e.x, 0.25 * e.y);
}

void ccsd_residual_dev(fc_ctx ctx, fc_ints I, const z* t1p, const z* t2p, z* r1p, z* r2p, int precision, z* fdiag) {
  StageTimer st(ctx, "residual");
  ensure_integrals(ctx, I);
  const ZTensor& Lvv = lvv(ctx, I);
  // mixed precision: every product outside the ladder's split kernels in FP32 arithmetic
  Fp32Gemms fp32(ctx, precision != FC_FP64);
  const long o = I->o, v = I->v, N = I->ncd;
  const z one = make_double2(1, 0), zero = make_double2(0, 0), half = make_double2(0.5, 0),
          mone = make_double2(-1, 0), mhalf = make_double2(-0.5, 0), quarter = make_double2(0.25, 0);
  ZT T1((z*)t1p, {o, v}), T2((z*)t2p, {o, o, v, v});
  ZT R1(r1p, {o, v}), R2(r2p, {o, o, v, v});
  const long n2 = o * o * v * v;

  ZTensor tau(ctx, {o, o, v, v}), taut(ctx, {o, o, v, v});
  hipLaunchKernelGGL(k_tau, dim3(nblk(n2)), dim3(TPB), 0, ctx->stream, t1p, t2p, tau.p(), taut.p(), o, v);
  FC_HIP(hipGetLastError());

  // ---- Cholesky-factorised three-virtual pieces
  ZTensor xP(ctx, {N});                 // x_P = sum_mf t_m^f L^P_mf
  zein(ctx, "mf,mfP->P", one, T1, I->Lov, zero, xP);
  ZTensor Y(ctx, {v, o, N});            // Y[a,m,P] = sum_f L^P_af t_m^f
  zgemm(ctx, 'N', 'N', o, N, v, one, t1p, v, Lvv.p(), N, zero, Y.p(), N, (int)v, 0, v * N, o * N);
  ZTensor Cm(ctx, {o, o, N});           // C[m,j,P] = sum_f L^P_mf t_j^f
  zgemm(ctx, 'N', 'N', o, N, v, one, t1p, v, I->Lov.p(), N, zero, Cm.p(), N, (int)o, 0, v * N, o * N);

  // ---- intermediates
  ZTensor Fme(ctx, {o, v}), Fae(ctx, {v, v}), Fmi(ctx, {o, o});
  zein(ctx, "nf,menf->me", one, T1, I->oovv_r, zero, Fme);
  // F_ae = sum_mf t_m^f <ma||fe> - 1/2 sum tau~_mn^af <mn||ef>,  <ma||fe> = (mf|ae) - (me|af)
  zein(ctx, "P,aeP->ae", one, xP, Lvv, zero, Fae);
  zein(ctx, "amP,meP->ae", mone, Y, I->Lov, one, Fae);
  // one (a x e) product per occupied pair (m, n), summed in pair order: no operand reordering
  zgemm_sum(ctx, 'N', 'T', v, v, v, mhalf, taut.p(), v, v * v, I->oovv.p(), v, v * v, (int)(o * o), one, Fae.p(), v);
  // F_mi = sum_ne t_n^e <mn||ie> + 1/2 sum tau~_in^ef <mn||ef>
  zein(ctx, "ne,mnie->mi", one, T1, I->ooov, zero, Fmi);
  zein(ctx, "inef,mnef->mi", half, taut, I->oovv, one, Fmi);
  // W0_mnij = <mn||ij> + P(ij) sum_e t_j^e <mn||ie>
  ZTensor W0(ctx, {o, o, o, o}), tmp4(ctx, {o, o, o, o});
  FC_HIP(hipMemcpyAsync(W0.p(), I->oooo.p(), sizeof(z) * W0.size(), hipMemcpyDeviceToDevice, ctx->stream));
  zein(ctx, "mnie,je->mnij", one, I->ooov, T1, zero, tmp4);
  hipLaunchKernelGGL(k_antisym_oooo, dim3(nblk(W0.size())), dim3(TPB), 0, ctx->stream, W0.p(), tmp4.p(), o);
  // X_ijmn = sum_ef tau_ij^ef <mn||ef>
  ZTensor X(ctx, {o, o, o, o});
  zein(ctx, "ijef,mnef->ijmn", one, tau, I->oovv, zero, X);
  // W_mbej = <mb||ej> + sum_f t_j^f <mb||ef> - sum_n t_n^b <mn||ej> - sum_nf (t_jn^fb/2 + t_j^f t_n^b) <mn||ef>
  //   sum_f t_j^f <mb||ef> = sum_P L^P_me Y[b,j,P] - sum_P C[m,j,P] L^P_be
  ZTensor Wmbej(ctx, {o, v, v, o});
  FC_HIP(hipMemcpyAsync(Wmbej.p(), I->ovvo.p(), sizeof(z) * Wmbej.size(), hipMemcpyDeviceToDevice, ctx->stream));
  zein(ctx, "meP,bjP->mbej", one, I->Lov, Y, one, Wmbej);
  zein(ctx, "mjP,beP->mbej", mone, Cm, Lvv, one, Wmbej);
  zein(ctx, "nb,mnej->mbej", mone, T1, I->oovo, one, Wmbej);
  {  // Z_jn^fb = t_jn^fb / 2 + t_j^f t_n^b, formed in the product's operand order [b][j][n][f]
    ZTensor Zr(ctx, {v, o, o, v});
    const long nbt = (v + 31) / 32;
    FC_REQUIRE(o * o <= 65535, FC_EARG, "ccsd residual: too many occupied pairs for one launch");
    if (nbt > 0 && o > 0)
      hipLaunchKernelGGL(k_ring_amp_t, dim3((unsigned)(nbt * nbt), (unsigned)(o * o)), dim3(256), 0, ctx->stream, t1p,
                         t2p, Zr.p(), o, v, 0.5);
    zein(ctx, "bjnf,menf->mbej", mone, Zr, I->oovv_r, one, Wmbej);
  }

  // t_im^ae as [i][a][m][e]: the two products that sum over (m, e) with (i, a) free read it in place
  ZTensor T2r(ctx, {o, v, o, v});
  permute(ctx, T2, {0, 2, 1, 3}, one, zero, T2r.p());

  // ---- T1 residual
  zein(ctx, "ie,ae->ia", one, T1, Fae, zero, R1);
  zein(ctx, "ma,mi->ia", mone, T1, Fmi, one, R1);
  zein(ctx, "iame,me->ia", one, T2r, Fme, one, R1);
  zein(ctx, "nf,nfai->ia", mone, T1, I->ovov, one, R1);
  {  // -1/2 sum_mef t_im^ef <ma||ef> = - sum_fP Q[i,f,P] L^P_af,  Q[i,f,P] = sum_me t_im^ef L^P_me
    ZTensor Q(ctx, {o, v, N});
    // (one product per i reading t2[i] transposed in place pads 160-row outputs to 64-row tiles
    // and measured slower than the reorder plus one product: 0.71 against 0.52 + 0.09 ms)
    zein(ctx, "imef,meP->ifP", one, T2, I->Lov, zero, Q);
    zein(ctx, "ifP,afP->ia", mone, Q, Lvv, one, R1);
  }
  // -1/2 sum_mne t_mn^ae <nm||ei> = +1/2 sum_mn sum_e t_mn^ae <mn||ei> (<nm||ei> = -<mn||ei> exactly,
  // as the block is assembled): one (i x a) product per occupied pair (m, n), summed in pair order
  zgemm_sum(ctx, 'T', 'T', o, v, v, half, I->oovo.p(), o, v * o, t2p, v, v * v, (int)(o * o), one, r1p, v);

  // ---- T2 residual: R2 = <ab||ij> + ..., the integral block read by the first antisymmetrising add
  ZTensor x(ctx, {o, o, v, v});
  {  // P(ab) sum_e t_ij^ae (F_be - 1/2 sum_m t_m^b F_me)
    ZTensor Fp(ctx, {v, v});
    FC_HIP(hipMemcpyAsync(Fp.p(), Fae.p(), sizeof(z) * Fp.size(), hipMemcpyDeviceToDevice, ctx->stream));
    zein(ctx, "mb,me->be", mhalf, T1, Fme, one, Fp);
    zein(ctx, "ijae,be->ijab", one, T2, Fp, zero, x);
    antisym_add(ctx, r2p, x.p(), o, v, 1, one, I->vvoo.p());
    if (fdiag) hipLaunchKernelGGL(k_diag_copy, dim3(1), dim3(TPB), 0, ctx->stream, Fp.p(), v, fdiag + o);
  }
  {  // -P(ij) sum_m t_im^ab (F_mj + 1/2 sum_e t_j^e F_me)
    ZTensor Fp(ctx, {o, o});
    FC_HIP(hipMemcpyAsync(Fp.p(), Fmi.p(), sizeof(z) * Fp.size(), hipMemcpyDeviceToDevice, ctx->stream));
    zein(ctx, "je,me->mj", half, T1, Fme, one, Fp);
    // one product per i: x[i] (j x ab) = Fp^T t2[i] (m x ab), no operand reordering
    zgemm(ctx, 'T', 'N', o, v * v, o, one, Fp.p(), o, t2p, v * v, zero, x.p(), v * v, (int)o, 0, o * v * v,
          o * v * v);
    antisym_add(ctx, r2p, x.p(), o, v, 2, mone);
    if (fdiag) hipLaunchKernelGGL(k_diag_copy, dim3(1), dim3(TPB), 0, ctx->stream, Fp.p(), o, fdiag);
  }
  zein(ctx, "mnab,mnij->ijab", half, tau, W0, one, R2);
  zein(ctx, "mnab,ijmn->ijab", quarter, T2, X, one, R2);
  // particle-particle ladder with T1-dressed Cholesky vectors, added into R2 by its scatter
  ladder_dev(ctx, I, tau.p(), t1p, r2p, precision, true);
  {  // P(ij)P(ab) sum_me (t_im^ae W_mbej - t_i^e t_m^a <mb||ej>)
    zein(ctx, "iame,mbej->ijab", one, T2r, Wmbej, zero, x);
    ZTensor U(ctx, {o, o, v, o});
    // U[i,m,b,j] = sum_e t_i^e <mb||ej> = -sum_e t_i^e <mb||je>: the stored ring-order block
    // [m][e][b][j] of <mb||je> (the exact negation of <mb||ej>, as it is assembled) read in place,
    // one (i) x (b,j) product per m.  (One o x o product per (m, b) on <mb||ej> itself measured
    // slower than a reorder plus one product.)
    zgemm(ctx, 'N', 'N', o, v * o, v, mone, t1p, v, I->ovov.p(), v * o, zero, U.p(), o * v * o, (int)o, 0, v * v * o,
          v * o);
    zein(ctx, "ma,imbj->ijab", mone, T1, U, one, x);
    antisym_add(ctx, r2p, x.p(), o, v, 3, one);
  }
  {  // P(ij) sum_e t_i^e <ab||ej> = P(ij) [sum_P Y[a,i,P] L^P_bj - sum_P L^P_aj Y[b,i,P]]
    zein(ctx, "aiP,bjP->ijab", one, Y, I->Lvo, zero, x);
    zein(ctx, "ajP,biP->ijab", mone, I->Lvo, Y, one, x);
    antisym_add(ctx, r2p, x.p(), o, v, 2, one);
  }
  {  // -P(ab) sum_m t_m^a <mb||ij>, and Omega = RHS - D t for the doubles in the same pass
    zein(ctx, "ma,mbij->ijab", one, T1, I->ovoo, zero, x);
    antisym_add(ctx, r2p, x.p(), o, v, 1, mone, nullptr, t2p, I->eps_d.as<double>());
  }
  // Omega = RHS - D t for the singles
  hipLaunchKernelGGL(k_sub_denom1, dim3(nblk(o * v)), dim3(TPB), 0, ctx->stream, r1p, t1p, I->eps_d.as<double>(), o, v);
  FC_HIP(hipGetLastError());
}

// Jacobi step out = t + Omega/D (exported for the solver); with fd (the dressed one-particle
// diagonals from the residual) the denominators are dressed
void jacobi_step(fc_ctx ctx, fc_ints I, const z* t1, const z* t2, const z* r1, const z* r2, z* o1, z* o2,
                 const z* fd) {
  const long o = I->o, v = I->v;
  if (fd) {
    hipLaunchKernelGGL(k_jacobi1_dressed, dim3(nblk(o * v)), dim3(TPB), 0, ctx->stream, t1, r1, o1,
                       I->eps_d.as<double>(), fd, o, v);
    hipLaunchKernelGGL(k_jacobi2_dressed, dim3(nblk(o * o * v * v)), dim3(TPB), 0, ctx->stream, t2, r2, o2,
                       I->eps_d.as<double>(), fd, o, v);
  } else {
    hipLaunchKernelGGL(k_jacobi1, dim3(nblk(o * v)), dim3(TPB), 0, ctx->stream, t1, r1, o1, I->eps_d.as<double>(), o, v);
    hipLaunchKernelGGL(k_jacobi2, dim3(nblk(o * o * v * v)), dim3(TPB), 0, ctx->stream, t2, r2, o2,
                       I->eps_d.as<double>(), o, v);
  }
  FC_HIP(hipGetLastError());
}

}  // namespace fc
