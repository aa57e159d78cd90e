// IP-EOM-CCSD: H-bar blocks (built once, Sec. 3), sigma = H-bar R on 1h + 2h1p (Eq. 17-18) and a
// non-Hermitian Davidson solver whose subspace eigenproblem runs in FP64 on the host.
//
// sigma_i    = -F_mi r_m + F_me r_im^e - 1/2 W_mnie r_mn^e
// sigma_ij^a = -W_maij r_m + F_ae r_ij^e - P(ij) F_mi r_mj^a + 1/2 W_mnij r_mn^a
//              + P(ij) W_maej r_im^e + X_e t_ij^ae,   X_e = 1/2 <mn||ef> r_mn^f
// The only three-virtual piece, 1/2 sum_ef <mb||ef> tau_ij^ef inside W_mbij, is formed once from
// the Cholesky vectors in occupied-index chunks, never stored whole.
#include <algorithm>
#include <cmath>

#include "fc_state.hpp"

namespace fc {
void jacobi_step(fc_ctx, fc_ints, const z*, const z*, const z*, const z*, z*, z*);
namespace {
constexpr int TPB = 256;
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(1048576L, (n + TPB * 4 - 1) / (TPB * 4))); }
#define GRID_STRIDE(i, n) for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)
__device__ inline z cmul(z a, z b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

__global__ void k_tau_full(const z* t1, const z* t2, z* tau, long o, long v) {
  GRID_STRIDE(t, o * o * v * v) {
    long b = t % v, a = (t / v) % v, j = (t / (v * v)) % o, i = t / (v * v * o);
    z x = cmul(t1[i * v + a], t1[j * v + b]), y = cmul(t1[i * v + b], t1[j * v + a]);
    tau[t] = make_double2(t2[t].x + x.x - y.x, t2[t].y + x.y - y.y);
  }
}
__global__ void k_ring_amp1(const z* t1, const z* t2, z* Z, long o, long v) {
  GRID_STRIDE(t, o * o * v * v) {
    long b = t % v, f = (t / v) % v, n = (t / (v * v)) % o, j = t / (v * v * o);
    z p = cmul(t1[j * v + f], t1[n * v + b]);
    Z[t] = make_double2(t2[t].x + p.x, t2[t].y + p.y);
  }
}
// W[..., i, j] += alpha (x[..., i, j] - x[..., j, i])
__global__ void k_antisym_last2(z* W, const z* x, long outer, long o, z alpha) {
  GRID_STRIDE(t, outer * o * o) {
    long j = t % o, i = (t / o) % o, q = t / (o * o);
    z a = x[t], b = x[(q * o + j) * o + i];
    z d = make_double2(a.x - b.x, a.y - b.y);
    z r = cmul(alpha, d);
    W[t].x += r.x; W[t].y += r.y;
  }
}
// add eps on the diagonal of an n x n block
__global__ void k_add_diag(z* F, const double* e, long n) {
  GRID_STRIDE(i, n) { F[i * n + i].x += e[i]; }
}
// [k][i][j][a] += alpha (x - x^(i<->j))
__global__ void k_antisym_ij_k(z* S, const z* x, long nk, long o, long v, z alpha) {
  GRID_STRIDE(t, nk * o * o * v) {
    long a = t % v, j = (t / v) % o, i = (t / (v * o)) % o, k = t / (v * o * o);
    z p = x[t], q = x[((k * o + j) * o + i) * v + a];
    z r = cmul(alpha, make_double2(p.x - q.x, p.y - q.y));
    S[t].x += r.x; S[t].y += r.y;
  }
}
// packed R [k][dim] -> r1 [k][o], r2 [k][o][o][v] (antisymmetric in ij)
__global__ void k_unpack(const z* R, z* r1, z* r2, long nk, long o, long v, long dim, const int2* po, long no) {
  GRID_STRIDE(t, nk * o * o * v) {
    long b = t % v, j = (t / v) % o, i = (t / (v * o)) % o, k = t / (v * o * o);
    z val = make_double2(0, 0);
    if (i != j) {
      long lo = i < j ? i : j, hi = i < j ? j : i;
      long p = lo * o - lo * (lo + 1) / 2 + (hi - lo - 1);  // index of pair (lo, hi)
      val = R[k * dim + o + p * v + b];
      if (i > j) { val.x = -val.x; val.y = -val.y; }
    }
    r2[t] = val;
    if (j == 0 && b == 0) r1[k * o + i] = R[k * dim + i];
  }
}
__global__ void k_pack(const z* s1, const z* s2, z* S, long nk, long o, long v, long dim, const int2* po, long no) {
  GRID_STRIDE(t, nk * dim) {
    long x = t % dim, k = t / dim;
    if (x < o) { S[t] = s1[k * o + x]; continue; }
    long q = x - o, b = q % v, p = q / v;
    int2 ij = po[p];
    S[t] = s2[((k * o + ij.x) * o + ij.y) * v + b];
  }
}
// delta_j = r_j / (theta_j - diag), guarded
__global__ void k_precond(const z* Rs, z* out, const z* diag, z theta, long dim) {
  GRID_STRIDE(x, dim) {
    double dr = theta.x - diag[x].x, di = theta.y - diag[x].y;
    double m = dr * dr + di * di;
    if (m < 1e-16) { dr = 1e-8; di = 0; m = 1e-16; }
    z r = Rs[x];
    out[x] = make_double2((r.x * dr + r.y * di) / m, (r.y * dr - r.x * di) / m);
  }
}
__global__ void k_diag(const z* Fmi, const z* Fae, z* d, long o, long v, long dim, const int2* po) {
  GRID_STRIDE(x, dim) {
    if (x < o) { d[x] = make_double2(-Fmi[x * o + x].x, -Fmi[x * o + x].y); continue; }
    long q = x - o, b = q % v, p = q / v;
    int2 ij = po[p];
    z fb = Fae[b * v + b], fi = Fmi[ij.x * o + ij.x], fj = Fmi[ij.y * o + ij.y];
    d[x] = make_double2(fb.x - fi.x - fj.x, fb.y - fi.y - fj.y);
  }
}
}  // namespace

// three-virtual part of W-bar_mbij: out[m,b,i,j] += sum_ef (me|bf) tau_ij^ef, chunked over m
static void wmbij_three_virtual(fc_ctx ctx, fc_ints I, const ZTensor& tau, z* out) {
  const long o = I->o, v = I->v, N = I->ncd;
  const z one = make_double2(1, 0), zero = make_double2(0, 0);
  const double budget = 1024.0 * 1024 * 1024;
  long mc = std::max(1L, std::min(o, (long)(budget / (16.0 * (double)v * v * v))));
  ZTensor Im(ctx, {mc, v, v, v});
  for (long m0 = 0; m0 < o; m0 += mc) {
    long nm = std::min(mc, o - m0);
    // Im[m,e,b,f] = sum_P L^P_me L^P_bf
    zgemm(ctx, 'N', 'T', nm * v, v * v, N, one, I->Lov.p() + m0 * v * N, N, I->Lvv.p(), N, zero, Im.p(), v * v);
    ZT Iv(Im.p(), {nm, v, v, v});
    ZT Ov(out + m0 * v * o * o, {nm, v, o, o});
    zein(ctx, "mebf,ijef->mbij", one, Iv, tau, one, Ov);
  }
}

void build_hbar(fc_ctx ctx, fc_ints I, fc_amps T) {
  StageTimer st(ctx, "hbar");
  HbarBlocks& H = T->hb;
  const long o = I->o, v = I->v, N = I->ncd;
  const z one = make_double2(1, 0), zero = make_double2(0, 0), half = make_double2(0.5, 0),
          mone = make_double2(-1, 0), mhalf = make_double2(-0.5, 0);
  ZT T1(T->t1.p(), {o, v}), T2(T->t2.p(), {o, o, v, v});
  const long n2 = o * o * v * v;
  ZTensor tau(ctx, {o, o, v, v});
  hipLaunchKernelGGL(k_tau_full, dim3(nblk(n2)), dim3(TPB), 0, ctx->stream, T->t1.p(), T->t2.p(), tau.p(), o, v);
  ZTensor xP(ctx, {N}), Y(ctx, {v, o, N}), Cm(ctx, {o, o, N});
  zein(ctx, "mf,mfP->P", one, T1, I->Lov, zero, xP);
  zgemm(ctx, 'N', 'N', o, N, v, one, T->t1.p(), v, I->Lvv.p(), N, zero, Y.p(), N, (int)v, 0, v * N, o * N);
  zgemm(ctx, 'N', 'N', o, N, v, one, T->t1.p(), v, I->Lov.p(), N, zero, Cm.p(), N, (int)o, 0, v * N, o * N);

  H.Fme = ZTensor(ctx, {o, v});
  zein(ctx, "nf,mnef->me", one, T1, I->oovv, zero, H.Fme);
  H.Fmi = ZTensor(ctx, {o, o});
  zein(ctx, "ne,mnie->mi", one, T1, I->ooov, zero, H.Fmi);
  zein(ctx, "inef,mnef->mi", half, tau, I->oovv, one, H.Fmi);
  hipLaunchKernelGGL(k_add_diag, dim3(1), dim3(TPB), 0, ctx->stream, H.Fmi.p(), I->eps_d.as<double>(), o);
  H.Fae = ZTensor(ctx, {v, v});
  zein(ctx, "P,aeP->ae", one, xP, I->Lvv, zero, H.Fae);
  zein(ctx, "amP,meP->ae", mone, Y, I->Lov, one, H.Fae);
  zein(ctx, "mnaf,mnef->ae", mhalf, tau, I->oovv, one, H.Fae);
  hipLaunchKernelGGL(k_add_diag, dim3(nblk(v)), dim3(TPB), 0, ctx->stream, H.Fae.p(), I->eps_d.as<double>() + o, v);
  // W_mnij = <mn||ij> + P(ij) t_j^e <mn||ie> + 1/2 tau_ij^ef <mn||ef>
  H.Wmnij = ZTensor(ctx, {o, o, o, o});
  FC_HIP(hipMemcpyAsync(H.Wmnij.p(), I->oooo.p(), sizeof(z) * H.Wmnij.size(), hipMemcpyDeviceToDevice, ctx->stream));
  {
    ZTensor tmp(ctx, {o, o, o, o});
    zein(ctx, "mnie,je->mnij", one, I->ooov, T1, zero, tmp);
    hipLaunchKernelGGL(k_antisym_last2, dim3(nblk(tmp.size())), dim3(TPB), 0, ctx->stream, H.Wmnij.p(), tmp.p(), o * o, o, one);
    zein(ctx, "ijef,mnef->mnij", half, tau, I->oovv, one, H.Wmnij);
  }
  // W_mnie = <mn||ie> + t_i^f <mn||fe>
  H.Wmnie = ZTensor(ctx, {o, o, o, v});
  FC_HIP(hipMemcpyAsync(H.Wmnie.p(), I->ooov.p(), sizeof(z) * H.Wmnie.size(), hipMemcpyDeviceToDevice, ctx->stream));
  zein(ctx, "if,mnfe->mnie", one, T1, I->oovv, one, H.Wmnie);
  // W_mbej = <mb||ej> + t_j^f <mb||ef> - t_n^b <mn||ej> - (t_jn^fb + t_j^f t_n^b) <mn||ef>
  H.Wmbej = ZTensor(ctx, {o, v, v, o});
  FC_HIP(hipMemcpyAsync(H.Wmbej.p(), I->ovvo.p(), sizeof(z) * H.Wmbej.size(), hipMemcpyDeviceToDevice, ctx->stream));
  zein(ctx, "meP,bjP->mbej", one, I->Lov, Y, one, H.Wmbej);
  zein(ctx, "mjP,beP->mbej", mone, Cm, I->Lvv, one, H.Wmbej);
  zein(ctx, "nb,mnej->mbej", mone, T1, I->oovo, one, H.Wmbej);
  {
    ZTensor Z(ctx, {o, o, v, v});
    hipLaunchKernelGGL(k_ring_amp1, dim3(nblk(n2)), dim3(TPB), 0, ctx->stream, T->t1.p(), T->t2.p(), Z.p(), o, v);
    zein(ctx, "jnfb,mnef->mbej", mone, Z, I->oovv, one, H.Wmbej);
  }
  // W_mbij = <mb||ij> - F_me t_ij^be - t_n^b W_mnij + 1/2 <mb||ef> tau_ij^ef
  //          + P(ij) [<mn||ie> t_jn^be + t_i^e (<mb||ej> - t_nj^bf <mn||ef>)]
  H.Wmbij = ZTensor(ctx, {o, v, o, o});
  FC_HIP(hipMemcpyAsync(H.Wmbij.p(), I->ovoo.p(), sizeof(z) * H.Wmbij.size(), hipMemcpyDeviceToDevice, ctx->stream));
  zein(ctx, "me,ijbe->mbij", mone, H.Fme, T2, one, H.Wmbij);
  zein(ctx, "nb,mnij->mbij", mone, T1, H.Wmnij, one, H.Wmbij);
  wmbij_three_virtual(ctx, I, tau, H.Wmbij.p());
  {
    ZTensor x(ctx, {o, v, o, o}), V(ctx, {o, v, v, o});
    zein(ctx, "mnie,jnbe->mbij", one, I->ooov, T2, zero, x);
    FC_HIP(hipMemcpyAsync(V.p(), I->ovvo.p(), sizeof(z) * V.size(), hipMemcpyDeviceToDevice, ctx->stream));
    zein(ctx, "njbf,mnef->mbej", mone, T2, I->oovv, one, V);
    zein(ctx, "ie,mbej->mbij", one, T1, V, one, x);
    hipLaunchKernelGGL(k_antisym_last2, dim3(nblk(x.size())), dim3(TPB), 0, ctx->stream, H.Wmbij.p(), x.p(), o * v, o, one);
  }
  FC_HIP(hipGetLastError());
  H.ready = true;
}

void sigma_dev(fc_ctx ctx, fc_ints I, fc_amps T, int nvec, const z* R, z* S) {
  StageTimer st(ctx, "sigma");
  if (!T->hb.ready) build_hbar(ctx, I, T);
  HbarBlocks& H = T->hb;
  const long o = I->o, v = I->v, k = nvec;
  const long no = o * (o - 1) / 2, dim = o + no * v;
  const z one = make_double2(1, 0), zero = make_double2(0, 0), half = make_double2(0.5, 0),
          mone = make_double2(-1, 0), mhalf = make_double2(-0.5, 0);
  if (k <= 0) return;
  std::vector<int2> hp;
  for (int i = 0; i < o; ++i) for (int j = i + 1; j < o; ++j) hp.push_back(make_int2(i, j));
  DBuf po(ctx, sizeof(int2) * std::max(1L, no));
  if (no) FC_HIP(hipMemcpyAsync(po.p, hp.data(), sizeof(int2) * no, hipMemcpyHostToDevice, ctx->stream));
  ZTensor r1(ctx, {k, o}), r2(ctx, {k, o, o, v}), s1(ctx, {k, o}), s2(ctx, {k, o, o, v}), x(ctx, {k, o, o, v});
  hipLaunchKernelGGL(k_unpack, dim3(nblk(r2.size())), dim3(TPB), 0, ctx->stream, R, r1.p(), r2.p(), k, o, v, dim,
                     po.as<int2>(), no);
  // sigma_i
  zein(ctx, "mi,km->ki", mone, H.Fmi, r1, zero, s1);
  zein(ctx, "me,kime->ki", one, H.Fme, r2, one, s1);
  zein(ctx, "mnie,kmne->ki", mhalf, H.Wmnie, r2, one, s1);
  // sigma_ij^a
  zein(ctx, "maij,km->kija", mone, H.Wmbij, r1, zero, s2);
  zein(ctx, "ae,kije->kija", one, H.Fae, r2, one, s2);
  zein(ctx, "mi,kmja->kija", one, H.Fmi, r2, zero, x);
  hipLaunchKernelGGL(k_antisym_ij_k, dim3(nblk(x.size())), dim3(TPB), 0, ctx->stream, s2.p(), x.p(), k, o, v, mone);
  zein(ctx, "mnij,kmna->kija", half, H.Wmnij, r2, one, s2);
  zein(ctx, "maej,kime->kija", one, H.Wmbej, r2, zero, x);
  hipLaunchKernelGGL(k_antisym_ij_k, dim3(nblk(x.size())), dim3(TPB), 0, ctx->stream, s2.p(), x.p(), k, o, v, one);
  {
    ZTensor X(ctx, {k, v});
    zein(ctx, "mnef,kmnf->ke", half, I->oovv, r2, zero, X);
    zein(ctx, "ke,ijae->kija", one, X, ZT(T->t2.p(), {o, o, v, v}), one, s2);
  }
  hipLaunchKernelGGL(k_pack, dim3(nblk(k * dim)), dim3(TPB), 0, ctx->stream, s1.p(), s2.p(), S, k, o, v, dim,
                     po.as<int2>(), no);
  FC_HIP(hipGetLastError());
}

// ------------------------------------------------------------------------------------ Davidson
static void lowest_by_real(const std::vector<z>& w, int k, std::vector<int>& idx) {
  idx.resize(w.size());
  for (size_t i = 0; i < w.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (w[a].x != w[b].x) return w[a].x < w[b].x;
    return w[a].y < w[b].y;
  });
  idx.resize(std::min<size_t>(k, w.size()));
}

int davidson_one(fc_ctx ctx, fc_ints I, fc_amps T, int k, const fc_eom_opts& op, z* omega, z* Rout, int* iters) {
  StageTimer st(ctx, "davidson");
  if (!T->hb.ready) build_hbar(ctx, I, T);
  const long o = I->o, v = I->v, no = o * (o - 1) / 2, dim = o + no * v;
  FC_REQUIRE(k >= 1 && k <= dim, FC_EARG, "ipeom_davidson: nroots out of range");
  const z one = make_double2(1, 0), zero = make_double2(0, 0), mone = make_double2(-1, 0);
  const int nguess = (int)std::min<long>(dim, std::max(k, op.guess_per_root * k));
  const int maxsub = (int)std::min<long>(dim, std::max<long>(op.max_subspace, nguess + k));
  // diagonal
  std::vector<int2> hp;
  for (int i = 0; i < o; ++i) for (int j = i + 1; j < o; ++j) hp.push_back(make_int2(i, j));
  DBuf po(ctx, sizeof(int2) * std::max(1L, no));
  if (no) FC_HIP(hipMemcpyAsync(po.p, hp.data(), sizeof(int2) * no, hipMemcpyHostToDevice, ctx->stream));
  DBuf diag(ctx, sizeof(z) * dim);
  hipLaunchKernelGGL(k_diag, dim3(nblk(dim)), dim3(TPB), 0, ctx->stream, T->hb.Fmi.p(), T->hb.Fae.p(), diag.as<z>(),
                     o, v, dim, po.as<int2>());
  std::vector<z> hdiag(dim);
  FC_HIP(hipMemcpyAsync(hdiag.data(), diag.p, sizeof(z) * dim, hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<int> order(dim);
  for (long i = 0; i < dim; ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hdiag[a].x < hdiag[b].x; });
  DBuf Vb(ctx, sizeof(z) * (size_t)maxsub * dim), Sb(ctx, sizeof(z) * (size_t)maxsub * dim);
  z* V = Vb.as<z>();
  z* S = Sb.as<z>();
  fill(ctx, V, (long)nguess * dim, zero);
  for (int g = 0; g < nguess; ++g)
    FC_HIP(hipMemcpyAsync(V + (size_t)g * dim + order[g], &one, sizeof(z), hipMemcpyHostToDevice, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  int m = nguess;
  sigma_dev(ctx, I, T, m, V, S);
  std::vector<z> theta_old;
  DBuf Xb(ctx, sizeof(z) * (size_t)k * dim), Rb(ctx, sizeof(z) * (size_t)k * dim), Db(ctx, sizeof(z) * (size_t)k * dim);
  DBuf Yd(ctx, sizeof(z) * (size_t)maxsub * std::max(k, 2 * k)), Cd(ctx, sizeof(z) * (size_t)maxsub * k);
  int it;
  for (it = 1; it <= op.max_iter; ++it) {
    // subspace matrix G = V^H S  (G[p][q] = <v_p | H v_q>)
    DBuf Gd(ctx, sizeof(z) * (size_t)m * m);
    zgemm(ctx, 'R', 'T', m, m, dim, one, V, dim, S, dim, zero, Gd.as<z>(), m);
    std::vector<z> G(m * (size_t)m), w, Y;
    FC_HIP(hipMemcpyAsync(G.data(), Gd.p, sizeof(z) * m * m, hipMemcpyDeviceToHost, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    gen_eig(m, G, w, Y);
    std::vector<int> sel;
    lowest_by_real(w, k, sel);
    // Yk (m x k), Ritz vectors X = Yk^T V, residuals R = Yk^T S - theta X
    std::vector<z> Yk(m * (size_t)k);
    for (int p = 0; p < m; ++p)
      for (int r = 0; r < k; ++r) Yk[p * (size_t)k + r] = Y[p * (size_t)m + sel[r]];
    FC_HIP(hipMemcpyAsync(Yd.p, Yk.data(), sizeof(z) * m * k, hipMemcpyHostToDevice, ctx->stream));
    zgemm(ctx, 'T', 'N', k, dim, m, one, Yd.as<z>(), k, V, dim, zero, Xb.as<z>(), dim);
    zgemm(ctx, 'T', 'N', k, dim, m, one, Yd.as<z>(), k, S, dim, zero, Rb.as<z>(), dim);
    std::vector<double> rn(k);
    double rmax = 0;
    for (int r = 0; r < k; ++r) {
      axpy(ctx, dim, make_double2(-w[sel[r]].x, -w[sel[r]].y), Xb.as<z>() + (size_t)r * dim, Rb.as<z>() + (size_t)r * dim);
      z nn = dotc(ctx, dim, Rb.as<z>() + (size_t)r * dim, Rb.as<z>() + (size_t)r * dim);
      rn[r] = std::sqrt(std::max(0.0, nn.x));
      rmax = std::max(rmax, rn[r]);
    }
    double dw = INFINITY;
    if (!theta_old.empty()) {
      dw = 0;
      for (int r = 0; r < k; ++r)
        dw = std::max(dw, std::hypot(w[sel[r]].x - theta_old[r].x, w[sel[r]].y - theta_old[r].y));
    }
    theta_old.assign(k, zero);
    for (int r = 0; r < k; ++r) theta_old[r] = w[sel[r]];
    if (ctx->verbose) {
      fprintf(stderr, "[davidson] it %d m %d rmax %.3e dw %.3e w0 %.10f\n", it, m, rmax, dw, w[sel[0]].x);
    }
    if (rmax < op.r_tol && dw < op.w_tol) break;
    // correction vectors
    int nnew = 0;
    for (int r = 0; r < k; ++r) {
      if (rn[r] < op.r_tol) continue;
      hipLaunchKernelGGL(k_precond, dim3(nblk(dim)), dim3(TPB), 0, ctx->stream, Rb.as<z>() + (size_t)r * dim,
                         Db.as<z>() + (size_t)nnew * dim, diag.as<z>(), w[sel[r]], dim);
      ++nnew;
    }
    if (nnew == 0) break;
    // collapse onto the lowest Ritz vectors when the subspace would overflow
    if (m + nnew > maxsub) {
      int keep = std::min(m, 2 * k);
      std::vector<int> sel2;
      lowest_by_real(w, keep, sel2);
      // orthonormalise the coefficient columns (V orthonormal => Ritz combinations orthonormal)
      std::vector<std::vector<std::complex<double>>> cols;
      for (int c = 0; c < keep; ++c) {
        std::vector<std::complex<double>> col(m);
        for (int p = 0; p < m; ++p) col[p] = {Y[p * (size_t)m + sel2[c]].x, Y[p * (size_t)m + sel2[c]].y};
        for (int pass = 0; pass < 2; ++pass)
          for (auto& q : cols) {
            std::complex<double> d = 0;
            for (int p = 0; p < m; ++p) d += std::conj(q[p]) * col[p];
            for (int p = 0; p < m; ++p) col[p] -= d * q[p];
          }
        double nr = 0;
        for (auto& x : col) nr += std::norm(x);
        nr = std::sqrt(nr);
        if (nr < 1e-12) continue;
        for (auto& x : col) x /= nr;
        cols.push_back(col);
      }
      int nk2 = (int)cols.size();
      std::vector<z> Yc(m * (size_t)nk2);
      for (int p = 0; p < m; ++p)
        for (int c = 0; c < nk2; ++c) Yc[p * (size_t)nk2 + c] = make_double2(cols[c][p].real(), cols[c][p].imag());
      DBuf Ycd(ctx, sizeof(z) * m * nk2), Vn(ctx, sizeof(z) * (size_t)nk2 * dim), Sn(ctx, sizeof(z) * (size_t)nk2 * dim);
      FC_HIP(hipMemcpyAsync(Ycd.p, Yc.data(), sizeof(z) * m * nk2, hipMemcpyHostToDevice, ctx->stream));
      zgemm(ctx, 'T', 'N', nk2, dim, m, one, Ycd.as<z>(), nk2, V, dim, zero, Vn.as<z>(), dim);
      zgemm(ctx, 'T', 'N', nk2, dim, m, one, Ycd.as<z>(), nk2, S, dim, zero, Sn.as<z>(), dim);
      FC_HIP(hipMemcpyAsync(V, Vn.p, sizeof(z) * nk2 * dim, hipMemcpyDeviceToDevice, ctx->stream));
      FC_HIP(hipMemcpyAsync(S, Sn.p, sizeof(z) * nk2 * dim, hipMemcpyDeviceToDevice, ctx->stream));
      m = nk2;
    }
    // orthogonalise the new block against V twice (classical Gram-Schmidt via GEMM), then among itself
    z* Dn = Db.as<z>();
    for (int pass = 0; pass < 2; ++pass) {
      zgemm(ctx, 'R', 'T', m, nnew, dim, one, V, dim, Dn, dim, zero, Cd.as<z>(), nnew);
      zgemm(ctx, 'T', 'N', nnew, dim, m, mone, Cd.as<z>(), nnew, V, dim, one, Dn, dim);
    }
    int added = 0;
    for (int j = 0; j < nnew; ++j) {
      z* x = Dn + (size_t)j * dim;
      for (int pass = 0; pass < 2; ++pass)
        for (int q = 0; q < added; ++q) {
          z* y = V + (size_t)(m + q) * dim;
          z d = dotc(ctx, dim, y, x);
          axpy(ctx, dim, make_double2(-d.x, -d.y), y, x);
        }
      z nn = dotc(ctx, dim, x, x);
      double nr = std::sqrt(std::max(0.0, nn.x));
      if (nr < 1e-10) continue;
      z* dst = V + (size_t)(m + added) * dim;
      FC_HIP(hipMemcpyAsync(dst, x, sizeof(z) * dim, hipMemcpyDeviceToDevice, ctx->stream));
      scale(ctx, dst, dim, make_double2(1.0 / nr, 0));
      ++added;
    }
    if (added == 0) break;
    sigma_dev(ctx, I, T, added, V + (size_t)m * dim, S + (size_t)m * dim);
    m += added;
  }
  for (int r = 0; r < k; ++r) omega[r] = theta_old[r];
  if (Rout) FC_HIP(hipMemcpyAsync(Rout, Xb.p, sizeof(z) * (size_t)k * dim, hipMemcpyDeviceToDevice, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  if (iters) *iters = std::min(it, op.max_iter);
  return it > op.max_iter ? FC_ENOCONV : FC_OK;
}

}  // namespace fc
