// IP-EOM-CCSD: H-bar blocks (built once, Sec. 3), sigma = H-bar R on 1h + 2h1p (Eq. 17-18) and a
// non-Hermitian Davidson solver whose subspace eigenproblem runs in FP64 on the host.
//
// sigma_i    = -F_mi r_m + F_me r_im^e - 1/2 W_mnie r_mn^e
// sigma_ij^a = -W_maij r_m + F_ae r_ij^e - P(ij) F_mi r_mj^a + 1/2 W_mnij r_mn^a
//              + P(ij) W_maej r_im^e + X_e t_ij^ae,   X_e = 1/2 <mn||ef> r_mn^f
// The only three-virtual piece, 1/2 sum_ef <mb||ef> tau_ij^ef inside W_mbij, is formed once from
// the Cholesky vectors in occupied-index chunks, never stored whole.  The sigma products
// themselves are evaluated as matrix products over the packed vector layout (fc_sigma.hip).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <exception>
#include <mutex>
#include <thread>

#include "fc_sigma.hpp"

namespace fc {
void jacobi_step(fc_ctx, fc_ints, const z*, const z*, const z*, const z*, z*, z*, const z* = nullptr);
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
  const ZTensor& Lvv = lvv(ctx, I);
  const double budget = 1024.0 * 1024 * 1024;
  long mc = std::max(1L, std::min(o, (long)(budget / (16.0 * (double)v * v * v))));
  ZTensor Im(ctx, {mc, v, v, v});
  for (long m0 = 0; m0 < o; m0 += mc) {
    long nm = std::min(mc, o - m0);
    // Im[m,e,b,f] = sum_P L^P_me L^P_bf
    zgemm(ctx, 'N', 'T', nm * v, v * v, N, one, I->Lov.p() + m0 * v * N, N, Lvv.p(), N, zero, Im.p(), v * v);
    ZT Iv(Im.p(), {nm, v, v, v});
    ZT Ov(out + m0 * v * o * o, {nm, v, o, o});
    zein(ctx, "mebf,ijef->mbij", one, Iv, tau, one, Ov);
  }
}

void build_hbar(fc_ctx ctx, fc_ints I, fc_amps T) {
  StageTimer st(ctx, "hbar");
  ensure_integrals(ctx, I);
  // with a split-precision integral handle (the mixed path) the H-bar products run in FP32
  // arithmetic like the residual's products outside the ladder; the blocks are stored in FP64 and
  // the Davidson sigma products that read them stay FP64
  Fp32Gemms fp32(ctx, I->precision != FC_FP64);
  const ZTensor& Lvv = lvv(ctx, I);
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
  zgemm(ctx, 'N', 'N', o, N, v, one, T->t1.p(), v, Lvv.p(), N, zero, Y.p(), N, (int)v, 0, v * N, o * N);
  zgemm(ctx, 'N', 'N', o, N, v, one, T->t1.p(), v, I->Lov.p(), N, zero, Cm.p(), N, (int)o, 0, v * N, o * N);

  H.Fme = ZTensor(ctx, {o, v});
  zein(ctx, "nf,menf->me", one, T1, I->oovv_r, zero, H.Fme);
  H.Fmi = ZTensor(ctx, {o, o});
  zein(ctx, "ne,mnie->mi", one, T1, I->ooov, zero, H.Fmi);
  zein(ctx, "inef,mnef->mi", half, tau, I->oovv, one, H.Fmi);
  hipLaunchKernelGGL(k_add_diag, dim3(1), dim3(TPB), 0, ctx->stream, H.Fmi.p(), I->eps_d.as<double>(), o);
  H.Fae = ZTensor(ctx, {v, v});
  zein(ctx, "P,aeP->ae", one, xP, Lvv, zero, H.Fae);
  zein(ctx, "amP,meP->ae", mone, Y, I->Lov, one, H.Fae);
  zgemm_sum(ctx, 'N', 'T', v, v, v, mhalf, tau.p(), v, v * v, I->oovv.p(), v, v * v, (int)(o * o), one, H.Fae.p(), v);
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
  zein(ctx, "mjP,beP->mbej", mone, Cm, Lvv, one, H.Wmbej);
  zein(ctx, "nb,mnej->mbej", mone, T1, I->oovo, one, H.Wmbej);
  {
    ZTensor Z(ctx, {o, o, v, v});
    hipLaunchKernelGGL(k_ring_amp1, dim3(nblk(n2)), dim3(TPB), 0, ctx->stream, T->t1.p(), T->t2.p(), Z.p(), o, v);
    zein(ctx, "jnfb,menf->mbej", mone, Z, I->oovv_r, one, H.Wmbej);
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
    zein(ctx, "njbf,menf->mbej", mone, T2, I->oovv_r, one, V);
    zein(ctx, "ie,mbej->mbij", one, T1, V, one, x);
    hipLaunchKernelGGL(k_antisym_last2, dim3(nblk(x.size())), dim3(TPB), 0, ctx->stream, H.Wmbij.p(), x.p(), o * v, o, one);
  }
  FC_HIP(hipGetLastError());
  H.ready = true;
}

void sigma_dev(fc_ctx ctx, fc_ints I, fc_amps T, int nvec, const z* R, z* S, bool left) {
  if (nvec <= 0) return;
  const long k = nvec;
  SigmaBatch sb(ctx, 1, &I, &T, &k, false, left);
  sb.run(&R, &S, &k);
}

// ------------------------------------------------------------------------------------ Davidson
// All instances advance in lockstep: every step below is one launch (or one transfer) for the
// whole batch, and the sigma products of all new trial vectors are one replay of a captured graph.
namespace {
struct RowJob {
  const z* X;        // source row
  z* R;              // destination row
  const z* diag;
  z theta;
  long dim, out;
};
// R -= theta X and |R|^2, one workgroup per row, summed in a fixed order
__global__ void k_resid_norm(const RowJob* __restrict__ jobs, double* __restrict__ nrm) {
  const RowJob j = jobs[blockIdx.x];
  double acc = 0;
  for (long x = threadIdx.x; x < j.dim; x += blockDim.x) {
    z r = j.R[x];
    const z xv = j.X[x];
    r.x -= j.theta.x * xv.x - j.theta.y * xv.y;
    r.y -= j.theta.x * xv.y + j.theta.y * xv.x;
    j.R[x] = r;
    acc += r.x * r.x + r.y * r.y;
  }
  __shared__ double sh[TPB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) nrm[j.out] = sh[0];
}
// correction vector R = X / (theta - diag), guarded against a vanishing denominator
__global__ void k_precond_rows(const RowJob* __restrict__ jobs) {
  const RowJob j = jobs[blockIdx.y];
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < j.dim; x += (long)gridDim.x * blockDim.x) {
    double dr = j.theta.x - j.diag[x].x, di = j.theta.y - j.diag[x].y;
    double m = dr * dr + di * di;
    if (m < 1e-16) { dr = 1e-8; di = 0; m = 1e-16; }
    const z r = j.X[x];
    j.R[x] = make_double2((r.x * dr + r.y * di) / m, (r.y * dr - r.x * di) / m);
  }
}
// scale each correction row to unit norm (one workgroup per row, fixed-order sum), so that the
// later test for vectors lost to the projection against V is relative to the vector's own size
__global__ void k_normalise_rows(const RowJob* __restrict__ jobs) {
  const RowJob j = jobs[blockIdx.x];
  double acc = 0;
  for (long x = threadIdx.x; x < j.dim; x += blockDim.x) acc += j.R[x].x * j.R[x].x + j.R[x].y * j.R[x].y;
  __shared__ double sh[TPB];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double n2 = sh[0];
  if (!(n2 > 0.0) || !(n2 < INFINITY)) return;
  const double f = 1.0 / sqrt(n2);
  for (long x = threadIdx.x; x < j.dim; x += blockDim.x) j.R[x] = make_double2(j.R[x].x * f, j.R[x].y * f);
}
__global__ void k_set_units(z* V, long dim, const long* idx, long n) {
  GRID_STRIDE(t, n) { V[t * dim + idx[t]] = make_double2(1.0, 0.0); }
}

void lowest_by_real(const std::vector<z>& w, int k, std::vector<int>& idx) {
  idx.resize(w.size());
  for (size_t i = 0; i < w.size(); ++i) idx[i] = (int)i;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
    if (w[a].x != w[b].x) return w[a].x < w[b].x;
    return w[a].y < w[b].y;
  });
  idx.resize(std::min<size_t>(k, w.size()));
}

// Pinned host buffer mirrored by a device buffer of the same size.
struct Mirror {
  fc_ctx ctx = nullptr;
  char* h = nullptr;
  DBuf d;
  size_t bytes = 0;
  Mirror(fc_ctx c, size_t n) : ctx(c), d(c, std::max<size_t>(n, 64)), bytes(std::max<size_t>(n, 64)) {
    FC_HIP(hipHostMalloc((void**)&h, bytes, hipHostMallocDefault));
  }
  ~Mirror() { if (h) (void)hipHostFree(h); }
  template <class T> T* host(size_t off) const { return reinterpret_cast<T*>(h + off); }
  template <class T> T* dev(size_t off) const { return reinterpret_cast<T*>(d.as<char>() + off); }
  void up(size_t off, size_t n) {
    if (n) FC_HIP(hipMemcpyAsync(d.as<char>() + off, h + off, n, hipMemcpyHostToDevice, ctx->stream));
  }
  void down(size_t off, size_t n) {
    if (n) FC_HIP(hipMemcpyAsync(h + off, d.as<char>() + off, n, hipMemcpyDeviceToHost, ctx->stream));
  }
};

struct Inst {
  fc_ints I;
  fc_amps T;
  int k = 0, nguess = 0, maxsub = 0;
  long o = 0, v = 0, dim = 0;
  DBuf V, S, X, Rr, D, D2, diag;
  int m = 0, gold = 0;            // vectors with sigma; leading block of G already known
  std::vector<z> G;               // maxsub x maxsub, row-major
  std::vector<z> Y, w;            // eigenvectors / values of the current subspace matrix
  std::vector<int> sel;
  std::vector<z> theta, theta_old;
  std::vector<double> rn;
  bool active = true;
  int iters = 0, status = FC_OK;
  // byte offsets in the staging mirror: this iteration's new G blocks and Ritz coefficients
  // (packed per iteration), projection coefficients, Gram matrix, orthonormalising
  // coefficients and residual norms (fixed)
  size_t off_g = 0, off_y = 0, off_c = 0, off_gram = 0, off_cc = 0, off_n = 0;
  int nnew = 0, added = 0;
  std::vector<int> roots;        // roots that get a correction vector this iteration
};

// fn(0..n-1) on up to 16 host threads (the calling thread included); the first exception
// thrown by any call is rethrown after all threads have joined.
template <class F>
void for_each_parallel(int n, F&& fn) {
  const int nt = std::max(1, std::min({n, 16, (int)std::thread::hardware_concurrency()}));
  if (nt <= 1) {
    for (int t = 0; t < n; ++t) fn(t);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex mu;
  auto worker = [&] {
    for (int t; (t = next.fetch_add(1)) < n;) {
      try {
        fn(t);
      } catch (...) {
        std::lock_guard<std::mutex> lk(mu);
        if (!err) err = std::current_exception();
      }
    }
  };
  std::vector<std::thread> th;
  for (int i = 1; i < nt; ++i) th.emplace_back(worker);
  worker();
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}

// split-K partial sums (complex elements) of one product under tiling `tl`
size_t split_elems(long M, long N, long K, const GroupTiling& tl) {
  if (K <= tl.kchunk) return 0;
  return (size_t)((K + tl.kchunk - 1) / tl.kchunk + 1) * M * N;
}
}  // namespace

// With `left` the trial vectors are multiplied from the left (sigma = V H-bar), so the solve
// finds the eigenvectors of the transposed matrix: the left eigenvectors of Eq. 19-20, with the
// same eigenvalues and the same diagonal preconditioner.
int davidson_batch(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* amps, const int* nroots,
                   const fc_eom_opts& op, z* omega, z* Rout, int* iters, bool left) {
  StageTimer st(ctx, "davidson");
  const z one = make_double2(1, 0), zero = make_double2(0, 0), mone = make_double2(-1, 0);
  const GroupTiling tl{0, 1024};
  std::vector<Inst> in(nb);
  size_t wmax = 0, gcap = 0, ycap = 0;
  long rows_total = 0;
  for (int b = 0; b < nb; ++b) {
    Inst& s = in[b];
    s.I = ints[b];
    s.T = amps[b];
    FC_REQUIRE(s.I && s.T && s.T->ints == s.I, FC_EARG, "ipeom_davidson: bad handles");
    if (!s.T->hb.ready) build_hbar(ctx, s.I, s.T);
    s.o = s.I->o; s.v = s.I->v;
    const long no = s.o * (s.o - 1) / 2;
    s.dim = s.o + no * s.v;
    s.k = nroots[b];
    FC_REQUIRE(s.k >= 1 && s.k <= s.dim, FC_EARG, "ipeom_davidson: nroots out of range");
    s.nguess = (int)std::min<long>(s.dim, std::max(s.k, op.guess_per_root * s.k));
    // 10 x roots by default: at o=24 v=160 with 8 roots, 18 iterations in 46 ms against 15 in
    // 68 ms with 20 x roots (the host eigenproblem of the projected matrix grows as its cube)
    const long msub = op.max_subspace > 0 ? op.max_subspace : 10L * s.k;
    s.maxsub = (int)std::min<long>(s.dim, std::max<long>(msub, s.nguess + s.k));
    s.V = DBuf(ctx, sizeof(z) * (size_t)s.maxsub * s.dim);
    s.S = DBuf(ctx, sizeof(z) * (size_t)s.maxsub * s.dim);
    s.X = DBuf(ctx, sizeof(z) * (size_t)s.k * s.dim);
    s.Rr = DBuf(ctx, sizeof(z) * (size_t)s.k * s.dim);
    s.D = DBuf(ctx, sizeof(z) * (size_t)s.k * s.dim);
    s.D2 = DBuf(ctx, sizeof(z) * (size_t)s.k * s.dim);
    s.diag = DBuf(ctx, sizeof(z) * s.dim);
    s.G.assign((size_t)s.maxsub * s.maxsub, zero);
    gcap += (size_t)s.maxsub * s.maxsub;
    ycap += (size_t)s.maxsub * s.k;
    rows_total += s.k;
    // split-K workspace of one iteration (upper bound): G blocks, Ritz vectors, two rounds of
    // two projections, Gram matrices and transforms
    const long ms = s.maxsub, k = s.k, d = s.dim;
    wmax += 2 * split_elems(ms, ms, d, tl) + 2 * split_elems(k, d, ms, tl) +
            4 * (split_elems(ms, k, d, tl) + split_elems(k, d, ms, tl)) + 2 * split_elems(k, k, d, tl) +
            2 * split_elems(k, d, k, tl);
  }
  // staging mirror, one contiguous range per kind so each transfer moves one range
  size_t moff = 0;
  auto take = [&](size_t n) { size_t a = moff; moff += (n + 255) / 256 * 256; return a; };
  const size_t rg_g = take(sizeof(z) * gcap), rg_y = take(sizeof(z) * ycap);
  const size_t rg_n = moff;
  for (Inst& s : in) s.off_n = take(sizeof(double) * s.k);
  const size_t rg_n_end = moff;
  for (Inst& s : in) s.off_gram = take(sizeof(z) * s.k * s.k);
  const size_t rg_gram_end = moff;
  const size_t rg_cc = moff;
  for (Inst& s : in) s.off_cc = take(sizeof(z) * s.k * s.k);
  const size_t rg_cc_end = moff;
  for (Inst& s : in) s.off_c = take(sizeof(z) * (size_t)s.maxsub * s.k);
  const size_t off_jobs = take(sizeof(RowJob) * rows_total);
  Mirror mir(ctx, moff);
  GroupArena arena(ctx, 64 * 1024 + (size_t)nb * 48 * 256, wmax);

  // diagonal guesses: unit vectors on the nguess smallest diagonal elements (by real part)
  for (Inst& s : in) {
    const long no = s.o * (s.o - 1) / 2;
    std::vector<int2> hp;
    for (int i = 0; i < s.o; ++i)
      for (int j = i + 1; j < s.o; ++j) hp.push_back(make_int2(i, j));
    DBuf pd(ctx, sizeof(int2) * std::max(1L, no));
    if (no) FC_HIP(hipMemcpyAsync(pd.p, hp.data(), sizeof(int2) * no, hipMemcpyHostToDevice, ctx->stream));
    hipLaunchKernelGGL(k_diag, dim3(nblk(s.dim)), dim3(TPB), 0, ctx->stream, s.T->hb.Fmi.p(), s.T->hb.Fae.p(),
                       s.diag.as<z>(), s.o, s.v, s.dim, pd.as<int2>());
    std::vector<z> hd(s.dim);
    FC_HIP(hipMemcpyAsync(hd.data(), s.diag.p, sizeof(z) * s.dim, hipMemcpyDeviceToHost, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    std::vector<long> order(s.dim);
    for (long i = 0; i < s.dim; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](long a, long c) { return hd[a].x < hd[c].x; });
    order.resize(s.nguess);
    DBuf id(ctx, sizeof(long) * s.nguess);
    FC_HIP(hipMemcpyAsync(id.p, order.data(), sizeof(long) * s.nguess, hipMemcpyHostToDevice, ctx->stream));
    fill(ctx, s.V.as<z>(), (long)s.nguess * s.dim, zero);
    hipLaunchKernelGGL(k_set_units, dim3(nblk(s.nguess)), dim3(TPB), 0, ctx->stream, s.V.as<z>(), s.dim,
                       id.as<long>(), (long)s.nguess);
    FC_HIP(hipGetLastError());
    FC_HIP(hipStreamSynchronize(ctx->stream));
  }

  std::vector<long> kmax(nb), nv(nb);
  std::vector<const z*> Rp(nb);
  std::vector<z*> Sp(nb);
  for (int b = 0; b < nb; ++b) kmax[b] = std::max(in[b].nguess, in[b].k);
  SigmaBatch sb(ctx, nb, ints, amps, kmax.data(), op.graph != 0, left);
  for (int b = 0; b < nb; ++b) {
    nv[b] = in[b].nguess;
    Rp[b] = in[b].V.as<z>();
    Sp[b] = in[b].S.as<z>();
    in[b].m = in[b].nguess;
  }
  sb.run(Rp.data(), Sp.data(), nv.data());

  std::vector<GroupGemm> g;
  int it;
  for (it = 1; it <= op.max_iter; ++it) {
    bool any = false;
    for (const Inst& s : in) any = any || s.active;
    if (!any) break;
    // the arena's pinned plans of the previous iteration must have been consumed
    FC_HIP(hipStreamSynchronize(ctx->stream));
    arena.reset();
    // (1) new blocks of G = V^H S, packed back to back
    g.clear();
    size_t gused = 0;
    for (Inst& s : in) {
      if (!s.active || s.gold == s.m) continue;
      const int nn = s.m - s.gold;
      s.off_g = rg_g + sizeof(z) * gused;
      gused += (size_t)s.m * nn + (size_t)nn * s.gold;
      z* gd = mir.dev<z>(s.off_g);
      GroupGemm p;
      p.opA = 'R'; p.opB = 'T'; p.M = s.m; p.N = nn; p.K = s.dim;
      p.A = s.V.as<z>(); p.lda = s.dim; p.B = s.S.as<z>() + (size_t)s.gold * s.dim; p.ldb = s.dim;
      p.C = gd; p.ldc = nn;
      g.push_back(p);
      if (s.gold > 0) {
        p = GroupGemm{};
        p.opA = 'R'; p.opB = 'T'; p.M = nn; p.N = s.gold; p.K = s.dim;
        p.A = s.V.as<z>() + (size_t)s.gold * s.dim; p.lda = s.dim; p.B = s.S.as<z>(); p.ldb = s.dim;
        p.C = gd + (size_t)s.m * nn; p.ldc = s.gold;
        g.push_back(p);
      }
    }
    arena.run(g, tl);
    mir.down(rg_g, sizeof(z) * gused);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    // (2) subspace eigenproblems on the host, the instances spread over host threads; Ritz
    // coefficients up
    size_t yused = 0;
    std::vector<Inst*> act;
    for (Inst& s : in) {
      if (!s.active) continue;
      s.off_y = rg_y + sizeof(z) * yused;
      yused += (size_t)s.m * s.k;
      act.push_back(&s);
    }
    for_each_parallel((int)act.size(), [&](int t) {
      Inst& s = *act[t];
      const int nn = s.m - s.gold;
      const z* gh = mir.host<z>(s.off_g);
      for (int p = 0; p < s.m; ++p)
        for (int c = 0; c < nn; ++c) s.G[(size_t)p * s.maxsub + s.gold + c] = gh[(size_t)p * nn + c];
      for (int r = 0; r < nn; ++r)
        for (int q = 0; q < s.gold; ++q)
          s.G[(size_t)(s.gold + r) * s.maxsub + q] = gh[(size_t)s.m * nn + (size_t)r * s.gold + q];
      s.gold = s.m;
      std::vector<z> Gm((size_t)s.m * s.m);
      for (int p = 0; p < s.m; ++p)
        for (int q = 0; q < s.m; ++q) Gm[(size_t)p * s.m + q] = s.G[(size_t)p * s.maxsub + q];
      gen_eig(s.m, Gm, s.w, s.Y);
      lowest_by_real(s.w, s.k, s.sel);
      z* yk = mir.host<z>(s.off_y);
      for (int p = 0; p < s.m; ++p)
        for (int r = 0; r < s.k; ++r) yk[(size_t)p * s.k + r] = s.Y[(size_t)p * s.m + s.sel[r]];
      s.theta.assign(s.k, zero);
      for (int r = 0; r < s.k; ++r) s.theta[r] = s.w[s.sel[r]];
    });
    mir.up(rg_y, sizeof(z) * yused);
    // (3) Ritz vectors X = Yk^T V and residuals R = Yk^T S - theta X with their norms
    g.clear();
    long nj = 0;
    RowJob* jobs = mir.host<RowJob>(off_jobs);
    for (Inst& s : in) {
      if (!s.active) continue;
      GroupGemm p;
      p.opA = 'T'; p.M = s.k; p.N = s.dim; p.K = s.m;
      p.A = mir.dev<z>(s.off_y); p.lda = s.k; p.B = s.V.as<z>(); p.ldb = s.dim;
      p.C = s.X.as<z>(); p.ldc = s.dim;
      g.push_back(p);
      p.B = s.S.as<z>(); p.C = s.Rr.as<z>();
      g.push_back(p);
      for (int r = 0; r < s.k; ++r)
        jobs[nj++] = RowJob{s.X.as<z>() + (size_t)r * s.dim, s.Rr.as<z>() + (size_t)r * s.dim, nullptr,
                            s.theta[r], s.dim, (long)(s.off_n / sizeof(double)) + r};
    }
    arena.run(g, tl);
    mir.up(off_jobs, sizeof(RowJob) * nj);
    if (nj) {
      hipLaunchKernelGGL(k_resid_norm, dim3((unsigned)nj), dim3(TPB), 0, ctx->stream, mir.dev<RowJob>(off_jobs),
                         mir.dev<double>(0));
      FC_HIP(hipGetLastError());
    }
    mir.down(rg_n, rg_n_end - rg_n);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    // (4) convergence, restarts and the correction vectors
    nj = 0;
    std::vector<Inst*> restart;
    for (Inst& s : in) {
      if (!s.active) continue;
      s.iters = it;
      const double* nh = mir.host<double>(s.off_n);
      s.rn.assign(s.k, 0.0);
      double rmax = 0;
      for (int r = 0; r < s.k; ++r) {
        s.rn[r] = std::sqrt(std::max(0.0, nh[r]));
        rmax = std::max(rmax, s.rn[r]);
      }
      double dw = INFINITY;
      if (!s.theta_old.empty()) {
        dw = 0;
        for (int r = 0; r < s.k; ++r)
          dw = std::max(dw, std::hypot(s.theta[r].x - s.theta_old[r].x, s.theta[r].y - s.theta_old[r].y));
      }
      s.theta_old = s.theta;
      if (ctx->verbose)
        fprintf(stderr, "[davidson] it %d m %d rmax %.3e dw %.3e w0 %.10f\n", it, s.m, rmax, dw, s.theta[0].x);
      if (rmax < op.r_tol && dw < op.w_tol) { s.active = false; continue; }
      s.roots.clear();
      for (int r = 0; r < s.k; ++r)
        if (s.rn[r] >= op.r_tol) s.roots.push_back(r);
      s.nnew = (int)s.roots.size();
      if (s.nnew == 0) { s.active = false; continue; }
      for (int j = 0; j < s.nnew; ++j)
        jobs[nj++] = RowJob{s.Rr.as<z>() + (size_t)s.roots[j] * s.dim, s.D.as<z>() + (size_t)j * s.dim,
                            s.diag.as<z>(), s.theta[s.roots[j]], s.dim, 0};
      if (s.m + s.nnew > s.maxsub) restart.push_back(&s);
    }
    if (nj) {
      // the previous job table has been read: the norms above were synchronised after it
      mir.up(off_jobs, sizeof(RowJob) * nj);
      hipLaunchKernelGGL(k_precond_rows, dim3(64, (unsigned)nj), dim3(TPB), 0, ctx->stream,
                         mir.dev<RowJob>(off_jobs));
      hipLaunchKernelGGL(k_normalise_rows, dim3((unsigned)nj), dim3(TPB), 0, ctx->stream, mir.dev<RowJob>(off_jobs));
      FC_HIP(hipGetLastError());
    }
    // (5) restart: collapse V and S onto the lowest Ritz vectors (orthonormalised combinations),
    // leaving room for this iteration's correction vectors
    for (Inst* sp : restart) {
      Inst& s = *sp;
      const int keep = std::min({s.m, 2 * s.k, s.maxsub - s.nnew});
      std::vector<int> sel2;
      lowest_by_real(s.w, keep, sel2);
      std::vector<std::vector<std::complex<double>>> cols;
      for (int c = 0; c < keep; ++c) {
        std::vector<std::complex<double>> col(s.m);
        for (int p = 0; p < s.m; ++p) col[p] = {s.Y[(size_t)p * s.m + sel2[c]].x, s.Y[(size_t)p * s.m + sel2[c]].y};
        for (int pass = 0; pass < 2; ++pass)
          for (auto& q : cols) {
            std::complex<double> d = 0;
            for (int p = 0; p < s.m; ++p) d += std::conj(q[p]) * col[p];
            for (int p = 0; p < s.m; ++p) col[p] -= d * q[p];
          }
        double nr = 0;
        for (auto& x : col) nr += std::norm(x);
        nr = std::sqrt(nr);
        if (nr < 1e-12) continue;
        for (auto& x : col) x /= nr;
        cols.push_back(col);
      }
      const int nk2 = (int)cols.size();
      std::vector<z> Yc((size_t)s.m * nk2);
      for (int p = 0; p < s.m; ++p)
        for (int c = 0; c < nk2; ++c) Yc[(size_t)p * nk2 + c] = make_double2(cols[c][p].real(), cols[c][p].imag());
      DBuf Ycd(ctx, sizeof(z) * s.m * nk2), Vn(ctx, sizeof(z) * (size_t)nk2 * s.dim),
          Sn(ctx, sizeof(z) * (size_t)nk2 * s.dim);
      FC_HIP(hipMemcpyAsync(Ycd.p, Yc.data(), sizeof(z) * s.m * nk2, hipMemcpyHostToDevice, ctx->stream));
      zgemm(ctx, 'T', 'N', nk2, s.dim, s.m, one, Ycd.as<z>(), nk2, s.V.as<z>(), s.dim, zero, Vn.as<z>(), s.dim);
      zgemm(ctx, 'T', 'N', nk2, s.dim, s.m, one, Ycd.as<z>(), nk2, s.S.as<z>(), s.dim, zero, Sn.as<z>(), s.dim);
      FC_HIP(hipMemcpyAsync(s.V.p, Vn.p, sizeof(z) * nk2 * s.dim, hipMemcpyDeviceToDevice, ctx->stream));
      FC_HIP(hipMemcpyAsync(s.S.p, Sn.p, sizeof(z) * nk2 * s.dim, hipMemcpyDeviceToDevice, ctx->stream));
      FC_HIP(hipStreamSynchronize(ctx->stream));
      s.m = nk2;
      s.gold = 0;   // recompute the (small) subspace matrix from the collapsed vectors
    }
    // (6) orthonormalise the correction vectors: project out V twice, then a Gram-matrix
    // (Loewdin) step; a second round when that Gram matrix was badly conditioned
    std::vector<Inst*> work;
    for (Inst& s : in) {
      s.added = 0;
      if (s.active && s.nnew > 0) work.push_back(&s);
    }
    std::vector<z*> src(nb, nullptr);
    for (Inst* sp : work) src[sp - in.data()] = sp->D.as<z>();
    for (int round = 0; round < 2 && !work.empty(); ++round) {
      for (int pass = 0; pass < 2; ++pass) {
        g.clear();
        for (Inst* sp : work) {
          Inst& s = *sp;
          GroupGemm p;
          p.opA = 'R'; p.opB = 'T'; p.M = s.m; p.N = s.nnew; p.K = s.dim;
          p.A = s.V.as<z>(); p.lda = s.dim; p.B = src[sp - in.data()]; p.ldb = s.dim;
          p.C = mir.dev<z>(s.off_c); p.ldc = s.nnew;
          g.push_back(p);
        }
        arena.run(g, tl);
        g.clear();
        for (Inst* sp : work) {
          Inst& s = *sp;
          GroupGemm p;
          p.opA = 'T'; p.M = s.nnew; p.N = s.dim; p.K = s.m; p.alpha = mone;
          p.A = mir.dev<z>(s.off_c); p.lda = s.nnew; p.B = s.V.as<z>(); p.ldb = s.dim;
          p.beta = one; p.C = src[sp - in.data()]; p.ldc = s.dim;
          g.push_back(p);
        }
        arena.run(g, tl);
      }
      g.clear();
      for (Inst* sp : work) {
        Inst& s = *sp;
        GroupGemm p;
        p.opA = 'R'; p.opB = 'T'; p.M = s.nnew; p.N = s.nnew; p.K = s.dim;
        p.A = src[sp - in.data()]; p.lda = s.dim; p.B = src[sp - in.data()]; p.ldb = s.dim;
        p.C = mir.dev<z>(s.off_gram); p.ldc = s.nnew;
        g.push_back(p);
      }
      arena.run(g, tl);
      mir.down(rg_n_end, rg_gram_end - rg_n_end);
      FC_HIP(hipStreamSynchronize(ctx->stream));
      std::vector<Inst*> again;
      g.clear();
      for (Inst* sp : work) {
        Inst& s = *sp;
        const int n = s.nnew;
        const z* gh = mir.host<z>(s.off_gram);
        // drop vectors that vanished under the projection, scale the rest to unit norm; the
        // corrections entered with unit norm, so d is the fraction of the vector outside span(V)
        std::vector<double> sc(n, 0.0);
        for (int j = 0; j < n; ++j) {
          const double d = gh[(size_t)j * n + j].x;
          sc[j] = d > 1e-20 ? 1.0 / std::sqrt(d) : 0.0;
        }
        std::vector<z> A((size_t)n * n);
        for (int j = 0; j < n; ++j)
          for (int l = 0; l < n; ++l) {
            const z u = gh[(size_t)j * n + l];
            A[(size_t)j * n + l] = make_double2(u.x * sc[j] * sc[l], u.y * sc[j] * sc[l]);
          }
        std::vector<double> lam;
        herm_eig(n, A, lam);
        std::vector<int> kept;
        for (int c = n - 1; c >= 0; --c)
          if (lam[c] > 1e-8) kept.push_back(c);
        const int na = (int)kept.size();
        if (na == 0) continue;
        z* cc = mir.host<z>(s.off_cc);
        double lmin = INFINITY;
        for (int c = 0; c < na; ++c) {
          const double f = 1.0 / std::sqrt(lam[kept[c]]);
          lmin = std::min(lmin, lam[kept[c]]);
          for (int j = 0; j < n; ++j) {
            const z u = A[(size_t)j * n + kept[c]];
            cc[(size_t)j * na + c] = make_double2(u.x * sc[j] * f, u.y * sc[j] * f);
          }
        }
        const bool redo = round == 0 && lmin < 1e-3;
        z* dst = redo ? s.D2.as<z>() : s.V.as<z>() + (size_t)s.m * s.dim;
        GroupGemm p;
        p.opA = 'T'; p.M = na; p.N = s.dim; p.K = n;
        p.A = mir.dev<z>(s.off_cc); p.lda = na; p.B = src[sp - in.data()]; p.ldb = s.dim;
        p.C = dst; p.ldc = s.dim;
        g.push_back(p);
        if (redo) {
          src[sp - in.data()] = dst;
          s.nnew = na;
          again.push_back(sp);
        } else {
          s.added = na;
        }
      }
      mir.up(rg_cc, rg_cc_end - rg_cc);
      arena.run(g, tl);
      work.swap(again);
    }
    // (7) sigma of every new trial vector, all instances in one graph replay
    bool anyadd = false;
    for (int b = 0; b < nb; ++b) {
      Inst& s = in[b];
      nv[b] = 0;
      if (!s.active) continue;
      if (s.added == 0) {
        // every correction lay in the subspace already while some residual is still above
        // r_tol: the solver cannot make progress, so the roots are reported unconverged
        s.active = false;
        s.status = FC_ENOCONV;
        continue;
      }
      nv[b] = s.added;
      Rp[b] = s.V.as<z>() + (size_t)s.m * s.dim;
      Sp[b] = s.S.as<z>() + (size_t)s.m * s.dim;
      anyadd = true;
    }
    if (anyadd) sb.run(Rp.data(), Sp.data(), nv.data());
    for (Inst& s : in)
      if (s.active) s.m += s.added;
  }
  int status = FC_OK;
  long off = 0, roff = 0;
  for (int b = 0; b < nb; ++b) {
    Inst& s = in[b];
    if (s.active) { s.status = FC_ENOCONV; s.iters = op.max_iter; }
    for (int r = 0; r < s.k; ++r) omega[off + r] = s.theta_old.empty() ? zero : s.theta_old[r];
    if (Rout) FC_HIP(hipMemcpyAsync(Rout + roff, s.X.p, sizeof(z) * (size_t)s.k * s.dim, hipMemcpyDeviceToDevice,
                                    ctx->stream));
    if (iters) iters[b] = s.iters;
    off += s.k;
    roff += (long)s.k * s.dim;
    if (s.status != FC_OK) status = s.status;
  }
  FC_HIP(hipStreamSynchronize(ctx->stream));
  return status;
}

// Left eigenvectors dual to given right ones (Eq. 19): the lowest roots of the transposed problem
// by the same Davidson, then L <- O^-1 L with the bilinear overlap O = L R^T, so that
// sum_x L_k[x] R_l[x] = delta_kl (no complex conjugation anywhere).  O^-1 rather than a
// per-root scale keeps the result right when roots are degenerate or come out of the two solves
// in a different order.  weight_k = sum_i l^i_k r_{k,i}, the one-hole part of that product.
int left_batch(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* amps, const int* nroots,
               const fc_eom_opts& op, const z* R, z* omega, z* L, z* weight, int* iters) {
  StageTimer st(ctx, "left");
  const int status = davidson_batch(ctx, nb, ints, amps, nroots, op, omega, L, iters, true);
  const z one = make_double2(1, 0), zero = make_double2(0, 0);
  long roff = 0, off = 0;
  for (int b = 0; b < nb; ++b) {
    const long o = ints[b]->o, v = ints[b]->v, dim = o + o * (o - 1) / 2 * v;
    const int k = nroots[b];
    const z* Rb = R + roff;
    z* Lb = L + roff;
    DBuf O(ctx, sizeof(z) * k * k), Oi(ctx, sizeof(z) * k * k), Ln(ctx, sizeof(z) * (size_t)k * dim);
    zgemm(ctx, 'N', 'T', k, k, dim, one, Lb, dim, Rb, dim, zero, O.as<z>(), k);
    std::vector<z> Oh((size_t)k * k), inv((size_t)k * k);
    FC_HIP(hipMemcpyAsync(Oh.data(), O.p, sizeof(z) * k * k, hipMemcpyDeviceToHost, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    // rows of L and R have unit norm, so a large inverse means the two solves found different roots
    double big = 0;
    for (int c = 0; c < k; ++c) {
      std::vector<z> e(k, zero);
      e[c] = one;
      FC_REQUIRE(lin_solve(k, Oh, e), FC_ENUMERIC, "ipeom_left: singular left-right overlap");
      for (int r = 0; r < k; ++r) {
        inv[(size_t)r * k + c] = e[r];
        big = std::max(big, std::hypot(e[r].x, e[r].y));
      }
    }
    FC_REQUIRE(big < 1e6, FC_ENUMERIC, "ipeom_left: left and right vectors belong to different roots");
    // report for right root k the eigenvalue of the left root that overlaps it most (the two
    // solves may order nearly equal real parts differently)
    std::vector<z> wl(omega + off, omega + off + k);
    for (int c = 0; c < k; ++c) {
      int best = c;
      for (int r = 0; r < k; ++r)
        if (std::hypot(Oh[(size_t)r * k + c].x, Oh[(size_t)r * k + c].y) >
            std::hypot(Oh[(size_t)best * k + c].x, Oh[(size_t)best * k + c].y))
          best = r;
      omega[off + c] = wl[best];
    }
    FC_HIP(hipMemcpyAsync(Oi.p, inv.data(), sizeof(z) * k * k, hipMemcpyHostToDevice, ctx->stream));
    zgemm(ctx, 'N', 'N', k, dim, k, one, Oi.as<z>(), k, Lb, dim, zero, Ln.as<z>(), dim);
    FC_HIP(hipMemcpyAsync(Lb, Ln.p, sizeof(z) * (size_t)k * dim, hipMemcpyDeviceToDevice, ctx->stream));
    std::vector<z> lh((size_t)k * o), rh((size_t)k * o);
    FC_HIP(hipMemcpy2DAsync(lh.data(), sizeof(z) * o, Lb, sizeof(z) * dim, sizeof(z) * o, k, hipMemcpyDeviceToHost,
                            ctx->stream));
    FC_HIP(hipMemcpy2DAsync(rh.data(), sizeof(z) * o, Rb, sizeof(z) * dim, sizeof(z) * o, k, hipMemcpyDeviceToHost,
                            ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < k; ++r) {
      z w = zero;
      for (long i = 0; i < o; ++i) {
        const z a = lh[(size_t)r * o + i], c = rh[(size_t)r * o + i];
        w.x += a.x * c.x - a.y * c.y;
        w.y += a.x * c.y + a.y * c.x;
      }
      weight[off + r] = w;
    }
    roff += (long)k * dim;
    off += k;
  }
  return status;
}

}  // namespace fc
