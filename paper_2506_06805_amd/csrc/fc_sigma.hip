// IP-EOM-CCSD sigma products (Eq. 17-18) as a few matrix products per instance, batched over
// instances of uneven size.
//
// With R packed as [r_i (o) | r_ij^a, i < j, a fastest] (row length dim = o + C(o,2) v):
//   sigma_i    = sum_x R[x] B1[x][i]                    F_mi r_m, F_me r_im^e, W_mnie r_mn^e
//   X_e        = sum_{q,f} R[(q, f)] <m_q n_q||ef>      the three-body piece 1/2 <mn||ef> r_mn^f
//   sigma_p^a  = sum_e R[(p, e)] F_ae                   F_ae r_ij^e
//              + sum_q Mp[p][q] R[(q, a)]               1/2 W_mnij r_mn^a and -P(ij) F_mi r_mj^a
//              + sum_{m} r_m (-W_maij) + sum_e X_e t_ij^ae
//              + x[i][j][a] - x[j][i][a],   x[i][(j, a)] = sum_{(m, e)} r_im^e W_maej
// Only the ring product x needs the unpacked, antisymmetric r_im^e.  Every product here is an
// FP64 MFMA GEMM; for all instances together they form two grouped persistent launches.
//
// The left product s = Y H-bar (row vectors l_i, l_b^ij of Eq. 20) applies the transpose of the
// same linear map.  Unpacking and packing are each other's transposes, so the left sequence keeps
// both kernels and transposes the products in between:
//   s_m        = sum_x Y[x] BL1[x][m]                   BL1 = [B1[:o]^T ; B2[:o]^T]
//   Z_e        = sum_{(p, a)} Y[(p, a)] t_ij^ae         (rows o + e of B2, transposed)
//   s_p^e      = sum_a Y[(p, a)] F_ae + sum_q Mp[q][p] Y[(q, e)]
//   s_(q, f)  += sum_i l_i B1[(q, f)][i] + sum_e Z_e <mn||ef>   = [l_i | Z_e] BL2
//              + x[m][n][f] - x[n][m][f],   x[m][(n, f)] = sum_{(j, a)} l_mj^a W_nafj
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fc_sigma.hpp"

namespace fc {
namespace {
constexpr int TPB = 256;
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(65536L, (n + TPB - 1) / TPB)); }
#define GRID_STRIDE(i, n) for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }
__device__ __host__ inline long pair_of(long lo, long hi, long o) { return lo * o - lo * (lo + 1) / 2 + (hi - lo - 1); }

// ------------------------------------------------------------------ operator preparation (once)
__global__ void k_prep_B1(z* B1, const z* Fmi, const z* Fme, const z* Wmnie, const int2* pairs, long o, long v,
                          long no) {
  const long dim = o + no * v;
  GRID_STRIDE(t, dim * o) {
    const long i = t % o, r = t / o;
    z val;
    if (r < o) {
      val = make_double2(-Fmi[r * o + i].x, -Fmi[r * o + i].y);
    } else {
      const long q = r - o, p = q / v, e = q % v;
      const int2 mn = pairs[p];
      const z w = Wmnie[((mn.x * o + mn.y) * o + i) * v + e];
      val = make_double2(-w.x, -w.y);
      if (i == mn.x) { val.x += Fme[mn.y * v + e].x; val.y += Fme[mn.y * v + e].y; }
      if (i == mn.y) { val.x -= Fme[mn.x * v + e].x; val.y -= Fme[mn.x * v + e].y; }
    }
    B1[t] = val;
  }
}
__global__ void k_prep_X(z* X, const z* oovv, const int2* pairs, long o, long v, long no) {
  GRID_STRIDE(t, no * v * v) {
    const long e = t % v, f = (t / v) % v, p = t / (v * v);
    const int2 mn = pairs[p];
    X[t] = oovv[((mn.x * o + mn.y) * v + e) * v + f];
  }
}
__global__ void k_prep_Wt(z* Wt, const z* Wmbej, long o, long v) {
  GRID_STRIDE(t, o * v * o * v) {
    const long a = t % v, j = (t / v) % o, e = (t / (v * o)) % v, m = t / (v * o * v);
    Wt[t] = Wmbej[((m * v + a) * v + e) * o + j];
  }
}
__global__ void k_prep_Mp(z* Mp, const z* Wmnij, const z* F, const int2* pairs, long o, long no) {
  GRID_STRIDE(t, no * no) {
    const long q = t % no, p = t / no;
    const int2 ij = pairs[p], mn = pairs[q];
    const long i = ij.x, j = ij.y, m = mn.x, n = mn.y;
    z val = Wmnij[((m * o + n) * o + i) * o + j];
    if (j == n) { val.x -= F[m * o + i].x; val.y -= F[m * o + i].y; }
    if (j == m) { val.x += F[n * o + i].x; val.y += F[n * o + i].y; }
    if (i == n) { val.x += F[m * o + j].x; val.y += F[m * o + j].y; }
    if (i == m) { val.x -= F[n * o + j].x; val.y -= F[n * o + j].y; }
    Mp[t] = val;
  }
}
__global__ void k_prep_B2(z* B2, const z* Wmbij, const z* t2, const int2* pairs, long o, long v, long no) {
  const long nc = no * v;
  GRID_STRIDE(t, (o + v) * nc) {
    const long c = t % nc, r = t / nc, p = c / v, a = c % v;
    const int2 ij = pairs[p];
    if (r < o) {
      const z w = Wmbij[((r * v + a) * o + ij.x) * o + ij.y];
      B2[t] = make_double2(-w.x, -w.y);
    } else {
      B2[t] = t2[((ij.x * o + ij.y) * v + a) * v + (r - o)];
    }
  }
}
// transposed operators of the left product, gathered from the right ones
__global__ void k_prep_BL1(z* BL1, const z* B1, const z* B2, long o, long nv) {
  GRID_STRIDE(t, (o + nv) * o) {
    const long m = t % o, x = t / o;
    BL1[t] = x < o ? B1[m * o + x] : B2[m * nv + (x - o)];
  }
}
__global__ void k_prep_BL2(z* BL2, const z* B1, const z* Xop, long o, long v, long nv) {
  GRID_STRIDE(t, (o + v) * nv) {
    const long c = t % nv, x = t / nv;
    BL2[t] = x < o ? B1[(o + c) * o + x] : Xop[c * v + (x - o)];
  }
}

// ------------------------------------------------------------------ per-call elementwise kernels
struct SigInst {
  long o, v, no, dim, k;
  const z* R;
  z* S;
  z* r2;    // [k][o][o][v], antisymmetric in the two occupied indices
  z* Y;     // [k][o + v]: r_m, then X_e
  z* x;     // [k][o][o][v] ring product
  z* s2b;   // [k][no][v] pair-mixing product
  const int2* pairs;
  long e0u, e0p;   // first element of this instance in the unpack and pack index spaces
};
struct SigHdr {
  long n, total_u, total_p, pad;
};
constexpr size_t TAB_HDR = 64;

template <long SigInst::*F>
__device__ inline long inst_find(const SigInst* d, long n, long x) {
  long lo = 0, hi = n - 1;
  while (lo < hi) {
    const long mid = (lo + hi + 1) >> 1;
    if (d[mid].*F <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_sig_unpack(const char* __restrict__ tab) {
  const SigHdr* h = reinterpret_cast<const SigHdr*>(tab);
  const SigInst* d = reinterpret_cast<const SigInst*>(tab + TAB_HDR);
  GRID_STRIDE(e, h->total_u) {
    const SigInst& s = d[inst_find<&SigInst::e0u>(d, h->n, e)];
    const long loc = e - s.e0u, o = s.o, v = s.v;
    const long n2 = s.k * o * o * v;
    if (loc < n2) {
      const long a = loc % v, m = (loc / v) % o, i = (loc / (v * o)) % o, kk = loc / (v * o * o);
      z val = make_double2(0.0, 0.0);
      if (i != m) {
        const long lo = i < m ? i : m, hi = i < m ? m : i;
        val = s.R[kk * s.dim + o + pair_of(lo, hi, o) * v + a];
        if (i > m) { val.x = -val.x; val.y = -val.y; }
      }
      s.r2[loc] = val;
    } else {
      const long q = loc - n2, kk = q / o, m = q % o;
      s.Y[kk * (o + v) + m] = s.R[kk * s.dim + m];
    }
  }
}

__global__ void k_sig_pack(const char* __restrict__ tab) {
  const SigHdr* h = reinterpret_cast<const SigHdr*>(tab);
  const SigInst* d = reinterpret_cast<const SigInst*>(tab + TAB_HDR);
  GRID_STRIDE(e, h->total_p) {
    const SigInst& s = d[inst_find<&SigInst::e0p>(d, h->n, e)];
    const long loc = e - s.e0p, o = s.o, v = s.v, nv = s.no * v;
    const long kk = loc / nv, q = loc % nv, p = q / v, a = q % v;
    const int2 ij = s.pairs[p];
    const z xa = s.x[((kk * o + ij.x) * o + ij.y) * v + a];
    const z xb = s.x[((kk * o + ij.y) * o + ij.x) * v + a];
    const z b = s.s2b[loc];
    z* out = s.S + kk * s.dim + o + q;
    z c = *out;
    c.x += b.x + xa.x - xb.x;
    c.y += b.y + xa.y - xb.y;
    *out = c;
  }
}
}  // namespace

static void prep_left_ops(fc_ctx ctx, fc_ints I, SigmaOps& so) {
  StageTimer st(ctx, "sigma_prep");
  const long o = I->o, v = I->v, no = o * (o - 1) / 2, nv = no * v;
  so.BL1 = ZTensor(ctx, {o + nv, o});
  so.BL2 = ZTensor(ctx, {o + v, nv});
  hipLaunchKernelGGL(k_prep_BL1, dim3(nblk((o + nv) * o)), dim3(TPB), 0, ctx->stream, so.BL1.p(), so.B1.p(),
                     so.B2.p(), o, nv);
  if (no)
    hipLaunchKernelGGL(k_prep_BL2, dim3(nblk((o + v) * nv)), dim3(TPB), 0, ctx->stream, so.BL2.p(), so.B1.p(),
                       so.Xop.p(), o, v, nv);
  FC_HIP(hipGetLastError());
  so.left_ready = true;
}

void prep_sigma_ops(fc_ctx ctx, fc_ints I, fc_amps T, bool left) {
  SigmaOps& so = T->so;
  if (so.ready) {
    if (left && !so.left_ready) prep_left_ops(ctx, I, so);
    return;
  }
  if (!T->hb.ready) build_hbar(ctx, I, T);
  StageTimer st(ctx, "sigma_prep");
  const HbarBlocks& H = T->hb;
  const long o = I->o, v = I->v, no = o * (o - 1) / 2, dim = o + no * v;
  std::vector<int2> hp;
  for (int i = 0; i < o; ++i)
    for (int j = i + 1; j < o; ++j) hp.push_back(make_int2(i, j));
  so.pairs = DBuf(ctx, sizeof(int2) * std::max(1L, no));
  if (no) FC_HIP(hipMemcpyAsync(so.pairs.p, hp.data(), sizeof(int2) * no, hipMemcpyHostToDevice, ctx->stream));
  const int2* pr = so.pairs.as<int2>();
  so.B1 = ZTensor(ctx, {dim, o});
  so.Xop = ZTensor(ctx, {no * v, v});
  so.Wt = ZTensor(ctx, {o * v, o * v});
  so.Mp = ZTensor(ctx, {no, no});
  so.B2 = ZTensor(ctx, {o + v, no * v});
  hipLaunchKernelGGL(k_prep_B1, dim3(nblk(dim * o)), dim3(TPB), 0, ctx->stream, so.B1.p(), H.Fmi.p(), H.Fme.p(),
                     H.Wmnie.p(), pr, o, v, no);
  if (no) {
    hipLaunchKernelGGL(k_prep_X, dim3(nblk(no * v * v)), dim3(TPB), 0, ctx->stream, so.Xop.p(), I->oovv.p(), pr, o,
                       v, no);
    hipLaunchKernelGGL(k_prep_Mp, dim3(nblk(no * no)), dim3(TPB), 0, ctx->stream, so.Mp.p(), H.Wmnij.p(),
                       H.Fmi.p(), pr, o, no);
    hipLaunchKernelGGL(k_prep_B2, dim3(nblk((o + v) * no * v)), dim3(TPB), 0, ctx->stream, so.B2.p(), H.Wmbij.p(),
                       T->t2.p(), pr, o, v, no);
  }
  hipLaunchKernelGGL(k_prep_Wt, dim3(nblk(o * v * o * v)), dim3(TPB), 0, ctx->stream, so.Wt.p(), H.Wmbej.p(), o, v);
  FC_HIP(hipGetLastError());
  so.ready = true;
  if (left) prep_left_ops(ctx, I, so);
}

// ------------------------------------------------------------------------------- SigmaBatch
SigmaBatch::SigmaBatch(fc_ctx ctx, int nb, const fc_ints* I, const fc_amps* T, const long* kmax, bool graph,
                       bool left)
    : ctx_(ctx), nb_(nb), I_(I, I + nb), T_(T, T + nb), kmax_(kmax, kmax + nb), graph_(graph), left_(left) {
  FC_REQUIRE(nb >= 1, FC_EARG, "sigma: no instances");
  for (int b = 0; b < nb; ++b) {
    FC_REQUIRE(I[b] && T[b] && T[b]->ints == I[b], FC_EARG, "sigma: bad handles");
    FC_REQUIRE(kmax[b] >= 0, FC_EARG, "sigma: negative vector count");
    prep_sigma_ops(ctx, I[b], T[b], left);
    const long o = I[b]->o, v = I[b]->v, no = o * (o - 1) / 2, k = std::max(1L, kmax[b]);
    r2_.emplace_back(ctx, std::vector<long>{k, o, o, v});
    x_.emplace_back(ctx, std::vector<long>{k, o, o, v});
    Y_.emplace_back(ctx, std::vector<long>{k, o + v});
    s2b_.emplace_back(ctx, std::vector<long>{k, std::max(1L, no), v});
  }
  // plan sizes do not depend on the tiling: count them once with the largest vector counts
  std::vector<GroupGemm> g1, g2;
  std::vector<const z*> R(nb, nullptr);
  std::vector<z*> S(nb, nullptr);
  lists(R.data(), S.data(), kmax_.data(), g1, g2, nullptr, &maxu_, &maxp_);
  cap_g1_ = align256(group_encode(g1, tl1_, nullptr, 0, nullptr, 0).plan_bytes);
  cap_g2_ = align256(group_encode(g2, tl2_, nullptr, 0, nullptr, 0).plan_bytes);
  const size_t tab = align256(TAB_HDR + sizeof(SigInst) * nb);
  off_g1_ = tab;
  off_g2_ = off_g1_ + cap_g1_;
  cap_ = off_g2_ + cap_g2_;
  dev_ = DBuf(ctx, cap_);
  FC_HIP(hipHostMalloc((void**)&host_, cap_, hipHostMallocDefault));
  FC_HIP(hipEventCreateWithFlags(&copied_, hipEventDisableTiming));
}

SigmaBatch::~SigmaBatch() {
  if (exec_) (void)hipGraphExecDestroy(exec_);
  if (g_) (void)hipGraphDestroy(g_);
  if (copied_) {
    (void)hipEventSynchronize(copied_);
    (void)hipEventDestroy(copied_);
  }
  if (host_) (void)hipHostFree(host_);
}

void SigmaBatch::lists(const z* const* R, z* const* S, const long* nvec, std::vector<GroupGemm>& g1,
                       std::vector<GroupGemm>& g2, std::vector<char>* tab, long* nu, long* np) const {
  const z one = make_double2(1, 0);
  long eu = 0, ep = 0;
  g1.clear();
  g2.clear();
  if (tab) tab->assign(TAB_HDR + sizeof(SigInst) * nb_, 0);
  for (int b = 0; b < nb_; ++b) {
    const long k = nvec[b];
    FC_REQUIRE(k >= 0 && k <= kmax_[b], FC_EARG, "sigma: more vectors than the batch was built for");
    const fc_ints I = I_[b];
    const SigmaOps& so = T_[b]->so;
    const long o = I->o, v = I->v, no = o * (o - 1) / 2, dim = o + no * v, nv = no * v, ov = o * v;
    SigInst s{};
    s.o = o; s.v = v; s.no = no; s.dim = dim; s.k = k;
    s.R = R[b]; s.S = S[b];
    s.r2 = r2_[b].p(); s.Y = Y_[b].p(); s.x = x_[b].p(); s.s2b = s2b_[b].p();
    s.pairs = so.pairs.as<int2>();
    s.e0u = eu; s.e0p = ep;
    if (tab) std::memcpy(tab->data() + TAB_HDR + sizeof(SigInst) * b, &s, sizeof(s));
    if (k == 0) continue;
    eu += k * o * o * v + k * o;
    ep += k * nv;
    GroupGemm p;
    if (left_) {
      const z* R2 = R[b] ? R[b] + o : nullptr;
      // s_m = Y BL1
      p = GroupGemm{}; p.M = k; p.N = o; p.K = dim;
      p.A = R[b]; p.lda = dim; p.B = so.BL1.p(); p.ldb = o; p.C = S[b]; p.ldc = dim;
      g1.push_back(p);
      // ring: x[(k, m)][(n, f)] = y2[(k, m)][(j, a)] Wt[(n, f)][(j, a)]
      p = GroupGemm{}; p.opB = 'T'; p.M = k * o; p.N = ov; p.K = ov;
      p.A = s.r2; p.lda = ov; p.B = so.Wt.p(); p.ldb = ov; p.C = s.x; p.ldc = ov;
      g1.push_back(p);
      if (no) {
        // Z_e into Y[:, o:]
        p = GroupGemm{}; p.opB = 'T'; p.M = k; p.N = v; p.K = nv;
        p.A = R2; p.lda = dim; p.B = so.B2.p() + o * nv; p.ldb = nv;
        p.C = s.Y + o; p.ldc = o + v;
        g1.push_back(p);
        // l_ij^a F_ae straight into the packed output, one batch entry per vector
        p = GroupGemm{}; p.M = no; p.N = v; p.K = v; p.batch = k;
        p.A = R2; p.lda = v; p.sA = dim; p.B = T_[b]->hb.Fae.p(); p.ldb = v;
        p.C = S[b] ? S[b] + o : nullptr; p.ldc = v; p.sC = dim;
        g1.push_back(p);
        // pair mixing, transposed, into s2b
        p = GroupGemm{}; p.opA = 'T'; p.M = no; p.N = v; p.K = no; p.batch = k;
        p.A = so.Mp.p(); p.lda = no; p.sA = 0;
        p.B = R2; p.ldb = v; p.sB = dim;
        p.C = s.s2b; p.ldc = v; p.sC = nv;
        g1.push_back(p);
        // [l_i | Z_e] BL2 added to the packed output
        p = GroupGemm{}; p.M = k; p.N = nv; p.K = o + v;
        p.A = s.Y; p.lda = o + v; p.B = so.BL2.p(); p.ldb = nv;
        p.beta = one; p.C = S[b] ? S[b] + o : nullptr; p.ldc = dim;
        g2.push_back(p);
      }
      continue;
    }
    // sigma_i = R B1
    p = GroupGemm{}; p.M = k; p.N = o; p.K = dim;
    p.A = R[b]; p.lda = dim; p.B = so.B1.p(); p.ldb = o; p.C = S[b]; p.ldc = dim;
    g1.push_back(p);
    // ring: x[(k, i)][(j, a)] = r2[(k, i)][(m, e)] Wt[(m, e)][(j, a)]
    p = GroupGemm{}; p.M = k * o; p.N = ov; p.K = ov;
    p.A = s.r2; p.lda = ov; p.B = so.Wt.p(); p.ldb = ov; p.C = s.x; p.ldc = ov;
    g1.push_back(p);
    if (no) {
      // X_e into Y[:, o:]
      p = GroupGemm{}; p.M = k; p.N = v; p.K = nv;
      p.A = R[b] ? R[b] + o : nullptr; p.lda = dim; p.B = so.Xop.p(); p.ldb = v;
      p.C = s.Y + o; p.ldc = o + v;
      g1.push_back(p);
      // F_ae r_ij^e straight into the packed output, one batch entry per vector
      p = GroupGemm{}; p.opB = 'T'; p.M = no; p.N = v; p.K = v; p.batch = k;
      p.A = R[b] ? R[b] + o : nullptr; p.lda = v; p.sA = dim;
      p.B = T_[b]->hb.Fae.p(); p.ldb = v;
      p.C = S[b] ? S[b] + o : nullptr; p.ldc = v; p.sC = dim;
      g1.push_back(p);
      // pair mixing into s2b
      p = GroupGemm{}; p.M = no; p.N = v; p.K = no; p.batch = k;
      p.A = so.Mp.p(); p.lda = no; p.sA = 0;
      p.B = R[b] ? R[b] + o : nullptr; p.ldb = v; p.sB = dim;
      p.C = s.s2b; p.ldc = v; p.sC = nv;
      g1.push_back(p);
      // [r_m | X_e] B2 added to the packed output
      p = GroupGemm{}; p.M = k; p.N = nv; p.K = o + v;
      p.A = s.Y; p.lda = o + v; p.B = so.B2.p(); p.ldb = nv;
      p.beta = one; p.C = S[b] ? S[b] + o : nullptr; p.ldc = dim;
      g2.push_back(p);
    }
  }
  if (tab) {
    SigHdr h{nb_, eu, ep, 0};
    std::memcpy(tab->data(), &h, sizeof(h));
  }
  if (nu) *nu = eu;
  if (np) *np = ep;
}

void SigmaBatch::configure(const GroupTiling& t1, const GroupTiling& t2) {
  tl1_ = t1;
  tl2_ = t2;
  std::vector<GroupGemm> g1, g2;
  std::vector<const z*> R(nb_, nullptr);
  std::vector<z*> S(nb_, nullptr);
  lists(R.data(), S.data(), kmax_.data(), g1, g2, nullptr, nullptr, nullptr);
  const GroupCounts c1 = group_encode(g1, tl1_, nullptr, 0, nullptr, 0);
  const GroupCounts c2 = group_encode(g2, tl2_, nullptr, 0, nullptr, 0);
  maxt1_ = c1.tiles; maxe1_ = c1.elems; wcap1_ = c1.work;
  maxt2_ = c2.tiles; maxe2_ = c2.elems; wcap2_ = c2.work;
  work1_ = DBuf(ctx_, sizeof(z) * wcap1_);
  work2_ = DBuf(ctx_, sizeof(z) * wcap2_);
  if (exec_) { (void)hipGraphExecDestroy(exec_); exec_ = nullptr; }
  if (g_) { (void)hipGraphDestroy(g_); g_ = nullptr; }
  configured_ = true;
}

void SigmaBatch::upload(const z* const* R, z* const* S, const long* nvec) {
  std::vector<GroupGemm> g1, g2;
  std::vector<char> tab;
  lists(R, S, nvec, g1, g2, &tab, nullptr, nullptr);
  // the previous upload must have left the pinned buffer before it is rewritten
  if (copy_pending_) FC_HIP(hipEventSynchronize(copied_));
  std::memcpy(host_, tab.data(), tab.size());
  group_encode(g1, tl1_, host_ + off_g1_, cap_g1_, work1_.as<z>(), wcap1_);
  group_encode(g2, tl2_, host_ + off_g2_, cap_g2_, work2_.as<z>(), wcap2_);
  FC_HIP(hipMemcpyAsync(dev_.p, host_, cap_, hipMemcpyHostToDevice, ctx_->stream));
  FC_HIP(hipEventRecord(copied_, ctx_->stream));
  copy_pending_ = true;
}

void SigmaBatch::launch_all() {
  const char* d = dev_.as<char>();
  k_sig_unpack<<<nblk(maxu_), TPB, 0, ctx_->stream>>>(d);
  FC_HIP(hipGetLastError());
  group_launch(ctx_, tl1_.cfg, d + off_g1_, maxt1_, maxe1_);
  group_launch(ctx_, tl2_.cfg, d + off_g2_, maxt2_, maxe2_);
  k_sig_pack<<<nblk(maxp_), TPB, 0, ctx_->stream>>>(d);
  FC_HIP(hipGetLastError());
}

// Times candidate tilings of the first grouped launch on this call's input and keeps the fastest.
void SigmaBatch::tune(const z* const* R, z* const* S, const long* nvec) {
  double flops = 0;
  for (int b = 0; b < nb_; ++b) {
    const double o = I_[b]->o, v = I_[b]->v;
    flops += 8.0 * nvec[b] * o * o * o * v * v;
  }
  char key[64];
  snprintf(key, sizeof(key), "sigma_%snb%d_f%d", left_ ? "left_" : "", nb_,
           (int)std::ceil(std::log2(std::max(1.0, flops))));
  auto it = ctx_->tune.find(key);
  if (it != ctx_->tune.end()) {
    const int c = it->second.first;
    configure(GroupTiling{c >> 5, 1L << (c & 31)}, GroupTiling{c >> 5, 512});
    return;
  }
  hipEvent_t e0, e1;
  FC_HIP(hipEventCreate(&e0));
  FC_HIP(hipEventCreate(&e1));
  float best = 1e30f;
  int bestc = (0 << 5) | 9;
  for (int cfg = 0; cfg < 3; ++cfg)
    for (int lg = 8; lg <= 11; ++lg) {
      configure(GroupTiling{cfg, 1L << lg}, GroupTiling{cfg, 512});
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        upload(R, S, nvec);
        FC_HIP(hipEventRecord(e0, ctx_->stream));
        launch_all();
        FC_HIP(hipEventRecord(e1, ctx_->stream));
        FC_HIP(hipEventSynchronize(e1));
        FC_HIP(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best) { best = ms; bestc = (cfg << 5) | lg; }
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx_->tune[key] = {bestc, best};
  configure(GroupTiling{bestc >> 5, 1L << (bestc & 31)}, GroupTiling{bestc >> 5, 512});
}

void SigmaBatch::run(const z* const* R, z* const* S, const long* nvec) {
  StageTimer st(ctx_, "sigma");
  if (!configured_) {
    if (ctx_->autotune) {
      tune(R, S, nvec);
    } else {
      // grouped tile configuration of both launches: FNSCC_SIGMA_CFG (0, 1, 2; a measurement
      // switch), else by size
      static const int env = [] {
        const char* e = getenv("FNSCC_SIGMA_CFG");
        const int c = e ? atoi(e) : -1;
        return c >= 0 && c <= 2 ? c : -1;
      }();
      // default: the direct-to-LDS three-product tile once the ring product k o x o v x o v has at
      // least three 128-row tiles (measured at o = 24, v = 160: k = 16 1.37 -> 1.31 ms, k = 32
      // 2.37 -> 2.07 ms per sigma; k = 8 0.83 -> 0.93 ms, so smaller blocks keep the 64 x 64 tile)
      long rows = 0;
      for (int b = 0; b < nb_; ++b) rows = std::max(rows, kmax_[b] * I_[b]->o);
      const int cfg = env >= 0 ? env : rows >= 384 ? 2 : 0;
      configure(GroupTiling{cfg, 512}, GroupTiling{cfg, 512});
    }
  }
  upload(R, S, nvec);
  if (!graph_) {
    launch_all();
    return;
  }
  if (!exec_) {
    // capture on a private stream: the context stream may be the legacy default stream
    hipStream_t cs;
    FC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipStream_t saved = ctx_->stream;
    ctx_->stream = cs;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      try {
        launch_all();
      } catch (...) {
        hipGraph_t junk = nullptr;
        (void)hipStreamEndCapture(cs, &junk);
        if (junk) (void)hipGraphDestroy(junk);
        ctx_->stream = saved;
        (void)hipStreamDestroy(cs);
        throw;
      }
      e = hipStreamEndCapture(cs, &g_);
    }
    ctx_->stream = saved;
    (void)hipStreamDestroy(cs);
    FC_HIP(e);
    FC_HIP(hipGraphInstantiate(&exec_, g_, nullptr, nullptr, 0));
  }
  FC_HIP(hipGraphLaunch(exec_, ctx_->stream));
}

}  // namespace fc
