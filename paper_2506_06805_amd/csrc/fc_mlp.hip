// Learned preconditioned T2 update: a 4 -> 64 -> 64 -> 2 tanh network that maps per-amplitude
// features to a complex gain g, applied as t_ij^ab <- t_ij^ab + (Omega_ij^ab / D_ij^ab)(1 + g).
// Omega = 0 gives a zero step, so the CCSD fixed point is unchanged; convergence is still judged
// on the plain FP64 residual, and the driver falls back to Jacobi + DIIS when the residual stalls.
//
// Features of amplitude (i,j,a,b): with D = e_i + e_j - e_a - e_b and dF = F_aa + F_bb - F_ii - F_jj
// (diagonals of the intermediates that multiply t_ij^ab in the residual), u = dF / D, and the
// ratio rho = Omega_k / Omega_{k-1} of the current and previous residual of that amplitude
// (0 at the first step, magnitude clipped to 1.5),
//   x = (Re u, Im u, Re rho, Im rho).
// The exact diagonal (Newton) step corresponds to g = u / (1 - u) and a geometric error decay with
// ratio rho to g = rho / (1 - rho) (Aitken); the network is trained on solver trajectories to
// reproduce the jump to the converged amplitudes.
//
// Training (FP32 master weights, Adam) runs as: per-sample forward with weights in LDS, per-sample
// loss gradient and backward, weight gradients as fixed-order sums over the minibatch (one row per
// workgroup, deterministic), Adam.  Inference uses the weights rounded to BF16 and accumulates in
// FP32.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fc_state.hpp"

struct fc_mlp_s {
  fc_ctx ctx = nullptr;
  int nin = 4, nh = 64, nout = 2;
  long np = 0;
  fc::DBuf params, grads, m, v, pbf;  // FP32 master, gradient, Adam moments, BF16-rounded copy (as FP32)
  long step = 0;
};

namespace fc {
namespace {
constexpr int NIN = 4, NH = 64, NOUT = 2;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr long NP = NH * NIN + NH + NH * NH + NH + NOUT * NH + NOUT;
constexpr int TPB = 256;
#define GRID_STRIDE(i, n) for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)
// parameter offsets
constexpr long OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
               OB3 = OW3 + NOUT * NH;

__device__ inline void features(double D, double fr, double fi, const z* rnow, const z* rprev, long idx, float* x) {
  const double ur = fr / D, ui = fi / D;
  x[0] = (float)ur;
  x[1] = (float)ui;
  double pr = 0.0, pi = 0.0;
  if (rprev) {
    const z a = rnow[idx], b = rprev[idx];
    const double den = b.x * b.x + b.y * b.y;
    if (den > 0.0) {
      pr = (a.x * b.x + a.y * b.y) / den;
      pi = (a.y * b.x - a.x * b.y) / den;
      const double m = sqrt(pr * pr + pi * pi);
      if (m > 1.5) { pr *= 1.5 / m; pi *= 1.5 / m; }
    }
  }
  x[2] = (float)pr;
  x[3] = (float)pi;
}

// forward of one sample with weights in LDS; h1, h2 optional outputs
__device__ inline void mlp_forward(const float* P, const float* x, float* h1, float* h2, float* y) {
  for (int p = 0; p < NH; ++p) {
    float s = P[OB1 + p];
#pragma unroll
    for (int q = 0; q < NIN; ++q) s += P[OW1 + p * NIN + q] * x[q];
    h1[p] = tanhf(s);
  }
  for (int p = 0; p < NH; ++p) {
    float s = P[OB2 + p];
#pragma unroll 16
    for (int q = 0; q < NH; ++q) s += P[OW2 + p * NH + q] * h1[q];
    h2[p] = tanhf(s);
  }
  for (int p = 0; p < NOUT; ++p) {
    float s = P[OB3 + p];
#pragma unroll 16
    for (int q = 0; q < NH; ++q) s += P[OW3 + p * NH + q] * h2[q];
    y[p] = s;
  }
}

__global__ __launch_bounds__(TPB) void k_forward(const float* __restrict__ params, const float* __restrict__ X, long B,
                                                 float* __restrict__ Y) {
  __shared__ float P[NP];
  for (long k = threadIdx.x; k < NP; k += blockDim.x) P[k] = params[k];
  __syncthreads();
  GRID_STRIDE(s, B) {
    float h1[NH], h2[NH], y[NOUT];
    mlp_forward(P, X + s * NIN, h1, h2, y);
    Y[s * NOUT] = y[0];
    Y[s * NOUT + 1] = y[1];
  }
}

// forward + loss gradient + backward per sample: writes H1, H2, dH1, dH2, dY and per-sample loss
__global__ __launch_bounds__(TPB) void k_train_sample(const float* __restrict__ params, const float* __restrict__ X,
                                                      const float* __restrict__ q, const float* __restrict__ r, long B,
                                                      float inv_w, float* __restrict__ H1, float* __restrict__ H2,
                                                      float* __restrict__ dH1, float* __restrict__ dH2,
                                                      float* __restrict__ dY, float* __restrict__ lossv) {
  __shared__ float P[NP];
  for (long k = threadIdx.x; k < NP; k += blockDim.x) P[k] = params[k];
  __syncthreads();
  GRID_STRIDE(s, B) {
    float h1[NH], h2[NH], y[NOUT];
    mlp_forward(P, X + s * NIN, h1, h2, y);
    // e = r - q g ; loss = |e|^2 / w ; dL/dRe g = -2 Re(conj(e) q) / w ; dL/dIm g = 2 Im(conj(e) q) / w
    const float qr = q[2 * s], qi = q[2 * s + 1];
    const float er = r[2 * s] - (qr * y[0] - qi * y[1]), ei = r[2 * s + 1] - (qr * y[1] + qi * y[0]);
    lossv[s] = (er * er + ei * ei) * inv_w;
    const float cr = er * qr + ei * qi, ci = er * qi - ei * qr;   // conj(e) q
    const float dy0 = -2.f * cr * inv_w, dy1 = 2.f * ci * inv_w;
    dY[2 * s] = dy0;
    dY[2 * s + 1] = dy1;
    float d2[NH];
    for (int p = 0; p < NH; ++p) {
      float g = P[OW3 + p] * dy0 + P[OW3 + NH + p] * dy1;
      d2[p] = g * (1.f - h2[p] * h2[p]);
      H2[s * NH + p] = h2[p];
      dH2[s * NH + p] = d2[p];
    }
    for (int p = 0; p < NH; ++p) {
      float g = 0.f;
#pragma unroll 16
      for (int k = 0; k < NH; ++k) g += P[OW2 + k * NH + p] * d2[k];
      H1[s * NH + p] = h1[p];
      dH1[s * NH + p] = g * (1.f - h1[p] * h1[p]);
    }
  }
}

// grad[row r of W][col c] = sum_s dOut[s][r] In[s][c]; bias row sums.  One workgroup per weight row,
// thread c accumulates over the minibatch in sample order (deterministic).
__global__ void k_weight_grad(const float* __restrict__ dOut, int nout, const float* __restrict__ In, int nin_, long B,
                              float* __restrict__ gW, float* __restrict__ gb) {
  const int rrow = blockIdx.x, c = threadIdx.x;
  if (c < nin_) {
    float acc = 0.f;
    for (long s = 0; s < B; ++s) acc += dOut[s * nout + rrow] * In[s * nin_ + c];
    gW[rrow * nin_ + c] = acc;
  }
  if (c == 0) {
    float acc = 0.f;
    for (long s = 0; s < B; ++s) acc += dOut[s * nout + rrow];
    gb[rrow] = acc;
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       float* __restrict__ pbf, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  GRID_STRIDE(k, n) {
    float gk = g[k];
    m[k] = b1 * m[k] + (1.f - b1) * gk;
    v[k] = b2 * v[k] + (1.f - b2) * gk * gk;
    p[k] -= lr * (m[k] / c1) / (sqrtf(v[k] / c2) + eps);
    pbf[k] = (float)(__bf16)p[k];
  }
}
__global__ void k_round_bf16(const float* __restrict__ p, float* __restrict__ pbf, long n) {
  GRID_STRIDE(k, n) { pbf[k] = (float)(__bf16)p[k]; }
}

__device__ inline unsigned long long mix64(unsigned long long x) {  // splitmix64 finaliser
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// r / (d - df), the solver's dressed Jacobi step (the residual's one-particle diagonals df taken
// off the orbital-energy difference d; the bare r / d where the dressing would bring the
// denominator below half the bare one's size)
__device__ inline z dressed_step(z r, double d, z df) {
  const double dr = d - df.x, di = -df.y;
  const double n2 = dr * dr + di * di;
  if (!(n2 >= 0.25 * d * d)) return make_double2(r.x / d, r.y / d);
  return make_double2((r.x * dr + r.y * di) / n2, (r.y * dr - r.x * di) / n2);
}

// samples: unique amplitude (i<j, a<b) chosen by a counter-based hash of (seed, k)
__global__ void k_samples(const z* __restrict__ t2, const z* __restrict__ r2, const z* __restrict__ r2prev,
                          const z* __restrict__ t2s,
                          const double* __restrict__ eps, const z* __restrict__ fd, long o, long v, long nsamp,
                          unsigned long long seed, float* __restrict__ X, float* __restrict__ q, float* __restrict__ r) {
  GRID_STRIDE(k, nsamp) {
    unsigned long long h1 = mix64(seed * 0x100000001b3ull + (unsigned long long)k);
    unsigned long long h2 = mix64(h1);
    long i = (long)(h1 % (unsigned long long)o), j = (long)((h1 >> 32) % (unsigned long long)(o - 1));
    if (j >= i) ++j;
    long a = (long)(h2 % (unsigned long long)v), b = (long)((h2 >> 32) % (unsigned long long)(v - 1));
    if (b >= a) ++b;
    const long idx = ((i * o + j) * v + a) * v + b;
    const double D = eps[i] + eps[j] - eps[o + a] - eps[o + b];
    const double fr = fd[o + a].x + fd[o + b].x - fd[i].x - fd[j].x;
    const double fi = fd[o + a].y + fd[o + b].y - fd[i].y - fd[j].y;
    features(D, fr, fi, r2, r2prev, idx, X + k * NIN);
    const z qd = dressed_step(r2[idx], D, make_double2(fr, fi));
    const double qr = qd.x, qi = qd.y;
    q[2 * k] = (float)qr;
    q[2 * k + 1] = (float)qi;
    r[2 * k] = (float)(t2s[idx].x - t2[idx].x - qr);
    r[2 * k + 1] = (float)(t2s[idx].y - t2[idx].y - qi);
  }
}

// tanh through one exponential: 1 - 2 / (exp(2x) + 1), exact limits +-1 for large |x|
__device__ inline float tanh_exp(float x) { return 1.0f - 2.0f / (__expf(2.0f * x) + 1.0f); }

// (i, j) of pair index p among the n(n-1)/2 pairs i < j in lexicographic order
__device__ inline void pair_of_index(long p, long n, long& i, long& j) {
  const double t = (double)(n * (n - 1) / 2 - 1 - p);
  long k = (long)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);   // t = k(k+1)/2 + r, 0 <= r <= k
  while ((k + 1) * (k + 2) / 2 <= (long)t) ++k;
  while (k * (k + 1) / 2 > (long)t) --k;
  i = n - 2 - k;
  j = i + 1 + (p - (i * n - i * (i + 1) / 2));
}

// t2_new = t2 + q (1 + g(x)), q the dressed Jacobi step, for every unique amplitude (i < j, a < b),
// written to its four antisymmetric images, with the BF16-rounded weights; the 64 x 64 hidden
// layer runs on the BF16 matrix cores with FP32 accumulation (h1 rounded to BF16), the rest in
// FP32.  Each wave takes 64
// unique amplitudes (one per lane), forms the features and the first hidden layer per lane,
// stages h1 as a 64 x 64 block in LDS, and multiplies it by W2^T with v_mfma_f32_16x16x32_bf16
// (4 x 4 output blocks, K = 64 in 2 steps; W2 fragments stay in registers for the whole kernel).
// Lane layout of the 16x16x32 product: A fragment A[l % 16][8 (l / 16) + 0..7], B fragment
// B[8 (l / 16) + 0..7][l % 16], accumulator r D[4 (l / 16) + r][l % 16].  tanh and the output layer act on the accumulators in place; the two output sums of a
// sample are reduced over the 16 lanes that hold its columns and handed back to the sample's
// lane through LDS.  (Evaluating the whole network per lane with weights in LDS took 3.9x as
// long: 2.5 against 0.64 ms per step at o = 24, v = 160.)
constexpr int LW = 4;              // waves per workgroup
constexpr int HS = NH + 1;         // LDS row of one sample's h1 (padded)
__global__ __launch_bounds__(64 * LW) void k_learned_t2_mfma(const float* __restrict__ pbf, const z* __restrict__ t2,
                                                            const z* __restrict__ r2, const z* __restrict__ r2prev,
                                                            const double* __restrict__ eps,
                                                            const z* __restrict__ fd, long o, long v, z* __restrict__ out) {
  __shared__ float Ps[NH * NIN + NH];        // W1, b1
  __shared__ float Hs[LW][64 * HS];          // per wave: h1 of its 64 samples, then (y0, y1)
  for (int k = threadIdx.x; k < NH * NIN + NH; k += blockDim.x) Ps[k] = pbf[OW1 + k];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, ln = lane & 15, lk = lane >> 4;
  // W2 fragments: B[k][n] of step kk and column block pb is W2[pb 16 + n][kk 32 + k], k = 8 lk + 0..7
  bf16x8 w2f[4][2];
#pragma unroll
  for (int pb = 0; pb < 4; ++pb)
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int e = 0; e < 8; ++e) w2f[pb][kk][e] = (__bf16)pbf[OW2 + (pb * 16 + ln) * NH + kk * 32 + 8 * lk + e];
  float b2c[4], w30[4], w31[4];
#pragma unroll
  for (int pb = 0; pb < 4; ++pb) {
    b2c[pb] = pbf[OB2 + pb * 16 + ln];
    w30[pb] = pbf[OW3 + pb * 16 + ln];
    w31[pb] = pbf[OW3 + NH + pb * 16 + ln];
  }
  const float b30 = pbf[OB3], b31 = pbf[OB3 + 1];
  __syncthreads();
  float* H = Hs[w];
  const long no = o * (o - 1) / 2, nv = v * (v - 1) / 2, nu = no * nv;
  const long groups = (nu + 63) / 64, stride = (long)gridDim.x * LW;
  for (long g0 = (long)blockIdx.x * LW; g0 < groups; g0 += stride) {   // uniform over the workgroup
    const long u = (g0 + w) * 64 + lane;
    const bool valid = u < nu;
    long i = 0, j = 1, a = 0, b = 1, x = 0;
    double D = 1.0;
    z df = make_double2(0.0, 0.0);
    float xin[NIN] = {0.f, 0.f, 0.f, 0.f};
    if (valid) {
      pair_of_index(u / nv, o, i, j);
      pair_of_index(u % nv, v, a, b);
      x = ((i * o + j) * v + a) * v + b;
      D = eps[i] + eps[j] - eps[o + a] - eps[o + b];
      const double fr = fd[o + a].x + fd[o + b].x - fd[i].x - fd[j].x;
      const double fi = fd[o + a].y + fd[o + b].y - fd[i].y - fd[j].y;
      df = make_double2(fr, fi);
      features(D, fr, fi, r2, r2prev, x, xin);
    }
#pragma unroll
    for (int p = 0; p < NH; p += 4) {
      float hv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float s = Ps[NH * NIN + p + e];
#pragma unroll
        for (int q = 0; q < NIN; ++q) s += Ps[(p + e) * NIN + q] * xin[q];
        hv[e] = tanh_exp(s);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) H[lane * HS + p + e] = hv[e];
    }
    __syncthreads();
    // h2 = tanh(h1 W2^T + b2): block (sb, pb) holds samples sb 16 + 4 lk + r, columns pb 16 + ln
    float y0[4][4], y1[4][4];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      f32x4 acc[4];
#pragma unroll
      for (int pb = 0; pb < 4; ++pb) acc[pb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        bf16x8 av;
#pragma unroll
        for (int e = 0; e < 8; ++e) av[e] = (__bf16)H[(sb * 16 + ln) * HS + kk * 32 + 8 * lk + e];
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) acc[pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, w2f[pb][kk], acc[pb], 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int pb = 0; pb < 4; ++pb) {
          const float h = tanh_exp(acc[pb][r] + b2c[pb]);
          s0 += w30[pb] * h;
          s1 += w31[pb] * h;
        }
        y0[sb][r] = s0;
        y1[sb][r] = s1;
      }
    }
    // sums over the 16 column lanes of each sample (lanes with the same lk)
#pragma unroll
    for (int m = 1; m < 16; m <<= 1)
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          y0[sb][r] += __shfl_xor(y0[sb][r], m, 16);
          y1[sb][r] += __shfl_xor(y1[sb][r], m, 16);
        }
    __syncthreads();   // every lane has read its h1 rows
    if (ln == 0) {
#pragma unroll
      for (int sb = 0; sb < 4; ++sb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int smp = sb * 16 + 4 * lk + r;
          H[2 * smp] = y0[sb][r];
          H[2 * smp + 1] = y1[sb][r];
        }
    }
    __syncthreads();
    if (valid) {
      const float g0 = H[2 * lane] + b30, g1 = H[2 * lane + 1] + b31;
      const z qd = dressed_step(r2[x], D, df);
      const double qr = qd.x, qi = qd.y;
      const double gr = 1.0 + (double)g0, gi = (double)g1;
      const z n = make_double2(t2[x].x + qr * gr - qi * gi, t2[x].y + qr * gi + qi * gr);
      const z mneg = make_double2(-n.x, -n.y);
      out[x] = n;
      out[((j * o + i) * v + a) * v + b] = mneg;
      out[((i * o + j) * v + b) * v + a] = mneg;
      out[((j * o + i) * v + b) * v + a] = n;
    }
    __syncthreads();   // the (y0, y1) slots are h1 rows of the next group
  }
}

// zeros where i == j or a == b (never visited by k_learned_t2_mfma)
__global__ void k_zero_diagonals(z* out, long o, long v) {
  GRID_STRIDE(t, o * v * v + o * o * v) {
    long x;
    if (t < o * v * v) {
      const long b = t % v, a = (t / v) % v, i = t / (v * v);
      x = ((i * o + i) * v + a) * v + b;
    } else {
      const long s = t - o * v * v, a = s % v, j = (s / v) % o, i = s / (v * o);
      x = ((i * o + j) * v + a) * v + a;
    }
    out[x] = make_double2(0.0, 0.0);
  }
}
__global__ void k_jacobi_t1(const z* t, const z* r, z* out, const double* eps, const z* fd, long o, long v) {
  GRID_STRIDE(x, o * v) {
    const long a = x % v, i = x / v;
    const z q = dressed_step(r[x], eps[i] - eps[o + a], make_double2(fd[o + a].x - fd[i].x, fd[o + a].y - fd[i].y));
    out[x] = make_double2(t[x].x + q.x, t[x].y + q.y);
  }
}
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(1048576L, (n + TPB - 1) / TPB)); }
}  // namespace

static void check_mlp(fc_mlp m) {
  FC_REQUIRE(m && m->nin == NIN && m->nh == NH && m->nout == NOUT, FC_EARG, "bad network handle");
}

int learned_step(fc_ctx ctx, fc_ints I, const void* mlpv, const z* t1, const z* t2, const z* r1, const z* r2,
                 const z* r2prev, const z* fd, z* o1, z* o2) {
  fc_mlp m = (fc_mlp)mlpv;
  check_mlp(m);
  const long o = I->o, v = I->v;
  k_jacobi_t1<<<nblk(o * v), TPB, 0, ctx->stream>>>(t1, r1, o1, I->eps_d.as<double>(), fd, o, v);
  k_zero_diagonals<<<nblk(o * v * v + o * o * v), TPB, 0, ctx->stream>>>(o2, o, v);
  const long nu = (o * (o - 1) / 2) * (v * (v - 1) / 2);
  if (nu > 0) {
    const long groups = (nu + 63) / 64;
    const unsigned nb = (unsigned)std::max(1L, std::min(2048L, (groups + LW - 1) / LW));
    k_learned_t2_mfma<<<nb, 64 * LW, 0, ctx->stream>>>(m->pbf.as<float>(), t2, r2, r2prev, I->eps_d.as<double>(),
                                                       fd, o, v, o2);
  }
  FC_HIP(hipGetLastError());
  return FC_OK;
}

// fd: F_mi diagonal (o entries) then F_ae diagonal (v entries), from the residual evaluation
void learn_samples(fc_ctx ctx, fc_ints I, const z* t2, const z* r2, const z* r2prev, const z* t2s, const z* fd,
                   long nsamp, unsigned long long seed, float* X, float* q, float* r) {
  const long o = I->o, v = I->v;
  FC_REQUIRE(o >= 2 && v >= 2, FC_EARG, "learn_samples: needs o >= 2 and v >= 2");
  k_samples<<<nblk(nsamp), TPB, 0, ctx->stream>>>(t2, r2, r2prev, t2s, I->eps_d.as<double>(), fd, o, v, nsamp, seed,
                                                  X, q, r);
  FC_HIP(hipGetLastError());
}

}  // namespace fc

using namespace fc;

extern "C" {

int fc_mlp_create(fc_ctx ctx, const float* params_host, unsigned long long seed, fc_mlp* out) {
  if (!ctx || !out) return FC_EARG;
  try {
    auto* m = new fc_mlp_s();
    m->ctx = ctx;
    m->np = NP;
    m->params = DBuf(ctx, sizeof(float) * NP);
    m->grads = DBuf(ctx, sizeof(float) * NP);
    m->m = DBuf(ctx, sizeof(float) * NP);
    m->v = DBuf(ctx, sizeof(float) * NP);
    m->pbf = DBuf(ctx, sizeof(float) * NP);
    std::vector<float> h(NP, 0.f);
    if (params_host) {
      std::memcpy(h.data(), params_host, sizeof(float) * NP);
    } else {
      // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a 64-bit LCG; output layer starts at zero
      unsigned long long s = seed * 6364136223846793005ull + 1442695040888963407ull;
      auto uni = [&]() { s = s * 6364136223846793005ull + 1442695040888963407ull; return (double)(s >> 11) * 0x1.0p-53; };
      for (long k = OW1; k < OB1; ++k) h[k] = (float)((2 * uni() - 1) / std::sqrt((double)NIN));
      for (long k = OW2; k < OB2; ++k) h[k] = (float)((2 * uni() - 1) / std::sqrt((double)NH));
    }
    FC_HIP(hipMemcpyAsync(m->params.p, h.data(), sizeof(float) * NP, hipMemcpyHostToDevice, ctx->stream));
    FC_HIP(hipMemsetAsync(m->m.p, 0, sizeof(float) * NP, ctx->stream));
    FC_HIP(hipMemsetAsync(m->v.p, 0, sizeof(float) * NP, ctx->stream));
    k_round_bf16<<<nblk(NP), TPB, 0, ctx->stream>>>(m->params.as<float>(), m->pbf.as<float>(), NP);
    FC_HIP(hipGetLastError());
    FC_HIP(hipStreamSynchronize(ctx->stream));
    *out = m;
    return FC_OK;
  } catch (const Error& e) {
    ctx->last_error = e.what();
    return e.code;
  }
}

void fc_mlp_free(fc_mlp m) { delete m; }

long fc_mlp_num_params(void) { return NP; }

int fc_mlp_get_params(fc_mlp m, float* host, int bf16_rounded) {
  if (!m || !host) return FC_EARG;
  try {
    FC_HIP(hipMemcpyAsync(host, bf16_rounded ? m->pbf.p : m->params.p, sizeof(float) * NP, hipMemcpyDeviceToHost,
                          m->ctx->stream));
    FC_HIP(hipStreamSynchronize(m->ctx->stream));
    return FC_OK;
  } catch (const Error& e) {
    m->ctx->last_error = e.what();
    return e.code;
  }
}

static void train_grads(fc_mlp m, const float* X, const float* q, const float* r, long B, float* loss_host) {
  fc_ctx ctx = m->ctx;
  // normalisation sum |q|^2 in FP64 on the host-visible side (fixed order)
  std::vector<float> hq(2 * B);
  FC_HIP(hipMemcpyAsync(hq.data(), q, sizeof(float) * 2 * B, hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  double w = 0;
  for (long s = 0; s < 2 * B; ++s) w += (double)hq[s] * hq[s];
  FC_REQUIRE(w > 0, FC_EARG, "mlp: all Jacobi steps in the minibatch are zero");
  DBuf H1(ctx, sizeof(float) * B * NH), H2(ctx, sizeof(float) * B * NH), dH1(ctx, sizeof(float) * B * NH),
      dH2(ctx, sizeof(float) * B * NH), dY(ctx, sizeof(float) * B * NOUT), lv(ctx, sizeof(float) * B);
  k_train_sample<<<nblk(B), TPB, 0, ctx->stream>>>(m->params.as<float>(), X, q, r, B, (float)(1.0 / w), H1.as<float>(),
                                                   H2.as<float>(), dH1.as<float>(), dH2.as<float>(), dY.as<float>(),
                                                   lv.as<float>());
  float* G = m->grads.as<float>();
  k_weight_grad<<<NOUT, 64, 0, ctx->stream>>>(dY.as<float>(), NOUT, H2.as<float>(), NH, B, G + OW3, G + OB3);
  k_weight_grad<<<NH, 64, 0, ctx->stream>>>(dH2.as<float>(), NH, H1.as<float>(), NH, B, G + OW2, G + OB2);
  k_weight_grad<<<NH, 64, 0, ctx->stream>>>(dH1.as<float>(), NH, X, NIN, B, G + OW1, G + OB1);
  FC_HIP(hipGetLastError());
  if (loss_host) {
    std::vector<float> hl(B);
    FC_HIP(hipMemcpyAsync(hl.data(), lv.p, sizeof(float) * B, hipMemcpyDeviceToHost, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    double s = 0;
    for (float x : hl) s += x;
    *loss_host = (float)s;
  }
}

int fc_mlp_grad(fc_mlp m, const float* X, const float* q, const float* r, long B, float* grad_host, float* loss) {
  if (!m || !X || !q || !r || B < 1) return FC_EARG;
  try {
    train_grads(m, X, q, r, B, loss);
    if (grad_host) {
      FC_HIP(hipMemcpyAsync(grad_host, m->grads.p, sizeof(float) * NP, hipMemcpyDeviceToHost, m->ctx->stream));
      FC_HIP(hipStreamSynchronize(m->ctx->stream));
    }
    return FC_OK;
  } catch (const Error& e) {
    m->ctx->last_error = e.what();
    return e.code;
  }
}

int fc_mlp_train_step(fc_mlp m, const float* X, const float* q, const float* r, long B, float lr, float* loss) {
  if (!m || !X || !q || !r || B < 1 || !(lr > 0)) return FC_EARG;
  try {
    train_grads(m, X, q, r, B, loss);
    m->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)m->step), c2 = 1.f - std::pow(b2, (float)m->step);
    k_adam<<<nblk(NP), TPB, 0, m->ctx->stream>>>(m->params.as<float>(), m->grads.as<float>(), m->m.as<float>(),
                                                 m->v.as<float>(), m->pbf.as<float>(), NP, lr, b1, b2, 1e-8f, c1, c2);
    FC_HIP(hipGetLastError());
    return FC_OK;
  } catch (const Error& e) {
    m->ctx->last_error = e.what();
    return e.code;
  }
}

int fc_mlp_forward(fc_mlp m, const float* X, long B, float* Y, int bf16_weights) {
  if (!m || !X || !Y || B < 1) return FC_EARG;
  try {
    k_forward<<<nblk(B), TPB, 0, m->ctx->stream>>>(bf16_weights ? m->pbf.as<float>() : m->params.as<float>(), X, B, Y);
    FC_HIP(hipGetLastError());
    FC_HIP(hipStreamSynchronize(m->ctx->stream));
    return FC_OK;
  } catch (const Error& e) {
    m->ctx->last_error = e.what();
    return e.code;
  }
}

}  // extern "C"
