// The step in front of the hot path: single-step pivoted Cholesky of the AO two-electron
// supermatrix (Eq. 21) and the two-component transform of its vectors to the spinor basis
// (Eq. 22), both on the device.
//
// Cholesky: vector j is l_j = (M[p_j, :] - sum_{k<j} l_k[p_j] l_k) / sqrt(d[p_j]) with p_j the
// largest remaining diagonal entry; d -= l_j^2 afterwards.  The loop is inherently sequential in
// j, so each step is one memory-bound pass over the vectors formed so far (j m doubles): the
// column kernel reads them once with every lane owning one composite index x and the waves of a
// workgroup splitting the sum over k; it updates d and leaves a per-workgroup argmax, and a
// one-workgroup kernel picks the next pivot.  Pivots stay on the device; the host only looks at
// the stop flag every few dozen steps.
//
// Transform: L^P = sum_s C_s^H L_AO^P C_s.  With Cs = [C_alpha | C_beta] (nao x 2n) one product
// X = L_AO Cs covers every P at once (rows (P, mu)); X^P read as [(mu, s)][q] then meets the
// coefficients with rows interleaved the same way, Ci[(mu, s)][p] = C_s[mu][p], in one batched
// product L^P = Ci^H X^P (K = 2 nao).
#include <algorithm>
#include <cmath>

#include "fc_state.hpp"

namespace fc {
namespace {
constexpr int CD_LANES = 64;   // composite indices per workgroup, one per lane
constexpr int CD_WAVES = 16;   // waves sharing the sum over earlier vectors
constexpr int CD_TPB = CD_LANES * CD_WAVES;
constexpr int PICK_TPB = 256;

struct ArgMax {
  double v;
  long i;
};
__device__ inline bool better(double v, long i, double bv, long bi) { return v > bv || (v == bv && i < bi); }

struct CdState {
  int stop;    // 0 running, 1 converged (largest diagonal < tau), 2 max_vec reached first
  int nvec;    // vectors formed (valid once stop != 0)
};

// d = diag(M) and one argmax per workgroup
__global__ void k_cd_init(const double* __restrict__ M, long m, double* __restrict__ d, ArgMax* __restrict__ part) {
  __shared__ double sv[CD_LANES];
  __shared__ long si[CD_LANES];
  const long x = blockIdx.x * (long)CD_LANES + threadIdx.x;
  double v = -INFINITY;
  if (x < m) {
    v = M[x * m + x];
    d[x] = v;
  }
  sv[threadIdx.x] = v;
  si[threadIdx.x] = x;
  __syncthreads();
  for (int s = CD_LANES / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && better(sv[threadIdx.x + s], si[threadIdx.x + s], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + s];
      si[threadIdx.x] = si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = ArgMax{sv[0], si[0]};
}

// Pivot of step j from the per-workgroup maxima, or the stop decision.
__global__ void k_cd_pick(const ArgMax* __restrict__ part, int nparts, int j, int max_vec, double tau,
                          int* __restrict__ piv, double* __restrict__ pval, CdState* __restrict__ st) {
  __shared__ double sv[PICK_TPB];
  __shared__ long si[PICK_TPB];
  if (st->stop) return;
  double bv = -INFINITY;
  long bi = 0x7fffffffffffffffL;
  for (int t = threadIdx.x; t < nparts; t += PICK_TPB)
    if (better(part[t].v, part[t].i, bv, bi)) { bv = part[t].v; bi = part[t].i; }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = PICK_TPB / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && better(sv[threadIdx.x + s], si[threadIdx.x + s], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + s];
      si[threadIdx.x] = si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (!(sv[0] >= tau)) {
      st->stop = 1;
      st->nvec = j;
    } else if (j == max_vec) {
      st->stop = 2;
      st->nvec = j;
    } else {
      piv[j] = (int)si[0];
      pval[j] = sv[0];
    }
  }
}

// Vector j: lane x of workgroup b owns composite index x = b * 64 + lane; wave w sums k = w, w + 16, ...
__global__ void __launch_bounds__(CD_TPB) k_cd_column(const double* __restrict__ M, long m, int j,
                                                      double* __restrict__ L, double* __restrict__ d,
                                                      const int* __restrict__ piv, const double* __restrict__ pval,
                                                      const CdState* __restrict__ st, ArgMax* __restrict__ part) {
  if (st->stop) return;
  __shared__ double acc[CD_WAVES][CD_LANES];
  __shared__ double sv[CD_LANES];
  __shared__ long si[CD_LANES];
  const int lane = threadIdx.x % CD_LANES, w = threadIdx.x / CD_LANES;
  const long x = blockIdx.x * (long)CD_LANES + lane;
  const long p = piv[j];
  // four independent partial sums keep four row loads of every wave in flight
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  if (x < m) {
    int k = w;
    for (; k + 3 * CD_WAVES < j; k += 4 * CD_WAVES) {
      const double* r = L + (long)k * m;
      const long step = (long)CD_WAVES * m;
      s0 += r[p] * r[x];
      s1 += r[step + p] * r[step + x];
      s2 += r[2 * step + p] * r[2 * step + x];
      s3 += r[3 * step + p] * r[3 * step + x];
    }
    for (; k < j; k += CD_WAVES) s0 += L[(long)k * m + p] * L[(long)k * m + x];
  }
  acc[w][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (w == 0) {
    double v = -INFINITY;
    if (x < m) {
      double s = 0;
      for (int q = 0; q < CD_WAVES; ++q) s += acc[q][lane];
      const double l = (M[p * m + x] - s) / sqrt(pval[j]);
      L[(long)j * m + x] = l;
      v = x == p ? 0.0 : d[x] - l * l;
      d[x] = v;
    }
    sv[lane] = v;
    si[lane] = x;
  }
  __syncthreads();
  for (int s = CD_LANES / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s && better(sv[threadIdx.x + s], si[threadIdx.x + s], sv[threadIdx.x], si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + s];
      si[threadIdx.x] = si[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = ArgMax{sv[0], si[0]};
}

constexpr int TPB = 256;
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(65536L, (n + TPB - 1) / TPB)); }
#define GRID_STRIDE(i, n) for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)

// Cs[nu][(s, q)] = C[s nao + nu][q];  Ci[(mu, s)][p] = C[s nao + mu][p]
__global__ void k_coeff_layouts(const z* __restrict__ C, long nao, long n, z* __restrict__ Cs, z* __restrict__ Ci) {
  GRID_STRIDE(t, 2 * nao * n) {
    const long q = t % n, r = t / n, s = r / nao, mu = r % nao;
    const z c = C[t];
    Cs[mu * 2 * n + s * n + q] = c;
    Ci[(2 * mu + s) * n + q] = c;
  }
}
__global__ void k_real_to_complex(const double* __restrict__ a, z* __restrict__ b, long n) {
  GRID_STRIDE(t, n) { b[t] = make_double2(a[t], 0.0); }
}
}  // namespace

int cd_pivoted_dev(fc_ctx ctx, long m, const double* M, double tau, int max_vec, double* L, int* nvec,
                   int* piv_host) {
  StageTimer stt(ctx, "ao_cd");
  const int nparts = (int)((m + CD_LANES - 1) / CD_LANES);
  DBuf d(ctx, sizeof(double) * m), part(ctx, sizeof(ArgMax) * nparts), piv(ctx, sizeof(int) * (max_vec + 1)),
      pval(ctx, sizeof(double) * (max_vec + 1)), st(ctx, sizeof(CdState));
  FC_HIP(hipMemsetAsync(st.p, 0, sizeof(CdState), ctx->stream));
  CdState* sh = nullptr;
  FC_HIP(hipHostMalloc((void**)&sh, sizeof(CdState), hipHostMallocDefault));
  struct Pinned {
    CdState* p;
    ~Pinned() { (void)hipHostFree(p); }
  } guard{sh};
  k_cd_init<<<nparts, CD_LANES, 0, ctx->stream>>>(M, m, d.as<double>(), part.as<ArgMax>());
  FC_HIP(hipGetLastError());
  // the host reads the stop flag after every `check` steps; steps after a stop return at once
  const int check = 32;
  for (int j = 0; j <= max_vec; ++j) {
    k_cd_pick<<<1, PICK_TPB, 0, ctx->stream>>>(part.as<ArgMax>(), nparts, j, max_vec, tau, piv.as<int>(),
                                                pval.as<double>(), st.as<CdState>());
    if (j < max_vec)
      k_cd_column<<<nparts, CD_TPB, 0, ctx->stream>>>(M, m, j, L, d.as<double>(), piv.as<int>(), pval.as<double>(),
                                                      st.as<CdState>(), part.as<ArgMax>());
    FC_HIP(hipGetLastError());
    if ((j + 1) % check == 0 || j == max_vec) {
      FC_HIP(hipMemcpyAsync(sh, st.p, sizeof(CdState), hipMemcpyDeviceToHost, ctx->stream));
      FC_HIP(hipStreamSynchronize(ctx->stream));
      if (sh->stop) break;
    }
  }
  FC_REQUIRE(sh->stop != 0, FC_ENUMERIC, "cd_ao_pivoted: no stop decision");
  *nvec = sh->nvec;
  if (piv_host && sh->nvec > 0)
    FC_HIP(hipMemcpyAsync(piv_host, piv.p, sizeof(int) * sh->nvec, hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  return sh->stop == 1 ? FC_OK : FC_ENOCONV;
}

void ao_to_spinor_dev(fc_ctx ctx, long nvec, long nao, long n, const double* Lao, const z* C, z* Lmo) {
  StageTimer stt(ctx, "ao_to_spinor");
  const z one = make_double2(1, 0), zero = make_double2(0, 0);
  ZTensor Cs(ctx, {nao, 2 * n}), Ci(ctx, {2 * nao, n});
  hipLaunchKernelGGL(k_coeff_layouts, dim3(nblk(2 * nao * n)), dim3(TPB), 0, ctx->stream, C, nao, n, Cs.p(), Ci.p());
  FC_HIP(hipGetLastError());
  // vectors per chunk: the complex copy of L_AO^P and X^P for a chunk stay within ~4 GB
  const double per = 16.0 * (nao * nao + nao * 2 * n);
  const long chunk = std::max(1L, std::min(nvec, (long)(4e9 / per)));
  ZTensor Lc(ctx, {chunk, nao, nao}), X(ctx, {chunk, nao, 2 * n});
  for (long P0 = 0; P0 < nvec; P0 += chunk) {
    const long np = std::min(chunk, nvec - P0);
    hipLaunchKernelGGL(k_real_to_complex, dim3(nblk(np * nao * nao)), dim3(TPB), 0, ctx->stream,
                       Lao + P0 * nao * nao, Lc.p(), np * nao * nao);
    FC_HIP(hipGetLastError());
    zgemm(ctx, 'N', 'N', np * nao, 2 * n, nao, one, Lc.p(), nao, Cs.p(), 2 * n, zero, X.p(), 2 * n);
    zgemm(ctx, 'C', 'N', n, n, 2 * nao, one, Ci.p(), n, X.p(), n, zero, Lmo + P0 * n * n, n, (int)np, 0,
          2 * nao * n, n * n);
  }
}

}  // namespace fc
