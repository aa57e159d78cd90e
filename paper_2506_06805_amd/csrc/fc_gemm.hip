// Complex GEMM on the FP64 matrix cores of gfx950.
//
// A complex product is four real products on v_mfma_f64_16x16x4f64:
//   Cre += Are*Bre - Aim*Bim,   Cim += Are*Bim + Aim*Bre
// (the "4M" form; no cancellation-prone 3M trick in FP64).  Operands are staged through LDS
// with their real and imaginary parts in separate planes, conjugation applied at staging time.
//
// MFMA f64 16x16x4 lane layout (lane l of a 64-wide wave):
//   A fragment: A[row = l % 16][k = l / 16];  B fragment: B[k = l / 16][col = l % 16];
//   accumulator register r: D[row = l / 16 + 4 * r][col = l % 16]  (measured on gfx950).
#include <algorithm>
#include <cstring>

#include "fc_internal.hpp"

namespace fc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 8;     // block tile (complex elements)
constexpr int PAD = 16;                     // LDS row padding (doubles): rows land 32 banks apart
constexpr int NT = 256;                     // 4 waves, 2 x 2, each a 32 x 32 sub-tile

struct GemmArgs {
  long M, N, K;
  const z* A; long lda; long sA;
  const z* B; long ldb; long sB;
  z* C; long ldc; long sC;
  z alpha, beta;
  int conjA, conjB;
  long kchunk;        // K range per split (multiple of BK); blockIdx.y selects the split
  z* part;            // split-K partial products [split][M][N] (nullptr: write C directly)
};

// TA: A stored K-major (A[k*lda+m]); TB: B stored K-minor (B[n*ldb+k]).
template <bool TA, bool TB>
__global__ __launch_bounds__(NT) void zgemm_f64_kernel(GemmArgs g) {
  __shared__ double sAr[2][BK][BM + PAD], sAi[2][BK][BM + PAD];
  __shared__ double sBr[2][BK][BN + PAD], sBi[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const long ntn = (g.N + BN - 1) / BN;
  const long tile = blockIdx.x;
  const long m0 = (tile / ntn) * BM, n0 = (tile % ntn) * BN;
  const z* __restrict__ A = g.A + (long)blockIdx.z * g.sA;
  const z* __restrict__ B = g.B + (long)blockIdx.z * g.sB;
  z* __restrict__ C = g.C + (long)blockIdx.z * g.sC;
  const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
  const long klo = (long)blockIdx.y * g.kchunk;
  const long khi = klo + g.kchunk < g.K ? klo + g.kchunk : g.K;

  // Each thread stages two complex elements of A and two of B per BK step.
  z ra[2], rb[2];
  auto load_tile = [&](long k0) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int e = tid + NT * r;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      long gm = m0 + mm, gk = k0 + kk;
      z val = make_double2(0.0, 0.0);
      if (gm < g.M && gk < khi) val = TA ? A[gk * g.lda + gm] : A[gm * g.lda + gk];
      ra[r] = val;
      int nn;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      long gn = n0 + nn; gk = k0 + kk;
      val = make_double2(0.0, 0.0);
      if (gn < g.N && gk < khi) val = TB ? B[gn * g.ldb + gk] : B[gk * g.ldb + gn];
      rb[r] = val;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      int e = tid + NT * r;
      int mm, kk;
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }
      sAr[buf][kk][mm] = ra[r].x;
      sAi[buf][kk][mm] = sa * ra[r].y;
      int nn;
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }
      sBr[buf][kk][nn] = rb[r].x;
      sBi[buf][kk][nn] = sb * rb[r].y;
    }
  };

  d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) { cr[i][j] = d4{0, 0, 0, 0}; ci[i][j] = d4{0, 0, 0, 0}; }

  const long nk = (khi - klo + BK - 1) / BK;
  load_tile(klo);
  store_tile(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (long kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) load_tile(klo + (kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double ar[2], ai[2], nai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = sAr[buf][ks + lk][wm + 16 * i + lr];
        ai[i] = sAi[buf][ks + lk][wm + 16 * i + lr];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        br[j] = sBr[buf][ks + lk][wn + 16 * j + lr];
        bi[j] = sBi[buf][ks + lk][wn + 16 * j + lr];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) {
      store_tile(buf ^ 1);
    }
    __syncthreads();
  }

  if (g.part) {  // split-K: raw partial sums, reduced in a fixed order by k_splitk_reduce
    z* P = g.part + (long)blockIdx.y * g.M * g.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          long m = m0 + wm + 16 * i + lk + 4 * r;
          long n = n0 + wn + 16 * j + lr;
          if (m < g.M && n < g.N) P[m * g.N + n] = make_double2(cr[i][j][r], ci[i][j][r]);
        }
    return;
  }
  const bool use_beta = (g.beta.x != 0.0 || g.beta.y != 0.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        long m = m0 + wm + 16 * i + lk + 4 * r;
        long n = n0 + wn + 16 * j + lr;
        if (m < g.M && n < g.N) {
          double re = cr[i][j][r], im = ci[i][j][r];
          z out = make_double2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
          if (use_beta) {
            z c0 = C[m * g.ldc + n];
            out.x += g.beta.x * c0.x - g.beta.y * c0.y;
            out.y += g.beta.x * c0.y + g.beta.y * c0.x;
          }
          C[m * g.ldc + n] = out;
        }
      }
}

// C = alpha * sum_s P[s] + beta * C, summed in split order (deterministic)
__global__ void k_splitk_reduce(const z* __restrict__ P, int ns, long M, long N, z* __restrict__ C, long ldc,
                                z alpha, z beta) {
  const long MN = M * N;
  const bool use_beta = (beta.x != 0.0 || beta.y != 0.0);
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < MN; t += (long)gridDim.x * blockDim.x) {
    double re = 0, im = 0;
    for (int s = 0; s < ns; ++s) { z p = P[s * MN + t]; re += p.x; im += p.y; }
    long m = t / N, n = t % N;
    z out = make_double2(alpha.x * re - alpha.y * im, alpha.x * im + alpha.y * re);
    if (use_beta) {
      z c0 = C[m * ldc + n];
      out.x += beta.x * c0.x - beta.y * c0.y;
      out.y += beta.x * c0.y + beta.y * c0.x;
    }
    C[m * ldc + n] = out;
  }
}

}  // namespace

void zgemm(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
           const z* B, long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  FC_REQUIRE(strchr("NTCR", opA) && strchr("NTCR", opB), FC_EARG, "zgemm: bad op");
  if (K <= 0) {  // C = beta C
    for (int b = 0; b < batch; ++b)
      for (long m = 0; m < M; ++m) scale(ctx, C + b * sC + m * ldc, N, beta);
    return;
  }
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.sA = sA;
  g.B = B; g.ldb = ldb; g.sB = sB;
  g.C = C; g.ldc = ldc; g.sC = sC;
  g.alpha = alpha; g.beta = beta;
  g.conjA = (opA == 'C' || opA == 'R');
  g.conjB = (opB == 'C' || opB == 'R');
  const bool ta = (opA == 'T' || opA == 'C');
  const bool tb = (opB == 'T' || opB == 'C');
  FC_REQUIRE(batch <= 65535, FC_EARG, "zgemm: batch too large");
  const long tiles = ((N + BN - 1) / BN) * ((M + BM - 1) / BM);
  FC_REQUIRE(tiles < (1L << 31), FC_EARG, "zgemm: problem too large for one launch");
  // Split K when the tile grid cannot fill the chip (256 CUs): each split covers >= 8 BK steps,
  // partials go to a workspace and are summed in split order, so results stay deterministic.
  long ksplit = 1;
  const long want = 1024;
  if (batch == 1 && tiles < want && K >= 16 * BK) {
    ksplit = std::min((want + tiles - 1) / tiles, K / (8 * BK));
    const long cap = std::max(1L, (256L << 20) / (long)(sizeof(z) * M * N));
    ksplit = std::max(1L, std::min({ksplit, cap, 4096L}));
  }
  g.kchunk = ((K + ksplit - 1) / ksplit + BK - 1) / BK * BK;
  ksplit = (K + g.kchunk - 1) / g.kchunk;
  g.part = nullptr;
  DBuf work;
  if (ksplit > 1) {
    work = DBuf(ctx, sizeof(z) * (size_t)ksplit * M * N);
    g.part = work.as<z>();
  }
  dim3 grid((unsigned)tiles, (unsigned)ksplit, (unsigned)batch);
  if (!ta && !tb) zgemm_f64_kernel<false, false><<<grid, NT, 0, ctx->stream>>>(g);
  else if (!ta && tb) zgemm_f64_kernel<false, true><<<grid, NT, 0, ctx->stream>>>(g);
  else if (ta && !tb) zgemm_f64_kernel<true, false><<<grid, NT, 0, ctx->stream>>>(g);
  else zgemm_f64_kernel<true, true><<<grid, NT, 0, ctx->stream>>>(g);
  FC_HIP(hipGetLastError());
  if (ksplit > 1) {
    const long MN = M * N;
    unsigned nb = (unsigned)std::max(1L, std::min(65536L, (MN + 255) / 256));
    k_splitk_reduce<<<nb, 256, 0, ctx->stream>>>(g.part, (int)ksplit, M, N, C, ldc, alpha, beta);
    FC_HIP(hipGetLastError());
  }
}

}  // namespace fc
