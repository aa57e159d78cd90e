// Complex GEMM on the FP64 matrix cores of gfx950.
//
// A complex product is four real products on v_mfma_f64_16x16x4f64:
//   Cre += Are*Bre - Aim*Bim,   Cim += Are*Bim + Aim*Bre
// (the "4M" form; no cancellation-prone 3M trick in FP64).  Operands are staged through LDS
// with their real and imaginary parts in separate planes, conjugation applied at staging time,
// double-buffered so the next K slice loads while the current one feeds the matrix cores.
//
// Two tile shapes: 64 x 64 (4 waves of 32 x 32) for small products and 128 x 128 (8 waves of
// 64 x 32) for large ones.  Workgroups are numbered so that each of the 8 XCDs walks a
// contiguous band of output tiles (consecutive tiles share a row of A in that XCD's L2).
//
// MFMA f64 16x16x4 lane layout (lane l of a 64-wide wave):
//   A fragment: A[row = l % 16][k = l / 16];  B fragment: B[k = l / 16][col = l % 16];
//   accumulator register r: D[row = l / 16 + 4 * r][col = l % 16]  (measured on gfx950).
#include <algorithm>
#include <cstring>

#include "fc_internal.hpp"
#include "fc_gemm.hpp"

namespace fc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int BK = 8;      // K slice (complex elements)
constexpr int PAD = 16;    // LDS row padding (doubles): consecutive K rows land 32 banks apart

struct GemmArgs {
  long M, N, K;
  const z* A; long lda; long sA;
  const z* B; long ldb; long sB;
  z* C; long ldc; long sC;
  z alpha, beta;
  int conjA, conjB;
  long kchunk;        // K range per split (multiple of BK); blockIdx.y selects the split
  z* part;            // split-K partial products [split][M][N] (nullptr: write C directly)
  long tiles;         // number of output tiles
  // ladder epilogue: C row m = (a - a0) v + e, column n = (b - b0) v + f is written to
  // C[((m / v) nB + n / v) v^2 + (m % v) v + n % v]; tiles with every a > every b are skipped
  long lv, lnB;
  int ltri;
};

// blockIdx -> tile so that XCD x (= bid % 8) owns the contiguous tiles [x * per, (x + 1) * per)
__device__ inline long xcd_tile(long bid, long tiles) {
  const long per = (tiles + 7) / 8;
  return (bid & 7) * per + (bid >> 3);
}

template <int BM, int BN, int WGM, int WGN, bool TA, bool TB, int EPI>
__global__ __launch_bounds__(WGM * WGN * 64) void zgemm_f64_kernel(GemmArgs g) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;           // wave tile
  constexpr int FI = WTM / 16, FJ = WTN / 16;             // MFMA tiles per wave
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;     // staged complex elements per thread
  __shared__ double sAr[2][BK][BM + PAD], sAi[2][BK][BM + PAD];
  __shared__ double sBr[2][BK][BN + PAD], sBi[2][BK][BN + PAD];

  const long tile = xcd_tile(blockIdx.x, g.tiles);   // the grid is padded to a multiple of 8
  if (tile >= g.tiles) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WTM, wn = (wave % WGN) * WTN;
  const long ntn = (g.N + BN - 1) / BN;
  const long m0 = (tile / ntn) * BM, n0 = (tile % ntn) * BN;
  if (EPI == 1 && g.ltri) {
    // diagonal ab block: skip tiles whose smallest a exceeds their largest b
    const long amin = m0 / g.lv, bmax = (n0 + BN - 1 < g.N ? n0 + BN - 1 : g.N - 1) / g.lv;
    if (amin > bmax) return;
  }
  const z* __restrict__ A = g.A + (long)blockIdx.z * g.sA;
  const z* __restrict__ B = g.B + (long)blockIdx.z * g.sB;
  z* __restrict__ C = g.C + (long)blockIdx.z * g.sC;
  const double sa = g.conjA ? -1.0 : 1.0, sb = g.conjB ? -1.0 : 1.0;
  const long klo = (long)blockIdx.y * g.kchunk;
  const long khi = klo + g.kchunk < g.K ? klo + g.kchunk : g.K;

  z ra[LA], rb[LB];
#define FC_LOAD_TILE(k0)                                                                 \
  do {                                                                                   \
    _Pragma("unroll") for (int r = 0; r < LA; ++r) {                                     \
      int e = tid + NT * r, mm, kk;                                                      \
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }           \
      long gm = m0 + mm, gk = (k0) + kk;                                                 \
      z val = make_double2(0.0, 0.0);                                                    \
      if (gm < g.M && gk < khi) val = TA ? A[gk * g.lda + gm] : A[gm * g.lda + gk];      \
      ra[r] = val;                                                                       \
    }                                                                                    \
    _Pragma("unroll") for (int r = 0; r < LB; ++r) {                                     \
      int e = tid + NT * r, nn, kk;                                                      \
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }           \
      long gn = n0 + nn, gk = (k0) + kk;                                                 \
      z val = make_double2(0.0, 0.0);                                                    \
      if (gn < g.N && gk < khi) val = TB ? B[gn * g.ldb + gk] : B[gk * g.ldb + gn];      \
      rb[r] = val;                                                                       \
    }                                                                                    \
  } while (0)
#define FC_STORE_TILE(buf)                                                               \
  do {                                                                                   \
    _Pragma("unroll") for (int r = 0; r < LA; ++r) {                                     \
      int e = tid + NT * r, mm, kk;                                                      \
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }           \
      sAr[buf][kk][mm] = ra[r].x;                                                        \
      sAi[buf][kk][mm] = sa * ra[r].y;                                                   \
    }                                                                                    \
    _Pragma("unroll") for (int r = 0; r < LB; ++r) {                                     \
      int e = tid + NT * r, nn, kk;                                                      \
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }           \
      sBr[buf][kk][nn] = rb[r].x;                                                        \
      sBi[buf][kk][nn] = sb * rb[r].y;                                                   \
    }                                                                                    \
  } while (0)

  d4 cr[FI][FJ], ci[FI][FJ];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) { cr[i][j] = d4{0, 0, 0, 0}; ci[i][j] = d4{0, 0, 0, 0}; }

  const long nk = (khi - klo + BK - 1) / BK;
  FC_LOAD_TILE(klo);
  FC_STORE_TILE(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (long kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) FC_LOAD_TILE(klo + (kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double ar[FI], ai[FI], nai[FI], br[FJ], bi[FJ];
#pragma unroll
      for (int i = 0; i < FI; ++i) {
        ar[i] = sAr[buf][ks + lk][wm + 16 * i + lr];
        ai[i] = sAi[buf][ks + lk][wm + 16 * i + lr];
        nai[i] = -ai[i];
      }
#pragma unroll
      for (int j = 0; j < FJ; ++j) {
        br[j] = sBr[buf][ks + lk][wn + 16 * j + lr];
        bi[j] = sBi[buf][ks + lk][wn + 16 * j + lr];
      }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], ci[i][j], 0, 0, 0);
        }
#pragma unroll
      for (int i = 0; i < FI; ++i)
#pragma unroll
        for (int j = 0; j < FJ; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(nai[i], bi[j], cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], ci[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) FC_STORE_TILE(buf ^ 1);
    __syncthreads();
  }
#undef FC_LOAD_TILE
#undef FC_STORE_TILE

  const bool use_beta = (g.beta.x != 0.0 || g.beta.y != 0.0);
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = m0 + wm + 16 * i + lk + 4 * r;
        const long n = n0 + wn + 16 * j + lr;
        if (m >= g.M || n >= g.N) continue;
        const double re = cr[i][j][r], im = ci[i][j][r];
        if (g.part) {  // split-K: raw partial sums, reduced in a fixed order afterwards
          g.part[((long)blockIdx.y * g.M + m) * g.N + n] = make_double2(re, im);
          continue;
        }
        long off;
        if (EPI == 1) {
          const long a = m / g.lv, e = m % g.lv, b = n / g.lv, f = n % g.lv;
          off = ((a * g.lnB + b) * g.lv + e) * g.lv + f;
        } else {
          off = m * g.ldc + n;
        }
        z out = make_double2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
        if (use_beta) {
          z c0 = C[off];
          out.x += g.beta.x * c0.x - g.beta.y * c0.y;
          out.y += g.beta.x * c0.y + g.beta.y * c0.x;
        }
        C[off] = out;
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

template <int BM, int BN, int WGM, int WGN, int EPI>
void launch(const GemmArgs& g, bool ta, bool tb, dim3 grid, hipStream_t s) {
  constexpr int NT = WGM * WGN * 64;
  if (!ta && !tb) zgemm_f64_kernel<BM, BN, WGM, WGN, false, false, EPI><<<grid, NT, 0, s>>>(g);
  else if (!ta && tb) zgemm_f64_kernel<BM, BN, WGM, WGN, false, true, EPI><<<grid, NT, 0, s>>>(g);
  else if (ta && !tb) zgemm_f64_kernel<BM, BN, WGM, WGN, true, false, EPI><<<grid, NT, 0, s>>>(g);
  else zgemm_f64_kernel<BM, BN, WGM, WGN, true, true, EPI><<<grid, NT, 0, s>>>(g);
}

// Tile configurations: 0 = 64 x 64 (4 waves), 1 = 128 x 64 (4 waves), 2 = 128 x 128 (8 waves).
constexpr int NCFG = 3;
constexpr int CFG_BM[NCFG] = {64, 128, 128}, CFG_BN[NCFG] = {64, 64, 128};

// Launch one configuration (split-K decided inside for configurations whose grid cannot fill the chip).
void zgemm_run(fc_ctx ctx, int cfg, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
               const z* B, long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC,
               const LadderEpilogue* lep);

// Shape bucket: operand layouts, sizes rounded to powers of two, batching and epilogue kind.
std::string bucket(char opA, char opB, long M, long N, long K, int batch, const LadderEpilogue* lep) {
  auto lg = [](long x) { int b = 0; while ((1L << b) < x) ++b; return b; };
  char buf[96];
  snprintf(buf, sizeof(buf), "%c%c_m%d_n%d_k%d_b%d_e%d", opA, opB, lg(M), lg(N), lg(K), batch > 1,
           lep ? 1 + lep->triangular : 0);
  return buf;
}

int heuristic_cfg(long M, long N, int batch) {
  const bool big = M >= 256 && N >= 256 && ((M + 127) / 128) * ((N + 127) / 128) * (long)batch >= 512;
  return big ? 2 : 0;
}

void zgemm_impl(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda, const z* B,
                long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC, const LadderEpilogue* lep) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  FC_REQUIRE(strchr("NTCR", opA) && strchr("NTCR", opB), FC_EARG, "zgemm: bad op");
  int cfg = heuristic_cfg(M, N, batch);
  if (ctx->autotune && K > 0) {
    const std::string key = bucket(opA, opB, M, N, K, batch, lep);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) {
      cfg = it->second.first;
    } else {
      // time every configuration once (after one warm-up launch) on a scratch copy of C, keep the fastest
      const long csz = lep ? (M / lep->v) * lep->nB * lep->v * lep->v
                           : ((long)(batch - 1) * sC + (M - 1) * ldc + N);
      DBuf scratch(ctx, sizeof(z) * (size_t)std::max(1L, csz));
      hipEvent_t e0, e1;
      FC_HIP(hipEventCreate(&e0));
      FC_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      int bestc = cfg;
      for (int c = 0; c < NCFG; ++c) {
        if (CFG_BM[c] > 64 && M < 128) continue;
        if (CFG_BN[c] > 64 && N < 128) continue;
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          if (!lep && (beta.x != 0.0 || beta.y != 0.0))
            FC_HIP(hipMemcpyAsync(scratch.p, C, sizeof(z) * csz, hipMemcpyDeviceToDevice, ctx->stream));
          FC_HIP(hipEventRecord(e0, ctx->stream));
          zgemm_run(ctx, c, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, scratch.as<z>(), ldc, batch, sA, sB, sC, lep);
          FC_HIP(hipEventRecord(e1, ctx->stream));
          FC_HIP(hipEventSynchronize(e1));
          FC_HIP(hipEventElapsedTime(&ms, e0, e1));
        }
        if (ms < best) { best = ms; bestc = c; }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      ctx->tune[key] = {bestc, best};
      cfg = bestc;
    }
  }
  zgemm_run(ctx, cfg, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch, sA, sB, sC, lep);
}

void zgemm_run(fc_ctx ctx, int cfg, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
               const z* B, long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC,
               const LadderEpilogue* lep) {
  FC_REQUIRE(strchr("NTCR", opA) && strchr("NTCR", opB), FC_EARG, "zgemm: bad op");
  if (K <= 0) {  // C = beta C
    FC_REQUIRE(!lep, FC_EARG, "zgemm: empty ladder product");
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
  g.lv = lep ? lep->v : 1;
  g.lnB = lep ? lep->nB : 1;
  g.ltri = lep ? lep->triangular : 0;
  const bool ta = (opA == 'T' || opA == 'C');
  const bool tb = (opB == 'T' || opB == 'C');
  FC_REQUIRE(batch <= 65535, FC_EARG, "zgemm: batch too large");
  FC_REQUIRE(cfg >= 0 && cfg < NCFG, FC_EARG, "zgemm: bad tile configuration");
  const long bm = CFG_BM[cfg], bn = CFG_BN[cfg];
  const long tiles = ((N + bn - 1) / bn) * ((M + bm - 1) / bm);
  FC_REQUIRE(tiles < (1L << 30), FC_EARG, "zgemm: problem too large for one launch");
  g.tiles = tiles;
  // Split K when the tile grid cannot fill the chip (256 CUs): each split covers >= 8 BK steps,
  // partials go to a workspace and are summed in split order, so results stay deterministic.
  long ksplit = 1;
  const long want = 1024;
  if (!lep && batch == 1 && tiles < want && K >= 16 * BK) {
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
  dim3 grid((unsigned)((tiles + 7) / 8 * 8), (unsigned)ksplit, (unsigned)batch);
  if (lep) {
    if (cfg == 2) launch<128, 128, 2, 4, 1>(g, ta, tb, grid, ctx->stream);
    else if (cfg == 1) launch<128, 64, 2, 2, 1>(g, ta, tb, grid, ctx->stream);
    else launch<64, 64, 2, 2, 1>(g, ta, tb, grid, ctx->stream);
  } else {
    if (cfg == 2) launch<128, 128, 2, 4, 0>(g, ta, tb, grid, ctx->stream);
    else if (cfg == 1) launch<128, 64, 2, 2, 0>(g, ta, tb, grid, ctx->stream);
    else launch<64, 64, 2, 2, 0>(g, ta, tb, grid, ctx->stream);
  }
  FC_HIP(hipGetLastError());
  if (ksplit > 1) {
    const long MN = M * N;
    unsigned nb = (unsigned)std::max(1L, std::min(65536L, (MN + 255) / 256));
    k_splitk_reduce<<<nb, 256, 0, ctx->stream>>>(g.part, (int)ksplit, M, N, C, ldc, alpha, beta);
    FC_HIP(hipGetLastError());
  }
}
}  // namespace

void zgemm(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda, const z* B, long ldb,
           z beta, z* C, long ldc, int batch, long sA, long sB, long sC) {
  zgemm_impl(ctx, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch, sA, sB, sC, nullptr);
}

void zgemm_ladder(fc_ctx ctx, long M, long N, long K, const z* A, long lda, const z* B, long ldb, z* W,
                  const LadderEpilogue& lep) {
  zgemm_impl(ctx, 'N', 'T', M, N, K, make_double2(1, 0), A, lda, B, ldb, make_double2(0, 0), W, 0, 1, 0, 0, 0, &lep);
}

}  // namespace fc
