// Split-precision complex GEMM on the 16-bit matrix cores of gfx950.
//
// Each FP64 real component x is stored as two 16-bit numbers, hi = round(s x) and
// lo = round(s x - hi) (s a power of two: 1 for BF16, chosen from max|x| for FP16 so that the
// lo parts stay normal), so x = (hi + lo) / s to ~2^-16 (BF16) or ~2^-22 (FP16) relative.  A real
// product keeps the three terms hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_{bf16,f16} with FP32
// accumulation; a complex product uses the real products Ar*Br, Ai*Bi and Ar*Bi + Ai*Br, i.e.
// 12 MFMAs per 16x16x32 complex block.
//
// Operands are split once into four planes (re_hi, re_lo, im_hi, im_lo), each [rows][kp] with the
// contraction index contiguous and padded to a multiple of 32; rows are padded to a multiple of
// the 128-row tile, so tile loads need no bounds checks.  C[m][n] = alpha sum_k A[m][k] B[n][k]
// + beta C[m][n] (FP64 complex output).
//
// Tiles are 128 x 128 (8 waves of 64 x 32), K slices of 32, double-buffered in LDS with an XOR
// chunk swizzle (see swz); with 128 KB of LDS and 222 registers one workgroup fits per CU, which
// is what the split-K count of skinny products is chosen for.
//
// MFMA 16x16x32 (bf16/f16) lane layout on gfx950 (measured): A fragment lane l holds
// A[row = l % 16][k = 8 (l / 16) + 0..7], B fragment B[k = 8 (l / 16) + 0..7][col = l % 16],
// accumulator register r holds D[row = 4 (l / 16) + r][col = l % 16].
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fc_split.hpp"

namespace fc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int TM = 128, TN = 128, TK = 32, NT = 512;   // 8 waves, 2 x 4, each 64 x 32
constexpr int LDK = TK;   // LDS row length (16-bit elements): 64 bytes, four 16-byte chunks
// Chunk c of LDS row r is stored at chunk c ^ swz(r).  Fragment reads (16 consecutive rows, one
// chunk) and staging stores (4 consecutive rows, all chunks) then touch distinct banks whether
// the LDS serves 8 lanes x 16 bytes or 16 lanes x 16 bytes per cycle (measured on gfx950: bank
// conflict cycles 50% of LDS-active cycles with rows padded to 80 bytes, 0 with this swizzle).
// swz depends on r % 16 only, so fragment rows wm + 16 i + lr share the swizzle of lr.
__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 2)) & 3; }

template <int PREC> __device__ inline u16 to16(float x);
template <> __device__ inline u16 to16<FC_SPLIT_BF16>(float x) { return __builtin_bit_cast(u16, (__bf16)x); }
template <> __device__ inline u16 to16<FC_SPLIT_FP16>(float x) { return __builtin_bit_cast(u16, (_Float16)x); }
template <int PREC> __device__ inline double from16(u16 x);
template <> __device__ inline double from16<FC_SPLIT_BF16>(u16 x) { return (double)(float)__builtin_bit_cast(__bf16, x); }
template <> __device__ inline double from16<FC_SPLIT_FP16>(u16 x) { return (double)(float)__builtin_bit_cast(_Float16, x); }

// X[r * ldx + k] (complex FP64, r < rows, k < K) -> planes [4][rows_pad][kp]
template <int PREC>
__global__ void k_split(const z* __restrict__ X, long rows, long K, long ldx, long rows_pad, long kp, double scale,
                        int conj, u16* __restrict__ out) {
  const long total = rows_pad * kp, plane = rows_pad * kp;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    long r = t / kp, k = t % kp;
    z x = (r < rows && k < K) ? X[r * ldx + k] : make_double2(0.0, 0.0);
    double re = x.x * scale, im = (conj ? -x.y : x.y) * scale;
    u16 rh = to16<PREC>((float)re);
    u16 rl = to16<PREC>((float)(re - from16<PREC>(rh)));
    u16 ih = to16<PREC>((float)im);
    u16 il = to16<PREC>((float)(im - from16<PREC>(ih)));
    out[t] = rh;
    out[plane + t] = rl;
    out[2 * plane + t] = ih;
    out[3 * plane + t] = il;
  }
}

// planes[p][r][k] = 0 for k0 <= k < kp, every row r < rows_pad of the four planes
__global__ void k_zero_kpad(u16* __restrict__ planes, long rows_pad, long kp, long k0) {
  const long w = kp - k0, total = 4 * rows_pad * w;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long r = t / w;   // plane-major rows: r = p * rows_pad + row
    planes[r * kp + k0 + (t - r * w)] = 0;
  }
}

__global__ void k_maxabs(const z* __restrict__ X, long rows, long K, long ldx, unsigned* out) {
  __shared__ float s[256];
  float m = 0.f;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < rows * K; t += (long)gridDim.x * blockDim.x) {
    z x = X[(t / K) * ldx + t % K];
    m = fmaxf(m, fmaxf((float)fabs(x.x), (float)fabs(x.y)));
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(s[0]));   // non-negative floats order as uints
}

struct SArgs {
  const u16* A; long a_plane; long a_row0;   // planes of A, first row of this product
  const u16* B; long b_plane; long b_row0;
  long M, N, kp;
  z* C; long ldc;
  z alpha, beta;
  double inv_scale;
  long kchunk;
  z* part;
  long tiles;
  // ladder epilogue (EPI = 1): FP32 complex output W[((m / v) nB + n / v) v^2 + (m % v) v + n % v],
  // tiles with every a = m / v above every b = n / v skipped when ltri is set
  float2* W;
  long lv, lnB;
  int ltri;
};

template <int PREC>
__device__ inline f4 mma(const u16* a, const u16* b, f4 c) {
  if constexpr (PREC == FC_SPLIT_BF16) {
    bf8 x = *reinterpret_cast<const bf8*>(a), y = *reinterpret_cast<const bf8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
  } else {
    h8 x = *reinterpret_cast<const h8*>(a), y = *reinterpret_cast<const h8*>(b);
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(x, y, c, 0, 0, 0);
  }
}

template <int PREC, int EPI>
__global__ __launch_bounds__(NT) void k_gemm_split(SArgs g) {
  // double-buffered: 2 x 64 KB
  __shared__ __attribute__((aligned(16))) u16 sA[2][4][TM][LDK];
  __shared__ __attribute__((aligned(16))) u16 sB[2][4][TN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 2) * 64, wn = (wave & 3) * 32;
  const long ntn = (g.N + TN - 1) / TN;
  // XCD x (= blockIdx.x % 8) walks the contiguous tiles [x * per, (x + 1) * per); the split index
  // rotates the slot so that the splits of one tile spread over all XCDs
  const long per = (g.tiles + 7) / 8;
  const long bx = ((long)blockIdx.x + blockIdx.y) % gridDim.x;
  const long tile = (bx & 7) * per + (bx >> 3);
  if (tile >= g.tiles) return;
  long mi = tile / ntn;
  if (EPI == 1 && g.ltri) {
    // triangular launches: fold the tile rows so every XCD's band mixes live and skipped tiles
    const long tm = g.tiles / ntn;
    mi = (mi & 1) ? tm - 1 - (mi >> 1) : (mi >> 1);
  }
  const long m0 = mi * TM, n0 = (tile % ntn) * TN;
  if (EPI == 1 && g.ltri) {
    const long amin = m0 / g.lv, bmax = (n0 + TN - 1 < g.N ? n0 + TN - 1 : g.N - 1) / g.lv;
    if (amin > bmax) return;
  }
  const long klo = (long)blockIdx.y * g.kchunk;
  const long khi = klo + g.kchunk < g.kp ? klo + g.kchunk : g.kp;
  const u16* A = g.A + (g.a_row0 + m0) * g.kp;
  const u16* B = g.B + (g.b_row0 + n0) * g.kp;

  // staging: 2048 16-byte chunks per operand per k-step, 4 per thread; chunk c = tid + NT q is
  // plane c / 512, row (c % 512) / 4, k offset 8 (c % 4)
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  const int srow = (tid & 511) >> 2, skc = 8 * (tid & 3);
  const long goffA = (long)srow * g.kp + skc, goffB = goffA;
  const int sk = 8 * ((skc >> 3) ^ swz(srow));   // LDS column of this thread's staging chunk
#define FC_GLOAD(k0)                                                                                 \
  do {                                                                                               \
    ra0 = *reinterpret_cast<const uint4*>(A + 0 * g.a_plane + goffA + (k0));                         \
    ra1 = *reinterpret_cast<const uint4*>(A + 1 * g.a_plane + goffA + (k0));                         \
    ra2 = *reinterpret_cast<const uint4*>(A + 2 * g.a_plane + goffA + (k0));                         \
    ra3 = *reinterpret_cast<const uint4*>(A + 3 * g.a_plane + goffA + (k0));                         \
    rb0 = *reinterpret_cast<const uint4*>(B + 0 * g.b_plane + goffB + (k0));                         \
    rb1 = *reinterpret_cast<const uint4*>(B + 1 * g.b_plane + goffB + (k0));                         \
    rb2 = *reinterpret_cast<const uint4*>(B + 2 * g.b_plane + goffB + (k0));                         \
    rb3 = *reinterpret_cast<const uint4*>(B + 3 * g.b_plane + goffB + (k0));                         \
  } while (0)
#define FC_SSTORE(buf)                                                                               \
  do {                                                                                               \
    *reinterpret_cast<uint4*>(&sA[buf][0][srow][sk]) = ra0;                                         \
    *reinterpret_cast<uint4*>(&sA[buf][1][srow][sk]) = ra1;                                         \
    *reinterpret_cast<uint4*>(&sA[buf][2][srow][sk]) = ra2;                                         \
    *reinterpret_cast<uint4*>(&sA[buf][3][srow][sk]) = ra3;                                         \
    *reinterpret_cast<uint4*>(&sB[buf][0][srow][sk]) = rb0;                                         \
    *reinterpret_cast<uint4*>(&sB[buf][1][srow][sk]) = rb1;                                         \
    *reinterpret_cast<uint4*>(&sB[buf][2][srow][sk]) = rb2;                                         \
    *reinterpret_cast<uint4*>(&sB[buf][3][srow][sk]) = rb3;                                         \
  } while (0)

  f4 rr[4][2], ii[4][2], im[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) { rr[i][j] = f4{0, 0, 0, 0}; ii[i][j] = f4{0, 0, 0, 0}; im[i][j] = f4{0, 0, 0, 0}; }

  const int lr = lane & 15, lk = 8 * ((lane >> 4) ^ swz(lr));
  // one barrier per K step: the loads of the next slice are issued before the products of this
  // one and stored to the other buffer after them
  if (klo < khi) {
    FC_GLOAD(klo);
    FC_SSTORE(0);
  }
  __syncthreads();
  int buf = 0;
  for (long k0 = klo; k0 < khi; k0 += TK, buf ^= 1) {
    const bool more = k0 + TK < khi;
    if (more) FC_GLOAD(k0 + TK);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ra_ = wm + 16 * i + lr;
      const u16 *aRh = &sA[buf][0][ra_][lk], *aRl = &sA[buf][1][ra_][lk], *aIh = &sA[buf][2][ra_][lk],
                *aIl = &sA[buf][3][ra_][lk];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int rb_ = wn + 16 * j + lr;
        const u16 *bRh = &sB[buf][0][rb_][lk], *bRl = &sB[buf][1][rb_][lk], *bIh = &sB[buf][2][rb_][lk],
                  *bIl = &sB[buf][3][rb_][lk];
        rr[i][j] = mma<PREC>(aRh, bRh, rr[i][j]);
        rr[i][j] = mma<PREC>(aRh, bRl, rr[i][j]);
        rr[i][j] = mma<PREC>(aRl, bRh, rr[i][j]);
        ii[i][j] = mma<PREC>(aIh, bIh, ii[i][j]);
        ii[i][j] = mma<PREC>(aIh, bIl, ii[i][j]);
        ii[i][j] = mma<PREC>(aIl, bIh, ii[i][j]);
        im[i][j] = mma<PREC>(aRh, bIh, im[i][j]);
        im[i][j] = mma<PREC>(aRh, bIl, im[i][j]);
        im[i][j] = mma<PREC>(aRl, bIh, im[i][j]);
        im[i][j] = mma<PREC>(aIh, bRh, im[i][j]);
        im[i][j] = mma<PREC>(aIh, bRl, im[i][j]);
        im[i][j] = mma<PREC>(aIl, bRh, im[i][j]);
      }
    }
    if (more) FC_SSTORE(buf ^ 1);
    __syncthreads();
  }

  const int orow = 4 * (lane >> 4), ocol = lane & 15;
  const bool use_beta = (g.beta.x != 0.0 || g.beta.y != 0.0);
  // ladder layout ((a nB + b) v + e) v + f as a row part plus a column part, one 32-bit division
  // per row or column of the lane
  long coff[2] = {0, 0};
  if (EPI == 1) {
    const unsigned lv = (unsigned)g.lv;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const unsigned n = (unsigned)(n0 + wn + 16 * j + ocol), b = n / lv;
      coff[j] = (long)b * g.lv * g.lv + (long)(n - b * lv);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long m = m0 + wm + 16 * i + orow + r;
      long roff = 0;
      if (EPI == 1) {
        const unsigned mu = (unsigned)m, lv = (unsigned)g.lv, a = mu / lv;
        roff = ((long)a * g.lnB * g.lv + (long)(mu - a * lv)) * g.lv;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const long n = n0 + wn + 16 * j + ocol;
        if (m >= g.M || n >= g.N) continue;
        double re = ((double)rr[i][j][r] - (double)ii[i][j][r]) * g.inv_scale, imv = (double)im[i][j][r] * g.inv_scale;
        if (EPI == 1) {
          g.W[roff + coff[j]] = make_float2((float)re, (float)imv);
          continue;
        }
        if (g.part) {
          g.part[((long)blockIdx.y * g.M + m) * g.N + n] = make_double2(re, imv);
          continue;
        }
        z out = make_double2(g.alpha.x * re - g.alpha.y * imv, g.alpha.x * imv + g.alpha.y * re);
        if (use_beta) {
          z c0 = g.C[m * g.ldc + n];
          out.x += g.beta.x * c0.x - g.beta.y * c0.y;
          out.y += g.beta.x * c0.y + g.beta.y * c0.x;
        }
        g.C[m * g.ldc + n] = out;
      }
    }
}

__global__ void k_split_reduce(const z* __restrict__ P, int ns, long M, long N, z* __restrict__ C, long ldc, z alpha,
                               z beta) {
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

SplitOp split_operand(fc_ctx ctx, int prec, const z* X, long rows, long K, long ldx, bool conj) {
  FC_REQUIRE(prec == FC_SPLIT_BF16 || prec == FC_SPLIT_FP16, FC_EARG, "split_operand: bad precision");
  SplitOp s;
  s.prec = prec;
  s.rows = rows;
  s.rows_pad = (rows + TM - 1) / TM * TM + TM;   // one spare zero tile for row-offset products
  s.kp = std::max<long>(TK, (K + TK - 1) / TK * TK);
  s.scale = 1.0;
  if (prec == FC_SPLIT_FP16 && rows > 0 && K > 0) {
    DBuf mx(ctx, sizeof(unsigned));
    FC_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned), ctx->stream));
    unsigned nb = (unsigned)std::max(1L, std::min(2048L, (rows * K + 255) / 256));
    k_maxabs<<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, mx.as<unsigned>());
    FC_HIP(hipGetLastError());
    unsigned h = 0;
    FC_HIP(hipMemcpyAsync(&h, mx.p, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    float m;
    std::memcpy(&m, &h, sizeof(m));
    // largest |x| maps into [2^13, 2^14): hi parts stay below the FP16 maximum with margin and
    // lo parts (~2^-11 of hi) stay normal for entries down to ~1e-4 of the maximum
    if (m > 0) s.scale = std::ldexp(1.0, 13 - std::ilogb((double)m));
  }
  s.buf = DBuf(ctx, sizeof(u16) * 4 * (size_t)s.rows_pad * s.kp);
  const long total = s.rows_pad * s.kp;
  unsigned nb = (unsigned)std::max(1L, std::min(1048576L, (total + 1023) / 1024));
  if (prec == FC_SPLIT_BF16)
    k_split<FC_SPLIT_BF16><<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, s.rows_pad, s.kp, s.scale, (int)conj, s.buf.as<u16>());
  else
    k_split<FC_SPLIT_FP16><<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, s.rows_pad, s.kp, s.scale, (int)conj, s.buf.as<u16>());
  FC_HIP(hipGetLastError());
  return s;
}

void split_zero_kpad(fc_ctx ctx, SplitOp& S, long k0) {
  FC_REQUIRE(k0 >= 0 && k0 <= S.kp, FC_EARG, "split_zero_kpad: column out of range");
  const long total = 4 * S.rows_pad * (S.kp - k0);
  if (total == 0) return;
  unsigned nb = (unsigned)std::max(1L, std::min(65536L, (total + 255) / 256));
  k_zero_kpad<<<nb, 256, 0, ctx->stream>>>(S.buf.as<u16>(), S.rows_pad, S.kp, k0);
  FC_HIP(hipGetLastError());
}

void gemm_split_nt(fc_ctx ctx, const SplitOp& A, long a_row0, long M, const SplitOp& B, long b_row0, long N, z alpha,
                   z beta, z* C, long ldc) {
  if (M <= 0 || N <= 0) return;
  FC_REQUIRE(A.prec == B.prec && A.kp == B.kp, FC_EARG, "gemm_split_nt: operand mismatch");
  // rows_pad >= rows + TM - 1, so whole 128-row tiles starting inside [row0, row0 + M) stay in
  // the allocated (zero-padded) planes whenever row0 + M <= rows
  FC_REQUIRE(a_row0 >= 0 && b_row0 >= 0 && a_row0 + M <= A.rows && b_row0 + N <= B.rows, FC_EARG,
             "gemm_split_nt: row range outside operand");
  SArgs g;
  g.A = A.buf.as<u16>(); g.a_plane = A.rows_pad * A.kp; g.a_row0 = a_row0;
  g.B = B.buf.as<u16>(); g.b_plane = B.rows_pad * B.kp; g.b_row0 = b_row0;
  g.M = M; g.N = N; g.kp = A.kp;
  g.C = C; g.ldc = ldc; g.alpha = alpha; g.beta = beta;
  g.inv_scale = 1.0 / (A.scale * B.scale);
  const long tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  g.tiles = tiles;
  g.W = nullptr; g.lv = 1; g.lnB = 1; g.ltri = 0;
  long ksplit = 1;
  const long nks = A.kp / TK;
  if (tiles < 512 && nks >= 16) {
    // one workgroup per CU (the double-buffered tile takes 128 KB of LDS): pick the split count
    // k minimising waves(k) x (K slices per split + 4), the 4 standing for a workgroup's fixed
    // cost, with at least 8 K slices per split, at most 16 splits and 1 GiB of partial sums
    const long cap = std::max(1L, (1L << 30) / (long)(sizeof(z) * M * N));
    const long kmax = std::max(1L, std::min({nks / 8, cap, 16L}));
    double best = 0.0;
    for (long k = 1; k <= kmax; ++k) {
      const long waves = (tiles * k + 255) / 256;
      const double t = (double)waves * ((double)nks / (double)k + 4.0);
      if (k == 1 || t < best - 1e-9) { best = t; ksplit = k; }
    }
  }
  g.kchunk = (nks + ksplit - 1) / ksplit * TK;
  ksplit = (A.kp + g.kchunk - 1) / g.kchunk;
  DBuf work;
  g.part = nullptr;
  if (ksplit > 1) {
    work = DBuf(ctx, sizeof(z) * (size_t)ksplit * M * N);
    g.part = work.as<z>();
  }
  dim3 grid((unsigned)((tiles + 7) / 8 * 8), (unsigned)ksplit);
  if (A.prec == FC_SPLIT_BF16) k_gemm_split<FC_SPLIT_BF16, 0><<<grid, NT, 0, ctx->stream>>>(g);
  else k_gemm_split<FC_SPLIT_FP16, 0><<<grid, NT, 0, ctx->stream>>>(g);
  FC_HIP(hipGetLastError());
  if (ksplit > 1) {
    const long MN = M * N;
    unsigned nb = (unsigned)std::max(1L, std::min(65536L, (MN + 255) / 256));
    k_split_reduce<<<nb, 256, 0, ctx->stream>>>(g.part, (int)ksplit, M, N, C, ldc, alpha, beta);
    FC_HIP(hipGetLastError());
  }
}

void gemm_split_ladder(fc_ctx ctx, const SplitOp& A, long a_row0, long M, const SplitOp& B, long b_row0, long N,
                       float2* W, const LadderEpilogue& lep) {
  if (M <= 0 || N <= 0) return;
  FC_REQUIRE(A.prec == B.prec && A.kp == B.kp, FC_EARG, "gemm_split_ladder: operand mismatch");
  FC_REQUIRE(a_row0 >= 0 && b_row0 >= 0 && a_row0 + M <= A.rows && b_row0 + N <= B.rows, FC_EARG,
             "gemm_split_ladder: row range outside operand");
  FC_REQUIRE(M < (1L << 31) && N < (1L << 31) && lep.v >= 1, FC_EARG, "gemm_split_ladder: product too large");
  SArgs g;
  g.A = A.buf.as<u16>(); g.a_plane = A.rows_pad * A.kp; g.a_row0 = a_row0;
  g.B = B.buf.as<u16>(); g.b_plane = B.rows_pad * B.kp; g.b_row0 = b_row0;
  g.M = M; g.N = N; g.kp = A.kp;
  g.C = nullptr; g.ldc = 0; g.alpha = make_double2(1, 0); g.beta = make_double2(0, 0);
  g.inv_scale = 1.0 / (A.scale * B.scale);
  g.tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  g.kchunk = A.kp;
  g.part = nullptr;
  g.W = W; g.lv = lep.v; g.lnB = lep.nB; g.ltri = lep.triangular;
  dim3 grid((unsigned)((g.tiles + 7) / 8 * 8), 1);
  if (A.prec == FC_SPLIT_BF16) k_gemm_split<FC_SPLIT_BF16, 1><<<grid, NT, 0, ctx->stream>>>(g);
  else k_gemm_split<FC_SPLIT_FP16, 1><<<grid, NT, 0, ctx->stream>>>(g);
  FC_HIP(hipGetLastError());
}

// Generic entry: only the layout with both operands contraction-contiguous (opA 'N'/'R', opB 'T'/'C').
void zgemm_split(fc_ctx ctx, int precision, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
                 const z* B, long ldb, z beta, z* C, long ldc) {
  FC_REQUIRE((opA == 'N' || opA == 'R') && (opB == 'T' || opB == 'C'), FC_EUNSUPPORTED,
             "zgemm_split: operands must be contraction-contiguous");
  SplitOp sa = split_operand(ctx, precision, A, M, K, lda, opA == 'R');
  SplitOp sb = split_operand(ctx, precision, B, N, K, ldb, opB == 'C');
  gemm_split_nt(ctx, sa, 0, M, sb, 0, N, alpha, beta, C, ldc);
}

}  // namespace fc
