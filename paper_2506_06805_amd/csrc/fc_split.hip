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
// Tiles are 128 x 128 (8 waves of 64 x 32), K slices of 32, in LDS with an XOR chunk swizzle (see
// swz).  By default both operands go straight from global memory into LDS (k_gemm_split_dma: three
// A buffers and two B buffers, 160 KB); the register-staged kernel (k_gemm_split: two buffers,
// 128 KB, 32 staging registers per lane) serves the other tile shapes and gives the same bits.
// Either way one workgroup fits per CU, which is what the split-K count of skinny products is
// chosen for.
//
// MFMA 16x16x32 (bf16/f16) lane layout on gfx950 (measured): A fragment lane l holds
// A[row = l % 16][k = 8 (l / 16) + 0..7], B fragment B[k = 8 (l / 16) + 0..7][col = l % 16],
// accumulator register r holds D[row = 4 (l / 16) + r][col = l % 16].
#include <algorithm>
#include <cmath>
#include <cstring>

#include "fc_dma.hpp"
#include "fc_split.hpp"

namespace fc {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16;

constexpr int TM = 128, TK = 32;   // row padding unit of split operands (the largest tile), K slice
constexpr long SKB = 128;          // K batch of the per-batch power-of-two scales of FP16 operands
static_assert(SKB % 64 == 0, "a wave's columns must lie in one scale batch");
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
// The scale is 2^bexp[k / kb] when bexp is given (one power of two per K batch), else `scale`.
template <int PREC>
__global__ void k_split(const z* __restrict__ X, long rows, long K, long ldx, long rows_pad, long kp, double scale,
                        const int* __restrict__ bexp, long kb, int conj, u16* __restrict__ out) {
  const long total = rows_pad * kp, plane = rows_pad * kp;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    long r = t / kp, k = t % kp;
    z x = (r < rows && k < K) ? X[r * ldx + k] : make_double2(0.0, 0.0);
    const double sc = bexp ? ldexp(1.0, bexp[k / kb]) : scale;
    double re = x.x * sc, im = (conj ? -x.y : x.y) * sc;
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

// X[r * ldx + colmap[k]] (colmap[k] < 0 or k >= K: zero) -> planes [4][rows_pad][kp]: the operand
// with its contraction index permuted (the blocked pair order of the ladder contraction)
template <int PREC>
__global__ void k_split_cols(const z* __restrict__ X, long rows, long K, long ldx, const int* __restrict__ colmap,
                             long rows_pad, long kp, double scale, u16* __restrict__ out) {
  const long total = rows_pad * kp, plane = rows_pad * kp;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long r = t / kp, k = t % kp;
    const int c = (r < rows && k < K) ? colmap[k] : -1;
    const z x = c >= 0 ? X[r * ldx + c] : make_double2(0.0, 0.0);
    const double re = x.x * scale, im = x.y * scale;
    const u16 rh = to16<PREC>((float)re), ih = to16<PREC>((float)im);
    out[t] = rh;
    out[plane + t] = to16<PREC>((float)(re - from16<PREC>(rh)));
    out[2 * plane + t] = ih;
    out[3 * plane + t] = to16<PREC>((float)(im - from16<PREC>(ih)));
  }
}

// T1-dressed virtual Cholesky vectors straight into split planes (the operand of the ladder
// assembly): planes row a v + e, column P = split(s (L[a][e][P] - sum_m t[m][a] Lov[m][e][P])).
// One workgroup per (e, 64 columns of P): the o x 64 slice of Lov sits in LDS, thread t owns column
// P0 + t % 64, and wave w takes the a values 4 (w + 4 k) + 0..3, so that each L_ov value read from
// LDS feeds four products and the t1 values are the same across the wave.  Columns N <= P < kp are
// written as zeros.
template <int PREC>
__device__ inline void put_split(u16* out, long plane, long off, double re, double im) {
  const u16 rh = to16<PREC>((float)re), ih = to16<PREC>((float)im);
  out[off] = rh;
  out[plane + off] = to16<PREC>((float)(re - from16<PREC>(rh)));
  out[2 * plane + off] = ih;
  out[3 * plane + off] = to16<PREC>((float)(im - from16<PREC>(ih)));
}
template <int PREC, class T>
__global__ __launch_bounds__(256) void k_split_dressed(const T* __restrict__ L, const z* __restrict__ Lov,
                                                       const z* __restrict__ t1, long o, long v, long N, long kp,
                                                       long rows_pad, double scale0, const int* __restrict__ bexp,
                                                       long kb, u16* __restrict__ out) {
  extern __shared__ z sl[];   // [o][64]
  const long e = blockIdx.y, P = (long)blockIdx.x * 64 + (threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long plane = rows_pad * kp;
  if (t1) {
    for (long i = threadIdx.x; i < o * 64; i += blockDim.x) {
      const long m = i / 64, q = (long)blockIdx.x * 64 + (i % 64);
      sl[i] = q < N ? Lov[(m * v + e) * N + q] : make_double2(0.0, 0.0);
    }
    __syncthreads();
  }
  if (P >= kp) return;
  const double scale = bexp ? ldexp(1.0, bexp[P / kb]) : scale0;   // 2^bexp per K batch of P
  for (long a0 = 4 * w; a0 < v; a0 += 16) {
    double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    if (P < N) {
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (a0 + d < v) {
          const T x = L[((a0 + d) * v + e) * N + P];
          re[d] = x.x;
          im[d] = x.y;
        }
      if (t1) {
        for (long m = 0; m < o; ++m) {
          const z y = sl[m * 64 + (threadIdx.x & 63)];
#pragma unroll
          for (int d = 0; d < 4; ++d) {
            const z t = a0 + d < v ? t1[m * v + a0 + d] : make_double2(0.0, 0.0);
            re[d] -= t.x * y.x - t.y * y.y;
            im[d] -= t.x * y.y + t.y * y.x;
          }
        }
      }
    }
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (a0 + d < v) put_split<PREC>(out, plane, ((a0 + d) * v + e) * kp + P, re[d] * scale, im[d] * scale);
  }
}

template <class T>
__global__ void k_maxabs_t(const T* __restrict__ X, long n, unsigned* out) {
  __shared__ float s[256];
  float m = 0.f;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    m = fmaxf(m, fmaxf((float)fabs((double)X[t].x), (float)fabs((double)X[t].y)));
  s[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(s[0]));   // non-negative floats order as uints
}

// out[k / kb] = max |component| of X[r * ldx + k] over r < rows (one K batch per entry); the
// workgroups of blockIdx.y take rows_per rows each.  kb is a multiple of 64, so the 64 columns of
// a wave lie in one batch: the wave reduces its maximum first and one lane updates the batch
// (per-lane atomics on the few batch words serialise in L2).
template <class T>
__global__ void k_maxabs_kbatch(const T* __restrict__ X, long rows, long K, long ldx, long kb, long rows_per,
                                unsigned* __restrict__ out) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  const long r0 = (long)blockIdx.y * rows_per, r1 = r0 + rows_per < rows ? r0 + rows_per : rows;
  float m = 0.f;
  if (k < K)
    for (long r = r0; r < r1; ++r) {
      const T x = X[r * ldx + k];
      m = fmaxf(m, fmaxf((float)fabs((double)x.x), (float)fabs((double)x.y)));
    }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  const long k0 = k - (threadIdx.x & 63);   // the wave's first column
  if ((threadIdx.x & 63) == 0 && k0 < K) atomicMax(out + k0 / kb, __float_as_uint(m));   // non-negative floats order as uints
}

// planes[p][r][k] = 0 for k0 <= k < kp, every row r < rows_pad of the four planes
__global__ void k_zero_kpad(u16* __restrict__ planes, long rows_pad, long kp, long k0) {
  const long w = kp - k0, total = 4 * rows_pad * w;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long r = t / w;   // plane-major rows: r = p * rows_pad + row
    planes[r * kp + k0 + (t - r * w)] = 0;
  }
}

struct SArgs {
  const u16* A; long a_plane; long a_row0;   // planes of A, first row of this product
  const u16* B; long b_plane; long b_row0;
  long M, N, kp;
  z* C; long ldc;
  z alpha, beta;
  double inv_scale;
  // per-K-batch scales (FP16 operands): the products of batch b carry 2^(eA_b + eB_b), eA_b from
  // a_bexp (or the constant a_e when a_bexp is null), likewise for B; kb = 0: constant scales only
  const int* a_bexp; const int* b_bexp;
  long kb;
  int a_e, b_e;
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
template <int PREC>
__device__ inline f4 mma_r(const uint4& a, const uint4& b, f4 c) {
  if constexpr (PREC == FC_SPLIT_BF16)
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, a), __builtin_bit_cast(h8, b), c, 0, 0, 0);
}

// Output tile of one workgroup: WM x WN waves, each owning WTM x WTN outputs (BI x BJ blocks of
// 16 x 16).  Staging: the NT threads cover RP = NT / 4 rows of one plane per pass (four 16-byte
// chunks per 64-byte row), so an operand of TM rows takes PA = TM / RP passes per plane.
template <int WM_, int WN_, int WTM_, int WTN_>
struct STile {
  static constexpr int WM = WM_, WN = WN_, WTM = WTM_, WTN = WTN_;
  static constexpr int NT = 64 * WM * WN, TM = WM * WTM, TN = WN * WTN;
  static constexpr int BI = WTM / 16, BJ = WTN / 16, RP = NT / 4;
  static constexpr int PA = (TM + RP - 1) / RP, PB = (TN + RP - 1) / RP;
  static_assert(RP % 16 == 0, "staging passes must keep the row swizzle");
};
// 8 waves of 64 x 32 at two waves per SIMD (256 registers each)
using TileW8 = STile<2, 4, 64, 32>;
// 4 waves of 64 x 64 at one wave per SIMD: the accumulators go to the AGPRs, and each wave reads
// a third fewer LDS bytes per MFMA than a 64 x 32 wave
using TileW4 = STile<2, 2, 64, 64>;
// 4 waves of 64 x 48: 96-column outputs (pair counts near 3 x 96, such as 276)
using TileW4n96 = STile<2, 2, 64, 48>;
// 8 waves of 32 x 48 at two waves per SIMD: 128 x 96 outputs
using TileW8n96 = STile<4, 2, 32, 48>;

// Origin (m0, n0) of this workgroup's output tile; false when the tile is past the product or is a
// skipped tile of a triangular ladder launch.  XCD x (= blockIdx.x % 8) walks the contiguous tiles
// [x * per, (x + 1) * per); the split index rotates the slot so that the splits of one tile spread
// over all XCDs.
template <int EPI, int TMt, int TNt>
__device__ __forceinline__ bool split_tile_origin(const SArgs& g, long& m0, long& n0) {
  const long ntn = (g.N + TNt - 1) / TNt;
  const long per = (g.tiles + 7) / 8;
  const long bx = ((long)blockIdx.x + blockIdx.y) % gridDim.x;
  const long tile = (bx & 7) * per + (bx >> 3);
  if (tile >= g.tiles) return false;
  long mi = tile / ntn;
  if (EPI == 1 && g.ltri) {
    // triangular launches: fold the tile rows so every XCD's band mixes live and skipped tiles
    const long tm = g.tiles / ntn;
    mi = (mi & 1) ? tm - 1 - (mi >> 1) : (mi >> 1);
  }
  m0 = mi * TMt;
  n0 = (tile % ntn) * TNt;
  if (EPI == 1 && g.ltri) {
    const long amin = m0 / g.lv, bmax = (n0 + TNt - 1 < g.N ? n0 + TNt - 1 : g.N - 1) / g.lv;
    if (amin > bmax) return false;
  }
  return true;
}

// Output of a wave's BI x BJ blocks: C = alpha (rr - ii + i im) / 2^ecur + beta C, or the split-K
// partial sums, or the ladder's FP32 W (EPI = 1).
template <int EPI, int BI, int BJ>
__device__ __forceinline__ void split_epilogue(const SArgs& g, const f4 (&rr)[BI][BJ], const f4 (&ii)[BI][BJ],
                                               const f4 (&im)[BI][BJ], long m0, long n0, int wm, int wn, int lane,
                                               int ecur) {
  const int orow = 4 * (lane >> 4), ocol = lane & 15;
  const bool use_beta = (g.beta.x != 0.0 || g.beta.y != 0.0);
  const double inv_scale = g.kb > 0 ? ldexp(1.0, -ecur) : g.inv_scale;
  // ladder layout ((a nB + b) v + e) v + f as a row part plus a column part, one 32-bit division
  // per row or column of the lane
  long coff[BJ];
#pragma unroll
  for (int j = 0; j < BJ; ++j) {
    coff[j] = 0;
    if (EPI == 1) {
      const unsigned lv = (unsigned)g.lv;
      const unsigned n = (unsigned)(n0 + wn + 16 * j + ocol), b = n / lv;
      coff[j] = (long)b * g.lv * g.lv + (long)(n - b * lv);
    }
  }
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long m = m0 + wm + 16 * i + orow + r;
      long roff = 0;
      if (EPI == 1) {
        const unsigned mu = (unsigned)m, lv = (unsigned)g.lv, a = mu / lv;
        roff = ((long)a * g.lnB * g.lv + (long)(mu - a * lv)) * g.lv;
      }
#pragma unroll
      for (int j = 0; j < BJ; ++j) {
        const long n = n0 + wn + 16 * j + ocol;
        if (m >= g.M || n >= g.N) continue;
        double re = ((double)rr[i][j][r] - (double)ii[i][j][r]) * inv_scale, imv = (double)im[i][j][r] * inv_scale;
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

template <int PREC, int EPI, class TL>
__global__ __launch_bounds__(TL::NT) void k_gemm_split(SArgs g) {
  constexpr int TMt = TL::TM, TNt = TL::TN, BI = TL::BI, BJ = TL::BJ, RP = TL::RP;
  constexpr int PA = TL::PA, PB = TL::PB;
  // double-buffered planes of both operands
  __shared__ __attribute__((aligned(16))) u16 sA[2][4][TMt][LDK];
  __shared__ __attribute__((aligned(16))) u16 sB[2][4][TNt][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / TL::WN) * TL::WTM, wn = (wave % TL::WN) * TL::WTN;
  long m0, n0;
  if (!split_tile_origin<EPI, TMt, TNt>(g, m0, n0)) return;
  const long klo = (long)blockIdx.y * g.kchunk;
  const long khi = klo + g.kchunk < g.kp ? klo + g.kchunk : g.kp;
  const u16* A = g.A + (g.a_row0 + m0) * g.kp;
  const u16* B = g.B + (g.b_row0 + n0) * g.kp;

  // staging: thread t holds, for each plane and pass, the 16-byte chunk of row (t / 4) + RP pass
  // at k offset 8 (t % 4); rows past the tile (TM or TN not a multiple of RP, or below RP) are
  // neither loaded nor stored -- a store past the tile's rows would land in the next plane
  const int srow = tid >> 2, skc = 8 * (tid & 3);
  const long goff = (long)srow * g.kp + skc;
  const int sk = 8 * ((skc >> 3) ^ swz(srow));   // LDS column of this thread's staging chunk
  // named staging registers (arrays here end up in scratch or LDS): pass 0 and, for tiles wider
  // than one pass (PA or PB = 2), pass 1 of each plane
  static_assert(PA <= 2 && PB <= 2, "at most two staging passes per operand");
  uint4 a00, a10, a20, a30, a01, a11, a21, a31, b00, b10, b20, b30, b01, b11, b21, b31;
  const bool a0ok = TMt >= RP || srow < TMt, b0ok = TNt >= RP || srow < TNt;
  const bool a1ok = PA > 1 && (TMt % RP == 0 || srow + RP < TMt);
  const bool b1ok = PB > 1 && (TNt % RP == 0 || srow + RP < TNt);
  const long gq = (long)RP * g.kp;   // global offset of the second pass
#define FC_LD(dst, base, plane_stride, p, q, k0) \
  dst = *reinterpret_cast<const uint4*>((base) + (p) * (plane_stride) + goff + (q) * gq + (k0))
#define FC_SGLOAD(k0)                                                                      \
  do {                                                                                     \
    if (a0ok) {                                                                            \
      FC_LD(a00, A, g.a_plane, 0, 0, k0); FC_LD(a10, A, g.a_plane, 1, 0, k0);              \
      FC_LD(a20, A, g.a_plane, 2, 0, k0); FC_LD(a30, A, g.a_plane, 3, 0, k0);              \
    }                                                                                      \
    if (b0ok) {                                                                            \
      FC_LD(b00, B, g.b_plane, 0, 0, k0); FC_LD(b10, B, g.b_plane, 1, 0, k0);              \
      FC_LD(b20, B, g.b_plane, 2, 0, k0); FC_LD(b30, B, g.b_plane, 3, 0, k0);              \
    }                                                                                      \
    if (a1ok) {                                                                            \
      FC_LD(a01, A, g.a_plane, 0, 1, k0); FC_LD(a11, A, g.a_plane, 1, 1, k0);              \
      FC_LD(a21, A, g.a_plane, 2, 1, k0); FC_LD(a31, A, g.a_plane, 3, 1, k0);              \
    }                                                                                      \
    if (b1ok) {                                                                            \
      FC_LD(b01, B, g.b_plane, 0, 1, k0); FC_LD(b11, B, g.b_plane, 1, 1, k0);              \
      FC_LD(b21, B, g.b_plane, 2, 1, k0); FC_LD(b31, B, g.b_plane, 3, 1, k0);              \
    }                                                                                      \
  } while (0)
#define FC_ST(arr, buf, p, row, val) *reinterpret_cast<uint4*>(&arr[buf][p][row][sk]) = val
#define FC_SSTORE(buf)                                                                     \
  do {                                                                                     \
    if (a0ok) {                                                                            \
      FC_ST(sA, buf, 0, srow, a00); FC_ST(sA, buf, 1, srow, a10);                          \
      FC_ST(sA, buf, 2, srow, a20); FC_ST(sA, buf, 3, srow, a30);                          \
    }                                                                                      \
    if (b0ok) {                                                                            \
      FC_ST(sB, buf, 0, srow, b00); FC_ST(sB, buf, 1, srow, b10);                          \
      FC_ST(sB, buf, 2, srow, b20); FC_ST(sB, buf, 3, srow, b30);                          \
    }                                                                                      \
    if (a1ok) {                                                                            \
      FC_ST(sA, buf, 0, srow + RP, a01); FC_ST(sA, buf, 1, srow + RP, a11);                \
      FC_ST(sA, buf, 2, srow + RP, a21); FC_ST(sA, buf, 3, srow + RP, a31);                \
    }                                                                                      \
    if (b1ok) {                                                                            \
      FC_ST(sB, buf, 0, srow + RP, b01); FC_ST(sB, buf, 1, srow + RP, b11);                \
      FC_ST(sB, buf, 2, srow + RP, b21); FC_ST(sB, buf, 3, srow + RP, b31);                \
    }                                                                                      \
  } while (0)

  f4 rr[BI][BJ], ii[BI][BJ], im[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) { rr[i][j] = f4{0, 0, 0, 0}; ii[i][j] = f4{0, 0, 0, 0}; im[i][j] = f4{0, 0, 0, 0}; }

  const int lr = lane & 15, lk = 8 * ((lane >> 4) ^ swz(lr));
  // one barrier per K step: the loads of the next slice are issued before the products of this
  // one and stored to the other buffer after them
  if (klo < khi) {
    FC_SGLOAD(klo);
    FC_SSTORE(0);
  }
  __syncthreads();
  // per-K-batch scales: the sums are kept in units of the current batch's factor 2^ecur and
  // rescaled by a power of two (exact in FP32) where a new batch starts
  int ecur = 0;
  if (g.kb > 0)
    ecur = (g.a_bexp ? g.a_bexp[klo / g.kb] : g.a_e) + (g.b_bexp ? g.b_bexp[klo / g.kb] : g.b_e);
  int buf = 0;
  for (long k0 = klo; k0 < khi; k0 += TK, buf ^= 1) {
    const bool more = k0 + TK < khi;
    if (g.kb > 0 && k0 > klo && k0 % g.kb == 0) {
      const long b = k0 / g.kb;
      const int enew = (g.a_bexp ? g.a_bexp[b] : g.a_e) + (g.b_bexp ? g.b_bexp[b] : g.b_e);
      if (enew != ecur) {
        const float f = ldexpf(1.0f, enew - ecur);
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
          for (int j = 0; j < BJ; ++j) { rr[i][j] *= f; ii[i][j] *= f; im[i][j] *= f; }
        ecur = enew;
      }
    }
    if (more) FC_SGLOAD(k0 + TK);
    if constexpr (TL::NT == 512) {
      // two waves per SIMD: fragments read per block pair, the other wave covers the latency
#pragma unroll
      for (int i = 0; i < BI; ++i) {
        const int ra_ = wm + 16 * i + lr;
        const u16 *aRh = &sA[buf][0][ra_][lk], *aRl = &sA[buf][1][ra_][lk], *aIh = &sA[buf][2][ra_][lk],
                  *aIl = &sA[buf][3][ra_][lk];
#pragma unroll
        for (int j = 0; j < BJ; ++j) {
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
    } else {
      // one wave per SIMD: every fragment of the slice in registers first (hi planes, then lo), then
      // the products term by term so consecutive MFMAs feed different accumulators
      uint4 fa[4][BI], fb[4][BJ];
#pragma unroll
      for (int pp = 0; pp < 4; ++pp) {
        const int p = ((pp & 1) << 1) | (pp >> 1);   // 0, 2, 1, 3: the hi planes first
#pragma unroll
        for (int i = 0; i < BI; ++i) fa[p][i] = *reinterpret_cast<const uint4*>(&sA[buf][p][wm + 16 * i + lr][lk]);
#pragma unroll
        for (int j = 0; j < BJ; ++j) fb[p][j] = *reinterpret_cast<const uint4*>(&sB[buf][p][wn + 16 * j + lr][lk]);
      }
      // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo; terms hi*hi, hi*lo, lo*hi
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int pa = t == 2 ? 1 : 0, pb = t == 1 ? 1 : 0;   // plane offsets of the lo factor
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
          for (int j = 0; j < BJ; ++j) {
            rr[i][j] = mma_r<PREC>(fa[0 + pa][i], fb[0 + pb][j], rr[i][j]);
            ii[i][j] = mma_r<PREC>(fa[2 + pa][i], fb[2 + pb][j], ii[i][j]);
            im[i][j] = mma_r<PREC>(fa[0 + pa][i], fb[2 + pb][j], im[i][j]);
            im[i][j] = mma_r<PREC>(fa[2 + pa][i], fb[0 + pb][j], im[i][j]);
          }
      }
    }
    if (more) FC_SSTORE(buf ^ 1);
    __syncthreads();
  }

  split_epilogue<EPI, BI, BJ>(g, rr, ii, im, m0, n0, wm, wn, lane, ecur);
}
#undef FC_SGLOAD
#undef FC_SSTORE
#undef FC_LD
#undef FC_ST

// The same product with both operands staged by direct-to-LDS loads (8-wave tiles, 128 rows of A).
// The register-staged kernel loads slice k + 1 while slice k's products run, through 32 staging
// registers per lane; the loads of a slice then have one slice of products to land, and the
// workgroup barrier waits for the slowest of its waves.  Here the loads bypass the registers and
// run further ahead: A rotates through three LDS buffers (slice k + 3 is requested at the end of
// slice k, into the buffer slice k has just left), B through two (slice k + 2 is requested once
// every wave holds slice k's B fragments in registers, after the slice's first twelve of its 96
// products per wave).  LDS: 3 x 32 KiB
// of A + 2 x 32 KiB of B = 160 KiB.  The layout in LDS is the register-staged kernel's (rows of
// 32 elements, 16-byte chunks XOR-swizzled by swz(row)): a 1 KiB run is 16 rows of one plane, lane
// l fetching row l / 4 and the chunk that belongs at position l % 4.  Fragments: B's of a whole
// slice and A's of one 16-row block, read one block ahead of the products; the MFMA order per
// accumulator is the register-staged kernel's, so both give the same bits.
template <int PREC, int EPI, class TL>
__global__ __launch_bounds__(TL::NT) void k_gemm_split_dma(SArgs g) {
  static_assert(TL::NT == 512 && TL::BI == 4 && TL::BJ == 2, "8 waves of 64 x 32");
  constexpr int TMt = TL::TM, TNt = TL::TN, BI = TL::BI, BJ = TL::BJ;
  constexpr int QA = 4, QB = 4;   // loads per wave and slice: one 16-row run of each plane
  static_assert(TMt == 16 * (TL::NT / 64) && TNt == 16 * (TL::NT / 64), "one 16-row block of each operand per wave");
  __shared__ __attribute__((aligned(16))) u16 sA[3][4][TMt][LDK];
  __shared__ __attribute__((aligned(16))) u16 sB[2][4][TNt][LDK];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = (wave / TL::WN) * TL::WTM, wn = (wave % TL::WN) * TL::WTN;
  long m0, n0;
  if (!split_tile_origin<EPI, TMt, TNt>(g, m0, n0)) return;
  const long klo = (long)blockIdx.y * g.kchunk;
  const long khi = klo + g.kchunk < g.kp ? klo + g.kchunk : g.kp;
  const int nk = khi > klo ? (int)((khi - klo) / TK) : 0;   // kchunk and kp are multiples of TK

  // wave w moves rows 16 w + 0..15 of each of the four planes of both operands (one 1 KiB run per
  // plane): lane l fetches row 16 w + l / 4, the chunk that belongs at position l % 4
  const int lrow = lane >> 2, lchunk = 8 * ((lane & 3) ^ swz(lrow));
  const u16* pa = g.A + (g.a_row0 + m0 + 16 * wave + lrow) * g.kp + klo + lchunk;
  const u16* pb = g.B + (g.b_row0 + n0 + 16 * wave + lrow) * g.kp + klo + lchunk;
#define FC_DMA_A(s, slot)                                                                           \
  _Pragma("unroll") for (int q = 0; q < 4; ++q)                                                     \
    lds_dma16(pa + q * g.a_plane + (long)(s) * TK, &sA[slot][q][16 * wave][0])
#define FC_DMA_B(s, slot)                                                                           \
  _Pragma("unroll") for (int q = 0; q < 4; ++q)                                                     \
    lds_dma16(pb + q * g.b_plane + (long)(s) * TK, &sB[slot][q][16 * wave][0])

  const int lr = lane & 15, lk = 8 * ((lane >> 4) ^ swz(lr));
#define FC_RD_A(slot, i, F) \
  _Pragma("unroll") for (int p = 0; p < 4; ++p) F[p] = *reinterpret_cast<const uint4*>(&sA[slot][p][wm + 16 * (i) + lr][lk])
#define FC_RD_BJ(slot, j, F) \
  _Pragma("unroll") for (int p = 0; p < 4; ++p) F[p][j] = *reinterpret_cast<const uint4*>(&sB[slot][p][wn + 16 * (j) + lr][lk])
  // planes 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo; terms hi*hi, hi*lo, lo*hi
#define FC_PROD_J(i, j, FA, FB)                                                                     \
  do {                                                                                              \
    rr[i][j] = mma_r<PREC>(FA[0], FB[0][j], rr[i][j]);                                              \
    rr[i][j] = mma_r<PREC>(FA[0], FB[1][j], rr[i][j]);                                              \
    rr[i][j] = mma_r<PREC>(FA[1], FB[0][j], rr[i][j]);                                              \
    ii[i][j] = mma_r<PREC>(FA[2], FB[2][j], ii[i][j]);                                              \
    ii[i][j] = mma_r<PREC>(FA[2], FB[3][j], ii[i][j]);                                              \
    ii[i][j] = mma_r<PREC>(FA[3], FB[2][j], ii[i][j]);                                              \
    im[i][j] = mma_r<PREC>(FA[0], FB[2][j], im[i][j]);                                              \
    im[i][j] = mma_r<PREC>(FA[0], FB[3][j], im[i][j]);                                              \
    im[i][j] = mma_r<PREC>(FA[1], FB[2][j], im[i][j]);                                              \
    im[i][j] = mma_r<PREC>(FA[2], FB[0][j], im[i][j]);                                              \
    im[i][j] = mma_r<PREC>(FA[2], FB[1][j], im[i][j]);                                              \
    im[i][j] = mma_r<PREC>(FA[3], FB[0][j], im[i][j]);                                              \
  } while (0)
#define FC_PROD(i, FA, FB) _Pragma("unroll") for (int j = 0; j < BJ; ++j) FC_PROD_J(i, j, FA, FB)

  f4 rr[BI][BJ], ii[BI][BJ], im[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) { rr[i][j] = f4{0, 0, 0, 0}; ii[i][j] = f4{0, 0, 0, 0}; im[i][j] = f4{0, 0, 0, 0}; }
  int ecur = 0;
  if (g.kb > 0)
    ecur = (g.a_bexp ? g.a_bexp[klo / g.kb] : g.a_e) + (g.b_bexp ? g.b_bexp[klo / g.kb] : g.b_e);

  // fragments: fb the B columns of the current slice (block j = 1 of the next slice arrives while
  // the first products of that slice run), fa0 / fa1 A row blocks, one block ahead of the products
  uint4 fa0[4], fa1[4], fb[4][BJ];
  if (nk > 0) {
    // slices 0 and 1 of both operands and slice 2 of A; then wait for slice 0
    FC_DMA_A(0, 0);
    FC_DMA_B(0, 0);
    if (nk > 1) { FC_DMA_A(1, 1); FC_DMA_B(1, 1); }
    if (nk > 2) {
      FC_DMA_A(2, 2);
      asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(2 * QA + QB) : "memory");
    } else if (nk > 1) {
      asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(QA + QB) : "memory");
    } else {
      asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
    }
    _Pragma("unroll") for (int j = 0; j < BJ; ++j) FC_RD_BJ(0, j, fb);
    FC_RD_A(0, 0, fa0);
  }
  int sa = 0, sb = 0;
  for (int kt = 0; kt < nk; ++kt) {
    const long k0 = klo + (long)TK * kt;
    if (g.kb > 0 && kt > 0 && k0 % g.kb == 0) {
      // FP16 operands: the sums move to the scale of the K batch that starts here (a uniform index,
      // so the exponents come through the scalar cache and no wait touches the loads in flight)
      typedef const __attribute__((address_space(4))) int* cint_p;   // read-only: scalar loads
      const int b = __builtin_amdgcn_readfirstlane((int)(k0 / g.kb));
      const int enew = (g.a_bexp ? ((cint_p)g.a_bexp)[b] : g.a_e) + (g.b_bexp ? ((cint_p)g.b_bexp)[b] : g.b_e);
      if (enew != ecur) {
        const float f = ldexpf(1.0f, enew - ecur);
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
          for (int j = 0; j < BJ; ++j) { rr[i][j] *= f; ii[i][j] *= f; im[i][j] *= f; }
        ecur = enew;
      }
    }
    const int san = sa == 2 ? 0 : sa + 1, sbn = sb ^ 1;
    FC_RD_A(sa, 1, fa1);
    __builtin_amdgcn_sched_barrier(0);
    FC_PROD_J(0, 0, fa0, fb);
    __builtin_amdgcn_sched_barrier(0);
    // every wave holds slice kt's B fragments: their buffer takes slice kt + 2
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 2 < nk) FC_DMA_B(kt + 2, sb);
    __builtin_amdgcn_sched_barrier(0);
    FC_PROD_J(0, 1, fa0, fb);
    __builtin_amdgcn_sched_barrier(0);
    FC_RD_A(sa, 2, fa0);
    __builtin_amdgcn_sched_barrier(0);
    FC_PROD(1, fa1, fb);
    __builtin_amdgcn_sched_barrier(0);
    FC_RD_A(sa, 3, fa1);
    __builtin_amdgcn_sched_barrier(0);
    FC_PROD(2, fa0, fb);
    __builtin_amdgcn_sched_barrier(0);
    // own loads of slice kt + 1 landed (those of kt + 2 may still run) and own reads of slice kt
    // done; then every wave's: slice kt's A buffer takes slice kt + 3.  The next slice's fragments
    // are read even after the last slice (stale LDS, unused): a read on one path only would make
    // the compiler wait for it before the products below.
    if (kt + 2 < nk) asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(QA + QB) : "memory");
    else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
    if (kt + 3 < nk) FC_DMA_A(kt + 3, sa);
    FC_RD_A(san, 0, fa0);
    __builtin_amdgcn_sched_barrier(0);
    // the last row block's products, each B column block followed by the next slice's copy of it
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      FC_PROD_J(3, j, fa1, fb);
      __builtin_amdgcn_sched_barrier(0);
      FC_RD_BJ(sbn, j, fb);
      __builtin_amdgcn_sched_barrier(0);
    }
    sa = san;
    sb = sbn;
  }
#undef FC_PROD
#undef FC_PROD_J
#undef FC_RD_A
#undef FC_RD_BJ
#undef FC_DMA_A
#undef FC_DMA_B
  split_epilogue<EPI, BI, BJ>(g, rr, ii, im, m0, n0, wm, wn, lane, ecur);
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
template <int EPI, class TL, bool DMA = false>
void launch_split_t(int prec, dim3 grid, const SArgs& g, hipStream_t st) {
  if constexpr (DMA) {
    if (prec == FC_SPLIT_BF16) k_gemm_split_dma<FC_SPLIT_BF16, EPI, TL><<<grid, TL::NT, 0, st>>>(g);
    else k_gemm_split_dma<FC_SPLIT_FP16, EPI, TL><<<grid, TL::NT, 0, st>>>(g);
  } else {
    if (prec == FC_SPLIT_BF16) k_gemm_split<FC_SPLIT_BF16, EPI, TL><<<grid, TL::NT, 0, st>>>(g);
    else k_gemm_split<FC_SPLIT_FP16, EPI, TL><<<grid, TL::NT, 0, st>>>(g);
  }
  FC_HIP(hipGetLastError());
}
}  // namespace

// Tile of a split product: 0 = 8 waves of 64 x 32 (128 x 128), 1 = 4 waves of 64 x 64 (128 x 128),
// 2 = 4 waves of 64 x 48 (128 x 96), 3 = 8 waves of 32 x 48 (128 x 96), 4 = tile 0 staged by
// direct-to-LDS loads.  The 96-wide tiles serve output widths that 96 pads much less than 128.
// n = 0: the ladder assembly (any width).  The context's staging choice (fc_set_split_config:
// 0 register-staged 8 waves, 1 four waves, 2 direct-to-LDS 8 waves), else FNSCC_SPLIT_TILE (the
// same numbers), overrides the default for the 128-wide outputs.
int split_tile_cfg(fc_ctx ctx, long n) {
  static const int env = [] {
    const char* e = getenv("FNSCC_SPLIT_TILE");
    const int v = e ? atoi(e) : -1;
    return v >= 0 && v < FC_SPLIT_NUM_CONFIGS ? v : -1;
  }();
  const int pick = ctx->split_cfg >= 0 ? ctx->split_cfg : env >= 0 ? env : FC_SPLIT_DEFAULT_CONFIG;
  const int base = pick == 1 ? 1 : pick == 2 ? 4 : 0;
  // 96-wide tiles when they pad at least 15% less than 128-wide ones (N = 276: 288 against 384)
  if (n > 96 && 100 * ((n + 95) / 96 * 96) < 85 * ((n + 127) / 128 * 128)) return base == 1 ? 2 : 3;
  return base;
}
long tile_tn(int cfg) { return (cfg == 2 || cfg == 3) ? 96 : 128; }
template <int EPI>
void launch_split(int cfg, int prec, dim3 grid, const SArgs& g, hipStream_t st) {
  if (cfg == 4) launch_split_t<EPI, TileW8, true>(prec, grid, g, st);
  else if (cfg == 1) launch_split_t<EPI, TileW4>(prec, grid, g, st);
  else if (cfg == 2) launch_split_t<EPI, TileW4n96>(prec, grid, g, st);
  else if (cfg == 3) launch_split_t<EPI, TileW8n96>(prec, grid, g, st);
  else launch_split_t<EPI, TileW8>(prec, grid, g, st);
}

// Per-K-batch maxima of |X[r * ldx + k]| (r < rows, k < K), batches of SKB, copied to the host.
template <class T>
static std::vector<double> kbatch_maxabs(fc_ctx ctx, const T* X, long rows, long K, long ldx, long nbatch) {
  std::vector<double> out((size_t)nbatch, 0.0);
  if (rows <= 0 || K <= 0) return out;
  DBuf mx(ctx, sizeof(unsigned) * (size_t)nbatch);
  FC_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned) * (size_t)nbatch, ctx->stream));
  const long rows_per = std::max(1L, (rows + 255) / 256);   // at most 256 row groups
  const dim3 grid((unsigned)((K + 255) / 256), (unsigned)((rows + rows_per - 1) / rows_per));
  k_maxabs_kbatch<T><<<grid, 256, 0, ctx->stream>>>(X, rows, K, ldx, SKB, rows_per, mx.as<unsigned>());
  FC_HIP(hipGetLastError());
  std::vector<unsigned> h((size_t)nbatch);
  FC_HIP(hipMemcpyAsync(h.data(), mx.p, sizeof(unsigned) * (size_t)nbatch, hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  for (long b = 0; b < nbatch; ++b) {
    float m;
    std::memcpy(&m, &h[(size_t)b], sizeof(m));
    out[(size_t)b] = m;
  }
  return out;
}

// One power-of-two scale per K batch of an FP16 operand: e_b = 13 - ilogb(bound_b), so that the
// batch's largest |x| maps into [2^13, 2^14) -- hi parts far below the FP16 maximum, lo parts
// (~2^-11 of hi) normal down to ~1e-4 of that batch's largest entry, whatever the batch's size
// relative to the others (Cholesky vectors decay over P).  A batch with no nonzero entry takes its
// neighbour's exponent, so no rescale happens there.  Exponents stay within 40 of the smallest, so
// that a product's FP32 sums, rescaled by 2^(eA + eB) differences at batch boundaries, stay far
// from overflow (entries more than 2^40 below their operand's largest keep fewer bits).
static void set_batch_scales(fc_ctx ctx, SplitOp& s, const std::vector<double>& bound) {
  const long nb = (long)bound.size();
  std::vector<int> e((size_t)nb, 0);
  long first = -1;
  int emin = 0;
  for (long b = 0; b < nb; ++b)
    if (bound[(size_t)b] > 0) {
      e[(size_t)b] = std::max(-200, std::min(200, 13 - std::ilogb(bound[(size_t)b])));
      emin = first < 0 ? e[(size_t)b] : std::min(emin, e[(size_t)b]);
      if (first < 0) first = b;
    }
  for (long b = 0; b < nb; ++b) {
    if (bound[(size_t)b] > 0) e[(size_t)b] = std::min(e[(size_t)b], emin + 40);
    else if (b > 0) e[(size_t)b] = e[(size_t)b - 1];
  }
  for (long b = 0; b < first; ++b) e[(size_t)b] = e[(size_t)first];
  s.bexp = DBuf(ctx, sizeof(int) * (size_t)nb);
  FC_HIP(hipMemcpyAsync(s.bexp.p, e.data(), sizeof(int) * (size_t)nb, hipMemcpyHostToDevice, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  s.kb = SKB;
  s.scale = 1.0;
}

SplitOp split_operand(fc_ctx ctx, int prec, const z* X, long rows, long K, long ldx, bool conj) {
  FC_REQUIRE(prec == FC_SPLIT_BF16 || prec == FC_SPLIT_FP16, FC_EARG, "split_operand: bad precision");
  SplitOp s;
  s.prec = prec;
  s.rows = rows;
  s.rows_pad = (rows + TM - 1) / TM * TM + TM;   // one spare zero tile for row-offset products
  s.kp = std::max<long>(TK, (K + TK - 1) / TK * TK);
  s.scale = 1.0;
  // FP16 (5 exponent bits): one power-of-two scale per K batch; BF16 keeps FP32's exponent range
  if (prec == FC_SPLIT_FP16 && rows > 0 && K > 0)
    set_batch_scales(ctx, s, kbatch_maxabs(ctx, X, rows, K, ldx, (s.kp + SKB - 1) / SKB));
  s.buf = DBuf(ctx, sizeof(u16) * 4 * (size_t)s.rows_pad * s.kp);
  const long total = s.rows_pad * s.kp;
  unsigned nb = (unsigned)std::max(1L, std::min(1048576L, (total + 1023) / 1024));
  const int* be = s.kb > 0 ? s.bexp.as<int>() : nullptr;
  if (prec == FC_SPLIT_BF16)
    k_split<FC_SPLIT_BF16><<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, s.rows_pad, s.kp, s.scale, be, s.kb, (int)conj,
                                                        s.buf.as<u16>());
  else
    k_split<FC_SPLIT_FP16><<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, s.rows_pad, s.kp, s.scale, be, s.kb, (int)conj,
                                                        s.buf.as<u16>());
  FC_HIP(hipGetLastError());
  return s;
}

template <class T>
static float device_maxabs(fc_ctx ctx, const T* X, long n) {
  if (n <= 0) return 0.f;
  DBuf mx(ctx, sizeof(unsigned));
  FC_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned), ctx->stream));
  const unsigned nb = (unsigned)std::max(1L, std::min(2048L, (n + 255) / 256));
  k_maxabs_t<T><<<nb, 256, 0, ctx->stream>>>(X, n, mx.as<unsigned>());
  FC_HIP(hipGetLastError());
  unsigned h = 0;
  FC_HIP(hipMemcpyAsync(&h, mx.p, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  float m;
  std::memcpy(&m, &h, sizeof(m));
  return m;
}

SplitOp split_operand_cols(fc_ctx ctx, int prec, const z* X, long rows, long K, long ldx, const int* colmap) {
  FC_REQUIRE(prec == FC_SPLIT_BF16 || prec == FC_SPLIT_FP16, FC_EARG, "split_operand_cols: bad precision");
  SplitOp s;
  s.prec = prec;
  s.rows = rows;
  s.rows_pad = (rows + TM - 1) / TM * TM + TM;
  s.kp = std::max<long>(TK, (K + TK - 1) / TK * TK);
  s.scale = 1.0;
  if (prec == FC_SPLIT_FP16) {
    // the permutation leaves the largest entry unchanged
    const float m = rows > 0 && K > 0 ? device_maxabs(ctx, X, rows * ldx) : 0.f;
    if (m > 0) s.scale = std::ldexp(1.0, 13 - std::ilogb((double)m));
  }
  s.buf = DBuf(ctx, sizeof(u16) * 4 * (size_t)s.rows_pad * s.kp);
  const long total = s.rows_pad * s.kp;
  const unsigned nb = (unsigned)std::max(1L, std::min(1048576L, (total + 1023) / 1024));
  if (prec == FC_SPLIT_BF16)
    k_split_cols<FC_SPLIT_BF16><<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, colmap, s.rows_pad, s.kp, s.scale, s.buf.as<u16>());
  else
    k_split_cols<FC_SPLIT_FP16><<<nb, 256, 0, ctx->stream>>>(X, rows, K, ldx, colmap, s.rows_pad, s.kp, s.scale, s.buf.as<u16>());
  FC_HIP(hipGetLastError());
  return s;
}

SplitOp split_lvv_dressed(fc_ctx ctx, int prec, const void* L, bool l_c64, const z* Lov, const z* t1, long o, long v,
                          long N) {
  FC_REQUIRE(prec == FC_SPLIT_BF16 || prec == FC_SPLIT_FP16, FC_EARG, "split_lvv_dressed: bad precision");
  FC_REQUIRE(!t1 || o <= 64, FC_EUNSUPPORTED, "split_lvv_dressed: dressing needs o <= 64 (LDS slice of L_ov)");
  SplitOp s;
  s.prec = prec;
  s.rows = v * v;
  s.rows_pad = (s.rows + TM - 1) / TM * TM + TM;
  s.kp = std::max<long>(TK, (N + TK - 1) / TK * TK);
  s.scale = 1.0;
  if (prec == FC_SPLIT_FP16) {
    // per K batch of P: |L_ae - sum_m t_m^a L_me| <= max|L_vv| + max_a sum_m |t_m^a| max|L_ov|
    const long nb = (s.kp + SKB - 1) / SKB;
    std::vector<double> bound = l_c64 ? kbatch_maxabs(ctx, (const float2*)L, v * v, N, N, nb)
                                      : kbatch_maxabs(ctx, (const z*)L, v * v, N, N, nb);
    if (t1) {
      std::vector<z> th((size_t)o * v);
      FC_HIP(hipMemcpyAsync(th.data(), t1, sizeof(z) * o * v, hipMemcpyDeviceToHost, ctx->stream));
      FC_HIP(hipStreamSynchronize(ctx->stream));
      double tmax = 0;
      for (long a = 0; a < v; ++a) {
        double sa = 0;
        for (long m = 0; m < o; ++m) sa += std::hypot(th[m * v + a].x, th[m * v + a].y);
        tmax = std::max(tmax, sa);
      }
      const std::vector<double> mo = kbatch_maxabs(ctx, Lov, o * v, N, N, nb);
      for (long b = 0; b < nb; ++b) bound[(size_t)b] += tmax * mo[(size_t)b] * std::sqrt(2.0);
    }
    set_batch_scales(ctx, s, bound);
  }
  s.buf = DBuf(ctx, sizeof(u16) * 4 * (size_t)s.rows_pad * s.kp);
  // rows past v^2 are padding: zero them (the columns past N are zeroed by the kernel)
  const size_t plane = (size_t)s.rows_pad * s.kp;
  for (int p = 0; p < 4; ++p)
    FC_HIP(hipMemsetAsync(s.buf.as<u16>() + p * plane + (size_t)s.rows * s.kp, 0,
                          sizeof(u16) * (size_t)(s.rows_pad - s.rows) * s.kp, ctx->stream));
  const dim3 grid((unsigned)((s.kp + 63) / 64), (unsigned)v);
  const size_t shm = t1 ? sizeof(z) * 64 * (size_t)o : 0;
  const int* be = s.kb > 0 ? s.bexp.as<int>() : nullptr;
  if (prec == FC_SPLIT_BF16) {
    if (l_c64)
      k_split_dressed<FC_SPLIT_BF16, float2><<<grid, 256, shm, ctx->stream>>>(
          (const float2*)L, Lov, t1, o, v, N, s.kp, s.rows_pad, s.scale, be, s.kb, s.buf.as<u16>());
    else
      k_split_dressed<FC_SPLIT_BF16, double2><<<grid, 256, shm, ctx->stream>>>(
          (const double2*)L, Lov, t1, o, v, N, s.kp, s.rows_pad, s.scale, be, s.kb, s.buf.as<u16>());
  } else {
    if (l_c64)
      k_split_dressed<FC_SPLIT_FP16, float2><<<grid, 256, shm, ctx->stream>>>(
          (const float2*)L, Lov, t1, o, v, N, s.kp, s.rows_pad, s.scale, be, s.kb, s.buf.as<u16>());
    else
      k_split_dressed<FC_SPLIT_FP16, double2><<<grid, 256, shm, ctx->stream>>>(
          (const double2*)L, Lov, t1, o, v, N, s.kp, s.rows_pad, s.scale, be, s.kb, s.buf.as<u16>());
  }
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

// Scale fields of a split product: per-K-batch exponents of either operand, else the operands'
// constant power-of-two scales folded into inv_scale.
static void set_scales(SArgs& g, const SplitOp& A, const SplitOp& B) {
  FC_REQUIRE(A.kb == 0 || B.kb == 0 || A.kb == B.kb, FC_EARG, "split product: operands batch K differently");
  g.kb = A.kb > 0 ? A.kb : B.kb;
  g.a_bexp = A.kb > 0 ? A.bexp.as<int>() : nullptr;
  g.b_bexp = B.kb > 0 ? B.bexp.as<int>() : nullptr;
  g.a_e = std::ilogb(A.scale);   // constant scales are powers of two
  g.b_e = std::ilogb(B.scale);
  g.inv_scale = 1.0 / (A.scale * B.scale);
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
  set_scales(g, A, B);
  const int tcfg = split_tile_cfg(ctx, N);
  const long tiles = ((M + 127) / 128) * ((N + tile_tn(tcfg) - 1) / tile_tn(tcfg));
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
  launch_split<0>(tcfg, A.prec, grid, g, ctx->stream);
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
  set_scales(g, A, B);
  const int tcfg = split_tile_cfg(ctx, 0);
  g.tiles = ((M + 127) / 128) * ((N + tile_tn(tcfg) - 1) / tile_tn(tcfg));
  g.kchunk = A.kp;
  g.part = nullptr;
  g.W = W; g.lv = lep.v; g.lnB = lep.nB; g.ltri = lep.triangular;
  dim3 grid((unsigned)((g.tiles + 7) / 8 * 8), 1);
  launch_split<1>(tcfg, A.prec, grid, g, ctx->stream);
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
