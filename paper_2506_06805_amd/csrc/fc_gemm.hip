// Complex GEMM on the FP64 matrix cores of gfx950.
//
// A complex product is four real products on the matrix cores (the "4M" form):
//   Cre += Are*Bre - Aim*Bim,   Cim += Are*Bim + Aim*Bre
// or Gauss's three (3M): Are*Bre, Aim*Bim and (Are + Aim)(Bre + Bim), giving Cre = P1 - P2 and
// Cim = P3 - P1 - P2.  3M issues a quarter fewer products; its error bound has the same form with
// (|Are| + |Aim|)(|Bre| + |Bim|) in place of |A||B| (Higham, "Stability of a method for multiplying
// complex matrices with three real matrix multiplications", SIAM J. Matrix Anal. Appl. 13, 1992).
// FP32 arithmetic (the mixed-precision residual) always uses 3M on v_mfma_f32_16x16x4f32; FP64
// (v_mfma_f64_16x16x4f64) uses 3M on its large products and 4M on the rest.
//
// Register-staged tiles: operands staged through LDS as interleaved complex rows, conjugation
// applied at staging time, double-buffered so the next K slice loads while the current one feeds
// the matrix cores; shapes 64 x 64 (4 waves of 32 x 32), 128 x 64 (4 waves of 64 x 32) and
// 128 x 128 (8 waves of 64 x 32), with K slices of 8 or 16 per pipeline step.  FP64 tiles staged by
// direct-to-LDS loads: 128 x 128 (4M) and 128 x 64 (3M, 8 waves of 32 x 32, K slices of 8 or 16),
// three buffers.  A heuristic or the autotuner picks one per product shape.  Workgroups are numbered so that each of the 8 XCDs walks a contiguous band
// of output tiles (consecutive tiles share a row of A in that XCD's L2).
//
// MFMA f64 16x16x4 lane layout (lane l of a 64-wide wave):
//   A fragment: A[row = l % 16][k = l / 16];  B fragment: B[k = l / 16][col = l % 16];
//   accumulator register r: D[row = l / 16 + 4 * r][col = l % 16]  (measured on gfx950).
#include <algorithm>
#include <cstring>
#include <mutex>

#include "fc_internal.hpp"
#include "fc_gemm.hpp"
#include "fc_dma.hpp"

namespace fc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Matrix-core arithmetic of a tile: FP64 (v_mfma_f64_16x16x4f64) or FP32 (v_mfma_f32_16x16x4f32),
// both 16 x 16 x 4 with one element of each operand per lane.  row(lk, r): output row of
// accumulator register r in lane group lk = lane / 16 (column = lane % 16).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
  using acc = d4;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct Mfma<float> {
  using acc = f4;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

constexpr int KQ = 16;     // K chunks of split products are multiples of this (and of every K slice)
constexpr int PADF = 2;    // LDS row padding of the FP32 complex rows (elements of 8 bytes)
constexpr int PADZ = 1;    // LDS row padding of the FP64 complex rows (elements of 16 bytes)

struct GemmArgs {
  long M, N, K;
  const z* A; long lda; long sA;
  const z* B; long ldb; long sB;
  z* C; long ldc; long sC;
  z alpha, beta;
  int conjA, conjB;
  long kchunk;        // K range per split (multiple of KQ); blockIdx.y selects the split
  z* part;            // split-K partial products [split][M][N] (nullptr: write C directly)
  long tiles;         // number of output tiles
  // ladder epilogue: C row m = (a - a0) v + e, column n = (b - b0) v + f is written to
  // C[((m / v) nB + n / v) v^2 + (m % v) v + n % v]; tiles with every a > every b are skipped
  long lv, lnB;
  int ltri;
  int omap;           // EPI 0: C laid out by `om` instead of row-major with ldc
  OutMap om;
};

// blockIdx -> tile so that XCD x (= bid % 8) owns the contiguous tiles [x * per, (x + 1) * per)
__device__ inline long xcd_tile(long bid, long tiles) {
  const long per = (tiles + 7) / 8;
  return (bid & 7) * per + (bid >> 3);
}

// K slice BK (complex elements) staged per step in the arithmetic type T, double-buffered.
// FP32: interleaved complex rows of 8-byte elements padded by two, so that the staging stores of a
// K-contiguous operand (8 K rows x 2 columns per 16 lanes) fall on distinct bank pairs.
template <int BM, int BN, int BK, typename T = double>
struct TileSmem {
  __attribute__((aligned(8))) float2 A[2][BK][BM + PADF];
  __attribute__((aligned(8))) float2 B[2][BK][BN + PADF];
  // cj: conjugate (the sign flip follows the rounding to FP32, so no FP64 multiply is needed)
  __device__ __forceinline__ void putA(int b, int k, int m, z v, bool cj) {
    const float im = (float)v.y;
    A[b][k][m] = make_float2((float)v.x, cj ? -im : im);
  }
  __device__ __forceinline__ void putB(int b, int k, int n, z v, bool cj) {
    const float im = (float)v.y;
    B[b][k][n] = make_float2((float)v.x, cj ? -im : im);
  }
  __device__ __forceinline__ void getA(int b, int k, int m, T& re, T& im) const {
    const float2 v = A[b][k][m];
    re = v.x; im = v.y;
  }
  __device__ __forceinline__ void getB(int b, int k, int n, T& re, T& im) const {
    const float2 v = B[b][k][n];
    re = v.x; im = v.y;
  }
};
// FP64: interleaved complex rows of 16-byte elements, one read yields the real and the imaginary
// part.  Rows of BM + 1 elements put the 8 K rows of a K-contiguous operand's staging store on
// distinct banks; fragment reads take 16 consecutive elements of one row.  (Measured on gfx950:
// bank-conflict cycles of a 4096^3 product 470M with split planes, 268M with a pad of 2, 201M with
// a pad of 1 or 3.)
template <int BM, int BN, int BK>
struct TileSmem<BM, BN, BK, double> {
  __attribute__((aligned(16))) z A[2][BK][BM + PADZ];
  __attribute__((aligned(16))) z B[2][BK][BN + PADZ];
  __device__ __forceinline__ void putA(int b, int k, int m, z v, bool cj) { A[b][k][m] = make_double2(v.x, cj ? -v.y : v.y); }
  __device__ __forceinline__ void putB(int b, int k, int n, z v, bool cj) { B[b][k][n] = make_double2(v.x, cj ? -v.y : v.y); }
  __device__ __forceinline__ void getA(int b, int k, int m, double& re, double& im) const {
    const z v = A[b][k][m];
    re = v.x; im = v.y;
  }
  __device__ __forceinline__ void getB(int b, int k, int n, double& re, double& im) const {
    const z v = B[b][k][n];
    re = v.x; im = v.y;
  }
};

// Source of the elements outside a product for loads that must issue on every path (the
// direct-to-LDS tiles and the FP32 two-slice pipeline).
__device__ __attribute__((aligned(16))) z g_dma_zero[1];

// One output tile [m0, m0 + BM) x [n0, n0 + BN) of one product over the K range [klo, khi).
struct TileJob {
  long M, N;
  const z* A; long lda;
  const z* B; long ldb;
  z* C; long ldc;
  z alpha, beta;
  int conjA, conjB;
  long m0, n0, klo, khi;
  z* part;        // split-K: raw sums over this K range as [M][N] (nullptr: write C)
  long lv, lnB;   // ladder epilogue (EPI == 1)
  int omap;       // EPI 0: C laid out by om
  OutMap om;
};

// Writes a finished tile: alpha, beta and the output layout (row-major C, the ladder layout, or
// raw split-K partial sums).  cr/ci hold the real/imaginary sums (FP64 4M), or with FP32 3M tiles
// cr = sum ar br, ci = sum ai bi and cx = sum (ar + ai)(br + bi).
template <int BM, int BN, int WGM, int WGN, int EPI, typename T, bool k3M, typename Acc, int FI, int FJ, int XI,
          int XJ>
__device__ __forceinline__ void tile_epilogue(const TileJob& g, const Acc (&cr)[FI][FJ], const Acc (&ci)[FI][FJ],
                                              const Acc (&cx)[XI][XJ], int wm, int wn, int lr, int lk) {
  const long m0 = g.m0, n0 = g.n0;
  z* __restrict__ C = g.C;
  const bool use_beta = (g.beta.x != 0.0 || g.beta.y != 0.0);
  // Ladder layout: off = ((a nB + b) v + e) v + f = (a nB v + e) v + (b v^2 + f) splits into a row
  // part and a column part, each formed once per row or column of the lane with 32-bit division
  // (a per-element 64-bit division cost more than a tenth of the assembly's time).
  // A general output map (EPI 0 with omap) splits the same way: (m / rd) rs1 + (m % rd) rs2 per row,
  // (n / cd) cs1 + (n % cd) cs2 per element (M, N < 2^31, checked by the host).
  const bool om = EPI == 0 && g.omap;
  long coff[FJ];
  if (EPI == 1) {
    const unsigned lv = (unsigned)g.lv;
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
      const unsigned n = (unsigned)(n0 + wn + 16 * j + lr), b = n / lv;
      coff[j] = (long)b * g.lv * g.lv + (long)(n - b * lv);
    }
  }
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long m = m0 + wm + 16 * i + Mfma<T>::row(lk, r);
      long roff = 0;
      if (EPI == 1) {
        const unsigned mu = (unsigned)m, lv = (unsigned)g.lv, a = mu / lv;
        roff = ((long)a * g.lnB * g.lv + (long)(mu - a * lv)) * g.lv;
      } else if (om) {
        const unsigned mu = (unsigned)m, rd = (unsigned)g.om.rd, q = mu / rd;
        roff = (long)q * g.om.rs1 + (long)(mu - q * rd) * g.om.rs2;
      }
#pragma unroll
      for (int j = 0; j < FJ; ++j) {
        const long n = n0 + wn + 16 * j + lr;
        if (m >= g.M || n >= g.N) continue;
        double re = (double)cr[i][j][r], im = (double)ci[i][j][r];
        if constexpr (k3M) {
          const double p1 = re, p2 = im;
          re = p1 - p2;
          im = (double)cx[i][j][r] - p1 - p2;
        }
        if (g.part) {  // split-K: raw partial sums, reduced in a fixed order afterwards
          g.part[m * g.N + n] = make_double2(re, im);
          continue;
        }
        long off = EPI == 1 ? roff + coff[j] : m * g.ldc + n;
        if (om) {  // column part formed here: a per-column array costs registers in every EPI 0 kernel
          const unsigned nu = (unsigned)n, cd = (unsigned)g.om.cd, q = nu / cd;
          off = roff + (long)q * g.om.cs1 + (long)(nu - q * cd) * g.om.cs2;
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
}

// Computes one tile with the whole workgroup, operands rounded to T at staging, products and
// sums in T, the result written in FP64.  The LDS buffers are free again on return.
template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB, int EPI, typename T = double>
__device__ __forceinline__ void gemm_tile(const TileJob& g, TileSmem<BM, BN, BK, T>& sm) {
  constexpr int NT = WGM * WGN * 64;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;           // wave tile
  constexpr int FI = WTM / 16, FJ = WTN / 16;             // MFMA tiles per wave
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;     // staged complex elements per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WGN) * WTM, wn = (wave % WGN) * WTN;
  const long m0 = g.m0, n0 = g.n0, klo = g.klo, khi = g.khi;
  const z* __restrict__ A = g.A;
  const z* __restrict__ B = g.B;
  const bool cja = g.conjA != 0, cjb = g.conjB != 0;

  z ra[LA], rb[LB];
#define FC_LOAD_TILE(k0, ra, rb)                                                                 \
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
#define FC_STORE_TILE(buf, ra, rb)                                                               \
  do {                                                                                   \
    _Pragma("unroll") for (int r = 0; r < LA; ++r) {                                     \
      int e = tid + NT * r, mm, kk;                                                      \
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }           \
      sm.putA(buf, kk, mm, ra[r], cja);                                                  \
    }                                                                                    \
    _Pragma("unroll") for (int r = 0; r < LB; ++r) {                                     \
      int e = tid + NT * r, nn, kk;                                                      \
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }           \
      sm.putB(buf, kk, nn, rb[r], cjb);                                                  \
    }                                                                                    \
  } while (0)
// The same loads with no branch: an element outside the product is read from a zero in global
// memory, so every load instruction issues on every path (no select after it either) and the
// compiler's count of loads in flight stays exact across the two-slice pipeline below.  (Forming
// the per-thread offsets once per tile, or interleaving the address arithmetic with the products
// through scheduling-group hints, measured slower on the 3840^3 product: 137.8 -> 135.5 and 132.3
// TFLOP/s.)
#define FC_LOAD_TILE_U(k0, ra, rb)                                                       \
  do {                                                                                   \
    _Pragma("unroll") for (int r = 0; r < LA; ++r) {                                     \
      int e = tid + NT * r, mm, kk;                                                      \
      if (TA) { kk = e / BM; mm = e % BM; } else { mm = e / BK; kk = e % BK; }           \
      const long gm = m0 + mm, gk = (k0) + kk;                                           \
      const z* src = (gm < g.M && gk < khi) ? A + (TA ? gk * g.lda + gm : gm * g.lda + gk) : g_dma_zero; \
      ra[r] = *src;                                                                      \
    }                                                                                    \
    _Pragma("unroll") for (int r = 0; r < LB; ++r) {                                     \
      int e = tid + NT * r, nn, kk;                                                      \
      if (TB) { nn = e / BK; kk = e % BK; } else { kk = e / BN; nn = e % BN; }           \
      const long gn = n0 + nn, gk = (k0) + kk;                                           \
      const z* src = (gn < g.N && gk < khi) ? B + (TB ? gn * g.ldb + gk : gk * g.ldb + gn) : g_dma_zero; \
      rb[r] = *src;                                                                      \
    }                                                                                    \
  } while (0)

  // 4M (FP64): cr = sum ar br - ai bi, ci = sum ar bi + ai br, four real products per complex
  // one.  3M (Gauss, FP32): cr = sum ar br, ci = sum ai bi, cx = sum (ar + ai)(br + bi), result
  // cr - ci + i (cx - cr - ci), three real products per complex one (measured: 4096^3 product
  // 127.6 -> 149.7 complex TFLOP/s).  FP64 keeps 4M: its third accumulator set (8 registers per
  // 16 x 16 block) spills in the 128 x 128 tiles and halves the occupancy of the 64 x 64 ones.
  constexpr bool k3M = sizeof(T) == sizeof(float);
  using Acc = typename Mfma<T>::acc;
  Acc cr[FI][FJ], ci[FI][FJ], cx[k3M ? FI : 1][k3M ? FJ : 1];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) { cr[i][j] = Acc{0, 0, 0, 0}; ci[i][j] = Acc{0, 0, 0, 0}; }
  if constexpr (k3M) {
#pragma unroll
    for (int i = 0; i < FI; ++i)
#pragma unroll
      for (int j = 0; j < FJ; ++j) cx[i][j] = Acc{0, 0, 0, 0};
  }

  constexpr bool kEarlyStore = sizeof(T) == sizeof(double);
  const long nk = (khi - klo + BK - 1) / BK;
  const int lr = lane & 15, lk = lane >> 4;
  // the products of one K slice from LDS buffer `buf`; with `early`, the next slice (registers RS,
  // RBS) is stored to the other buffer before the last K quarter's products
#define FC_SLICE_PRODUCTS(buf, kt, early, RS, RBS)                                                \
  _Pragma("unroll") for (int ks = 0; ks < BK; ks += 4) {                                          \
    T ar[FI], ai[FI], nai[FI], br[FJ], bi[FJ];                                                    \
    _Pragma("unroll") for (int i = 0; i < FI; ++i) {                                              \
      sm.getA(buf, ks + lk, wm + 16 * i + lr, ar[i], ai[i]);                                      \
      nai[i] = -ai[i];                                                                            \
    }                                                                                             \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j) sm.getB(buf, ks + lk, wn + 16 * j + lr, br[j], bi[j]); \
    if ((early) && ks == BK - 4 && (kt) + 1 < nk) FC_STORE_TILE((buf) ^ 1, RS, RBS);              \
    if constexpr (k3M) {                                                                          \
      T sa_[FI], sb_[FJ];                                                                         \
      _Pragma("unroll") for (int i = 0; i < FI; ++i) sa_[i] = ar[i] + ai[i];                      \
      _Pragma("unroll") for (int j = 0; j < FJ; ++j) sb_[j] = br[j] + bi[j];                      \
      _Pragma("unroll") for (int i = 0; i < FI; ++i)                                              \
        _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                          \
          cr[i][j] = Mfma<T>::mac(ar[i], br[j], cr[i][j]);                                        \
          ci[i][j] = Mfma<T>::mac(ai[i], bi[j], ci[i][j]);                                        \
          cx[i][j] = Mfma<T>::mac(sa_[i], sb_[j], cx[i][j]);                                      \
        }                                                                                         \
    } else {                                                                                      \
      _Pragma("unroll") for (int i = 0; i < FI; ++i)                                              \
        _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                          \
          cr[i][j] = Mfma<T>::mac(ar[i], br[j], cr[i][j]);                                        \
          ci[i][j] = Mfma<T>::mac(ar[i], bi[j], ci[i][j]);                                        \
        }                                                                                         \
      _Pragma("unroll") for (int i = 0; i < FI; ++i)                                              \
        _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                          \
          cr[i][j] = Mfma<T>::mac(nai[i], bi[j], cr[i][j]);                                       \
          ci[i][j] = Mfma<T>::mac(ai[i], br[j], ci[i][j]);                                        \
        }                                                                                         \
    }                                                                                             \
  }

  // FP32 128 x 128 with 8-deep slices: global loads two K slices ahead into two register sets
  // (even slices in ra/rb, odd ones in ra2/rb2), the loop unrolled by two so that each half names
  // its sets statically: a slice's FP32 products are too short to cover the load latency on their
  // own, and this tile (one workgroup per CU) has registers to spare below the next occupancy
  // step.  The smaller FP32 tiles would lose a wave per SIMD and keep loads one slice ahead, as do
  // the FP64 tiles (the 16-deep variant would spill).
  constexpr bool kDepth2 = sizeof(T) == sizeof(float) && BM == 128 && BN == 128 && BK == 8;
  if constexpr (kDepth2) {
    z ra2[LA], rb2[LB];
    FC_LOAD_TILE_U(klo, ra, rb);
    FC_STORE_TILE(0, ra, rb);
    FC_LOAD_TILE_U(klo + BK, ra2, rb2);
    __syncthreads();
    // the next slice's registers were loaded a slice earlier, so they go to LDS before the last
    // K quarter's products, among which the compiler can spread the conversions and stores
    for (long kt = 0; kt < nk; kt += 2) {
      FC_LOAD_TILE_U(klo + (kt + 2) * BK, ra, rb);
      FC_SLICE_PRODUCTS(0, kt, true, ra2, rb2);
      __syncthreads();
      if (kt + 1 < nk) {
        FC_LOAD_TILE_U(klo + (kt + 3) * BK, ra2, rb2);
        FC_SLICE_PRODUCTS(1, kt + 1, true, ra, rb);
        __syncthreads();
      }
    }
  } else {
    FC_LOAD_TILE(klo, ra, rb);
    FC_STORE_TILE(0, ra, rb);
    __syncthreads();
    for (long kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) FC_LOAD_TILE(klo + (kt + 1) * BK, ra, rb);
      // FP64: the next tile goes to the other buffer while the last products of this one run
      // (measured: +6-10% on skinny and long-K products, neutral on large ones); FP32 products
      // are twice as fast, too short to cover the global loads, and store after the step instead
      FC_SLICE_PRODUCTS(buf, kt, kEarlyStore, ra, rb);
      if (!kEarlyStore && kt + 1 < nk) FC_STORE_TILE(buf ^ 1, ra, rb);
      __syncthreads();
    }
  }
#undef FC_SLICE_PRODUCTS
#undef FC_LOAD_TILE
#undef FC_LOAD_TILE_U
#undef FC_STORE_TILE

  tile_epilogue<BM, BN, WGM, WGN, EPI, T, k3M>(g, cr, ci, cx, wm, wn, lr, lk);
}

// ------------------------------------------------------------------------------------------------
// FP64 tiles fed by direct-to-LDS loads (global_load_lds_dwordx4).  Each lane moves 16 bytes -- one
// complex FP64 element -- from global memory into LDS without passing through vector registers:
// lane i of the wave writes slot i of a 64-slot (1 KiB) run whose base (M0) is uniform over the
// wave.  Which element a lane fetches therefore fixes the LDS layout of a K slice (8 deep):
//  * K-contiguous operand (A 'N'/'R', B 'T'/'C'): a run covers 8 rows x 8 K, the 8 lanes of a row
//    fetching its 128-byte line; row m keeps its elements at slots 8m + (k ^ sw(m)), where sw puts
//    the 16 rows of a fragment read on distinct 16-byte bank groups whether LDS serves 8 or 16
//    lanes of a 128-bit read per pass.
//  * M-contiguous operand (A 'T'/'C', B 'N'/'R'): a run covers 64 consecutive rows of one k.
// LDS receives the raw elements, so conjugation flips the sign of the imaginary part in the
// fragments.  Elements outside the product (rows >= M, k >= the split's end) come from a zero.
//
// Three LDS buffers, loads two slices ahead, fragments one K quarter ahead: step kt requests
// slice kt + 2 into the buffer slice kt - 1 left, reads the fragments of slice kt's second quarter,
// runs the first quarter's products, waits (own loads of slice kt + 1, then a workgroup barrier),
// reads slice kt + 1's first quarter and runs the second quarter's products.  The loads are issued
// from inline assembly: the compiler would otherwise make every later LDS read wait for all of
// them, and the waits here are explicit.

template <int BM, int BN, int BK>
struct DmaSmem {
  __attribute__((aligned(16))) z A[3][BM * BK];
  __attribute__((aligned(16))) z B[3][BN * BK];
};

// bank spread of a K-contiguous row of BK elements (see above); with BK = 16 a row is 256 bytes and
// the row index itself spreads the 16 rows of a fragment read
template <int BK>
__device__ __forceinline__ int dma_sw(int m) {
  if constexpr (BK == 8) return ((m >> 1) & 7) ^ ((m & 1) << 2);
  else return m & 15;
}

// LDS slot of element (row m, k) of a slice whose operand tile has R rows
template <bool KC, int R, int BK>
__device__ __forceinline__ int dma_slot(int m, int k) { return KC ? BK * m + (k ^ dma_sw<BK>(m)) : k * R + m; }

// the element of run r that lane `lane` fetches: row m and k within the slice
template <bool KC, int R, int BK>
__device__ __forceinline__ void dma_elem(int r, int lane, int& m, int& k) {
  if (KC) { m = (64 / BK) * r + lane / BK; k = (lane % BK) ^ dma_sw<BK>(m); }
  else { k = r / (R / 64); m = (r % (R / 64)) * 64 + lane; }
}

__device__ __forceinline__ double flip_sign(double x, unsigned long long mask) {
  return __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, x) ^ mask);
}

template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB, int EPI, bool G3M, typename T>
__device__ __forceinline__ void gemm_tile_dma(const TileJob& g, DmaSmem<BM, BN, BK>& sm) {
  static_assert(BK == 8 || BK == 16, "K slices of 8 or 16");
  static_assert(G3M || sizeof(T) == sizeof(double), "FP32 arithmetic uses the three-product form");
  constexpr int NQ = BK / 4;                              // K quarters (one MFMA deep) per slice
  constexpr int NW = WGM * WGN;
  constexpr int WTM = BM / WGM, WTN = BN / WGN;           // wave tile
  constexpr int FI = WTM / 16, FJ = WTN / 16;             // MFMA tiles per wave
  constexpr int QA = BM * BK / 64 / NW, QB = BN * BK / 64 / NW;   // runs per wave and K slice
  static_assert(QA * NW * 64 == BM * BK && QB * NW * 64 == BN * BK && BM % 64 == 0 && BN % 64 == 0,
                "run split");
  constexpr bool KCA = !TA, KCB = TB;
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = (wave / WGN) * WTM, wn = (wave % WGN) * WTN;
  const long klo = g.klo, khi = g.khi;

  // per-lane load plan: the element of each run at K slice 0, its k, whether its row exists
  const z* pa[QA]; const z* pb[QB];
  int ka[QA], kb[QB];
  bool oka[QA], okb[QB];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    int m;
    dma_elem<KCA, BM, BK>(wave + NW * q, lane, m, ka[q]);
    long gm = g.m0 + m;
    oka[q] = gm < g.M;
    if (!oka[q]) gm = g.M - 1;
    pa[q] = KCA ? g.A + gm * g.lda + klo + ka[q] : g.A + (klo + ka[q]) * g.lda + gm;
  }
#pragma unroll
  for (int q = 0; q < QB; ++q) {
    int n;
    dma_elem<KCB, BN, BK>(wave + NW * q, lane, n, kb[q]);
    long gn = g.n0 + n;
    okb[q] = gn < g.N;
    if (!okb[q]) gn = g.N - 1;
    pb[q] = KCB ? g.B + gn * g.ldb + klo + kb[q] : g.B + (klo + kb[q]) * g.ldb + gn;
  }
  const long stepA = KCA ? BK : BK * g.lda, stepB = KCB ? BK : BK * g.ldb;
  const long kspan = khi - klo;
#define FC_DMA_SLICE(s, buf)                                                                       \
  do {                                                                                             \
    _Pragma("unroll") for (int q = 0; q < QA; ++q)                                                 \
      lds_dma16((oka[q] && ka[q] + (s) * BK < kspan) ? pa[q] + (s) * stepA : g_dma_zero,           \
                &sm.A[buf][64 * (wave + NW * q)]);                                                 \
    _Pragma("unroll") for (int q = 0; q < QB; ++q)                                                 \
      lds_dma16((okb[q] && kb[q] + (s) * BK < kspan) ? pb[q] + (s) * stepB : g_dma_zero,           \
                &sm.B[buf][64 * (wave + NW * q)]);                                                 \
  } while (0)

  using Acc = typename Mfma<T>::acc;
  Acc cr[FI][FJ], ci[FI][FJ], cx[G3M ? FI : 1][G3M ? FJ : 1];
#pragma unroll
  for (int i = 0; i < FI; ++i)
#pragma unroll
    for (int j = 0; j < FJ; ++j) {
      cr[i][j] = Acc{0, 0, 0, 0};
      ci[i][j] = Acc{0, 0, 0, 0};
      if constexpr (G3M) cx[i][j] = Acc{0, 0, 0, 0};
    }

  const unsigned long long cmA = g.conjA ? 0x8000000000000000ull : 0ull;
  const unsigned long long cmB = g.conjB ? 0x8000000000000000ull : 0ull;
  const int lr = lane & 15, lk = lane >> 4;
  const long nk = (khi - klo + BK - 1) / BK;
  // fragments of one K quarter as the raw FP64 elements (A rows, B columns).  Conjugation and the
  // rounding to T happen in the products' step: an operation on a fragment right after its read
  // would make the wave wait for the read there, before the products it is meant to overlap.
  struct Frag { z a[FI], b[FJ]; };
#define FC_DMA_READ(buf, h, F)                                                                     \
  do {                                                                                             \
    _Pragma("unroll") for (int i = 0; i < FI; ++i)                                                 \
      F.a[i] = sm.A[buf][dma_slot<KCA, BM, BK>(wm + 16 * i + lr, 4 * (h) + lk)];                   \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j)                                                 \
      F.b[j] = sm.B[buf][dma_slot<KCB, BN, BK>(wn + 16 * j + lr, 4 * (h) + lk)];                   \
  } while (0)
  // 4M: cr += ar br - ai bi, ci += ar bi + ai br, the minus sign on bi (the same products as -ai
  // times bi, bit for bit).  3M: cr += ar br, ci += ai bi, cx += (ar + ai)(br + bi).
#define FC_DMA_MAC(F)                                                                              \
  do {                                                                                             \
    T ar_[FI], ai_[FI], br_[FJ], bi_[FJ];                                                          \
    _Pragma("unroll") for (int i = 0; i < FI; ++i) {                                               \
      ar_[i] = (T)F.a[i].x;                                                                        \
      ai_[i] = (T)flip_sign(F.a[i].y, cmA);                                                        \
    }                                                                                              \
    _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                               \
      br_[j] = (T)F.b[j].x;                                                                        \
      bi_[j] = (T)flip_sign(F.b[j].y, cmB);                                                        \
    }                                                                                              \
    if constexpr (G3M) {                                                                           \
      T sa_[FI], sb_[FJ];                                                                          \
      _Pragma("unroll") for (int i = 0; i < FI; ++i) sa_[i] = ar_[i] + ai_[i];                   \
      _Pragma("unroll") for (int j = 0; j < FJ; ++j) sb_[j] = br_[j] + bi_[j];                   \
      _Pragma("unroll") for (int i = 0; i < FI; ++i)                                               \
        _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                           \
          cr[i][j] = Mfma<T>::mac(ar_[i], br_[j], cr[i][j]);                                     \
          ci[i][j] = Mfma<T>::mac(ai_[i], bi_[j], ci[i][j]);                                     \
          cx[i][j] = Mfma<T>::mac(sa_[i], sb_[j], cx[i][j]);                                       \
        }                                                                                          \
    } else {                                                                                       \
      T nbi[FJ];                                                                                   \
      _Pragma("unroll") for (int j = 0; j < FJ; ++j) nbi[j] = -bi_[j];                            \
      _Pragma("unroll") for (int i = 0; i < FI; ++i)                                               \
        _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                           \
          cr[i][j] = Mfma<double>::mac(ar_[i], br_[j], cr[i][j]);                                \
          ci[i][j] = Mfma<double>::mac(ar_[i], bi_[j], ci[i][j]);                                \
        }                                                                                          \
      _Pragma("unroll") for (int i = 0; i < FI; ++i)                                               \
        _Pragma("unroll") for (int j = 0; j < FJ; ++j) {                                           \
          cr[i][j] = Mfma<double>::mac(ai_[i], nbi[j], cr[i][j]);                                 \
          ci[i][j] = Mfma<double>::mac(ai_[i], br_[j], ci[i][j]);                                \
        }                                                                                          \
    }                                                                                              \
  } while (0)

  FC_DMA_SLICE(0, 0);
  if (nk > 1) {
    FC_DMA_SLICE(1, 1);
    asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(QA + QB) : "memory");
  } else {
    asm volatile("s_waitcnt vmcnt(0)\n\ts_barrier" ::: "memory");
  }
  // fragments ping-pong between two sets, one K quarter ahead of the products
  Frag f[2];
  FC_DMA_READ(0, 0, f[0]);
  int buf = 0;
  for (long kt = 0; kt < nk; ++kt) {
    const int nbuf = buf == 2 ? 0 : buf + 1;
    if (kt + 2 < nk) FC_DMA_SLICE(kt + 2, nbuf == 2 ? 0 : nbuf + 1);
#pragma unroll
    for (int h = 0; h < NQ; ++h) {
      if (h + 1 < NQ) {
        FC_DMA_READ(buf, h + 1, f[(h + 1) & 1]);
      } else if (kt + 1 < nk) {
        // own loads of slice kt + 1 done (those of slice kt + 2 may still run), own reads of
        // slice kt done; then every wave's
        if (kt + 2 < nk) asm volatile("s_waitcnt vmcnt(%0) lgkmcnt(0)\n\ts_barrier" ::"n"(QA + QB) : "memory");
        else asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)\n\ts_barrier" ::: "memory");
        FC_DMA_READ(nbuf, 0, f[(h + 1) & 1]);
      }
      // keep the next quarter's reads ahead of this quarter's products (the scheduler would
      // otherwise sink them below the products or hoist the products' waits above them)
      __builtin_amdgcn_sched_barrier(0);
      FC_DMA_MAC(f[h & 1]);
      __builtin_amdgcn_sched_barrier(0);
    }
    buf = nbuf;
  }
#undef FC_DMA_SLICE
#undef FC_DMA_READ
#undef FC_DMA_MAC
  tile_epilogue<BM, BN, WGM, WGN, EPI, T, G3M>(g, cr, ci, cx, wm, wn, lr, lk);
}

template <int BM, int BN, int WGM, int WGN, int BK, bool TA, bool TB, int EPI, typename T, int DMA = 0>
__global__ __launch_bounds__(WGM * WGN * 64) void zgemm_f64_kernel(GemmArgs g) {
  // The x extent is a multiple of 8, so a workgroup runs on XCD blockIdx.x % 8 whatever its split
  // (y) and batch (z) index.  Rotating x by those indices spreads the splits and batch entries
  // of a product with few tiles over all XCDs instead of stacking them on the XCD of tile 0.
  const long bx = ((long)blockIdx.x + blockIdx.y + (long)gridDim.y * blockIdx.z) % gridDim.x;
  const long tile = xcd_tile(bx, g.tiles);
  if (tile >= g.tiles) return;
  const long ntn = (g.N + BN - 1) / BN;
  long mi = tile / ntn;
  if (EPI == 1 && g.ltri) {
    // triangular launches: fold the tile rows (0, tm-1, 1, tm-2, ...) so that every XCD's band
    // mixes rows with many and with few live tiles
    const long tm = g.tiles / ntn;
    mi = (mi & 1) ? tm - 1 - (mi >> 1) : (mi >> 1);
  }
  const long m0 = mi * BM, n0 = (tile % ntn) * BN;
  if (EPI == 1 && g.ltri) {
    // diagonal ab block: skip tiles whose smallest a exceeds their largest b
    const long amin = m0 / g.lv, bmax = (n0 + BN - 1 < g.N ? n0 + BN - 1 : g.N - 1) / g.lv;
    if (amin > bmax) return;
  }
  TileJob j;
  j.M = g.M; j.N = g.N;
  j.A = g.A + (long)blockIdx.z * g.sA; j.lda = g.lda;
  j.B = g.B + (long)blockIdx.z * g.sB; j.ldb = g.ldb;
  j.C = g.C + (long)blockIdx.z * g.sC; j.ldc = g.ldc;
  j.alpha = g.alpha; j.beta = g.beta;
  j.conjA = g.conjA; j.conjB = g.conjB;
  j.m0 = m0; j.n0 = n0;
  j.klo = (long)blockIdx.y * g.kchunk;
  j.khi = j.klo + g.kchunk < g.K ? j.klo + g.kchunk : g.K;
  j.part = g.part ? g.part + (long)blockIdx.y * g.M * g.N : nullptr;
  j.lv = g.lv; j.lnB = g.lnB;
  j.omap = g.omap; j.om = g.om;
  if constexpr (DMA) {
    __shared__ DmaSmem<BM, BN, BK> sm;
    gemm_tile_dma<BM, BN, WGM, WGN, BK, TA, TB, EPI, DMA == 2, T>(j, sm);
  } else {
    __shared__ TileSmem<BM, BN, BK, T> sm;
    gemm_tile<BM, BN, WGM, WGN, BK, TA, TB, EPI, T>(j, sm);
  }
}

// C = alpha * sum_s P[s] + beta * C.  Lane x of a workgroup owns output t = 64 b + x; its W waves
// take the splits s = w, w + W, ... in ascending order (two running sums each) and wave 0 adds
// the W results in wave order.  The order depends only on (ns, W), so results repeat bit for bit,
// and many splits of a small output are summed by W waves at once instead of one serial loop.
// With omap, C is laid out by om (the product's output map) instead of row-major with ldc.
template <int W>
__global__ void __launch_bounds__(64 * W) k_splitk_reduce(const z* __restrict__ P, int ns, long M, long N,
                                                          z* __restrict__ C, long ldc, z alpha, z beta, int omap,
                                                          OutMap om) {
  __shared__ z acc[W][64];
  const long MN = M * N;
  const bool use_beta = (beta.x != 0.0 || beta.y != 0.0);
  const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
  for (long base = blockIdx.x * 64L; base < MN; base += (long)gridDim.x * 64) {
    const long t = base + lane;
    double re0 = 0, im0 = 0, re1 = 0, im1 = 0;
    if (t < MN) {
      int s = w;
      for (; s + W < ns; s += 2 * W) {
        const z p = P[s * MN + t], q = P[(s + W) * MN + t];
        re0 += p.x; im0 += p.y;
        re1 += q.x; im1 += q.y;
      }
      if (s < ns) { const z p = P[s * MN + t]; re0 += p.x; im0 += p.y; }
    }
    acc[w][lane] = make_double2(re0 + re1, im0 + im1);
    __syncthreads();
    if (w == 0 && t < MN) {
      double re = 0, im = 0;
      for (int q = 0; q < W; ++q) { re += acc[q][lane].x; im += acc[q][lane].y; }
      const long m = t / N, n = t % N;
      const long off = omap ? (m / om.rd) * om.rs1 + (m % om.rd) * om.rs2 + (n / om.cd) * om.cs1 + (n % om.cd) * om.cs2
                            : m * ldc + n;
      z out = make_double2(alpha.x * re - alpha.y * im, alpha.x * im + alpha.y * re);
      if (use_beta) {
        const z c0 = C[off];
        out.x += beta.x * c0.x - beta.y * c0.y;
        out.y += beta.x * c0.y + beta.y * c0.x;
      }
      C[off] = out;
    }
    __syncthreads();
  }
}

void splitk_reduce(hipStream_t st, const z* part, long ns, long M, long N, z* C, long ldc, z alpha, z beta,
                   const OutMap* om) {
  const long MN = M * N;
  const unsigned nb = (unsigned)std::max(1L, std::min(65536L, (MN + 63) / 64));
  const int f = om ? 1 : 0;
  const OutMap m = om ? *om : OutMap{};
  if (ns >= 64) k_splitk_reduce<16><<<nb, 64 * 16, 0, st>>>(part, (int)ns, M, N, C, ldc, alpha, beta, f, m);
  else if (ns >= 8) k_splitk_reduce<4><<<nb, 64 * 4, 0, st>>>(part, (int)ns, M, N, C, ldc, alpha, beta, f, m);
  else k_splitk_reduce<1><<<nb, 64, 0, st>>>(part, (int)ns, M, N, C, ldc, alpha, beta, f, m);
}

template <int BM, int BN, int WGM, int WGN, int BK, int EPI, typename T, int DMA = 0>
void launch(const GemmArgs& g, bool ta, bool tb, dim3 grid, hipStream_t s) {
  constexpr int NT = WGM * WGN * 64;
  if (!ta && !tb) zgemm_f64_kernel<BM, BN, WGM, WGN, BK, false, false, EPI, T, DMA><<<grid, NT, 0, s>>>(g);
  else if (!ta && tb) zgemm_f64_kernel<BM, BN, WGM, WGN, BK, false, true, EPI, T, DMA><<<grid, NT, 0, s>>>(g);
  else if (ta && !tb) zgemm_f64_kernel<BM, BN, WGM, WGN, BK, true, false, EPI, T, DMA><<<grid, NT, 0, s>>>(g);
  else zgemm_f64_kernel<BM, BN, WGM, WGN, BK, true, true, EPI, T, DMA><<<grid, NT, 0, s>>>(g);
}

// Tile configurations: 64 x 64 (4 waves), 128 x 64 (4 waves) and 128 x 128 (8 waves), each with
// K slices of 8 (configurations 0-2) or 16 (3-5) complex elements per pipeline step; 128 x 96
// (4 waves of 64 x 48, configuration 6) for outputs about 300 columns wide, whose 64- and 128-wide
// tiles leave up to a third of the last column of tiles idle; 32 x 32 (one wave, configuration 7)
// for outputs of a few hundred elements with long K, which a 64 x 64 tile would mostly pad;
// with direct-to-LDS staging: 128 x 128, 8 waves of 64 x 32 (configuration 8: four real products
// per complex one in FP64, Gauss's three in FP32), and 128 x 64, 8 waves of 32 x 32, Gauss's three,
// with K slices of 8 (9) or 16 (10).
constexpr int NCFG = 11;
constexpr int CFG_BM[NCFG] = {64, 128, 128, 64, 128, 128, 128, 32, 128, 128, 128},
              CFG_BN[NCFG] = {64, 64, 128, 64, 64, 128, 96, 32, 128, 64, 64};

template <int EPI, typename T>
void launch_cfg(int cfg, const GemmArgs& g, bool ta, bool tb, dim3 grid, hipStream_t s) {
  switch (cfg) {
    case 0: launch<64, 64, 2, 2, 8, EPI, T>(g, ta, tb, grid, s); break;
    case 1: launch<128, 64, 2, 2, 8, EPI, T>(g, ta, tb, grid, s); break;
    case 2: launch<128, 128, 2, 4, 8, EPI, T>(g, ta, tb, grid, s); break;
    case 3: launch<64, 64, 2, 2, 16, EPI, T>(g, ta, tb, grid, s); break;
    case 4: launch<128, 64, 2, 2, 16, EPI, T>(g, ta, tb, grid, s); break;
    case 5: launch<128, 128, 2, 4, 16, EPI, T>(g, ta, tb, grid, s); break;
    case 6: launch<128, 96, 2, 2, 8, EPI, T>(g, ta, tb, grid, s); break;
    case 7: launch<32, 32, 1, 1, 8, EPI, T>(g, ta, tb, grid, s); break;
    case 8: launch<128, 128, 2, 4, 8, EPI, T, sizeof(T) == sizeof(double) ? 1 : 2>(g, ta, tb, grid, s); break;
    case 9: launch<128, 64, 4, 2, 8, EPI, T, 2>(g, ta, tb, grid, s); break;
    default: launch<128, 64, 4, 2, 16, EPI, T, 2>(g, ta, tb, grid, s); break;
  }
}

// Launch one configuration (split-K decided inside for configurations whose grid cannot fill the chip).
// fixed_part: when given, split-K partial sums go there (at most NOALLOC_SCRATCH_BYTES) instead
// of into a buffer from the context's allocator.
// om: when given, C is laid out by the output map (batch 1, no ladder epilogue).
void zgemm_run(fc_ctx ctx, int cfg, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
               const z* B, long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC,
               const LadderEpilogue* lep, z* fixed_part = nullptr, const OutMap* om = nullptr);

// Shape bucket: operand layouts, sizes rounded to powers of two, batching and epilogue kind.
std::string bucket(char opA, char opB, long M, long N, long K, int batch, const LadderEpilogue* lep, int fp32) {
  auto lg = [](long x) { int b = 0; while ((1L << b) < x) ++b; return b; };
  char buf[96];
  snprintf(buf, sizeof(buf), "%c%c_m%d_n%d_k%d_b%d_e%d%s", opA, opB, lg(M), lg(N), lg(K), batch > 1,
           lep ? 1 + lep->triangular : 0, fp32 ? "_s" : "");
  return buf;
}

// Default tile choice, from timing every configuration on the hot path's shapes: 32 x 32 for
// tiny outputs; in FP64 the direct-to-LDS 128 x 64 tile with Gauss's three products and K slices
// of 16 when its tiles fill the chip and pad the output by at most a quarter (4096^3 66 -> 81
// complex TFLOP/s, the ladder's assembly 64 -> 76 and contraction 54 -> 70); 128 x 128 when there
// are enough such
// tiles to fill the chip; otherwise 64 x 64, with 16-element K slices in FP64 when K is long
// (skinny and split-K products), and 128 x 96 in FP32 for outputs about 300 columns wide.
int heuristic_cfg(long M, long N, long K, int batch, bool fp32) {
  if (M <= 32 && N <= 32) return 7;
  if (!fp32) {
    const long tm = (M + 127) / 128, tn = (N + 63) / 64;
    // enough tiles to fill the chip, or outputs of a few hundred squared with K long enough for
    // split K to fill it (576 x 576 x 25600: 47 -> 58 TFLOP/s; 3840 x 500 x 3840: 56 -> 71)
    const bool fills = tm * tn * batch >= 256 || (M >= 256 && N >= 256 && K >= 2048 && batch == 1);
    if (M >= 256 && N >= 64 && fills && 4 * (tm * 128) * (tn * 64) <= 5 * M * N) return 10;
  }
  const long t128 = ((M + 127) / 128) * ((N + 127) / 128), t64 = ((M + 63) / 64) * ((N + 63) / 64);
  // 128 x 128 unless its padding costs a quarter more work than 64 x 64 tiles (e.g. 300 x 300)
  const bool big = M >= 256 && N >= 256 && t128 * (long)batch >= 512 && 4 * t128 * 4 <= 5 * t64;
  if (big) return 2;
  if (fp32) return (M >= 1024 && N > 192 && N <= 288) ? 6 : 0;
  return K >= 2048 ? 3 : 0;
}
// A configuration fits a product when its tile is not larger than the padded output needs.
bool cfg_fits(int c, long M, long N) {
  return (CFG_BM[c] <= 64 || M >= 128) && (CFG_BN[c] <= 64 || N >= 96);
}

// Tuning override: the context's configuration (fc_set_gemm_config), else FNSCC_GEMM_CFG, selects
// one configuration for every product it fits.
int forced_cfg(fc_ctx ctx, long M, long N) {
  static const int env = [] {
    const char* e = getenv("FNSCC_GEMM_CFG");
    return e ? atoi(e) : -1;
  }();
  const int forced = ctx->gemm_cfg >= 0 ? ctx->gemm_cfg : env;
  return (forced >= 0 && forced < NCFG && cfg_fits(forced, M, N)) ? forced : -1;
}

void zgemm_impl(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda, const z* B,
                long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC, const LadderEpilogue* lep,
                const OutMap* om = nullptr) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  FC_REQUIRE(strchr("NTCR", opA) && strchr("NTCR", opB), FC_EARG, "zgemm: bad op");
  int cfg = heuristic_cfg(M, N, K, batch, !lep && ctx->gemm_fp32);
  const int forced = forced_cfg(ctx, M, N);
  if (forced >= 0) {
    cfg = forced;
  } else if (ctx->autotune && K > 0) {
    const std::string key = bucket(opA, opB, M, N, K, batch, lep, lep ? 0 : ctx->gemm_fp32);
    auto it = ctx->tune.find(key);
    if (it != ctx->tune.end()) {
      cfg = it->second.first;
    } else {
      // time every configuration once (after one warm-up launch) on a scratch copy of C, keep the fastest
      const long csz = lep  ? (M / lep->v) * lep->nB * lep->v * lep->v
                       : om ? (long)(batch - 1) * sC + om->span(M, N)
                            : ((long)(batch - 1) * sC + (M - 1) * ldc + N);
      DBuf trial(ctx, sizeof(z) * (size_t)std::max(1L, csz));
      hipEvent_t e0, e1;
      FC_HIP(hipEventCreate(&e0));
      FC_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      int bestc = cfg;
      for (int c = 0; c < NCFG; ++c) {
        if (!cfg_fits(c, M, N)) continue;
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          if (!lep && (beta.x != 0.0 || beta.y != 0.0))
            FC_HIP(hipMemcpyAsync(trial.p, C, sizeof(z) * csz, hipMemcpyDeviceToDevice, ctx->stream));
          FC_HIP(hipEventRecord(e0, ctx->stream));
          zgemm_run(ctx, c, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, trial.as<z>(), ldc, batch, sA, sB, sC, lep,
                    nullptr, om);
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
  zgemm_run(ctx, cfg, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch, sA, sB, sC, lep, nullptr, om);
}

void zgemm_run(fc_ctx ctx, int cfg, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
               const z* B, long ldb, z beta, z* C, long ldc, int batch, long sA, long sB, long sC,
               const LadderEpilogue* lep, z* fixed_part, const OutMap* om) {
  FC_REQUIRE(strchr("NTCR", opA) && strchr("NTCR", opB), FC_EARG, "zgemm: bad op");
  FC_REQUIRE(!om || (!lep && om->rd >= 1 && om->cd >= 1 && M % om->rd == 0 && N % om->cd == 0 &&
                     M < (1L << 31) && N < (1L << 31)),
             FC_EARG, "zgemm: bad output map");
  if (K <= 0) {  // C = beta C
    FC_REQUIRE(!lep && !om, FC_EARG, "zgemm: empty ladder or mapped product");
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
  g.omap = om ? 1 : 0;
  g.om = om ? *om : OutMap{};
  const bool ta = (opA == 'T' || opA == 'C');
  const bool tb = (opB == 'T' || opB == 'C');
  FC_REQUIRE(batch <= 65535, FC_EARG, "zgemm: batch too large");
  FC_REQUIRE(cfg >= 0 && cfg < NCFG, FC_EARG, "zgemm: bad tile configuration");
  FC_REQUIRE(!lep || (M < (1L << 31) && N < (1L << 31) && lep->v >= 1), FC_EARG, "zgemm: ladder product too large");
  const long bm = CFG_BM[cfg], bn = CFG_BN[cfg];
  const long tiles = ((N + bn - 1) / bn) * ((M + bm - 1) / bm);
  FC_REQUIRE(tiles < (1L << 30), FC_EARG, "zgemm: problem too large for one launch");
  g.tiles = tiles;
  // Split K when the tile grid cannot fill the chip (256 CUs): each split covers >= 4 KQ elements,
  // partials go to a workspace and are summed in split order, so results stay deterministic.
  long ksplit = 1;
  const long want = 1024;
  if (!lep && batch == 1 && tiles < want && K >= 8 * KQ) {
    ksplit = std::min((want + tiles - 1) / tiles, K / (4 * KQ));
    const long cap = std::max(1L, (256L << 20) / (long)(sizeof(z) * M * N));
    ksplit = std::max(1L, std::min({ksplit, cap, 4096L}));
  }
  g.kchunk = ((K + ksplit - 1) / ksplit + KQ - 1) / KQ * KQ;
  ksplit = (K + g.kchunk - 1) / g.kchunk;
  g.part = nullptr;
  DBuf work;
  if (ksplit > 1) {
    const size_t need = sizeof(z) * (size_t)ksplit * M * N;
    if (fixed_part) {
      FC_REQUIRE(need <= NOALLOC_SCRATCH_BYTES, FC_EARG,
                 "fc_zgemm_noalloc: the split-K partial sums of this product need " + std::to_string(need) +
                     " bytes, more than the " + std::to_string(NOALLOC_SCRATCH_BYTES) + "-byte fixed workspace");
      g.part = fixed_part;
    } else {
      work = DBuf(ctx, need);
      g.part = work.as<z>();
    }
  }
  dim3 grid((unsigned)((tiles + 7) / 8 * 8), (unsigned)ksplit, (unsigned)batch);
  // FNSCC_VERBOSE >= 3: every product is timed on its own (synchronising) and logged
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->verbose >= 3) {
    FC_HIP(hipEventCreate(&e0));
    FC_HIP(hipEventCreate(&e1));
    FC_HIP(hipEventRecord(e0, ctx->stream));
  }
  if (lep) launch_cfg<1, double>(cfg, g, ta, tb, grid, ctx->stream);
  else if (ctx->gemm_fp32) launch_cfg<0, float>(cfg, g, ta, tb, grid, ctx->stream);
  else launch_cfg<0, double>(cfg, g, ta, tb, grid, ctx->stream);
  FC_HIP(hipGetLastError());
  if (ksplit > 1) {
    splitk_reduce(ctx->stream, g.part, ksplit, M, N, C, ldc, alpha, beta, om);
    FC_HIP(hipGetLastError());
  }
  if (e0) {
    FC_HIP(hipEventRecord(e1, ctx->stream));
    FC_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    FC_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double fl = 8.0 * M * N * K * batch;
    fprintf(stderr, "[gemm] %c%c M %ld N %ld K %ld batch %d cfg %d ksplit %ld %s %.3f ms %.1f TF/s\n", opA, opB,
            M, N, K, batch, cfg, ksplit, lep ? "ladder" : ctx->gemm_fp32 ? "fp32" : "fp64", ms,
            fl / (ms * 1e-3) / 1e12);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
}

// ------------------------------------------------------------------------------------------------
// Grouped products: one persistent launch walks the output tiles of many independent products
// (different shapes, operands and layouts) listed in a device-resident plan.  The plan is read at
// run time, so a captured graph replays with whatever products the plan holds at that moment.
struct GroupHeader {
  long nprob, total_tiles, total_elems, pad;
};
struct GroupDesc {
  long M, N, K;
  const z* A; long lda, sA;
  const z* B; long ldb, sB;
  z* C; long ldc, sC;
  z alpha, beta;
  int ta, tb, conjA, conjB;
  long batch, ksplit, kchunk, tn, tiles;   // tiles: output tiles of one (split, batch) slice
  long tile0, elem0;                       // first global tile, first reduced element
  z* part;                                 // split-K partials [ksplit][batch][M][N]
};
constexpr size_t PLAN_HDR = 64;

// index of the last entry whose key field is <= x (keys non-decreasing; the entry holding x)
template <long GroupDesc::*F>
__device__ inline long group_find(const GroupDesc* d, long np, long x) {
  long lo = 0, hi = np - 1;
  while (lo < hi) {
    const long mid = (lo + hi + 1) >> 1;
    if (d[mid].*F <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int BM, int BN, int WGM, int WGN, int BK>
__global__ __launch_bounds__(WGM * WGN * 64) void k_group_gemm(const char* __restrict__ plan) {
  __shared__ TileSmem<BM, BN, BK> sm;
  const GroupHeader* h = reinterpret_cast<const GroupHeader*>(plan);
  const GroupDesc* d = reinterpret_cast<const GroupDesc*>(plan + PLAN_HDR);
  const long total = h->total_tiles, np = h->nprob;
  const long span = (total + 7) / 8 * 8;
  // the grid is a multiple of 8, so virtual tile vt runs on XCD vt % 8 and each XCD walks a
  // contiguous band of tiles
  for (long vt = blockIdx.x; vt < span; vt += gridDim.x) {
    const long t = xcd_tile(vt, total);
    if (t >= total) continue;
    const GroupDesc g = d[group_find<&GroupDesc::tile0>(d, np, t)];
    const long loc = t - g.tile0;
    const long tt = loc % g.tiles, r = loc / g.tiles;
    const long b = r % g.batch, s = r / g.batch;
    TileJob j;
    j.M = g.M; j.N = g.N;
    j.A = g.A + b * g.sA; j.lda = g.lda;
    j.B = g.B + b * g.sB; j.ldb = g.ldb;
    j.C = g.C + b * g.sC; j.ldc = g.ldc;
    j.alpha = g.alpha; j.beta = g.beta;
    j.conjA = g.conjA; j.conjB = g.conjB;
    j.m0 = (tt / g.tn) * BM; j.n0 = (tt % g.tn) * BN;
    j.klo = s * g.kchunk;
    j.khi = j.klo + g.kchunk < g.K ? j.klo + g.kchunk : g.K;
    j.part = g.ksplit > 1 ? g.part + (s * g.batch + b) * g.M * g.N : nullptr;
    j.lv = 1; j.lnB = 1; j.omap = 0;
    if (g.ta) {
      if (g.tb) gemm_tile<BM, BN, WGM, WGN, BK, true, true, 0>(j, sm);
      else gemm_tile<BM, BN, WGM, WGN, BK, true, false, 0>(j, sm);
    } else {
      if (g.tb) gemm_tile<BM, BN, WGM, WGN, BK, false, true, 0>(j, sm);
      else gemm_tile<BM, BN, WGM, WGN, BK, false, false, 0>(j, sm);
    }
  }
}

// The same persistent walk over the plan's tiles on the 128 x 64 direct-to-LDS tile with Gauss's
// three real products (8 waves, one workgroup per CU).  The tile ends without a barrier after its
// last LDS reads, so one is taken before the next tile's loads reuse the buffers.
template <int BM, int BN, int WGM, int WGN, int BK>
__global__ __launch_bounds__(WGM * WGN * 64) void k_group_gemm_dma(const char* __restrict__ plan) {
  __shared__ DmaSmem<BM, BN, BK> sm;
  const GroupHeader* h = reinterpret_cast<const GroupHeader*>(plan);
  const GroupDesc* d = reinterpret_cast<const GroupDesc*>(plan + PLAN_HDR);
  const long total = h->total_tiles, np = h->nprob;
  const long span = (total + 7) / 8 * 8;
  bool first = true;
  for (long vt = blockIdx.x; vt < span; vt += gridDim.x) {
    const long t = xcd_tile(vt, total);
    if (t >= total) continue;
    const GroupDesc g = d[group_find<&GroupDesc::tile0>(d, np, t)];
    const long loc = t - g.tile0;
    const long tt = loc % g.tiles, r = loc / g.tiles;
    const long b = r % g.batch, s = r / g.batch;
    TileJob j;
    j.M = g.M; j.N = g.N;
    j.A = g.A + b * g.sA; j.lda = g.lda;
    j.B = g.B + b * g.sB; j.ldb = g.ldb;
    j.C = g.C + b * g.sC; j.ldc = g.ldc;
    j.alpha = g.alpha; j.beta = g.beta;
    j.conjA = g.conjA; j.conjB = g.conjB;
    j.m0 = (tt / g.tn) * BM; j.n0 = (tt % g.tn) * BN;
    j.klo = s * g.kchunk;
    j.khi = j.klo + g.kchunk < g.K ? j.klo + g.kchunk : g.K;
    j.part = g.ksplit > 1 ? g.part + (s * g.batch + b) * g.M * g.N : nullptr;
    j.lv = 1; j.lnB = 1; j.omap = 0;
    if (!first) __syncthreads();   // every wave has left the previous tile's buffers
    first = false;
    if (g.ta) {
      if (g.tb) gemm_tile_dma<BM, BN, WGM, WGN, BK, true, true, 0, true, double>(j, sm);
      else gemm_tile_dma<BM, BN, WGM, WGN, BK, true, false, 0, true, double>(j, sm);
    } else {
      if (g.tb) gemm_tile_dma<BM, BN, WGM, WGN, BK, false, true, 0, true, double>(j, sm);
      else gemm_tile_dma<BM, BN, WGM, WGN, BK, false, false, 0, true, double>(j, sm);
    }
  }
}

// C = alpha * sum_s part[s] + beta * C for every split product of the plan, in split order.
__global__ void k_group_reduce(const char* __restrict__ plan) {
  const GroupHeader* h = reinterpret_cast<const GroupHeader*>(plan);
  const GroupDesc* d = reinterpret_cast<const GroupDesc*>(plan + PLAN_HDR);
  const long total = h->total_elems, np = h->nprob;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const GroupDesc& g = d[group_find<&GroupDesc::elem0>(d, np, e)];
    const long MN = g.M * g.N, loc = e - g.elem0;
    const long b = loc / MN, mn = loc % MN, m = mn / g.N, n = mn % g.N;
    double re = 0, im = 0;
    for (long s = 0; s < g.ksplit; ++s) {
      const z p = g.part[(s * g.batch + b) * MN + mn];
      re += p.x; im += p.y;
    }
    z out = make_double2(g.alpha.x * re - g.alpha.y * im, g.alpha.x * im + g.alpha.y * re);
    z* c = g.C + b * g.sC + m * g.ldc + n;
    if (g.beta.x != 0.0 || g.beta.y != 0.0) {
      const z c0 = *c;
      out.x += g.beta.x * c0.x - g.beta.y * c0.y;
      out.y += g.beta.x * c0.y + g.beta.y * c0.x;
    }
    *c = out;
  }
}
}  // namespace

// grouped tiles: 0 = 64 x 64 and 1 = 128 x 64 register-staged (four products), 2 = 128 x 64
// direct-to-LDS with three products
constexpr int GROUP_NCFG = 3;
constexpr long GROUP_BM[GROUP_NCFG] = {64, 128, 128}, GROUP_BN[GROUP_NCFG] = {64, 64, 64};

GroupCounts group_encode(const std::vector<GroupGemm>& probs, const GroupTiling& tl, void* host_plan,
                         size_t plan_cap, z* work, size_t work_cap) {
  FC_REQUIRE(tl.cfg >= 0 && tl.cfg < GROUP_NCFG, FC_EARG, "grouped gemm: bad tile configuration");
  FC_REQUIRE(tl.kchunk >= KQ, FC_EARG, "grouped gemm: K chunk below one K slice");
  const long bm = GROUP_BM[tl.cfg], bn = GROUP_BN[tl.cfg];
  GroupCounts c;
  c.plan_bytes = PLAN_HDR + sizeof(GroupDesc) * probs.size();
  GroupDesc* d = host_plan ? reinterpret_cast<GroupDesc*>((char*)host_plan + PLAN_HDR) : nullptr;
  if (host_plan) FC_REQUIRE(c.plan_bytes <= plan_cap, FC_EARG, "grouped gemm: plan buffer too small");
  for (size_t i = 0; i < probs.size(); ++i) {
    const GroupGemm& p = probs[i];
    FC_REQUIRE(strchr("NTCR", p.opA) && strchr("NTCR", p.opB), FC_EARG, "grouped gemm: bad op");
    FC_REQUIRE(p.M >= 0 && p.N >= 0 && p.K >= 0 && p.batch >= 0, FC_EARG, "grouped gemm: negative size");
    GroupDesc g{};
    g.M = p.M; g.N = p.N; g.K = p.K;
    g.A = p.A; g.lda = p.lda; g.sA = p.sA;
    g.B = p.B; g.ldb = p.ldb; g.sB = p.sB;
    g.C = p.C; g.ldc = p.ldc; g.sC = p.sC;
    g.alpha = p.alpha; g.beta = p.beta;
    g.ta = (p.opA == 'T' || p.opA == 'C');
    g.tb = (p.opB == 'T' || p.opB == 'C');
    g.conjA = (p.opA == 'C' || p.opA == 'R');
    g.conjB = (p.opB == 'C' || p.opB == 'R');
    g.batch = p.batch;
    const long tm = (p.M + bm - 1) / bm;
    g.tn = std::max(1L, (p.N + bn - 1) / bn);
    g.tiles = std::max(1L, tm * ((p.N + bn - 1) / bn));
    if (p.K > tl.kchunk) {
      const long ks = (p.K + tl.kchunk - 1) / tl.kchunk;
      g.kchunk = ((p.K + ks - 1) / ks + KQ - 1) / KQ * KQ;
      g.ksplit = (p.K + g.kchunk - 1) / g.kchunk;
    } else {
      g.kchunk = std::max<long>(p.K, 1);
      g.ksplit = 1;
    }
    const bool empty = p.M == 0 || p.N == 0 || p.batch == 0;
    g.tile0 = c.tiles;
    g.elem0 = c.elems;
    g.part = nullptr;
    if (!empty) {
      c.tiles += g.ksplit * g.batch * g.tiles;
      if (g.ksplit > 1) {
        g.part = work ? work + c.work : nullptr;
        c.work += (size_t)(g.ksplit * g.batch * p.M * p.N);
        c.elems += g.batch * p.M * p.N;
      }
    } else {
      g.batch = 1; g.ksplit = 1;   // never visited: no tiles, no reduced elements
    }
    if (d) d[i] = g;
  }
  if (host_plan) {
    FC_REQUIRE(!work || c.work <= work_cap, FC_EARG, "grouped gemm: split-K workspace too small");
    FC_REQUIRE(work || c.work == 0, FC_EARG, "grouped gemm: split-K workspace missing");
    GroupHeader* h = reinterpret_cast<GroupHeader*>(host_plan);
    h->nprob = (long)probs.size();
    h->total_tiles = c.tiles;
    h->total_elems = c.elems;
    h->pad = 0;
  }
  return c;
}

void group_launch(fc_ctx ctx, int cfg, const void* dplan, long max_tiles, long max_elems) {
  const char* p = static_cast<const char*>(dplan);
  // persistent grid: at most 4 workgroups per CU of 256 CUs, a multiple of 8
  const long g1 = std::max(8L, std::min(1024L, (max_tiles + 7) / 8 * 8));
  if (cfg == 2) {
    // 144 KB of LDS: one workgroup per CU
    const long gd = std::max(8L, std::min(256L, (max_tiles + 7) / 8 * 8));
    k_group_gemm_dma<128, 64, 4, 2, 16><<<(unsigned)gd, 512, 0, ctx->stream>>>(p);
  } else if (cfg == 1) {
    k_group_gemm<128, 64, 2, 2, 8><<<(unsigned)g1, 256, 0, ctx->stream>>>(p);
  } else {
    k_group_gemm<64, 64, 2, 2, 8><<<(unsigned)g1, 256, 0, ctx->stream>>>(p);
  }
  FC_HIP(hipGetLastError());
  if (max_elems > 0) {
    const long g2 = std::max(1L, std::min(2048L, (max_elems + 255) / 256));
    k_group_reduce<<<(unsigned)g2, 256, 0, ctx->stream>>>(p);
    FC_HIP(hipGetLastError());
  }
}

void group_gemm(fc_ctx ctx, const std::vector<GroupGemm>& probs, const GroupTiling& tl) {
  if (probs.empty()) return;
  const GroupCounts c = group_encode(probs, tl, nullptr, 0, nullptr, 0);
  if (c.tiles == 0) return;
  std::vector<char> host(c.plan_bytes);
  DBuf work(ctx, sizeof(z) * c.work), dplan(ctx, c.plan_bytes);
  group_encode(probs, tl, host.data(), host.size(), work.as<z>(), c.work);
  FC_HIP(hipMemcpyAsync(dplan.p, host.data(), c.plan_bytes, hipMemcpyHostToDevice, ctx->stream));
  group_launch(ctx, tl.cfg, dplan.p, c.tiles, c.elems);
  // the host plan must outlive the copy
  FC_HIP(hipStreamSynchronize(ctx->stream));
}

GroupArena::GroupArena(fc_ctx c, size_t plan_bytes, size_t work_elems)
    : ctx(c), dev(c, plan_bytes), work(c, sizeof(z) * work_elems), cap(plan_bytes), wcap(work_elems) {
  FC_HIP(hipHostMalloc((void**)&host, plan_bytes, hipHostMallocDefault));
}

GroupArena::~GroupArena() {
  if (host) (void)hipHostFree(host);
}

void GroupArena::run(const std::vector<GroupGemm>& probs, const GroupTiling& tl) {
  if (probs.empty()) return;
  const GroupCounts c0 = group_encode(probs, tl, nullptr, 0, nullptr, 0);
  if (c0.tiles == 0) return;
  const size_t at = (off + 255) / 256 * 256;
  FC_REQUIRE(at + c0.plan_bytes <= cap, FC_EARG, "grouped gemm: plan arena exhausted");
  FC_REQUIRE(woff + c0.work <= wcap, FC_EARG, "grouped gemm: workspace arena exhausted");
  group_encode(probs, tl, host + at, cap - at, work.as<z>() + woff, wcap - woff);
  FC_HIP(hipMemcpyAsync(dev.as<char>() + at, host + at, c0.plan_bytes, hipMemcpyHostToDevice, ctx->stream));
  group_launch(ctx, tl.cfg, dev.as<char>() + at, c0.tiles, c0.elems);
  off = at + c0.plan_bytes;
  woff += c0.work;
}

int gemm_num_configs() { return NCFG; }

// ------------------------------------------------------------------------------------------------
// Fixed workspace of the allocation-free product.  Each device holds its own copy of this array
// from module load until the process ends.  Host code never uses the array's name as an address:
// noalloc_scratch_init looks its device address up once per device (with that device current)
// and every kernel argument uses that pointer.  Sized for every split the default tile choice
// makes: fewer than 1024 + tiles - 1 split tiles of at most 64 x 64 outputs each, i.e. under
// 2048 x 4096 complex partial sums.
__device__ __align__(256) static double2 scratch[NOALLOC_SCRATCH_BYTES / sizeof(double2)];

namespace {
std::mutex g_scratch_mu;
constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

void noalloc_scratch_init(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  FC_REQUIRE(device >= 0 && device < MAX_DEVICES, FC_EARG, "device index out of range");
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  FC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  FC_REQUIRE(p != nullptr, FC_EHIP, "hipGetSymbolAddress returned no address for the fixed workspace");
  g_scratch_ptr[device] = p;
}

void zgemm_noalloc(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
                   const z* B, long ldb, z beta, z* C, long ldc) {
  if (M <= 0 || N <= 0) return;
  FC_REQUIRE(strchr("NTCR", opA) && strchr("NTCR", opB), FC_EARG, "zgemm: bad op");
  void* part = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (ctx->device >= 0 && ctx->device < MAX_DEVICES) part = g_scratch_ptr[ctx->device];
  }
  FC_REQUIRE(part != nullptr, FC_EHIP, "fc_zgemm_noalloc: fixed workspace not set up on this device");
  // the size heuristic (or the forced configuration), never the autotuner: timing trial products
  // needs a buffer of its own
  int cfg = heuristic_cfg(M, N, K, 1, ctx->gemm_fp32);
  const int forced = forced_cfg(ctx, M, N);
  if (forced >= 0) cfg = forced;
  zgemm_run(ctx, cfg, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 1, 0, 0, 0, nullptr,
            static_cast<z*>(part));
}

void zgemm(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda, const z* B, long ldb,
           z beta, z* C, long ldc, int batch, long sA, long sB, long sC) {
  zgemm_impl(ctx, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, batch, sA, sB, sC, nullptr);
}

void zgemm_sum(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda, long sA,
               const z* B, long ldb, long sB, int batch, z beta, z* C, long ldc) {
  if (M <= 0 || N <= 0) return;
  if (batch <= 0 || K <= 0) {
    for (long m = 0; m < M; ++m) scale(ctx, C + m * ldc, N, beta);
    return;
  }
  DBuf part(ctx, sizeof(z) * (size_t)batch * M * N);
  zgemm(ctx, opA, opB, M, N, K, make_double2(1, 0), A, lda, B, ldb, make_double2(0, 0), part.as<z>(), N, batch,
        sA, sB, M * N);
  splitk_reduce(ctx->stream, part.as<z>(), batch, M, N, C, ldc, alpha, beta, nullptr);
  FC_HIP(hipGetLastError());
}

void zgemm_mapped(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
                  const z* B, long ldb, z beta, z* C, const OutMap& om, int batch, long sA, long sB, long sC) {
  zgemm_impl(ctx, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, 0, batch, sA, sB, sC, nullptr, &om);
}

void zgemm_ladder(fc_ctx ctx, long M, long N, long K, const z* A, long lda, const z* B, long ldb, z* W,
                  const LadderEpilogue& lep) {
  zgemm_impl(ctx, 'N', 'T', M, N, K, make_double2(1, 0), A, lda, B, ldb, make_double2(0, 0), W, 0, 1, 0, 0, 0, &lep);
}

}  // namespace fc
