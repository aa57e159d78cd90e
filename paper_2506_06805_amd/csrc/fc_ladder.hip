// Particle-particle ladder R_ij^ab = sum_ef tau_ij^ef sum_P Lb^P_ae Lb^P_bf (Eq. 21, 23), with the
// four-virtual integrals rebuilt from the Cholesky vectors on every call and never stored whole.
//
// The unique outputs (i<j, a<b) are produced in chunks of (a,b) pairs:
//  1. assembly: for a block pair (A, B), W[(a,e),(b,f)] = sum_P Lb[a,e,P] Lb[b,f,P] is one GEMM
//     with K = N_CD whose epilogue writes W in [(a,b)][e][f] order (diagonal block pairs skip the
//     output tiles with every a > every b);
//  2. antisymmetrisation: Wp[ab][k(e,f)] = W[ab][e][f] - W[ab][f][e] for e < f, LDS-tiled so both
//     the tile and its transpose are read coalesced (split precision: written directly as hi/lo
//     planes).  The contraction index k runs over 32 x 32 blocks of (e, f) (block pairs E <= F in
//     order, then rows of the block), so each block of a pair is one contiguous run of Wp;
//  3. contraction: Rp[ab][i<j] = sum_k Wp[ab][k] tau[i<j][k], one GEMM per chunk with K = v(v-1)/2
//     (tau packed in the same blocked order);
//  4. the chunk's Rp written to the output: all four antisymmetric images of a full R, or the
//     packed R[i<j][a<b].
// The T1 dressing Lb = L_ae - sum_m t_m^a L_me is folded into the split of L_vv in split precision
// (complex64 or complex128 vectors, never a dressed copy); in FP64 it is a dressed complex128 copy.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "fc_split.hpp"
#include "fc_state.hpp"

namespace fc {
namespace {
constexpr int TPB = 256;
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(1048576L, (n + TPB * 4 - 1) / (TPB * 4))); }
#define GRID_STRIDE(i, n) for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < (n); i += (long)gridDim.x * blockDim.x)
typedef unsigned short u16;

// taup[pij][pef] = tau[i,j,e,f] for i<j, e<f (natural pair order)
__global__ void k_pack_tau(const z* __restrict__ tau, z* __restrict__ taup, long o, long v, const int2* po,
                           const int2* pv, long no, long nv) {
  GRID_STRIDE(t, no * nv) {
    long pe = t % nv, pi = t / nv;
    int2 ij = po[pi], ef = pv[pe];
    taup[t] = tau[((ij.x * o + ij.y) * v + ef.x) * v + ef.y];
  }
}
// out[r][k] = in[r][colmap[k]] (the FP64 contraction operand in blocked order)
__global__ void k_gather_cols(const z* __restrict__ in, z* __restrict__ out, long rows, long K, const int* colmap) {
  GRID_STRIDE(t, rows * K) {
    const long r = t / K, k = t % K;
    out[t] = in[r * K + colmap[k]];
  }
}

// Wp[s][boff(E,F) + local(e,f)] = W[s][e][f] - W[s][f][e] for valid slots (a < b); one 32 x 32
// block pair (E <= F) per workgroup, both tiles staged in LDS.  local = (e - 32E) nF + f - 32F for
// E < F, the row-major index of e < f inside the triangle for E = F.  T: double2 (FP64 path) or
// float2 (split path).
template <class T>
struct AntiOut;
template <>
struct AntiOut<double2> {
  z* Wp;
  long nv;
  // one 16-byte slot per lane, consecutive lanes on consecutive slots (runs of four per lane
  // measured 10% slower here)
  static constexpr bool kRun4 = false;
  __device__ void put(long s, long pe, double re, double im) const { Wp[s * nv + pe] = make_double2(re, im); }
  __device__ void put4(long, long, const double (&)[4], const double (&)[4]) const {}
};
template <int PREC>
__device__ inline u16 to16(float x) {
  if constexpr (PREC == FC_SPLIT_BF16) return __builtin_bit_cast(u16, (__bf16)x);
  else return __builtin_bit_cast(u16, (_Float16)x);
}
template <int PREC>
__device__ inline double from16(u16 x) {
  if constexpr (PREC == FC_SPLIT_BF16) return (double)(float)__builtin_bit_cast(__bf16, x);
  else return (double)(float)__builtin_bit_cast(_Float16, x);
}
template <int PREC>
struct SplitOut {
  // runs of four slots per lane: one 8-byte store per plane instead of four 2-byte ones
  static constexpr bool kRun4 = true;
  u16* planes;
  long plane, kp;
  double scale;
  __device__ void put(long s, long pe, double re, double im) const {
    re *= scale; im *= scale;
    const u16 rh = to16<PREC>((float)re), ih = to16<PREC>((float)im);
    const long off = s * kp + pe;
    planes[off] = rh;
    planes[plane + off] = to16<PREC>((float)(re - from16<PREC>(rh)));
    planes[2 * plane + off] = ih;
    planes[3 * plane + off] = to16<PREC>((float)(im - from16<PREC>(ih)));
  }
  // four consecutive slots pe .. pe + 3 (pe a multiple of 4): one 8-byte store per plane
  __device__ void put4(long s, long pe, const double (&re)[4], const double (&im)[4]) const {
    u16 h[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double r = re[q] * scale, i = im[q] * scale;
      h[0][q] = to16<PREC>((float)r);
      h[1][q] = to16<PREC>((float)(r - from16<PREC>(h[0][q])));
      h[2][q] = to16<PREC>((float)i);
      h[3][q] = to16<PREC>((float)(i - from16<PREC>(h[2][q])));
    }
    const long off = s * kp + pe;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      uint2 w;
      w.x = (unsigned)h[p][0] | ((unsigned)h[p][1] << 16);
      w.y = (unsigned)h[p][2] | ((unsigned)h[p][3] << 16);
      *reinterpret_cast<uint2*>(planes + p * plane + off) = w;
    }
  }
};

// One workgroup per (E <= F) block pair and group of slots: it walks the slots s = blockIdx.y,
// blockIdx.y + gridDim.y, ... (a few per workgroup: one slot per workgroup made the pass
// dispatch-bound, about 193,000 small workgroups per evaluation at v = 160).
template <class T, class Out>
__global__ __launch_bounds__(256) void k_ladder_anti(const T* __restrict__ W, const int* __restrict__ compact, long v,
                                                    long nbv, const long* __restrict__ boff, long ns, Out out) {
  __shared__ T X[32][33], Y[32][33];
  // block pair (E, F), E <= F, from the linear id
  long q = blockIdx.x, E = 0;
  while (q >= nbv - E) { q -= nbv - E; ++E; }
  const long F = E + q;
  const long off = boff[blockIdx.x];
  const long nE = std::min(32L, v - 32 * E), nF = std::min(32L, v - 32 * F);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (long s = blockIdx.y; s < ns; s += gridDim.y) {
    const int c = compact[s];   // row of the valid pair (a < b) in Wp, or -1 (uniform over the workgroup)
    if (c < 0) continue;
    const T* Ws = W + s * v * v;
    __syncthreads();   // the previous slot's reads of X and Y are done
    for (int r = ty; r < 32; r += 8) {
      long e = E * 32 + r, f = F * 32 + tx;
      X[r][tx] = (e < v && f < v) ? Ws[e * v + f] : T{};
      long e2 = F * 32 + r, f2 = E * 32 + tx;
      Y[r][tx] = (e2 < v && f2 < v) ? Ws[e2 * v + f2] : T{};
    }
    __syncthreads();
    if constexpr (!Out::kRun4) {
      for (int r = ty; r < 32; r += 8) {
        if (r >= nE || tx >= nF) continue;
        long local;
        if (E < F) local = r * nF + tx;
        else if (r < tx) local = (long)r * (2 * nE - r - 1) / 2 + (tx - r - 1);
        else continue;
        const T x = X[r][tx], y = Y[tx][r];
        out.put(c, off + local, (double)x.x - (double)y.x, (double)x.y - (double)y.y);
      }
      continue;
    }
    // runs: thread t takes row r = t / 8 of the block and its columns 4 (t % 8) + 0..3, written as
    // one 4-slot run where the run is whole and 4-aligned (every off-diagonal run when v is a
    // multiple of 32), slot by slot otherwise
    const int r = threadIdx.x >> 3, c0 = 4 * (threadIdx.x & 7);
    if (r >= nE) continue;
    if (E < F) {
      const long pe = off + r * nF + c0;
      if (c0 + 4 <= nF && (pe & 3) == 0) {
        double re[4], im[4];
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const T x = X[r][c0 + q4], y = Y[c0 + q4][r];
          re[q4] = (double)x.x - (double)y.x;
          im[q4] = (double)x.y - (double)y.y;
        }
        out.put4(c, pe, re, im);
      } else {
        for (int q4 = 0; q4 < 4 && c0 + q4 < nF; ++q4) {
          const T x = X[r][c0 + q4], y = Y[c0 + q4][r];
          out.put(c, pe + q4, (double)x.x - (double)y.x, (double)x.y - (double)y.y);
        }
      }
    } else {
      for (int q4 = 0; q4 < 4; ++q4) {
        const int f = c0 + q4;
        if (f >= nE || f <= r) continue;
        const T x = X[r][f], y = Y[f][r];
        out.put(c, off + (long)r * (2 * nE - r - 1) / 2 + (f - r - 1), (double)x.x - (double)y.x,
                (double)x.y - (double)y.y);
      }
    }
  }
}

__global__ void k_maxabs_slots(const float2* __restrict__ W, const int* __restrict__ compact, long nslots, long vv,
                               unsigned* out) {
  __shared__ float sm[TPB];
  float m = 0.f;
  GRID_STRIDE(t, nslots * vv) {
    if (compact[t / vv] >= 0) m = fmaxf(m, fmaxf(fabsf(W[t].x), fabsf(W[t].y)));
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = TPB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = fmaxf(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  // the maximum of non-negative floats equals the maximum of their bit patterns
  if (threadIdx.x == 0) atomicMax(out, __float_as_uint(sm[0]));
}

__device__ inline long upair(long i, long j, long n) { return i * (2 * n - i - 1) / 2 + (j - i - 1); }

// Rp is [pair][i<j] (the contraction runs with the long (a,b)-pair dimension as rows, so the tiles
// that share a panel of Wp are neighbours on one XCD and Wp is read from HBM about once).
// Full output: R[i,j,a,b] and its three antisymmetric images.
// acc: add into R (each of the four images belongs to one unique amplitude, so no two threads
// touch the same element)
__global__ void k_ladder_scatter(const z* __restrict__ Rp, z* __restrict__ R, long o, long v, const int2* pairs,
                                 long npairs, const int2* po, long no, int acc) {
  GRID_STRIDE(t, no * npairs) {
    const long s = t % npairs, pi = t / npairs;
    const int2 ab = pairs[s];
    const int2 ij = po[pi];
    const z r = Rp[s * no + pi], m = make_double2(-r.x, -r.y);
    const long i = ij.x, j = ij.y, a = ab.x, b = ab.y;
    const long x0 = ((i * o + j) * v + a) * v + b, x1 = ((j * o + i) * v + a) * v + b,
               x2 = ((i * o + j) * v + b) * v + a, x3 = ((j * o + i) * v + b) * v + a;
    if (acc) {
      const z y0 = R[x0], y1 = R[x1], y2 = R[x2], y3 = R[x3];
      R[x0] = make_double2(y0.x + r.x, y0.y + r.y);
      R[x1] = make_double2(y1.x + m.x, y1.y + m.y);
      R[x2] = make_double2(y2.x + m.x, y2.y + m.y);
      R[x3] = make_double2(y3.x + r.x, y3.y + r.y);
    } else {
      R[x0] = r;
      R[x1] = m;
      R[x2] = m;
      R[x3] = r;
    }
  }
}
// Packed output: Rk[i<j][a<b]
__global__ void k_ladder_scatter_packed(const z* __restrict__ Rp, z* __restrict__ Rk, long v, const int2* pairs,
                                        long npairs, long no) {
  const long nv = v * (v - 1) / 2;
  GRID_STRIDE(t, no * npairs) {
    const long s = t % npairs, pi = t / npairs;
    const int2 ab = pairs[s];
    Rk[pi * nv + upair(ab.x, ab.y, v)] = Rp[s * no + pi];
  }
}
}  // namespace

static DBuf pair_table(fc_ctx ctx, long n, long& np) {
  std::vector<int2> h;
  for (long i = 0; i < n; ++i)
    for (long j = i + 1; j < n; ++j) h.push_back(make_int2((int)i, (int)j));
  np = (long)h.size();
  DBuf d(ctx, sizeof(int2) * std::max(1L, np));
  if (np) FC_HIP(hipMemcpyAsync(d.p, h.data(), sizeof(int2) * np, hipMemcpyHostToDevice, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  return d;
}

// Memory for one chunk of the assembled W (bytes); the chunk covers as many (a,b) pairs as fit.
static double ladder_budget_bytes() {
  const char* s = getenv("FNSCC_LADDER_BUDGET_GB");
  return (s ? atof(s) : 8.0) * 1e9;
}

namespace {
struct Sink {
  bool packed;
  z* R;
  bool accumulate = false;   // full layout: add into R
};

// The blocked contraction order: for each 32 x 32 block pair (E <= F) in the anti kernel's
// enumeration, its first slot (boff) and, for every slot, the natural index of its (e, f) pair.
struct BlockedOrder {
  DBuf boff, colmap;
  long nbv = 0, ntri = 0;
  BlockedOrder(fc_ctx ctx, long v) {
    nbv = (v + 31) / 32;
    ntri = nbv * (nbv + 1) / 2;
    std::vector<long> hb;
    std::vector<int> hc;
    for (long E = 0; E < nbv; ++E)
      for (long F = E; F < nbv; ++F) {
        hb.push_back((long)hc.size());
        const long nE = std::min(32L, v - 32 * E), nF = std::min(32L, v - 32 * F);
        for (long r = 0; r < nE; ++r)
          for (long c = (E == F ? r + 1 : 0); c < nF; ++c) {
            const long e = 32 * E + r, f = 32 * F + c;
            hc.push_back((int)(e * (2 * v - e - 1) / 2 + (f - e - 1)));
          }
      }
    FC_REQUIRE((long)hc.size() == v * (v - 1) / 2, FC_EARG, "ladder: blocked pair order incomplete");
    boff = DBuf(ctx, sizeof(long) * hb.size());
    colmap = DBuf(ctx, sizeof(int) * std::max<size_t>(1, hc.size()));
    FC_HIP(hipMemcpyAsync(boff.p, hb.data(), sizeof(long) * hb.size(), hipMemcpyHostToDevice, ctx->stream));
    if (!hc.empty())
      FC_HIP(hipMemcpyAsync(colmap.p, hc.data(), sizeof(int) * hc.size(), hipMemcpyHostToDevice, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
  }
};
}  // namespace

// taup: [i<j][e<f] natural order (device, complex128); the chunks' results go to the sink.
static void ladder_core(fc_ctx ctx, fc_ints I, const z* taup, const z* t1dress, int precision, const Sink& sink,
                        long no, const DBuf& po) {
  const long o = I->o, v = I->v, N = I->ncd;
  const z one = make_double2(1, 0), zero = make_double2(0, 0);
  const bool split = precision != FC_FP64;
  const long nv = v * (v - 1) / 2;
  if (no <= 0 || nv <= 0) return;
  BlockedOrder bo(ctx, v);
  // block size T (pairs per block pair T^2) and chunk capacity in (a,b) slots
  const double esz = split ? 8.0 : 16.0;
  const long cap_slots = std::max(1L, (long)(ladder_budget_bytes() / (esz * (double)v * (double)v)));
  long T = std::max(1L, std::min({v, 64L, (long)std::floor(std::sqrt((double)cap_slots))}));
  struct BP { long a0, nA, b0, nB; };
  std::vector<BP> bps;
  for (long a0 = 0; a0 < v; a0 += T)
    for (long b0 = a0; b0 < v; b0 += T) bps.push_back({a0, std::min(T, v - a0), b0, std::min(T, v - b0)});
  long max_slots = 0;
  {  // size the chunk buffers for the largest chunk
    long cur = 0;
    for (auto& bp : bps) {
      if (cur > 0 && cur + bp.nA * bp.nB > cap_slots) { max_slots = std::max(max_slots, cur); cur = 0; }
      cur += bp.nA * bp.nB;
    }
    max_slots = std::max(max_slots, cur);
  }
  FC_REQUIRE(max_slots <= 65535, FC_EARG, "ladder: chunk has too many (a,b) slots");
  // operands: the (dressed) virtual vectors and tau in the blocked contraction order
  SplitOp Ls, Ts, Wps;
  ZTensor Lb, taub;
  DBuf Wp64;
  if (split) {
    if (I->Lvv64.p && (!t1dress || o <= 64)) {
      Ls = split_lvv_dressed(ctx, precision, I->Lvv64.p, true, I->Lov.p(), t1dress, o, v, N);
    } else if (!t1dress || o <= 64) {
      Ls = split_lvv_dressed(ctx, precision, I->Lvv.p(), false, I->Lov.p(), t1dress, o, v, N);
    } else {
      Lb = ZTensor(ctx, {v, v, N});
      const ZTensor& L = lvv(ctx, I);
      FC_HIP(hipMemcpyAsync(Lb.p(), L.p(), sizeof(z) * Lb.size(), hipMemcpyDeviceToDevice, ctx->stream));
      zein(ctx, "ma,meP->aeP", make_double2(-1, 0), ZT((z*)t1dress, {o, v}), I->Lov, one, Lb);
      Ls = split_lvv_dressed(ctx, precision, Lb.p(), false, I->Lov.p(), nullptr, o, v, N);
      Lb = ZTensor();
    }
    Ts = split_operand_cols(ctx, precision, taup, no, nv, nv, bo.colmap.as<int>());
    Wps.prec = precision;
    Wps.kp = Ts.kp;
    Wps.rows_pad = (max_slots + 127) / 128 * 128 + 128;
    Wps.buf = DBuf(ctx, sizeof(u16) * 4 * (size_t)Wps.rows_pad * Wps.kp);
    // the contraction padding (k >= nv) is never written by the chunks: clear it once.  Rows
    // past a chunk's valid pairs reach only output rows that are never stored.
    split_zero_kpad(ctx, Wps, nv);
  } else {
    // dressed vectors Lb^P_ae = L^P_ae - sum_m t_m^a L^P_me
    const ZTensor& L = lvv(ctx, I);
    Lb = ZTensor(ctx, {v, v, N});
    FC_HIP(hipMemcpyAsync(Lb.p(), L.p(), sizeof(z) * Lb.size(), hipMemcpyDeviceToDevice, ctx->stream));
    if (t1dress) zein(ctx, "ma,meP->aeP", make_double2(-1, 0), ZT((z*)t1dress, {o, v}), I->Lov, one, Lb);
    taub = ZTensor(ctx, {no, nv});
    hipLaunchKernelGGL(k_gather_cols, dim3(nblk(no * nv)), dim3(TPB), 0, ctx->stream, taup, taub.p(), no, nv,
                       bo.colmap.as<int>());
    FC_HIP(hipGetLastError());
    Wp64 = DBuf(ctx, sizeof(z) * (size_t)max_slots * nv);
  }
  DBuf Wbuf(ctx, (size_t)esz * max_slots * v * v);
  DBuf Rp(ctx, sizeof(z) * no * max_slots);
  DBuf slots_d(ctx, sizeof(int2) * max_slots), compact_d(ctx, sizeof(int) * max_slots);
  DBuf mx(ctx, sizeof(unsigned));
  size_t next = 0;
  // FNSCC_VERBOSE: a line per twentieth of the block pairs (long evaluations at large shapes)
  const auto t_start = std::chrono::steady_clock::now();
  size_t reported = 0;
  while (next < bps.size()) {
    if (ctx->verbose && next >= reported) {
      const double s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
      fprintf(stderr, "[ladder] block pair %zu of %zu, %.1f s\n", next, bps.size(), s);
      fflush(stderr);
      reported = next + std::max<size_t>(1, bps.size() / 20);
    }
    // gather a chunk of block pairs and run their assembly GEMMs
    std::vector<int2> hslots;
    while (next < bps.size() && (hslots.empty() || (long)hslots.size() + bps[next].nA * bps[next].nB <= cap_slots)) {
      const BP& bp = bps[next];
      LadderEpilogue lep;
      lep.v = v; lep.nB = bp.nB; lep.triangular = (bp.a0 == bp.b0);
      const long base = (long)hslots.size();
      if (!split)
        zgemm_ladder(ctx, bp.nA * v, bp.nB * v, N, Lb.p() + bp.a0 * v * N, N, Lb.p() + bp.b0 * v * N, N,
                     Wbuf.as<z>() + base * v * v, lep);
      else
        gemm_split_ladder(ctx, Ls, bp.a0 * v, bp.nA * v, Ls, bp.b0 * v, bp.nB * v,
                          Wbuf.as<float2>() + base * v * v, lep);
      for (long ia = 0; ia < bp.nA; ++ia)
        for (long ib = 0; ib < bp.nB; ++ib) hslots.push_back(make_int2((int)(bp.a0 + ia), (int)(bp.b0 + ib)));
      ++next;
    }
    const long ns = (long)hslots.size();
    // valid pairs (a < b) get consecutive rows of Wp; the others (below-diagonal slots of diagonal
    // block pairs) are skipped by the antisymmetrisation, the contraction and the scatter
    std::vector<int> hcompact(ns, -1);
    std::vector<int2> hpairs;
    for (long s = 0; s < ns; ++s)
      if (hslots[s].x < hslots[s].y) { hcompact[s] = (int)hpairs.size(); hpairs.push_back(hslots[s]); }
    const long nvalid = (long)hpairs.size();
    if (nvalid == 0) {   // only below-diagonal slots in this chunk
      FC_HIP(hipStreamSynchronize(ctx->stream));
      continue;
    }
    FC_HIP(hipMemcpyAsync(slots_d.p, hpairs.data(), sizeof(int2) * nvalid, hipMemcpyHostToDevice, ctx->stream));
    FC_HIP(hipMemcpyAsync(compact_d.p, hcompact.data(), sizeof(int) * ns, hipMemcpyHostToDevice, ctx->stream));
    // a few slots per workgroup (see k_ladder_anti)
    dim3 agrid((unsigned)bo.ntri, (unsigned)std::min(ns, 2048L));
    if (!split) {
      AntiOut<double2> out{Wp64.as<z>(), nv};
      k_ladder_anti<double2, AntiOut<double2>><<<agrid, 256, 0, ctx->stream>>>(
          Wbuf.as<double2>(), compact_d.as<int>(), v, bo.nbv, bo.boff.as<long>(), ns, out);
      FC_HIP(hipGetLastError());
      zgemm(ctx, 'N', 'T', nvalid, no, nv, one, Wp64.as<z>(), nv, taub.p(), nv, zero, Rp.as<z>(), no);
    } else {
      Wps.scale = 1.0;
      if (precision == FC_SPLIT_FP16) {
        FC_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned), ctx->stream));
        // at most 2048 workgroups: one atomic per workgroup on a single word
        k_maxabs_slots<<<std::min(2048u, nblk(ns * v * v)), TPB, 0, ctx->stream>>>(Wbuf.as<float2>(), compact_d.as<int>(),
                                                                                    ns, v * v, mx.as<unsigned>());
        FC_HIP(hipGetLastError());
        unsigned hb = 0;
        FC_HIP(hipMemcpyAsync(&hb, mx.p, sizeof(unsigned), hipMemcpyDeviceToHost, ctx->stream));
        FC_HIP(hipStreamSynchronize(ctx->stream));
        float m;
        std::memcpy(&m, &hb, sizeof(m));
        // differences are at most twice the largest entry; keep them below 2^14
        if (m > 0) Wps.scale = std::ldexp(1.0, 12 - std::ilogb((double)m));
      }
      Wps.rows = nvalid;
      const long plane = Wps.rows_pad * Wps.kp;
      if (precision == FC_SPLIT_BF16) {
        SplitOut<FC_SPLIT_BF16> out{Wps.buf.as<u16>(), plane, Wps.kp, Wps.scale};
        k_ladder_anti<float2, SplitOut<FC_SPLIT_BF16>><<<agrid, 256, 0, ctx->stream>>>(
            Wbuf.as<float2>(), compact_d.as<int>(), v, bo.nbv, bo.boff.as<long>(), ns, out);
      } else {
        SplitOut<FC_SPLIT_FP16> out{Wps.buf.as<u16>(), plane, Wps.kp, Wps.scale};
        k_ladder_anti<float2, SplitOut<FC_SPLIT_FP16>><<<agrid, 256, 0, ctx->stream>>>(
            Wbuf.as<float2>(), compact_d.as<int>(), v, bo.nbv, bo.boff.as<long>(), ns, out);
      }
      FC_HIP(hipGetLastError());
      gemm_split_nt(ctx, Wps, 0, nvalid, Ts, 0, no, one, zero, Rp.as<z>(), no);
    }
    if (sink.packed)
      hipLaunchKernelGGL(k_ladder_scatter_packed, dim3(nblk(no * nvalid)), dim3(TPB), 0, ctx->stream, Rp.as<z>(),
                         sink.R, v, slots_d.as<int2>(), nvalid, no);
    else
      hipLaunchKernelGGL(k_ladder_scatter, dim3(nblk(no * nvalid)), dim3(TPB), 0, ctx->stream, Rp.as<z>(), sink.R, o,
                         v, slots_d.as<int2>(), nvalid, po.as<int2>(), no, sink.accumulate ? 1 : 0);
    FC_HIP(hipGetLastError());
    // the slot table is rewritten by the next chunk: keep host and device in order
    FC_HIP(hipStreamSynchronize(ctx->stream));
  }
}

namespace {
struct LadderEvents {
  fc_ctx ctx;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  explicit LadderEvents(fc_ctx c) : ctx(c) {
    if (ctx->timing & 2) {
      FC_HIP(hipEventCreate(&ev0));
      FC_HIP(hipEventCreate(&ev1));
      FC_HIP(hipEventRecord(ev0, ctx->stream));
    }
  }
  void done() {
    if (ev0) {
      FC_HIP(hipEventRecord(ev1, ctx->stream));
      ctx->ladder_events.emplace_back(ev0, ev1);
      ev0 = nullptr;
    }
  }
  ~LadderEvents() {
    if (ev0) { (void)hipEventDestroy(ev0); (void)hipEventDestroy(ev1); }
  }
};
}  // namespace

void ladder_dev(fc_ctx ctx, fc_ints I, const z* tau, const z* t1dress, z* R, int precision, bool accumulate) {
  StageTimer st(ctx, "ladder");
  LadderEvents evs(ctx);
  const long o = I->o, v = I->v;
  long no, nv;
  DBuf po = pair_table(ctx, o, no), pv = pair_table(ctx, v, nv);
  // the scatter writes every element with i != j and a != b; the rest of the ladder term is zero
  if (!accumulate) fill(ctx, R, o * o * v * v, make_double2(0, 0));
  if (no > 0 && nv > 0) {
    DBuf taup(ctx, sizeof(z) * no * nv);
    hipLaunchKernelGGL(k_pack_tau, dim3(nblk(no * nv)), dim3(TPB), 0, ctx->stream, tau, taup.as<z>(), o, v,
                       po.as<int2>(), pv.as<int2>(), no, nv);
    FC_HIP(hipGetLastError());
    ladder_core(ctx, I, taup.as<z>(), t1dress, precision, Sink{false, R, accumulate}, no, po);
  }
  evs.done();
}

void ladder_packed_dev(fc_ctx ctx, fc_ints I, const z* taup, const z* t1dress, z* Rk, int precision) {
  StageTimer st(ctx, "ladder");
  LadderEvents evs(ctx);
  const long o = I->o;
  long no;
  DBuf po = pair_table(ctx, o, no);
  ladder_core(ctx, I, taup, t1dress, precision, Sink{true, Rk}, no, po);
  evs.done();
}

}  // namespace fc
