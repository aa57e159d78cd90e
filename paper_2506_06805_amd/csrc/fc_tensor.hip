// Streaming tensor kernels (HBM-bound) and the two-operand contraction planner.
#include <algorithm>
#include <cstring>

#include "fc_internal.hpp"

namespace fc {

// ------------------------------------------------------------------------------ memory
static size_t round_up(size_t b) {
  const size_t g = 256;
  return (b + g - 1) / g * g;
}

void* dmalloc(fc_ctx ctx, size_t bytes) {
  size_t rb = round_up(bytes);
  auto it = ctx->cache.lower_bound(rb);
  // reuse a cached block of the same size class (at most 1/8 larger)
  if (it != ctx->cache.end() && it->first <= rb + rb / 8) {
    void* p = it->second;
    size_t sz = it->first;
    ctx->cache.erase(it);
    ctx->cached_bytes -= sz;
    ctx->live[p] = sz;
    return p;
  }
  void* p = nullptr;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (ctx->alloc) {
      p = ctx->alloc(rb, (void*)ctx->stream, ctx->user);
    } else {
      if (hipMalloc(&p, rb) != hipSuccess) { (void)hipGetLastError(); p = nullptr; }
    }
    if (p) break;
    release_cache(ctx);  // give cached blocks back and retry once
  }
  if (!p) throw Error(FC_ENOMEM, "device allocation of " + std::to_string(rb) + " bytes failed");
  ctx->live[p] = rb;
  return p;
}

void dfree(fc_ctx ctx, void* p) {
  auto it = ctx->live.find(p);
  if (it == ctx->live.end()) return;
  ctx->cache.emplace(it->second, p);
  ctx->cached_bytes += it->second;
  ctx->live.erase(it);
}

void release_cache(fc_ctx ctx) {
  if (ctx->cache.empty()) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->cache) {
    if (ctx->release) ctx->release(kv.second, kv.first, (void*)ctx->stream, ctx->user);
    else (void)hipFree(kv.second);
  }
  ctx->cache.clear();
  ctx->cached_bytes = 0;
}

// ------------------------------------------------------------------------------ timers
StageTimer::StageTimer(fc_ctx c, const char* n) : ctx(c), name(n) {
  if (ctx->timing & 1) {
    FC_HIP(hipEventCreate(&a));
    FC_HIP(hipEventCreate(&b));
    FC_HIP(hipEventRecord(a, ctx->stream));
  }
}
StageTimer::~StageTimer() {
  if (!a) return;
  float ms = 0.f;
  if (hipEventRecord(b, ctx->stream) == hipSuccess && hipEventSynchronize(b) == hipSuccess &&
      hipEventElapsedTime(&ms, a, b) == hipSuccess) {
    ctx->stage_ms[name] += ms;
    ctx->stage_calls[name] += 1;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
}

// ------------------------------------------------------------------------------ elementwise
namespace {
constexpr int TPB = 256;
inline unsigned nblocks(long n, long per = 1) {
  long b = (n + TPB * per - 1) / (TPB * per);
  if (b < 1) b = 1;
  if (b > 1048576) b = 1048576;
  return (unsigned)b;
}
__device__ inline z cmul(z a, z b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline z cadd(z a, z b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline z csub(z a, z b) { return make_double2(a.x - b.x, a.y - b.y); }

__global__ void k_fill(z* p, long n, z v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_scale(z* p, long n, z a) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = cmul(a, p[i]);
}
__global__ void k_axpy(long n, z a, const z* x, z* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = cadd(y[i], cmul(a, x[i]));
}
__global__ void k_copy(long n, const z* x, z* y, int conj) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    z v = x[i];
    if (conj) v.y = -v.y;
    y[i] = v;
  }
}

constexpr int MAXD = 8;
struct PermArgs {
  int nd;
  long odims[MAXD];   // output dims (row-major)
  long istr[MAXD];    // input stride of each output dim
  long n;
  z alpha, beta;
  int conj, use_beta;
};
__global__ void k_permute(const z* __restrict__ in, z* __restrict__ out, PermArgs a) {
  for (long o = blockIdx.x * (long)blockDim.x + threadIdx.x; o < a.n; o += (long)gridDim.x * blockDim.x) {
    long rem = o, ioff = 0;
    for (int d = a.nd - 1; d >= 0; --d) {
      long c = rem % a.odims[d];
      rem /= a.odims[d];
      ioff += c * a.istr[d];
    }
    z v = in[ioff];
    if (a.conj) v.y = -v.y;
    z r = cmul(a.alpha, v);
    if (a.use_beta) r = cadd(r, cmul(a.beta, out[o]));
    out[o] = r;
  }
}

// The same with 32-bit index arithmetic (every tensor here has fewer than 2^31 elements): the
// 64-bit divisions of the general kernel cost more than its memory traffic.
struct PermArgs32 {
  int nd;
  unsigned odims[MAXD], istr[MAXD];
  unsigned n;
  z alpha, beta;
  int conj, use_beta;
};
__global__ void k_permute32(const z* __restrict__ in, z* __restrict__ out, PermArgs32 a) {
  for (unsigned o = blockIdx.x * blockDim.x + threadIdx.x; o < a.n; o += gridDim.x * blockDim.x) {
    unsigned rem = o, ioff = 0;
    for (int d = a.nd - 1; d >= 0; --d) {
      const unsigned q = rem / a.odims[d];
      ioff += (rem - q * a.odims[d]) * a.istr[d];
      rem = q;
    }
    z v = in[ioff];
    if (a.conj) v.y = -v.y;
    z r = cmul(a.alpha, v);
    if (a.use_beta) r = cadd(r, cmul(a.beta, out[o]));
    out[o] = r;
  }
}

// Permutes whose innermost output index is not the innermost input index, as 32 x 32 tiles
// through LDS: reads run along the input's contiguous index p, writes along the output's last
// index q, both coalesced.  blockIdx.x walks the (p, q) tiles, blockIdx.y the remaining indices.
struct TransArgs {
  int nouter;
  unsigned odim[MAXD], istr[MAXD], ostr[MAXD];   // the remaining output indices, outermost first
  unsigned Dp, Dq, istr_q, ostr_p, ntq, nouter_total;
  z alpha, beta;
  int conj, use_beta;
};
constexpr int TT = 32, TR = 8;
__global__ void __launch_bounds__(TT * TR) k_permute_tiled(const z* __restrict__ in, z* __restrict__ out, TransArgs a) {
  __shared__ z tile[TT][TT + 1];
  const unsigned tq = blockIdx.x % a.ntq, tp = blockIdx.x / a.ntq;
  const unsigned p0 = tp * TT, q0 = tq * TT;
  const int tx = threadIdx.x % TT, ty = threadIdx.x / TT;
  for (unsigned ob = blockIdx.y; ob < a.nouter_total; ob += gridDim.y) {
    unsigned rem = ob, ib = 0, obase = 0;
    for (int d = a.nouter - 1; d >= 0; --d) {
      const unsigned q = rem / a.odim[d], c = rem - q * a.odim[d];
      ib += c * a.istr[d];
      obase += c * a.ostr[d];
      rem = q;
    }
#pragma unroll
    for (int r = 0; r < TT / TR; ++r) {
      const unsigned pp = p0 + tx, qq = q0 + ty + TR * r;
      if (pp < a.Dp && qq < a.Dq) tile[ty + TR * r][tx] = in[ib + pp + qq * a.istr_q];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < TT / TR; ++r) {
      const unsigned qq = q0 + tx, pp = p0 + ty + TR * r;
      if (pp < a.Dp && qq < a.Dq) {
        z v = tile[tx][ty + TR * r];
        if (a.conj) v.y = -v.y;
        z res = cmul(a.alpha, v);
        z* dst = out + obase + pp * a.ostr_p + qq;
        if (a.use_beta) res = cadd(res, cmul(a.beta, *dst));
        *dst = res;
      }
    }
    __syncthreads();
  }
}

// r[i,j,a,b] += alpha * P(..) x over 16 x 16 (a, b) tiles, each element of x read once: val (the antisymmetrised
// x of the mode) is antisymmetric in the swapped index pairs, so one workgroup forms it for a tile
// and adds it, with the sign of each image, to every image of the tile -- the (a, b)-transposed
// images through LDS, so that reads and writes stay coalesced.  Images are negations of the same
// floating-point value, so the update is exactly antisymmetric.  Grid: x = (A, B) tile pair (A <= B
// for modes 1 and 3, every pair for mode 2), y = (i, j) (every plane for mode 1, i < j otherwise:
// val vanishes at i = j).
constexpr int AT = 16;
__device__ inline z cneg(z a) { return make_double2(-a.x, -a.y); }
__global__ __launch_bounds__(AT * AT) void k_antisym_tiles(z* r, const z* __restrict__ x, long o, long v, int mode,
                                                           z alpha, const z* base, const z* __restrict__ tsub,
                                                           const double* __restrict__ eps) {
  __shared__ z T[4][AT][AT + 1];
  const int tx = threadIdx.x % AT, ty = threadIdx.x / AT;
  const long nb = (v + AT - 1) / AT;
  long A, B;
  if (mode == 2) {
    A = blockIdx.x / nb;
    B = blockIdx.x % nb;
  } else {
    long q = blockIdx.x;
    A = 0;
    while (q >= nb - A) { q -= nb - A; ++A; }
    B = A + q;
  }
  long i, j;
  if (mode == 1) {
    i = blockIdx.y / o;
    j = blockIdx.y % o;
  } else {
    long q = blockIdx.y;
    i = 0;
    while (q >= o - 1 - i) { q -= o - 1 - i; ++i; }
    j = i + 1 + q;
  }
  const long pij = (i * o + j) * v * v, pji = (j * o + i) * v * v;
  const long A0 = A * AT, B0 = B * AT;
  auto load = [&](int k, long plane, long R0, long C0) {
    const long e = R0 + ty, f = C0 + tx;
    T[k][ty][tx] = (e < v && f < v) ? x[plane + e * v + f] : make_double2(0.0, 0.0);
  };
  // base == r: accumulate; otherwise r = base + alpha val (mode 1 writes every element once);
  // tsub (mode 1): then subtract (eps_i + eps_j - eps_e - eps_f) tsub
  auto add = [&](long plane, long R0, long C0, z val) {
    const long e = R0 + ty, f = C0 + tx;
    if (e < v && f < v) {
      const long off = plane + e * v + f;
      z out = cadd(base[off], cmul(alpha, val));
      if (tsub) {
        const double d = eps[i] + eps[j] - eps[o + e] - eps[o + f];
        const z t = tsub[off];
        out.x -= d * t.x;
        out.y -= d * t.y;
      }
      r[off] = out;
    }
  };
  if (mode == 2) {
    // val = x_ijab - x_jiab: no transpose; r_ij += val, r_ji -= val
    const long e = A0 + ty, f = B0 + tx;
    if (e < v && f < v) {
      const z val = csub(x[pij + e * v + f], x[pji + e * v + f]);
      add(pij, A0, B0, val);
      add(pji, A0, B0, cneg(val));
    }
    return;
  }
  load(0, pij, A0, B0);
  if (A != B) load(1, pij, B0, A0);
  if (mode == 3) {
    load(2, pji, A0, B0);
    if (A != B) load(3, pji, B0, A0);
  }
  __syncthreads();
  const int kBA = A != B ? 1 : 0, kJBA = A != B ? 3 : 2;   // tiles holding x_ijba, x_jiba
  // val of element (a, b) = (A0 + ra, B0 + cb) from the tiles, in the order x_ijab - x_ijba - x_jiab + x_jiba
  auto val_at = [&](int ra, int cb) {
    z w = csub(T[0][ra][cb], T[kBA][cb][ra]);
    if (mode == 3) w = cadd(csub(w, T[2][ra][cb]), T[kJBA][cb][ra]);
    return w;
  };
  const z vab = val_at(ty, tx);          // this thread's element of the (A, B) tile
  add(pij, A0, B0, vab);
  if (mode == 3) add(pji, A0, B0, cneg(vab));
  if (A != B) {
    const z vba = val_at(tx, ty);        // the element whose (B, A) image this thread writes
    add(pij, B0, A0, cneg(vba));
    if (mode == 3) add(pji, B0, A0, vba);
  }
}

// Deterministic dot product: fixed grid, fixed per-thread striding, fixed tree.
constexpr int DOT_BLOCKS = 1024;
constexpr int MAXV = 16;
__global__ void k_dot_partial(long n, const z* __restrict__ x, const z* __restrict__ y, int conjx, z* part) {
  __shared__ double sr[TPB], si[TPB];
  double ar = 0, ai = 0;
  for (long i = blockIdx.x * (long)TPB + threadIdx.x; i < n; i += (long)DOT_BLOCKS * TPB) {
    z a = x[i], b = y[i];
    if (conjx) a.y = -a.y;
    ar += a.x * b.x - a.y * b.y;
    ai += a.x * b.y + a.y * b.x;
  }
  sr[threadIdx.x] = ar; si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; si[threadIdx.x] += si[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = make_double2(sr[0], si[0]);
}
__global__ void k_dot_final(const z* part, z* out) {
  __shared__ double sr[TPB], si[TPB];
  double ar = 0, ai = 0;
  for (int i = threadIdx.x; i < DOT_BLOCKS; i += TPB) { ar += part[i].x; ai += part[i].y; }
  sr[threadIdx.x] = ar; si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; si[threadIdx.x] += si[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = make_double2(sr[0], si[0]);
}
// Several vectors at once (DIIS): one pass over x for all dot products, one pass over the inputs
// of a linear combination.  Vector k is base + slot[k] * stride.
struct MultiArgs {
  int m;
  int slot[MAXV];
  z c[MAXV];
};
// part[b * m + k] = sum over this block's fixed stripe of conj(x) * Y_k
__global__ void k_multi_dot_partial(long n, const z* __restrict__ x, const z* __restrict__ base, long stride,
                                    MultiArgs a, z* __restrict__ part) {
  __shared__ double sr[TPB], si[TPB];
  double ar[MAXV], ai[MAXV];
#pragma unroll
  for (int k = 0; k < MAXV; ++k) { ar[k] = 0; ai[k] = 0; }
  for (long i = blockIdx.x * (long)TPB + threadIdx.x; i < n; i += (long)DOT_BLOCKS * TPB) {
    const z xv = x[i];
#pragma unroll
    for (int k = 0; k < MAXV; ++k) {
      if (k >= a.m) break;
      const z y = base[(long)a.slot[k] * stride + i];
      ar[k] += xv.x * y.x + xv.y * y.y;
      ai[k] += xv.x * y.y - xv.y * y.x;
    }
  }
  for (int k = 0; k < a.m; ++k) {
    sr[threadIdx.x] = ar[k]; si[threadIdx.x] = ai[k];
    __syncthreads();
    for (int s = TPB / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; si[threadIdx.x] += si[threadIdx.x + s]; }
      __syncthreads();
    }
    if (threadIdx.x == 0) part[(long)blockIdx.x * a.m + k] = make_double2(sr[0], si[0]);
    __syncthreads();
  }
}
// out[k] = sum over blocks of part[b * m + k], one workgroup per k, fixed tree
__global__ void k_multi_dot_final(const z* __restrict__ part, int m, z* __restrict__ out) {
  __shared__ double sr[TPB], si[TPB];
  const int k = blockIdx.x;
  double ar = 0, ai = 0;
  for (int b = threadIdx.x; b < DOT_BLOCKS; b += TPB) { ar += part[(long)b * m + k].x; ai += part[(long)b * m + k].y; }
  sr[threadIdx.x] = ar; si[threadIdx.x] = ai;
  __syncthreads();
  for (int s = TPB / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) { sr[threadIdx.x] += sr[threadIdx.x + s]; si[threadIdx.x] += si[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = make_double2(sr[0], si[0]);
}
__global__ void k_lincomb(long n, const z* __restrict__ base, long stride, MultiArgs a, z* __restrict__ out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    z acc = make_double2(0, 0);
    for (int k = 0; k < a.m; ++k) acc = cadd(acc, cmul(a.c[k], base[(long)a.slot[k] * stride + i]));
    out[i] = acc;
  }
}
// v = tnew, e = tnew - told
// Amplitude vectors over the unique entries: t1 (o v), then t2_ij^ab for i < j, a < b in
// lexicographic pair order, b fastest: packed index o v + pij C(v, 2) + pab with
// pij = i (2 o - i - 1) / 2 + j - i - 1 and pab likewise.  One thread per entry of the full layout.
__device__ inline long upair(long i, long j, long n) { return i * (2 * n - i - 1) / 2 + (j - i - 1); }
// v = pack(tnew), e = pack(tnew) - pack(told)
__global__ void k_diis_push_packed(long o, long v, const z* __restrict__ tnew, const z* __restrict__ told,
                                   z* __restrict__ pv, z* __restrict__ pe) {
  const long n1 = o * v, n2 = o * o * v * v, nvp = v * (v - 1) / 2;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < n1 + n2; x += (long)gridDim.x * blockDim.x) {
    long k;
    if (x < n1) {
      k = x;
    } else {
      const long y = x - n1, b = y % v, a = (y / v) % v, j = (y / (v * v)) % o, i = y / (v * v * o);
      if (!(i < j && a < b)) continue;
      k = n1 + upair(i, j, o) * nvp + upair(a, b, v);
    }
    const z p = tnew[x], q = told[x];
    pv[k] = p;
    pe[k] = make_double2(p.x - q.x, p.y - q.y);
  }
}
// full t1 | t2 from the packed vector (antisymmetric images, zeros where i == j or a == b)
__global__ void k_unpack_amps(long o, long v, const z* __restrict__ pk, z* __restrict__ t) {
  const long n1 = o * v, n2 = o * o * v * v, nvp = v * (v - 1) / 2;
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < n1 + n2; x += (long)gridDim.x * blockDim.x) {
    if (x < n1) { t[x] = pk[x]; continue; }
    const long y = x - n1, b = y % v, a = (y / v) % v, j = (y / (v * v)) % o, i = y / (v * v * o);
    if (i == j || a == b) { t[x] = make_double2(0, 0); continue; }
    const bool si = i > j, sa = a > b;
    const z p = pk[n1 + upair(si ? j : i, si ? i : j, o) * nvp + upair(sa ? b : a, sa ? a : b, v)];
    t[x] = (si != sa) ? make_double2(-p.x, -p.y) : p;
  }
}
}  // namespace

void diis_push_packed(fc_ctx ctx, long o, long v, const z* tnew, const z* told, z* pv, z* pe) {
  const long n = o * v + o * o * v * v;
  hipLaunchKernelGGL(k_diis_push_packed, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, o, v, tnew, told, pv, pe);
  FC_HIP(hipGetLastError());
}
void unpack_amps(fc_ctx ctx, long o, long v, const z* packed, z* t) {
  const long n = o * v + o * o * v * v;
  hipLaunchKernelGGL(k_unpack_amps, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, o, v, packed, t);
  FC_HIP(hipGetLastError());
}

void multi_dotc(fc_ctx ctx, long n, const z* x, const z* base, long stride, const int* slot, int m, z* out) {
  FC_REQUIRE(m >= 1 && m <= MAXV, FC_EARG, "multi_dotc: 1..16 vectors");
  MultiArgs a{};
  a.m = m;
  for (int k = 0; k < m; ++k) a.slot[k] = slot[k];
  DBuf part(ctx, sizeof(z) * ((size_t)DOT_BLOCKS * m + m));
  z* fin = part.as<z>() + (size_t)DOT_BLOCKS * m;
  hipLaunchKernelGGL(k_multi_dot_partial, dim3(DOT_BLOCKS), dim3(TPB), 0, ctx->stream, n, x, base, stride, a,
                     part.as<z>());
  hipLaunchKernelGGL(k_multi_dot_final, dim3(m), dim3(TPB), 0, ctx->stream, part.as<z>(), m, fin);
  FC_HIP(hipGetLastError());
  FC_HIP(hipMemcpyAsync(out, fin, sizeof(z) * m, hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
}
void lincomb(fc_ctx ctx, long n, const z* base, long stride, const int* slot, const z* c, int m, z* out) {
  FC_REQUIRE(m >= 1 && m <= MAXV, FC_EARG, "lincomb: 1..16 vectors");
  MultiArgs a{};
  a.m = m;
  for (int k = 0; k < m; ++k) { a.slot[k] = slot[k]; a.c[k] = c[k]; }
  hipLaunchKernelGGL(k_lincomb, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, n, base, stride, a, out);
  FC_HIP(hipGetLastError());
}
void fill(fc_ctx ctx, z* p, long n, z value) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, p, n, value);
  FC_HIP(hipGetLastError());
}
void scale(fc_ctx ctx, z* p, long n, z alpha) {
  if (n <= 0) return;
  if (alpha.x == 0.0 && alpha.y == 0.0) { fill(ctx, p, n, make_double2(0, 0)); return; }
  hipLaunchKernelGGL(k_scale, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, p, n, alpha);
  FC_HIP(hipGetLastError());
}
void axpy(fc_ctx ctx, long n, z alpha, const z* x, z* y) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_axpy, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, n, alpha, x, y);
  FC_HIP(hipGetLastError());
}
void copy_conj(fc_ctx ctx, long n, const z* x, z* y, bool conj) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_copy, dim3(nblocks(n, 4)), dim3(TPB), 0, ctx->stream, n, x, y, (int)conj);
  FC_HIP(hipGetLastError());
}

void permute(fc_ctx ctx, const ZT& in, const std::vector<int>& perm, z alpha, z beta, z* out, bool conj) {
  const int nd = (int)in.dims.size();
  FC_REQUIRE((int)perm.size() == nd && nd <= MAXD, FC_EARG, "permute: bad rank");
  PermArgs a;
  a.nd = nd;
  std::vector<long> istr(nd);
  long s = 1;
  for (int d = nd - 1; d >= 0; --d) { istr[d] = s; s *= in.dims[d]; }
  a.n = s;
  for (int d = 0; d < nd; ++d) { a.odims[d] = in.dims[perm[d]]; a.istr[d] = istr[perm[d]]; }
  a.alpha = alpha; a.beta = beta; a.conj = conj;
  a.use_beta = (beta.x != 0.0 || beta.y != 0.0);
  if (a.n <= 0) return;
  if (a.n >= (1L << 31)) {
    hipLaunchKernelGGL(k_permute, dim3(nblocks(a.n, 4)), dim3(TPB), 0, ctx->stream, in.p, out, a);
    FC_HIP(hipGetLastError());
    return;
  }
  // p: the output index that is contiguous in the input; q: the last output index
  int p = -1;
  for (int d = 0; d < nd; ++d)
    if (a.istr[d] == 1 && a.odims[d] > 1) p = d;
  const int q = nd - 1;
  if (p >= 0 && p != q && a.odims[p] >= 8 && a.odims[q] >= 8) {
    TransArgs t{};
    std::vector<long> ostr(nd);
    long os = 1;
    for (int d = nd - 1; d >= 0; --d) { ostr[d] = os; os *= a.odims[d]; }
    t.nouter = 0;
    long nout = 1;
    for (int d = 0; d < nd; ++d) {
      if (d == p || d == q) continue;
      t.odim[t.nouter] = (unsigned)a.odims[d];
      t.istr[t.nouter] = (unsigned)a.istr[d];
      t.ostr[t.nouter] = (unsigned)ostr[d];
      ++t.nouter;
      nout *= a.odims[d];
    }
    t.Dp = (unsigned)a.odims[p]; t.Dq = (unsigned)a.odims[q];
    t.istr_q = (unsigned)a.istr[q]; t.ostr_p = (unsigned)ostr[p];
    t.ntq = (unsigned)((t.Dq + TT - 1) / TT);
    t.nouter_total = (unsigned)nout;
    t.alpha = alpha; t.beta = beta; t.conj = conj; t.use_beta = a.use_beta;
    const long ntiles = (long)t.ntq * ((t.Dp + TT - 1) / TT);
    FC_REQUIRE(ntiles < (1L << 31), FC_EARG, "permute: too many tiles");
    const unsigned gy = (unsigned)std::max(1L, std::min(nout, 65535L));
    hipLaunchKernelGGL(k_permute_tiled, dim3((unsigned)ntiles, gy), dim3(TT * TR), 0, ctx->stream, in.p, out, t);
    FC_HIP(hipGetLastError());
    return;
  }
  PermArgs32 b{};
  b.nd = nd;
  for (int d = 0; d < nd; ++d) { b.odims[d] = (unsigned)a.odims[d]; b.istr[d] = (unsigned)a.istr[d]; }
  b.n = (unsigned)a.n;
  b.alpha = alpha; b.beta = beta; b.conj = conj; b.use_beta = a.use_beta;
  hipLaunchKernelGGL(k_permute32, dim3(nblocks(a.n, 4)), dim3(TPB), 0, ctx->stream, in.p, out, b);
  FC_HIP(hipGetLastError());
}

void antisym_add(fc_ctx ctx, z* r, const z* x, long o, long v, int mode, z alpha, const z* base, const z* tsub,
                 const double* eps) {
  FC_REQUIRE((!base && !tsub) || mode == 1, FC_EARG, "antisym_add: a separate base or tsub needs mode 1");
  FC_REQUIRE(!tsub || eps, FC_EARG, "antisym_add: tsub needs eps");
  long n = o * o * v * v;
  if (n <= 0) return;
  const long nb = (v + AT - 1) / AT;
  const long gx = mode == 2 ? nb * nb : nb * (nb + 1) / 2, gy = mode == 1 ? o * o : o * (o - 1) / 2;
  if (gy <= 0) return;
  FC_REQUIRE(gx < (1L << 31) && gy <= 65535, FC_EARG, "antisym_add: too many tiles");
  hipLaunchKernelGGL(k_antisym_tiles, dim3((unsigned)gx, (unsigned)gy), dim3(AT * AT), 0, ctx->stream, r, x, o, v,
                     mode, alpha, base ? base : r, tsub, eps);
  FC_HIP(hipGetLastError());
}

static z dot_impl(fc_ctx ctx, long n, const z* x, const z* y, int conjx) {
  if (n <= 0) return make_double2(0, 0);
  DBuf part(ctx, sizeof(z) * (DOT_BLOCKS + 1));
  hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(TPB), 0, ctx->stream, n, x, y, conjx, part.as<z>());
  hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(TPB), 0, ctx->stream, part.as<z>(), part.as<z>() + DOT_BLOCKS);
  FC_HIP(hipGetLastError());
  z h;
  FC_HIP(hipMemcpyAsync(&h, part.as<z>() + DOT_BLOCKS, sizeof(z), hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  return h;
}
z dotu(fc_ctx ctx, long n, const z* x, const z* y) { return dot_impl(ctx, n, x, y, 0); }
z dotc(fc_ctx ctx, long n, const z* x, const z* y) { return dot_impl(ctx, n, x, y, 1); }

// ------------------------------------------------------------------------------ contraction planner
// Transpose-transpose-GEMM-transpose: permute operands only when their index order does not
// already form [free, summed] blocks, run one complex GEMM, and permute the product into C only
// when C's order is neither [freeA, freeB] nor [freeB, freeA].
namespace {
struct Spec { std::string a, b, c; };
Spec parse(const char* s) {
  Spec r;
  std::string str(s);
  auto comma = str.find(','), arrow = str.find("->");
  FC_REQUIRE(comma != std::string::npos && arrow != std::string::npos, FC_EARG, "zein: bad spec");
  r.a = str.substr(0, comma);
  r.b = str.substr(comma + 1, arrow - comma - 1);
  r.c = str.substr(arrow + 2);
  return r;
}
bool is_perm_of(const std::string& x, const std::string& set) {
  if (x.size() != set.size()) return false;
  for (char ch : x) if (set.find(ch) == std::string::npos) return false;
  return true;
}
std::vector<int> perm_to(const std::string& from, const std::string& to) {
  std::vector<int> p;
  for (char ch : to) p.push_back((int)from.find(ch));
  return p;
}
// Output map for a product whose rows run over rowOrd and columns over colOrd (each row-major)
// into C with index order cOrd: possible when each side's indices (those of extent > 1) form at
// most two runs that are also consecutive and contiguous in C.
bool out_map(const std::string& cOrd, std::map<char, long>& dim, const std::string& rowOrd,
             const std::string& colOrd, OutMap& om) {
  std::map<char, long> str;
  long st = 1;
  for (int k = (int)cOrd.size() - 1; k >= 0; --k) { str[cOrd[k]] = st; st *= dim[cOrd[k]]; }
  auto side = [&](const std::string& ord, long& d, long& s1, long& s2) {
    std::vector<std::string> runs;
    for (char ch : ord) {
      if (dim[ch] == 1) continue;
      if (!runs.empty() && str[runs.back().back()] == dim[ch] * str[ch]) runs.back() += ch;
      else runs.push_back(std::string(1, ch));
    }
    auto ext = [&](const std::string& r) { long e = 1; for (char ch : r) e *= dim[ch]; return e; };
    if (runs.size() > 2) return false;
    if (runs.empty()) { d = 1; s1 = 0; s2 = 0; }
    else if (runs.size() == 1) { d = ext(runs[0]); s1 = 0; s2 = str[runs[0].back()]; }
    else { d = ext(runs[1]); s1 = str[runs[0].back()]; s2 = str[runs[1].back()]; }
    return true;
  };
  return side(rowOrd, om.rd, om.rs1, om.rs2) && side(colOrd, om.cd, om.cs1, om.cs2);
}
}  // namespace

void zein(fc_ctx ctx, const char* spec, z alpha, const ZT& A, const ZT& B, z beta, const ZT& C, bool conjA, bool conjB) {
  Spec s = parse(spec);
  FC_REQUIRE(s.a.size() == A.dims.size() && s.b.size() == B.dims.size() && s.c.size() == C.dims.size(),
             FC_EARG, std::string("zein: rank mismatch in ") + spec);
  std::map<char, long> dim;
  auto reg = [&](const std::string& idx, const ZT& t) {
    for (size_t k = 0; k < idx.size(); ++k) {
      auto it = dim.find(idx[k]);
      FC_REQUIRE(it == dim.end() || it->second == t.dims[k], FC_EARG, std::string("zein: dim mismatch in ") + spec);
      dim[idx[k]] = t.dims[k];
    }
  };
  reg(s.a, A); reg(s.b, B); reg(s.c, C);
  std::string K, FA, FB;
  for (char ch : s.a) {
    bool inb = s.b.find(ch) != std::string::npos, inc = s.c.find(ch) != std::string::npos;
    FC_REQUIRE(!(inb && inc), FC_EARG, std::string("zein: batch index unsupported in ") + spec);
    FC_REQUIRE(inb || inc, FC_EARG, std::string("zein: index summed in one operand only in ") + spec);
    if (inb) K += ch; else FA += ch;
  }
  for (char ch : s.b) {
    bool ina = s.a.find(ch) != std::string::npos, inc = s.c.find(ch) != std::string::npos;
    FC_REQUIRE(ina || inc, FC_EARG, std::string("zein: index summed in one operand only in ") + spec);
    if (!ina) FB += ch;
  }
  FC_REQUIRE(is_perm_of(s.c, FA + FB), FC_EARG, std::string("zein: output indices mismatch in ") + spec);
  auto prod = [&](const std::string& x) { long p = 1; for (char ch : x) p *= dim[ch]; return p; };
  const long M = prod(FA), N = prod(FB), KK = prod(K);

  // Plan: the order of the summed indices (kOrd) decides which operands can be used in place.
  // Candidates are the orders in which either operand already holds its summed indices
  // contiguously; the plan that moves the fewest bytes through permutations wins.
  struct Plan {
    std::string kOrd, faOrd, fbOrd;
    bool permA = false, permB = false, permC = false, mapC = false, flipC = false;
    char opA = 'N', opB = 'N';
    OutMap om;
    double cost = 0;
  };
  std::string cFA, cFB;   // free indices in the output's order
  for (char ch : s.c) (FA.find(ch) != std::string::npos ? cFA : cFB) += ch;
  // A mapped output is stored coalesced when consecutive columns of the product are consecutive in
  // C (the column side's innermost run has stride 1): the matrix-core tile stores 16 consecutive
  // columns per row.  Other maps scatter every element to its own cache line and cost more than
  // the permutation they replace (measured), so they are not used.
  auto coalesced = [](const OutMap& m) { return m.cs2 == 1; };
  // forceA / forceB: reorder that operand into the output's index order even when it could be used
  // in place (a small operand reordered can turn a large output permutation into a coalesced map)
  auto plan_for = [&](const std::string& kOrd, bool forceA, bool forceB) {
    Plan p;
    p.kOrd = kOrd;
    const std::string pre = s.a.substr(0, FA.size()), post = s.a.substr(FA.size());
    const std::string pre2 = s.a.substr(0, K.size()), post2 = s.a.substr(K.size());
    if (!forceA && is_perm_of(pre, FA) && post == kOrd) { p.faOrd = pre; p.opA = conjA ? 'R' : 'N'; }
    else if (!forceA && pre2 == kOrd && is_perm_of(post2, FA)) { p.faOrd = post2; p.opA = conjA ? 'C' : 'T'; }
    else { p.faOrd = cFA; p.permA = true; p.opA = 'N'; }
    const std::string bpre = s.b.substr(0, K.size()), bpost = s.b.substr(K.size());
    const std::string bpre2 = s.b.substr(0, FB.size()), bpost2 = s.b.substr(FB.size());
    if (!forceB && bpre == kOrd && is_perm_of(bpost, FB)) { p.fbOrd = bpost; p.opB = conjB ? 'R' : 'N'; }
    else if (!forceB && bpost2 == kOrd && is_perm_of(bpre2, FB)) { p.fbOrd = bpre2; p.opB = conjB ? 'C' : 'T'; }
    else { p.fbOrd = cFB; p.permB = true; p.opB = 'N'; }
    p.permC = !(s.c == p.faOrd + p.fbOrd || s.c == p.fbOrd + p.faOrd);
    // an output the product can store in place, coalesced, through an output map needs no
    // permutation; flipC: as the transposed product (rows from B, columns from A)
    if (p.permC && KK > 0 && M < (1L << 31) && N < (1L << 31)) {
      OutMap m;
      if (out_map(s.c, dim, p.faOrd, p.fbOrd, m) && coalesced(m)) { p.mapC = true; p.om = m; }
      else if (out_map(s.c, dim, p.fbOrd, p.faOrd, m) && coalesced(m)) { p.mapC = p.flipC = true; p.om = m; }
      if (p.mapC) p.permC = false;
    }
    p.cost = (p.permA ? 2.0 * A.size() : 0.0) + (p.permB ? 2.0 * B.size() : 0.0) + (p.permC ? 3.0 * M * N : 0.0);
    return p;
  };
  std::vector<std::string> cands;
  auto add = [&](const std::string& k) {
    if (is_perm_of(k, K) && std::find(cands.begin(), cands.end(), k) == cands.end()) cands.push_back(k);
  };
  add(s.a.substr(FA.size()));
  add(s.a.substr(0, K.size()));
  add(s.b.substr(0, K.size()));
  add(s.b.substr(FB.size()));
  add(K);
  Plan best;
  best.cost = -1;
  for (const auto& k : cands)
    for (int f = 0; f < 4; ++f) {
      Plan p = plan_for(k, f & 1, f & 2);
      if (best.cost < 0 || p.cost < best.cost) best = p;
    }
  if (ctx->verbose >= 2 && (best.cost > 0 || best.mapC))
    fprintf(stderr, "[zein] %s permutes A:%d B:%d C:%d%s (%.1f MB moved)\n", spec, best.permA, best.permB, best.permC,
            best.mapC ? " (output mapped)" : "", best.cost * sizeof(z) / 1e6);
  const std::string& kOrd = best.kOrd;
  const std::string faOrd = best.faOrd, fbOrd = best.fbOrd;
  const z* Ap = A.p; char opA = best.opA; DBuf Atmp;
  if (best.permA) {
    Atmp = DBuf(ctx, sizeof(z) * std::max(1L, A.size()));
    permute(ctx, A, perm_to(s.a, faOrd + kOrd), make_double2(1, 0), make_double2(0, 0), Atmp.as<z>(), conjA);
    Ap = Atmp.as<z>();
  }
  const z* Bp = B.p; char opB = best.opB; DBuf Btmp;
  if (best.permB) {
    Btmp = DBuf(ctx, sizeof(z) * std::max(1L, B.size()));
    permute(ctx, B, perm_to(s.b, kOrd + fbOrd), make_double2(1, 0), make_double2(0, 0), Btmp.as<z>(), conjB);
    Bp = Btmp.as<z>();
  }
  const long lda = (opA == 'N' || opA == 'R') ? KK : M;
  const long ldb = (opB == 'N' || opB == 'R') ? N : KK;
  // C^T = op(B)^T op(A)^T: swap operands and flip their transposition.
  auto flip = [](char op) { return op == 'N' ? 'T' : op == 'T' ? 'N' : op == 'R' ? 'C' : 'R'; };
  if (best.mapC && !best.flipC) {
    zgemm_mapped(ctx, opA, opB, M, N, KK, alpha, Ap, lda, Bp, ldb, beta, C.p, best.om);
  } else if (best.mapC) {
    zgemm_mapped(ctx, flip(opB), flip(opA), N, M, KK, alpha, Bp, ldb, Ap, lda, beta, C.p, best.om);
  } else if (s.c == faOrd + fbOrd) {
    zgemm(ctx, opA, opB, M, N, KK, alpha, Ap, lda, Bp, ldb, beta, C.p, N);
  } else if (s.c == fbOrd + faOrd) {
    zgemm(ctx, flip(opB), flip(opA), N, M, KK, alpha, Bp, ldb, Ap, lda, beta, C.p, M);
  } else {
    DBuf Ctmp(ctx, sizeof(z) * std::max(1L, M * N));
    zgemm(ctx, opA, opB, M, N, KK, make_double2(1, 0), Ap, lda, Bp, ldb, make_double2(0, 0), Ctmp.as<z>(), N);
    std::vector<long> tdims;
    std::string tord = faOrd + fbOrd;
    for (char ch : tord) tdims.push_back(dim[ch]);
    permute(ctx, ZT(Ctmp.as<z>(), tdims), perm_to(tord, s.c), alpha, beta, C.p);
  }
}

}  // namespace fc
