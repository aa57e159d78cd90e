// Internal declarations of libfnscc (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fnscc.h"

namespace fc {

using z = double2;  // complex FP64, interleaved (re, im)

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define FC_HIP(call)                                                                        \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      throw ::fc::Error(FC_EHIP, std::string(#call) + ": " + hipGetErrorString(e_) + " at " + \
                                     __FILE__ + ":" + std::to_string(__LINE__));            \
  } while (0)

#define FC_REQUIRE(cond, code, msg)                 \
  do {                                              \
    if (!(cond)) throw ::fc::Error((code), (msg));  \
  } while (0)

}  // namespace fc

// ----------------------------------------------------------------------------------------------
// Context: device, stream, allocator callbacks, a size-keyed cache of freed blocks.
struct fc_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  fc_alloc_fn alloc = nullptr;
  fc_free_fn release = nullptr;
  void* user = nullptr;
  std::string last_error;
  std::multimap<size_t, void*> cache;          // freed blocks kept for reuse
  std::unordered_map<void*, size_t> live;      // pointer -> rounded size
  size_t cached_bytes = 0;
  int verbose = 0;
  // per-stage timers (ms), filled when timing is enabled
  int timing = 0;          // bit 0: per-stage timers (synchronising); bit 1: ladder events only
  std::map<std::string, double> stage_ms;
  std::map<std::string, long> stage_calls;
  // hipEvents bracketing ladder launches (measured on this context's stream)
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ladder_events;
  // while set, zgemm products run on the FP32 matrix cores (operands rounded to FP32 at staging,
  // FP32 sums, FP64 result); the particle-particle ladder's own products are not affected
  int gemm_fp32 = 0;
  // GEMM autotuning: shape bucket -> chosen configuration (and its measured time in ms)
  int autotune = 0;
  std::map<std::string, std::pair<int, float>> tune;
  // forced tile configuration of single products (-1: heuristic or autotuner)
  int gemm_cfg = -1;
  // forced staging of the 128-wide split-precision tiles (-1: default)
  int split_cfg = -1;
};

namespace fc {

void* dmalloc(fc_ctx ctx, size_t bytes);
void dfree(fc_ctx ctx, void* p);
void release_cache(fc_ctx ctx);

// Owning device buffer (freed back into the context cache).
struct DBuf {
  fc_ctx ctx = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(fc_ctx c, size_t b) : ctx(c), p(b ? dmalloc(c, b) : nullptr), bytes(b) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : ctx(o.ctx), p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) { reset(); ctx = o.ctx; p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() { if (p && ctx) dfree(ctx, p); p = nullptr; bytes = 0; }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Non-owning row-major complex tensor view.
struct ZT {
  z* p = nullptr;
  std::vector<long> dims;
  long size() const { long s = 1; for (long d : dims) s *= d; return s; }
  ZT() = default;
  ZT(z* p_, std::vector<long> d) : p(p_), dims(std::move(d)) {}
};

// Owning complex tensor.
struct ZTensor {
  DBuf buf;
  std::vector<long> dims;
  ZTensor() = default;
  ZTensor(fc_ctx c, std::vector<long> d) : dims(std::move(d)) {
    long s = 1; for (long x : dims) s *= x;
    buf = DBuf(c, (size_t)s * sizeof(z));
  }
  z* p() const { return buf.as<z>(); }
  long size() const { long s = 1; for (long d : dims) s *= d; return s; }
  ZT view() const { return ZT(p(), dims); }
  operator ZT() const { return view(); }
};

// ---------------------------------------------------------------- kernels (fc_gemm.hip)
// Row-major complex GEMM, C = alpha * op(A) op(B) + beta * C, FP64 MFMA.
// opA: 'N' A[m*lda+k], 'T' A[k*lda+m], 'C' conj(A[k*lda+m]), 'R' conj(A[m*lda+k]).
// opB: 'N' B[k*ldb+n], 'T' B[n*ldb+k], 'C' conj(B[n*ldb+k]), 'R' conj(B[k*ldb+n]).
void zgemm(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
           const z* B, long ldb, z beta, z* C, long ldc, int batch = 1, long sA = 0, long sB = 0,
           long sC = 0);
// Output layout of a product whose row and column indices each split into two sub-indices with
// strides of their own (a contraction whose free indices interleave in the output tensor):
// element (m, n) is C[(m / rd) rs1 + (m % rd) rs2 + (n / cd) cs1 + (n % cd) cs2].  rd divides M
// and cd divides N, so the map is known to reach exactly its largest offset (span()).
struct OutMap {
  long rd = 1, rs1 = 0, rs2 = 0, cd = 1, cs1 = 0, cs2 = 0;
  long span(long M, long N) const {
    return (M / rd - 1) * rs1 + (rd - 1) * rs2 + (N / cd - 1) * cs1 + (cd - 1) * cs2 + 1;
  }
};
// C = alpha sum_b op(A_b) op(B_b) + beta C over b < batch (A_b = A + b sA, B_b = B + b sB): one
// batched product into a workspace, then the partial products summed in batch order (a contraction
// whose summed indices include the operands' leading ones, e.g. a pair index).
void zgemm_sum(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda, long sA,
               const z* B, long ldb, long sB, int batch, z beta, z* C, long ldc);
// C_b = alpha op(A_b) op(B_b) + beta C_b with each C_b (at C + b sC) laid out by `om`.
void zgemm_mapped(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
                  const z* B, long ldb, z beta, z* C, const OutMap& om, int batch = 1, long sA = 0, long sB = 0,
                  long sC = 0);

// Split-precision variant (hi/lo BF16 or FP16 parts, FP32 accumulation, three products).
void zgemm_split(fc_ctx ctx, int precision, char opA, char opB, long M, long N, long K, z alpha,
                 const z* A, long lda, const z* B, long ldb, z beta, z* C, long ldc);

// ---------------------------------------------------------------- tensor ops (fc_tensor.hip)
void fill(fc_ctx ctx, z* p, long n, z value);
void scale(fc_ctx ctx, z* p, long n, z alpha);
void axpy(fc_ctx ctx, long n, z alpha, const z* x, z* y);               // y += alpha x
void copy_conj(fc_ctx ctx, long n, const z* x, z* y, bool conj);
// out[perm index] = alpha * op(in) + beta * out; in has dims `dims` (row-major), the output
// dims are dims[perm[0]], dims[perm[1]], ...
void permute(fc_ctx ctx, const ZT& in, const std::vector<int>& perm, z alpha, z beta, z* out,
             bool conj = false);
// Einstein-summation contraction of two tensors into a third (two operands, no batch indices):
// C = alpha * sum A B + beta * C; conjA/conjB conjugate an operand.
void zein(fc_ctx ctx, const char* spec, z alpha, const ZT& A, const ZT& B, z beta, const ZT& C,
          bool conjA = false, bool conjB = false);
// r[i,j,a,b] += x - x^(a<->b) (mode 1), x - x^(i<->j) (mode 2),
// x - x^(ij) - x^(ab) + x^(ij,ab) (mode 3); dims o,o,v,v.
// base (mode 1 only, which writes every element once): r = base + alpha P(ab) x instead of r += ...
// tsub, eps (mode 1 only): afterwards r -= (eps_i + eps_j - eps_a - eps_b) tsub (the doubles
// residual's Omega = RHS - D t in the same pass)
void antisym_add(fc_ctx ctx, z* r, const z* x, long o, long v, int mode, z alpha, const z* base = nullptr,
                 const z* tsub = nullptr, const double* eps = nullptr);
// Dot products with FP64 accumulation in a fixed order (deterministic).
z dotu(fc_ctx ctx, long n, const z* x, const z* y);    // sum x*y
z dotc(fc_ctx ctx, long n, const z* x, const z* y);    // sum conj(x)*y
// Vectors base + slot[k] * stride, k < m <= 16 (DIIS history): out[k] = dotc(x, vector k) on the
// host (one pass over x, fixed order); out = sum_k c[k] vector k (one pass).
void multi_dotc(fc_ctx ctx, long n, const z* x, const z* base, long stride, const int* slot, int m, z* out);
void lincomb(fc_ctx ctx, long n, const z* base, long stride, const int* slot, const z* c, int m, z* out);
// Packed amplitude vectors (t1, then t2 over i < j, a < b): pv = pack(tnew), pe = pack(tnew - told)
// from full-layout t1 | t2 vectors; unpack_amps writes the full layout back (antisymmetric images).
void diis_push_packed(fc_ctx ctx, long o, long v, const z* tnew, const z* told, z* pv, z* pe);
void unpack_amps(fc_ctx ctx, long o, long v, const z* packed, z* t);

// Scope in which zgemm runs in FP32 arithmetic (the mixed-precision residual).
struct Fp32Gemms {
  fc_ctx ctx;
  int saved;
  Fp32Gemms(fc_ctx c, bool on) : ctx(c), saved(c->gemm_fp32) { c->gemm_fp32 = on ? 1 : 0; }
  ~Fp32Gemms() { ctx->gemm_fp32 = saved; }
  Fp32Gemms(const Fp32Gemms&) = delete;
  Fp32Gemms& operator=(const Fp32Gemms&) = delete;
};

// Timing helper: adds elapsed stream time of a scope to ctx->stage_ms[name] when enabled.
struct StageTimer {
  fc_ctx ctx; std::string name; hipEvent_t a = nullptr, b = nullptr;
  StageTimer(fc_ctx c, const char* n);
  ~StageTimer();
};

}  // namespace fc
