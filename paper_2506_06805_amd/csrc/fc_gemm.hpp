// GEMM variants used by the particle-particle ladder.
#pragma once
#include "fc_internal.hpp"

namespace fc {

// Output layout of the ladder assembly product: row m = (a - a0) v + e, column n = (b - b0) v + f
// is written to W[((m / v) nB + n / v) v^2 + (m % v) v + n % v], i.e. [(a, b)][e][f].  With
// `triangular` (a diagonal block pair, a0 == b0) output tiles whose smallest a exceeds their
// largest b are not computed.
struct LadderEpilogue {
  long v = 1, nB = 1;
  int triangular = 0;
};

// Number of tile configurations the FP64 product kernels offer (autotuner table entries).
int gemm_num_configs();

// Allocation-free complex product (fc_zgemm_noalloc): split-K partial sums in a fixed per-device
// workspace of NOALLOC_SCRATCH_BYTES instead of an allocated buffer.  noalloc_scratch_init looks
// the workspace address up for `device` (which must be current); fc_create calls it.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
void noalloc_scratch_init(int device);
void zgemm_noalloc(fc_ctx ctx, char opA, char opB, long M, long N, long K, z alpha, const z* A, long lda,
                   const z* B, long ldb, z beta, z* C, long ldc);

// W = A B^T in the ladder layout, FP64 (A[m * lda + k], B[n * ldb + k]).
void zgemm_ladder(fc_ctx ctx, long M, long N, long K, const z* A, long lda, const z* B, long ldb, z* W,
                  const LadderEpilogue& lep);

// ---------------------------------------------------------------------------- grouped products
// One product of a grouped launch: C_b = alpha op(A_b) op(B_b) + beta C_b for b < batch, with the
// operand conventions of zgemm and batch strides sA, sB, sC.  Products of one launch must not
// write memory that another product of the same launch reads or writes.
struct GroupGemm {
  char opA = 'N', opB = 'N';
  long M = 0, N = 0, K = 0;
  z alpha{1, 0};
  const z* A = nullptr; long lda = 0, sA = 0;
  const z* B = nullptr; long ldb = 0, sB = 0;
  z beta{0, 0};
  z* C = nullptr; long ldc = 0, sC = 0;
  long batch = 1;
};
// Tile configuration (0: 64 x 64, 1: 128 x 64) and the longest K range one tile covers; longer
// products are split over K and summed in a fixed order by a second kernel.
struct GroupTiling {
  int cfg = 0;
  long kchunk = 512;
};
struct GroupCounts {
  size_t plan_bytes = 0, work = 0;   // plan size (bytes), split-K workspace (complex elements)
  long tiles = 0, elems = 0;         // tiles of the persistent launch, elements of the reduction
};
// Writes the device plan for `probs` into host memory (nullptr: only count).  `work` is the
// split-K workspace the plan will point into.
GroupCounts group_encode(const std::vector<GroupGemm>& probs, const GroupTiling& tl, void* host_plan,
                         size_t plan_cap, z* work, size_t work_cap);
// Launches the persistent product kernel and the split-K reduction over a device plan.  The grids
// are sized for at most max_tiles tiles and max_elems reduced elements, so a graph captured with
// the largest plan replays correctly with any smaller one written to the same address.
void group_launch(fc_ctx ctx, int cfg, const void* dplan, long max_tiles, long max_elems);
// Plans, uploads and runs one grouped launch (synchronises the stream before returning).
void group_gemm(fc_ctx ctx, const std::vector<GroupGemm>& probs, const GroupTiling& tl);

// Pinned host + device staging for a sequence of grouped launches between two synchronisations:
// each run() encodes its plan into the next free slice, uploads it and launches.  reset() after
// the stream has drained makes the whole arena free again.
struct GroupArena {
  fc_ctx ctx = nullptr;
  char* host = nullptr;
  DBuf dev, work;
  size_t cap = 0, off = 0, wcap = 0, woff = 0;
  GroupArena() = default;
  GroupArena(fc_ctx c, size_t plan_bytes, size_t work_elems);
  GroupArena(const GroupArena&) = delete;
  GroupArena& operator=(const GroupArena&) = delete;
  ~GroupArena();
  void reset() { off = 0; woff = 0; }
  void run(const std::vector<GroupGemm>& probs, const GroupTiling& tl);
};

}  // namespace fc
