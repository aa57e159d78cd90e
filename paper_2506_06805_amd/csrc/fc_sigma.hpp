// Batched IP-EOM sigma products (Eq. 17-18) over many instances of uneven size.
#pragma once
#include "fc_gemm.hpp"
#include "fc_state.hpp"

namespace fc {

// Forms T->so from the H-bar blocks (building those first if needed); with `left`, also the two
// matrices of the left products.
void prep_sigma_ops(fc_ctx ctx, fc_ints I, fc_amps T, bool left = false);

// sigma = H-bar R (or the left product R H-bar) for a set of instances, each with its own block of
// trial vectors, as one sequence of four launches shared by every instance: unpack r_ij^a, one
// grouped launch of the products that read R only, one of the products that need X_e (or its left
// counterpart Z_e), and a pack that applies P(ij).
// The launch plans live at fixed device addresses and are rewritten before every call, so with
// `graph` the sequence is captured once into a HIP graph and replayed for any vector counts up to
// the kmax given at construction.  Buffers for kmax vectors per instance are held for the
// object's lifetime; calls are ordered on the context stream.
class SigmaBatch {
 public:
  // left: row vectors times H-bar (Eq. 19-20) instead of H-bar times column vectors (Eq. 18)
  SigmaBatch(fc_ctx ctx, int nb, const fc_ints* I, const fc_amps* T, const long* kmax, bool graph,
             bool left = false);
  ~SigmaBatch();
  SigmaBatch(const SigmaBatch&) = delete;
  SigmaBatch& operator=(const SigmaBatch&) = delete;
  // S_b[0, nvec_b) = sigma(R_b[0, nvec_b)), rows of length dim_b; nvec_b = 0 skips instance b.
  void run(const z* const* R, z* const* S, const long* nvec);
  GroupTiling tiling(int phase) const { return phase == 1 ? tl1_ : tl2_; }

 private:
  void lists(const z* const* R, z* const* S, const long* nvec, std::vector<GroupGemm>& g1,
             std::vector<GroupGemm>& g2, std::vector<char>* tab, long* nu, long* np) const;
  void configure(const GroupTiling& t1, const GroupTiling& t2);
  void upload(const z* const* R, z* const* S, const long* nvec);
  void launch_all();
  void tune(const z* const* R, z* const* S, const long* nvec);

  fc_ctx ctx_;
  int nb_;
  std::vector<fc_ints> I_;
  std::vector<fc_amps> T_;
  std::vector<long> kmax_;
  std::vector<ZTensor> r2_, Y_, x_, s2b_;
  bool graph_, left_;
  bool configured_ = false;
  GroupTiling tl1_, tl2_;
  char* host_ = nullptr;
  DBuf dev_, work1_, work2_;
  size_t cap_ = 0, off_g1_ = 0, off_g2_ = 0, cap_g1_ = 0, cap_g2_ = 0, wcap1_ = 0, wcap2_ = 0;
  long maxt1_ = 0, maxe1_ = 0, maxt2_ = 0, maxe2_ = 0, maxu_ = 0, maxp_ = 0;
  hipEvent_t copied_ = nullptr;
  bool copy_pending_ = false;
  hipGraph_t g_ = nullptr;
  hipGraphExec_t exec_ = nullptr;
};

}  // namespace fc
