// Cholesky-vector staging and assembly of the stored antisymmetrised integrals.
//
// Eq. 21/23: (pr|qs) = sum_P L^P_pr L^P_qs and <pq||rs> = (pr|qs) - (ps|qr).  Each Mulliken block
// is one complex GEMM over P (K = ncd) with both operands P-contiguous; the antisymmetrised block
// is then formed by index permutation.  Only blocks with at most two virtual indices are stored.
#include "fc_state.hpp"

namespace fc {
namespace {
constexpr int TPB = 256;

// Staging of one block: out[p - p0][q - q0][P] = L[P][p][q] (complex128 or complex64 in, O = double2
// or float2 out), as a transpose per bra spinor p: 32 x 32 tiles
// of (P, q) through LDS so that both the read (q fastest) and the write (P fastest) are coalesced.
// grid: (ceil(nq / 32), ceil(ncd / 32), np), 256 threads.
template <class T, class O>
__global__ __launch_bounds__(256) void k_stage_block_t(const T* __restrict__ L, long n, long ncd, long p0, long q0,
                                                       long nq, O* __restrict__ out) {
  __shared__ O tile[32][33];
  const long p = blockIdx.z, qb = (long)blockIdx.x * 32, Pb = (long)blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const long P = Pb + r, q = qb + tx;
    O val{};
    if (P < ncd && q < nq) {
      const T x = L[(P * n + p0 + p) * n + q0 + q];
      val.x = x.x;
      val.y = x.y;
    }
    tile[r][tx] = val;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const long q = qb + r, P = Pb + tx;
    if (q < nq && P < ncd) out[(p * nq + q) * ncd + P] = tile[tx][r];
  }
}

__global__ void k_widen(const float2* __restrict__ in, z* __restrict__ out, long n) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    out[t] = make_double2((double)in[t].x, (double)in[t].y);
}
}  // namespace

const ZTensor& lvv(fc_ctx ctx, fc_ints I) {
  if (!I->Lvv.p()) {
    FC_REQUIRE(I->Lvv64.p, FC_EARG, "no virtual-virtual Cholesky block staged");
    const long v = I->v, N = I->ncd, n = v * v * N;
    I->Lvv = ZTensor(ctx, {v, v, N});
    hipLaunchKernelGGL(k_widen, dim3((unsigned)std::min<long>(1048576, (n + TPB * 4 - 1) / (TPB * 4))), dim3(TPB), 0,
                       ctx->stream, I->Lvv64.as<float2>(), I->Lvv.p(), n);
    FC_HIP(hipGetLastError());
  }
  return I->Lvv;
}

void ensure_integrals(fc_ctx ctx, fc_ints I) {
  if (I->assembled) return;
  assemble_integrals(ctx, I);
  I->assembled = true;
}

// Stage the L blocks from L[P][p][q] (device, complex128 or complex64).  The occupied blocks are
// complex128; L_vv keeps the input type (complex64 vectors: Lvv64, widened only on demand).
void stage_cholesky(fc_ctx ctx, fc_ints I, const void* Ldev, int l_dtype) {
  const long o = I->o, v = I->v, n = o + v, N = I->ncd;
  I->Loo = ZTensor(ctx, {o, o, N});
  I->Lov = ZTensor(ctx, {o, v, N});
  I->Lvo = ZTensor(ctx, {v, o, N});
  const bool c64 = l_dtype == FC_C64;
  if (c64) I->Lvv64 = DBuf(ctx, sizeof(float2) * (size_t)v * v * N);
  else I->Lvv = ZTensor(ctx, {v, v, N});
  struct B { void* out; bool f32; long p0, np, q0, nq; } blocks[4] = {
      {I->Loo.p(), false, 0, o, 0, o}, {I->Lov.p(), false, 0, o, o, v}, {I->Lvo.p(), false, o, v, 0, o},
      {c64 ? I->Lvv64.p : (void*)I->Lvv.p(), c64, o, v, o, v}};
  for (auto& b : blocks) {
    FC_REQUIRE(b.np <= 65535, FC_EARG, "stage_cholesky: more than 65535 spinors in a block");
    const dim3 grid((unsigned)((b.nq + 31) / 32), (unsigned)((N + 31) / 32), (unsigned)b.np);
    if (!c64)
      hipLaunchKernelGGL((k_stage_block_t<double2, double2>), grid, dim3(TPB), 0, ctx->stream, (const double2*)Ldev,
                         n, N, b.p0, b.q0, b.nq, (double2*)b.out);
    else if (b.f32)
      hipLaunchKernelGGL((k_stage_block_t<float2, float2>), grid, dim3(TPB), 0, ctx->stream, (const float2*)Ldev, n,
                         N, b.p0, b.q0, b.nq, (float2*)b.out);
    else
      hipLaunchKernelGGL((k_stage_block_t<float2, double2>), grid, dim3(TPB), 0, ctx->stream, (const float2*)Ldev,
                         n, N, b.p0, b.q0, b.nq, (double2*)b.out);
    FC_HIP(hipGetLastError());
  }
}

// J[(p,r),(q,s)] = sum_P X[p,r,P] Y[q,s,P]   (Mulliken block, one GEMM, K = ncd)
static void mulliken(fc_ctx ctx, int precision, const ZTensor& X, const ZTensor& Y, ZTensor& J) {
  const long M = X.dims[0] * X.dims[1], Nn = Y.dims[0] * Y.dims[1], K = X.dims[2];
  J = ZTensor(ctx, {X.dims[0], X.dims[1], Y.dims[0], Y.dims[1]});
  if (precision == FC_FP64)
    zgemm(ctx, 'N', 'T', M, Nn, K, make_double2(1, 0), X.p(), K, Y.p(), K, make_double2(0, 0), J.p(), Nn);
  else
    zgemm_split(ctx, precision, 'N', 'T', M, Nn, K, make_double2(1, 0), X.p(), K, Y.p(), K, make_double2(0, 0),
                J.p(), Nn);
}

void assemble_integrals(fc_ctx ctx, fc_ints I) {
  StageTimer st(ctx, "assemble");
  const long o = I->o, v = I->v;
  const z one = make_double2(1, 0), mone = make_double2(-1, 0), zero = make_double2(0, 0);
  const int prec = I->precision;
  ZTensor J, J2;
  // <mn||ij> = (mi|nj) - (mj|ni);  J[m,i,n,j]
  mulliken(ctx, prec, I->Loo, I->Loo, J);
  I->oooo = ZTensor(ctx, {o, o, o, o});
  permute(ctx, J, {0, 2, 1, 3}, one, zero, I->oooo.p());     // (m,n,i,j) <- J[m,i,n,j]
  permute(ctx, J, {0, 2, 3, 1}, mone, one, I->oooo.p());     // -(mj|ni) = -J[m,j,n,i]
  // <mn||ie> = (mi|ne) - (me|ni);  J[m,i,n,e], (me|ni) = (ni|me) = J[n,i,m,e]
  mulliken(ctx, prec, I->Loo, I->Lov, J);
  I->ooov = ZTensor(ctx, {o, o, o, v});
  permute(ctx, J, {0, 2, 1, 3}, one, zero, I->ooov.p());     // (m,n,i,e) <- J[m,i,n,e]
  permute(ctx, J, {2, 0, 1, 3}, mone, one, I->ooov.p());     // (m,n,i,e) <- J[n,i,m,e]
  // <mn||ef> = (me|nf) - (mf|ne);  J[m,e,n,f]
  mulliken(ctx, prec, I->Lov, I->Lov, J);
  I->oovv = ZTensor(ctx, {o, o, v, v});
  permute(ctx, J, {0, 2, 1, 3}, one, zero, I->oovv.p());
  permute(ctx, J, {0, 2, 3, 1}, mone, one, I->oovv.p());
  // <mb||ej> = (me|bj) - (mj|be);  J[m,e,b,j], J2[m,j,b,e]
  mulliken(ctx, prec, I->Lov, I->Lvo, J);
  mulliken(ctx, prec, I->Loo, lvv(ctx, I), J2);
  I->ovvo = ZTensor(ctx, {o, v, v, o});
  permute(ctx, J, {0, 2, 1, 3}, one, zero, I->ovvo.p());     // (m,b,e,j) <- J[m,e,b,j]
  permute(ctx, J2, {0, 2, 3, 1}, mone, one, I->ovvo.p());    // (m,b,e,j) <- J2[m,j,b,e]
  J = ZTensor(); J2 = ZTensor();
  // symmetry copies
  I->oovo = ZTensor(ctx, {o, o, v, o});                      // <mn||ej> = -<mn||je>
  permute(ctx, I->ooov, {0, 1, 3, 2}, mone, zero, I->oovo.p());
  I->ovov = ZTensor(ctx, {o, v, v, o});                      // <ma||if> = -<ma||fi> as (m,f,a,i)
  permute(ctx, I->ovvo, {0, 2, 1, 3}, mone, zero, I->ovov.p());
  I->ovoo = ZTensor(ctx, {o, v, o, o});                      // <mb||ij> = conj <ij||mb>
  permute(ctx, I->ooov, {2, 3, 0, 1}, one, zero, I->ovoo.p(), true);
  I->vvoo = ZTensor(ctx, {o, o, v, v});                      // <ab||ij> stored as [i][j][a][b]
  copy_conj(ctx, I->oovv.size(), I->oovv.p(), I->vvoo.p(), true);
  I->oovv_r = ZTensor(ctx, {o, v, o, v});                    // (m,e,n,f) <- <mn||ef>
  permute(ctx, I->oovv, {0, 2, 1, 3}, one, zero, I->oovv_r.p());
}

}  // namespace fc
