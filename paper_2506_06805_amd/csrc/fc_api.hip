// C ABI entry points of libfnscc: context, integral and amplitude handles, CCSD driver (Jacobi +
// complex DIIS), frozen natural spinors, IP-EOM sigma and Davidson.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <sstream>

#include "fc_gemm.hpp"
#include "fc_split.hpp"
#include "fc_state.hpp"

namespace fc {
void stage_cholesky(fc_ctx ctx, fc_ints I, const void* Ldev, int l_dtype);
void jacobi_step(fc_ctx ctx, fc_ints I, const z* t1, const z* t2, const z* r1, const z* r2, z* o1, z* o2,
                 const z* fd = nullptr);
int davidson_batch(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* amps, const int* nroots,
                   const fc_eom_opts& op, z* omega, z* Rout, int* iters, bool left = false);
int left_batch(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* amps, const int* nroots,
               const fc_eom_opts& op, const z* R, z* omega, z* L, z* weight, int* iters);

namespace {
constexpr int TPB = 256;
inline unsigned nblk(long n) { return (unsigned)std::max(1L, std::min(1048576L, (n + TPB * 4 - 1) / (TPB * 4))); }
__global__ void k_mp2_amp(const z* vvoo, const double* eps, z* t, long o, long v) {
  for (long x = blockIdx.x * (long)blockDim.x + threadIdx.x; x < o * o * v * v; x += (long)gridDim.x * blockDim.x) {
    long b = x % v, a = (x / v) % v, j = (x / (v * v)) % o, i = x / (v * v * o);
    double d = eps[i] + eps[j] - eps[o + a] - eps[o + b];
    t[x] = make_double2(vvoo[x].x / d, vvoo[x].y / d);
  }
}
}  // namespace

// ------------------------------------------------------------------------------ CCSD driver
// DIIS history over the unique amplitudes (t1, then t2 for i < j, a < b): a quarter of the doubles
// of the full layout per vector.  Inner products weight the packed t2 part by 4, so the Gram
// matrix and the extrapolation are those of the full antisymmetric vectors.
struct DiisState {
  int size = 8;
  long o = 0, v = 0, n1 = 0, nt = 0;   // nt: packed length
  DBuf vecs, errs, tmp;
  std::deque<int> order;          // slots, oldest first
  std::vector<z> B;               // size x size, by slot
  void init(fc_ctx ctx, int sz, long o_, long v_) {
    size = sz; o = o_; v = v_;
    n1 = o * v;
    nt = n1 + (o * (o - 1) / 2) * (v * (v - 1) / 2);
    vecs = DBuf(ctx, sizeof(z) * (size_t)sz * nt);
    errs = DBuf(ctx, sizeof(z) * (size_t)sz * nt);
    tmp = DBuf(ctx, sizeof(z) * (size_t)nt);
    B.assign((size_t)sz * sz, make_double2(0, 0));
    order.clear();
  }
  z* vec(int s) { return vecs.as<z>() + (size_t)s * nt; }
  z* err(int s) { return errs.as<z>() + (size_t)s * nt; }
};

// push (t_new, t_new - t_old) (full layout) and write the extrapolated amplitudes (full layout) into out
static void diis_push_extrapolate(fc_ctx ctx, DiisState& D, const z* tnew, const z* told, z* out) {
  int slot;
  if ((int)D.order.size() < D.size) {
    std::vector<bool> used(D.size, false);
    for (int s : D.order) used[s] = true;
    slot = 0;
    while (used[slot]) ++slot;
  } else {
    slot = D.order.front();
    D.order.pop_front();
  }
  diis_push_packed(ctx, D.o, D.v, tnew, told, D.vec(slot), D.err(slot));
  D.order.push_back(slot);
  {
    const std::vector<int> sl(D.order.begin(), D.order.end());
    std::vector<z> b1(sl.size()), b2(sl.size());
    multi_dotc(ctx, D.n1, D.err(slot), D.err(0), D.nt, sl.data(), (int)sl.size(), b1.data());
    multi_dotc(ctx, D.nt - D.n1, D.err(slot) + D.n1, D.err(0) + D.n1, D.nt, sl.data(), (int)sl.size(), b2.data());
    for (size_t k = 0; k < sl.size(); ++k) {
      const z bs = make_double2(b1[k].x + 4.0 * b2[k].x, b1[k].y + 4.0 * b2[k].y);
      D.B[slot * D.size + sl[k]] = bs;
      D.B[sl[k] * D.size + slot] = make_double2(bs.x, -bs.y);
    }
  }
  while (D.order.size() >= 2) {
    const int m = (int)D.order.size();
    std::vector<z> A((m + 1) * (size_t)(m + 1), make_double2(0, 0)), rhs(m + 1, make_double2(0, 0));
    double sc = 0;
    for (int k = 0; k < m; ++k) sc = std::max(sc, std::hypot(D.B[D.order[k] * D.size + D.order[k]].x, D.B[D.order[k] * D.size + D.order[k]].y));
    if (sc == 0.0) break;
    for (int k = 0; k < m; ++k)
      for (int l = 0; l < m; ++l) {
        z b = D.B[D.order[k] * D.size + D.order[l]];
        A[k * (m + 1) + l] = make_double2(b.x / sc, b.y / sc);
      }
    for (int k = 0; k < m; ++k) { A[m * (m + 1) + k] = make_double2(1, 0); A[k * (m + 1) + m] = make_double2(1, 0); }
    rhs[m] = make_double2(1, 0);
    if (cond_herm(m + 1, A) < 1e12 && lin_solve(m + 1, A, rhs)) {
      const std::vector<int> sl(D.order.begin(), D.order.end());
      lincomb(ctx, D.nt, D.vec(0), D.nt, sl.data(), rhs.data(), m, D.tmp.as<z>());
      unpack_amps(ctx, D.o, D.v, D.tmp.as<z>(), out);
      return;
    }
    D.order.pop_front();  // ill-conditioned: drop the oldest vector
  }
  unpack_amps(ctx, D.o, D.v, D.vec(D.order.back()), out);
}

static int solve_one(fc_ctx ctx, fc_ints I, const fc_ccsd_opts& op, fc_amps* tout, z* ecorr, int* iters) {
  StageTimer st(ctx, "ccsd");
  const long o = I->o, v = I->v, n1 = o * v, n2 = o * o * v * v, nt = n1 + n2;
  const int prec = op.precision >= 0 ? op.precision : I->precision;
  // tolerances <= 0 pick the precision's own: converging the residual far below the error of the
  // split products only chases rounding noise
  const double e_tol = op.e_tol > 0 ? op.e_tol : (prec == FC_FP64 ? 1e-10 : 1e-8);
  const double r_tol = op.r_tol > 0 ? op.r_tol : (prec == FC_FP64 ? 1e-9 : 1e-7);
  ZTensor t(ctx, {nt}), tn(ctx, {nt}), r(ctx, {nt}), tx(ctx, {nt});
  if (op.t1_init && op.t2_init) {
    FC_HIP(hipMemcpyAsync(t.p(), op.t1_init, sizeof(z) * n1, hipMemcpyDeviceToDevice, ctx->stream));
    FC_HIP(hipMemcpyAsync(t.p() + n1, op.t2_init, sizeof(z) * n2, hipMemcpyDeviceToDevice, ctx->stream));
  } else {
    fill(ctx, t.p(), nt, make_double2(0, 0));
  }
  DiisState D;
  if (op.diis_dim > 1) D.init(ctx, op.diis_dim, o, v);
  z e_old = ccsd_energy_dev(ctx, I, t.p(), t.p() + n1);
  const double nuniq = (double)n1 + (double)(o * (o - 1) / 2) * (double)(v * (v - 1) / 2);
  int status = FC_ENOCONV, it;
  z e = e_old;
  // learned step: used until the residual stops decreasing for stall_window iterations, then
  // plain Jacobi (DIIS history restarted, since the iteration map changes)
  bool learned = op.learned && op.mlp;
  DBuf fd(ctx, sizeof(z) * (o + v));
  ZTensor tgood, rprev;
  bool have_good = false, have_prev = false;
  if (learned) { tgood = ZTensor(ctx, {nt}); rprev = ZTensor(ctx, {n2}); }
  double best_rms = INFINITY;
  int since_best = 0;
  for (it = 1; it <= op.max_iter; ++it) {
    if (op.on_iter) {
      FC_HIP(hipStreamSynchronize(ctx->stream));
      op.on_iter(it, t.p(), t.p() + n1, op.user);
    }
    ccsd_residual_dev(ctx, I, t.p(), t.p() + n1, r.p(), r.p() + n1, prec,
                      (learned || op.precond == 1) ? fd.as<z>() : nullptr);
    z a = dotc(ctx, n1, r.p(), r.p()), b = dotc(ctx, n2, r.p() + n1, r.p() + n1);
    double rms = std::sqrt(std::max(0.0, (a.x + 0.25 * b.x) / std::max(1.0, nuniq)));
    if (!std::isfinite(a.x + b.x) && learned && have_good) {
      // the learned step produced a non-finite iterate: return to the last good one, go plain
      FC_HIP(hipMemcpyAsync(t.p(), tgood.p(), sizeof(z) * nt, hipMemcpyDeviceToDevice, ctx->stream));
      learned = false;
      D.order.clear();
      if (ctx->verbose) fprintf(stderr, "[ccsd] it %3d learned step not finite: back to the last good iterate\n", it);
      ccsd_residual_dev(ctx, I, t.p(), t.p() + n1, r.p(), r.p() + n1, prec, nullptr);
      a = dotc(ctx, n1, r.p(), r.p());
      b = dotc(ctx, n2, r.p() + n1, r.p() + n1);
      rms = std::sqrt(std::max(0.0, (a.x + 0.25 * b.x) / std::max(1.0, nuniq)));
    }
    if (!std::isfinite(rms)) throw Error(FC_ENUMERIC, "ccsd_solve: residual is not finite");
    if (learned) {
      FC_HIP(hipMemcpyAsync(tgood.p(), t.p(), sizeof(z) * nt, hipMemcpyDeviceToDevice, ctx->stream));
      have_good = true;
      if (rms < best_rms * 0.999) {
        best_rms = rms;
        since_best = 0;
      } else if (++since_best >= std::max(1, op.stall_window)) {
        learned = false;
        D.order.clear();
        if (ctx->verbose) fprintf(stderr, "[ccsd] it %3d learned step stalled: Jacobi + DIIS from here\n", it);
      }
    }
    if (learned) {
      learned_step(ctx, I, op.mlp, t.p(), t.p() + n1, r.p(), r.p() + n1, have_prev ? rprev.p() : nullptr, fd.as<z>(),
                   tn.p(), tn.p() + n1);
      FC_HIP(hipMemcpyAsync(rprev.p(), r.p() + n1, sizeof(z) * n2, hipMemcpyDeviceToDevice, ctx->stream));
      have_prev = true;
    } else {
      jacobi_step(ctx, I, t.p(), t.p() + n1, r.p(), r.p() + n1, tn.p(), tn.p() + n1,
                  op.precond == 1 ? fd.as<z>() : nullptr);
    }
    if (op.diis_dim > 1 && it >= op.diis_start) {
      diis_push_extrapolate(ctx, D, tn.p(), t.p(), tx.p());
      std::swap(t, tx);
    } else {
      std::swap(t, tn);
    }
    e = ccsd_energy_dev(ctx, I, t.p(), t.p() + n1);
    const double de = std::hypot(e.x - e_old.x, e.y - e_old.y);
    if (ctx->verbose)
      fprintf(stderr, "[ccsd] it %3d E %.12f %+.2e dE %.2e rms %.2e %s\n", it, e.x, e.y, de, rms, learned ? "learned" : "jacobi");
    if (de < e_tol && rms < r_tol) { status = FC_OK; break; }
    e_old = e;
  }
  *ecorr = e;
  *iters = std::min(it, op.max_iter);
  auto* T = new fc_amps_s();
  T->ctx = ctx; T->ints = I;
  T->t1 = ZTensor(ctx, {o, v});
  T->t2 = ZTensor(ctx, {o, o, v, v});
  FC_HIP(hipMemcpyAsync(T->t1.p(), t.p(), sizeof(z) * n1, hipMemcpyDeviceToDevice, ctx->stream));
  FC_HIP(hipMemcpyAsync(T->t2.p(), t.p() + n1, sizeof(z) * n2, hipMemcpyDeviceToDevice, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  *tout = T;
  return status;
}

// ------------------------------------------------------------------------------ FNS
static fc_ints fns_impl(fc_ctx ctx, fc_ints I, double thresh, int* v_kept, double* occ_out, void* U_out) {
  StageTimer st(ctx, "fns");
  ensure_integrals(ctx, I);
  const long o = I->o, v = I->v, N = I->ncd;
  const z one = make_double2(1, 0), zero = make_double2(0, 0);
  ZTensor t(ctx, {o, o, v, v}), Dv(ctx, {v, v});
  hipLaunchKernelGGL(k_mp2_amp, dim3(nblk(t.size())), dim3(TPB), 0, ctx->stream, I->vvoo.p(), I->eps_d.as<double>(), t.p(), o, v);
  // D_ab = 1/2 sum_ijc t_ij^ac conj(t_ij^bc)   (Eq. 24)
  zein(ctx, "ijac,ijbc->ab", make_double2(0.5, 0), t, t, zero, Dv, false, true);
  std::vector<z> Dh(v * v);
  FC_HIP(hipMemcpyAsync(Dh.data(), Dv.p(), sizeof(z) * v * v, hipMemcpyDeviceToHost, ctx->stream));
  FC_HIP(hipStreamSynchronize(ctx->stream));
  std::vector<double> nocc;
  herm_eig((int)v, Dh, nocc);                   // ascending; columns are natural spinors (Eq. 25)
  std::vector<int> keep;
  for (long c = v - 1; c >= 0; --c)
    if (nocc[c] > thresh) keep.push_back((int)c);  // descending occupation
  const long vp = (long)keep.size();
  FC_REQUIRE(vp >= 2, FC_EUNSUPPORTED, "fns_truncate: the threshold keeps fewer than two virtual spinors");
  if (occ_out) for (long c = 0; c < v; ++c) occ_out[c] = nocc[v - 1 - c];
  // F^NS = V~^H diag(eps_v) V~ (Eq. 26), semicanonical Z~ (Eq. 27), U = V~ Z~ (Eq. 28)
  std::vector<z> F(vp * vp);
  for (long p = 0; p < vp; ++p)
    for (long q = 0; q < vp; ++q) {
      double re = 0, im = 0;
      for (long a = 0; a < v; ++a) {
        z x = Dh[a * v + keep[p]], y = Dh[a * v + keep[q]];
        double e = I->eps[o + a];
        re += e * (x.x * y.x + x.y * y.y);
        im += e * (x.x * y.y - x.y * y.x);
      }
      F[p * vp + q] = make_double2(re, im);
    }
  std::vector<double> enew;
  herm_eig((int)vp, F, enew);
  std::vector<z> U(v * vp);
  for (long a = 0; a < v; ++a)
    for (long c = 0; c < vp; ++c) {
      double re = 0, im = 0;
      for (long p = 0; p < vp; ++p) {
        z x = Dh[a * v + keep[p]], y = F[p * vp + c];
        re += x.x * y.x - x.y * y.y;
        im += x.x * y.y + x.y * y.x;
      }
      U[a * vp + c] = make_double2(re, im);
    }
  if (U_out) std::memcpy(U_out, U.data(), sizeof(z) * v * vp);
  *v_kept = (int)vp;
  auto* J = new fc_ints_s();
  J->ctx = ctx; J->o = (int)o; J->v = (int)vp; J->ncd = (int)N; J->precision = I->precision;
  J->eps.assign(I->eps.begin(), I->eps.begin() + o);
  for (double e : enew) J->eps.push_back(e);
  J->eps_d = DBuf(ctx, sizeof(double) * J->eps.size());
  FC_HIP(hipMemcpyAsync(J->eps_d.p, J->eps.data(), sizeof(double) * J->eps.size(), hipMemcpyHostToDevice, ctx->stream));
  ZTensor Ud(ctx, {v, vp});
  FC_HIP(hipMemcpyAsync(Ud.p(), U.data(), sizeof(z) * v * vp, hipMemcpyHostToDevice, ctx->stream));
  J->Loo = ZTensor(ctx, {o, o, N});
  FC_HIP(hipMemcpyAsync(J->Loo.p(), I->Loo.p(), sizeof(z) * J->Loo.size(), hipMemcpyDeviceToDevice, ctx->stream));
  J->Lov = ZTensor(ctx, {o, vp, N});
  zein(ctx, "iaP,ak->ikP", one, I->Lov, Ud, zero, J->Lov);
  J->Lvo = ZTensor(ctx, {vp, o, N});
  zein(ctx, "ak,aiP->kiP", one, Ud, I->Lvo, zero, J->Lvo, true, false);
  ZTensor tmp(ctx, {vp, v, N});
  zein(ctx, "ak,abP->kbP", one, Ud, lvv(ctx, I), zero, tmp, true, false);
  J->Lvv = ZTensor(ctx, {vp, vp, N});
  zein(ctx, "kbP,bl->klP", one, tmp, Ud, zero, J->Lvv);
  ensure_integrals(ctx, J);
  FC_HIP(hipStreamSynchronize(ctx->stream));
  return J;
}

}  // namespace fc

using namespace fc;

#define FC_TRY(ctx, ...)                                                   \
  try {                                                                    \
    __VA_ARGS__                                                            \
  } catch (const fc::Error& e_) {                                          \
    if (ctx) (ctx)->last_error = e_.what();                                \
    return e_.code;                                                        \
  } catch (const std::exception& e_) {                                     \
    if (ctx) (ctx)->last_error = e_.what();                                \
    return FC_ENUMERIC;                                                    \
  }

extern "C" {

int fc_create(fc_ctx* out, int device, void* stream, fc_alloc_fn alloc, fc_free_fn release, void* user) {
  if (!out) return FC_EARG;
  *out = nullptr;
  auto* c = new fc_ctx_s();
  c->device = device;
  c->stream = (hipStream_t)stream;
  c->alloc = alloc;
  c->release = release;
  c->user = user;
  const char* vb = getenv("FNSCC_VERBOSE");
  c->verbose = vb ? atoi(vb) : 0;
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return FC_EHIP;
  }
  try {
    noalloc_scratch_init(device);   // the device address of the fixed workspace, once per device
  } catch (const fc::Error&) {
    (void)hipGetLastError();
    delete c;
    return FC_EHIP;
  }
  *out = c;
  return FC_OK;
}

void fc_destroy(fc_ctx ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& e : ctx->ladder_events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  release_cache(ctx);
  delete ctx;
}

const char* fc_last_error(fc_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

int fc_set_timing(fc_ctx ctx, int on) {
  if (!ctx) return FC_EARG;
  ctx->timing = on;
  return FC_OK;
}

int fc_take_timings(fc_ctx ctx, char* buf, size_t len) {
  if (!ctx || !buf || len == 0) return FC_EARG;
  FC_TRY(ctx, {
    FC_HIP(hipStreamSynchronize(ctx->stream));
    std::ostringstream os;
    for (auto& kv : ctx->stage_ms) os << kv.first << "=" << kv.second << ";";
    // ladder launches: per-launch durations from events on the context stream
    double tot = 0;
    for (auto& e : ctx->ladder_events) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) tot += ms;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    os << "ladder_events=" << ctx->ladder_events.size() << ";ladder_event_ms=" << tot << ";";
    ctx->ladder_events.clear();
    for (auto& kv : ctx->stage_calls) os << "calls_" << kv.first << "=" << kv.second << ";";
    ctx->stage_ms.clear();
    ctx->stage_calls.clear();
    std::string s = os.str();
    size_t n = std::min(len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
    return FC_OK;
  })
}

int fc_set_autotune(fc_ctx ctx, int on) {
  if (!ctx) return FC_EARG;
  ctx->autotune = on;
  return FC_OK;
}

int fc_autotune_save(fc_ctx ctx, const char* path) {
  if (!ctx || !path) return FC_EARG;
  FILE* f = fopen(path, "w");
  if (!f) { ctx->last_error = std::string("cannot write ") + path; return FC_EARG; }
  for (auto& kv : ctx->tune) fprintf(f, "%s %d %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
  fclose(f);
  return FC_OK;
}

int fc_autotune_load(fc_ctx ctx, const char* path) {
  if (!ctx || !path) return FC_EARG;
  FILE* f = fopen(path, "r");
  if (!f) { ctx->last_error = std::string("cannot read ") + path; return FC_EARG; }
  char key[128];
  int cfg;
  float ms;
  while (fscanf(f, "%127s %d %f", key, &cfg, &ms) == 3) {
    // GEMM entries name a tile configuration; sigma entries pack (configuration, log2 K chunk)
    const bool sigma = std::strncmp(key, "sigma_", 6) == 0;
    const bool ok = sigma ? (cfg >> 5) >= 0 && (cfg >> 5) < 2 && (cfg & 31) >= 4 && (cfg & 31) <= 20
                          : cfg >= 0 && cfg < gemm_num_configs();
    if (ok) ctx->tune[key] = {cfg, ms};
  }
  fclose(f);
  return FC_OK;
}

int fc_autotune_size(fc_ctx ctx) { return ctx ? (int)ctx->tune.size() : 0; }

int fc_set_gemm_config(fc_ctx ctx, int cfg) {
  if (!ctx || cfg < -1 || cfg >= gemm_num_configs()) return FC_EARG;
  ctx->gemm_cfg = cfg;
  return FC_OK;
}

int fc_gemm_num_configs(void) { return gemm_num_configs(); }

int fc_set_split_config(fc_ctx ctx, int cfg) {
  if (!ctx || cfg < -1 || cfg >= fc::FC_SPLIT_NUM_CONFIGS) return FC_EARG;
  ctx->split_cfg = cfg;
  return FC_OK;
}

int fc_split_num_configs(void) { return fc::FC_SPLIT_NUM_CONFIGS; }

int cd_ao_pivoted(fc_ctx ctx, long m, const double* M, double tau, int max_vec, double* L, int* nvec, int* piv) {
  if (!ctx || m < 1 || !M || !L || !nvec || max_vec < 1 || !(tau > 0)) return FC_EARG;
  FC_TRY(ctx, {
    *nvec = 0;
    // m vectors exhaust any m x m matrix: reaching them is convergence, not a cap
    const int cap = (int)std::min<long>(max_vec, m);
    int s = cd_pivoted_dev(ctx, m, M, tau, cap, L, nvec, piv);
    if (s == FC_ENOCONV && cap == m) s = FC_OK;
    if (s == FC_ENOCONV) ctx->last_error = "cd_ao_pivoted: max_vec vectors formed before the diagonal fell below tau";
    return s;
  })
}

int ao_to_spinor(fc_ctx ctx, int nvec, int nao, int n, const double* Lao, const void* C, void* Lmo) {
  if (!ctx || nvec < 1 || nao < 1 || n < 1 || !Lao || !C || !Lmo) return FC_EARG;
  FC_TRY(ctx, {
    ao_to_spinor_dev(ctx, nvec, nao, n, Lao, (const z*)C, (z*)Lmo);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

int cd_integrals(fc_ctx ctx, int o, int v, int ncd, const double* eps, const void* L, int l_dtype, int l_on_device,
                 int precision, fc_ints* out) {
  if (!ctx || !out) return FC_EARG;
  *out = nullptr;
  FC_TRY(ctx, {
    FC_REQUIRE(o >= 1 && v >= 1 && ncd >= 1, FC_EARG, "cd_integrals: o, v and ncd must be >= 1");
    // one occupied or one virtual spinor leaves no doubles (and no 2h1p space): not supported
    FC_REQUIRE(o >= 2 && v >= 2, FC_EUNSUPPORTED, "cd_integrals: needs at least two occupied and two virtual spinors");
    FC_REQUIRE(eps && L, FC_EARG, "cd_integrals: NULL eps or L");
    FC_REQUIRE(l_dtype == FC_C128 || l_dtype == FC_C64, FC_EARG, "cd_integrals: l_dtype must be FC_C128 or FC_C64");
    FC_REQUIRE(precision >= FC_FP64 && precision <= FC_SPLIT_FP16, FC_EARG, "cd_integrals: bad precision");
    StageTimer st(ctx, "cd_integrals");
    auto* I = new fc_ints_s();
    std::unique_ptr<fc_ints_s> guard(I);
    I->ctx = ctx; I->o = o; I->v = v; I->ncd = ncd; I->precision = precision;
    const long n = (long)o + v;
    I->eps.assign(eps, eps + n);
    I->eps_d = DBuf(ctx, sizeof(double) * n);
    FC_HIP(hipMemcpyAsync(I->eps_d.p, eps, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    const size_t esz = l_dtype == FC_C128 ? 16 : 8;
    const size_t lbytes = esz * (size_t)ncd * n * n;
    DBuf Ld;
    const void* Lsrc = L;
    if (!l_on_device) {
      Ld = DBuf(ctx, lbytes);
      FC_HIP(hipMemcpyAsync(Ld.p, L, lbytes, hipMemcpyHostToDevice, ctx->stream));
      Lsrc = Ld.p;
    }
    stage_cholesky(ctx, I, Lsrc, l_dtype);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    *out = guard.release();
    return FC_OK;
  })
}

int fc_ints_info(fc_ints I, int* o, int* v, int* ncd) {
  if (!I) return FC_EARG;
  if (o) *o = I->o;
  if (v) *v = I->v;
  if (ncd) *ncd = I->ncd;
  return FC_OK;
}

void fc_free_ints(fc_ints I) { delete I; }

int fns_truncate(fc_ctx ctx, fc_ints in, double occ_thresh, fc_ints* out, int* v_kept, double* occ, void* U) {
  if (!ctx || !in || !out || !v_kept) return FC_EARG;
  *out = nullptr;
  FC_TRY(ctx, {
    *out = fns_impl(ctx, in, occ_thresh, v_kept, occ, U);
    return FC_OK;
  })
}

void fc_ccsd_default_opts(fc_ccsd_opts* op) {
  if (!op) return;
  std::memset(op, 0, sizeof(*op));
  op->e_tol = 0;   // 0: by precision (FP64 1e-10 / 1e-9, split 1e-8 / 1e-7)
  op->r_tol = 0;
  op->max_iter = 200;
  op->diis_dim = 10;
  op->learned = 0;
  op->precision = -1;  // inherit from the integral handle
  op->stall_window = 3;
  op->diis_start = 1;
  op->precond = 1;
}

int ccsd_solve(fc_ctx ctx, int nb, const fc_ints* ints, const fc_ccsd_opts* opts, fc_amps* t, double* e_corr, int* iters) {
  if (!ctx || nb < 1 || !ints || !t || !e_corr || !iters) return FC_EARG;
  FC_TRY(ctx, {
    fc_ccsd_opts op;
    if (opts) op = *opts; else fc_ccsd_default_opts(&op);
    FC_REQUIRE(op.max_iter >= 1, FC_EARG, "ccsd_solve: max_iter must be >= 1");
    FC_REQUIRE(op.diis_dim <= 16, FC_EARG, "ccsd_solve: diis_dim must be <= 16");
    FC_REQUIRE(op.diis_start >= 1, FC_EARG, "ccsd_solve: diis_start must be >= 1");
    FC_REQUIRE(op.precond == 0 || op.precond == 1, FC_EARG, "ccsd_solve: precond must be 0 or 1");
    int status = FC_OK;
    for (int b = 0; b < nb; ++b) {
      FC_REQUIRE(ints[b], FC_EARG, "ccsd_solve: NULL integral handle");
      z e;
      int s = solve_one(ctx, ints[b], op, &t[b], &e, &iters[b]);
      e_corr[2 * b] = e.x;
      e_corr[2 * b + 1] = e.y;
      if (s != FC_OK) status = s;
    }
    if (status == FC_ENOCONV) ctx->last_error = "ccsd_solve: not converged within max_iter";
    return status;
  })
}

int ccsd_residual(fc_ctx ctx, fc_ints I, const void* t1, const void* t2, void* r1, void* r2, int precision) {
  if (!ctx || !I || !t1 || !t2 || !r1 || !r2) return FC_EARG;
  FC_TRY(ctx, {
    ccsd_residual_dev(ctx, I, (const z*)t1, (const z*)t2, (z*)r1, (z*)r2, precision < 0 ? I->precision : precision);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

int fc_ladder(fc_ctx ctx, fc_ints I, const void* tau, const void* t1, void* R, int precision) {
  if (!ctx || !I || !tau || !R) return FC_EARG;
  FC_TRY(ctx, {
    ladder_dev(ctx, I, (const z*)tau, (const z*)t1, (z*)R, precision < 0 ? I->precision : precision);
    return FC_OK;
  })
}

int fc_ladder_packed(fc_ctx ctx, fc_ints I, const void* taup, const void* t1, void* Rp, int precision) {
  if (!ctx || !I || !taup || !Rp) return FC_EARG;
  FC_TRY(ctx, {
    const int prec = precision < 0 ? I->precision : precision;
    FC_REQUIRE(prec >= FC_FP64 && prec <= FC_SPLIT_FP16, FC_EARG, "fc_ladder_packed: bad precision");
    ladder_packed_dev(ctx, I, (const z*)taup, (const z*)t1, (z*)Rp, prec);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

int fc_learned_step(fc_ctx ctx, fc_ints I, fc_mlp mlp, const void* t1, const void* t2, const void* r1, const void* r2,
                    const void* r2prev, const void* fdiag, void* t1_out, void* t2_out) {
  if (!ctx || !I || !mlp || !t1 || !t2 || !r1 || !r2 || !fdiag || !t1_out || !t2_out) return FC_EARG;
  FC_TRY(ctx, {
    learned_step(ctx, I, mlp, (const z*)t1, (const z*)t2, (const z*)r1, (const z*)r2, (const z*)r2prev,
                 (const z*)fdiag, (z*)t1_out, (z*)t2_out);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

int fc_zgemm(fc_ctx ctx, char opA, char opB, long M, long N, long K, const double* alpha, const void* A,
             long lda, const void* B, long ldb, const double* beta, void* C, long ldc, int precision) {
  if (!ctx || !alpha || !beta || M < 0 || N < 0 || K < 0) return FC_EARG;
  const bool split = precision == FC_SPLIT_BF16 || precision == FC_SPLIT_FP16;
  if (precision != FC_FP64 && precision != FC_FP32 && !split) return FC_EARG;
  if (M == 0 || N == 0) return FC_OK;
  if (!C || (K > 0 && (!A || !B))) return FC_EARG;
  FC_TRY(ctx, {
    if (split) {
      // contraction-contiguous layouts only (FC_EUNSUPPORTED otherwise, before any launch)
      zgemm_split(ctx, precision, opA, opB, M, N, K, make_double2(alpha[0], alpha[1]), (const z*)A, lda, (const z*)B,
                  ldb, make_double2(beta[0], beta[1]), (z*)C, ldc);
      return FC_OK;
    }
    Fp32Gemms fp32(ctx, precision == FC_FP32);
    zgemm(ctx, opA, opB, M, N, K, make_double2(alpha[0], alpha[1]), (const z*)A, lda, (const z*)B, ldb,
          make_double2(beta[0], beta[1]), (z*)C, ldc);
    return FC_OK;
  })
}

int fc_zgemm_noalloc(fc_ctx ctx, char opA, char opB, long M, long N, long K, const double* alpha, const void* A,
                     long lda, const void* B, long ldb, const double* beta, void* C, long ldc, int precision) {
  if (!ctx || !alpha || !beta || M < 0 || N < 0 || K < 0) return FC_EARG;
  if (precision != FC_FP64 && precision != FC_FP32) return FC_EARG;
  if (M == 0 || N == 0) return FC_OK;
  if (!C || (K > 0 && (!A || !B))) return FC_EARG;
  FC_TRY(ctx, {
    Fp32Gemms fp32(ctx, precision == FC_FP32);
    zgemm_noalloc(ctx, opA, opB, M, N, K, make_double2(alpha[0], alpha[1]), (const z*)A, lda, (const z*)B, ldb,
                  make_double2(beta[0], beta[1]), (z*)C, ldc);
    return FC_OK;
  })
}

int fc_learn_samples(fc_ctx ctx, fc_ints I, const void* t1, const void* t2, const void* t1prev, const void* t2prev,
                     const void* t2_star, long nsamp, unsigned long long seed, float* X, float* q, float* r) {
  if (!ctx || !I || !t1 || !t2 || !t2_star || nsamp < 1 || !X || !q || !r) return FC_EARG;
  FC_TRY(ctx, {
    const long o = I->o, v = I->v;
    ZTensor r1(ctx, {o, v}), r2(ctx, {o, o, v, v}), p2;
    DBuf fd(ctx, sizeof(z) * (o + v));
    if (t1prev && t2prev) {
      p2 = ZTensor(ctx, {o, o, v, v});
      ccsd_residual_dev(ctx, I, (const z*)t1prev, (const z*)t2prev, r1.p(), p2.p(), I->precision, nullptr);
    }
    ccsd_residual_dev(ctx, I, (const z*)t1, (const z*)t2, r1.p(), r2.p(), I->precision, fd.as<z>());
    learn_samples(ctx, I, (const z*)t2, r2.p(), p2.size() ? p2.p() : nullptr, (const z*)t2_star, fd.as<z>(), nsamp,
                  seed, X, q, r);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

int fc_amps_create(fc_ctx ctx, fc_ints I, const void* t1, const void* t2, fc_amps* out) {
  if (!ctx || !I || !t1 || !t2 || !out) return FC_EARG;
  FC_TRY(ctx, {
    auto* T = new fc_amps_s();
    T->ctx = ctx; T->ints = I;
    const long o = I->o, v = I->v;
    T->t1 = ZTensor(ctx, {o, v});
    T->t2 = ZTensor(ctx, {o, o, v, v});
    FC_HIP(hipMemcpyAsync(T->t1.p(), t1, sizeof(z) * o * v, hipMemcpyDeviceToDevice, ctx->stream));
    FC_HIP(hipMemcpyAsync(T->t2.p(), t2, sizeof(z) * o * o * v * v, hipMemcpyDeviceToDevice, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    *out = T;
    return FC_OK;
  })
}

int fc_amps_read(fc_amps T, void* t1, void* t2) {
  if (!T) return FC_EARG;
  fc_ctx ctx = T->ctx;
  FC_TRY(ctx, {
    if (t1) FC_HIP(hipMemcpyAsync(t1, T->t1.p(), sizeof(z) * T->t1.size(), hipMemcpyDeviceToDevice, ctx->stream));
    if (t2) FC_HIP(hipMemcpyAsync(t2, T->t2.p(), sizeof(z) * T->t2.size(), hipMemcpyDeviceToDevice, ctx->stream));
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

void fc_free_amps(fc_amps T) { delete T; }

int ipeom_sigma(fc_ctx ctx, fc_ints I, fc_amps T, int nvec, const void* R, void* S) {
  if (!ctx || !I || !T || nvec < 0 || (nvec > 0 && (!R || !S))) return FC_EARG;
  if (nvec == 0) return T->ints == I ? FC_OK : FC_EARG;   // nothing to compute, no launch
  FC_TRY(ctx, {
    FC_REQUIRE(T->ints == I, FC_EARG, "ipeom_sigma: amplitudes belong to another integral handle");
    sigma_dev(ctx, I, T, nvec, (const z*)R, (z*)S);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

int ipeom_sigma_left(fc_ctx ctx, fc_ints I, fc_amps T, int nvec, const void* Y, void* S) {
  if (!ctx || !I || !T || nvec < 0 || (nvec > 0 && (!Y || !S))) return FC_EARG;
  if (nvec == 0) return T->ints == I ? FC_OK : FC_EARG;   // nothing to compute, no launch
  FC_TRY(ctx, {
    FC_REQUIRE(T->ints == I, FC_EARG, "ipeom_sigma_left: amplitudes belong to another integral handle");
    sigma_dev(ctx, I, T, nvec, (const z*)Y, (z*)S, true);
    FC_HIP(hipStreamSynchronize(ctx->stream));
    return FC_OK;
  })
}

void fc_eom_default_opts(fc_eom_opts* op) {
  if (!op) return;
  op->r_tol = 1e-9;
  op->w_tol = 1e-10;
  op->max_iter = 200;
  op->max_subspace = 0;  // 0 = 10 x roots
  op->guess_per_root = 2;
  op->graph = 1;
}

int ipeom_davidson(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* t, const int* nroots,
                   const fc_eom_opts* opts, double* omega, void* R_out, int* iters) {
  if (!ctx || nb < 1 || !ints || !t || !nroots || !omega) return FC_EARG;
  FC_TRY(ctx, {
    fc_eom_opts op;
    if (opts) op = *opts; else fc_eom_default_opts(&op);
    FC_REQUIRE(op.max_iter >= 1, FC_EARG, "ipeom_davidson: max_iter must be >= 1");
    long total = 0;
    for (int b = 0; b < nb; ++b) {
      FC_REQUIRE(nroots[b] >= 1, FC_EARG, "ipeom_davidson: nroots must be >= 1");
      total += nroots[b];
    }
    std::vector<z> w(total);
    const int s = davidson_batch(ctx, nb, ints, t, nroots, op, w.data(), (z*)R_out, iters);
    for (long r = 0; r < total; ++r) { omega[2 * r] = w[r].x; omega[2 * r + 1] = w[r].y; }
    if (s == FC_ENOCONV) ctx->last_error = "ipeom_davidson: not converged within max_iter";
    return s;
  })
}

int ipeom_left(fc_ctx ctx, int nb, const fc_ints* ints, const fc_amps* t, const int* nroots,
               const fc_eom_opts* opts, const void* R, double* omega, void* L_out, double* weight, int* iters) {
  if (!ctx || nb < 1 || !ints || !t || !nroots || !R || !omega || !L_out || !weight) return FC_EARG;
  FC_TRY(ctx, {
    fc_eom_opts op;
    if (opts) op = *opts; else fc_eom_default_opts(&op);
    FC_REQUIRE(op.max_iter >= 1, FC_EARG, "ipeom_left: max_iter must be >= 1");
    long total = 0;
    for (int b = 0; b < nb; ++b) {
      FC_REQUIRE(nroots[b] >= 1, FC_EARG, "ipeom_left: nroots must be >= 1");
      total += nroots[b];
    }
    std::vector<z> w(total), wt(total);
    const int s = left_batch(ctx, nb, ints, t, nroots, op, (const z*)R, w.data(), (z*)L_out, wt.data(), iters);
    for (long r = 0; r < total; ++r) {
      omega[2 * r] = w[r].x; omega[2 * r + 1] = w[r].y;
      weight[2 * r] = wt[r].x; weight[2 * r + 1] = wt[r].y;
    }
    if (s == FC_ENOCONV) ctx->last_error = "ipeom_left: not converged within max_iter";
    return s;
  })
}

}  // extern "C"
