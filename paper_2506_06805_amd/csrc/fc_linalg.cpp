// Host FP64 dense linear algebra: the small eigenproblems and linear systems the method keeps in
// double precision on the CPU (natural-spinor density and semicanonical Fock block, the Davidson
// subspace matrix, the DIIS system).
//
// Hermitian: Householder reduction to tridiagonal form, diagonal phase scaling to a real
// symmetric tridiagonal, implicit QL with Wilkinson-type shifts, back-transformation.  The QL
// sweep is the published tql2 procedure (Bowdler, Martin, Reinsch and Wilkinson, "The QR and QL
// algorithms for symmetric matrices", Numer. Math. 11 (1968) 293, reprinted in Wilkinson and
// Reinsch, Handbook for Automatic Computation II, and in EISPACK as TQL2); its rotation
// recurrences are therefore the textbook ones.
// General complex: Householder reduction to Hessenberg form, single-shift implicit QR sweeps
// with Givens rotations to a complex Schur form (the complex QR algorithm of Francis and
// Kublanovskaya with Wilkinson's shift, as in EISPACK COMQR2), eigenvectors of the triangular
// factor by back substitution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <limits>
#include <numeric>
#include <vector>

#include "fc_state.hpp"

namespace fc {
using C = std::complex<double>;
static inline C toc(z a) { return C(a.x, a.y); }
static inline z toz(C a) { return make_double2(a.real(), a.imag()); }

// ---- Hermitian eigenproblem ----------------------------------------------------------------
void herm_eig(int n, std::vector<z>& Az, std::vector<double>& w) {
  std::vector<C> A(n * (size_t)n), Q(n * (size_t)n, C(0));
  for (size_t i = 0; i < A.size(); ++i) A[i] = toc(Az[i]);
  for (int i = 0; i < n; ++i) Q[i * (size_t)n + i] = 1.0;
  auto a = [&](int i, int j) -> C& { return A[i * (size_t)n + j]; };
  auto q = [&](int i, int j) -> C& { return Q[i * (size_t)n + j]; };
  std::vector<C> v(n), p(n), wv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of the column below the diagonal
    double nx = 0;
    for (int i = 0; i < m; ++i) nx += std::norm(a(k + 1 + i, k));
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    C x0 = a(k + 1, k);
    C phase = std::abs(x0) > 0 ? x0 / std::abs(x0) : C(1.0);
    C alpha = -phase * nx;
    for (int i = 0; i < m; ++i) v[i] = a(k + 1 + i, k);
    v[0] -= alpha;
    double vn2 = 0;
    for (int i = 0; i < m; ++i) vn2 += std::norm(v[i]);
    if (vn2 == 0.0) continue;
    const double tau = 2.0 / vn2;
    // p = tau A_sub v ; K = tau/2 v^H p ; w = p - K v ; A_sub -= v w^H + w v^H
    for (int i = 0; i < m; ++i) {
      C s = 0;
      for (int j = 0; j < m; ++j) s += a(k + 1 + i, k + 1 + j) * v[j];
      p[i] = tau * s;
    }
    C vhp = 0;
    for (int i = 0; i < m; ++i) vhp += std::conj(v[i]) * p[i];
    const double K = 0.5 * tau * vhp.real();
    for (int i = 0; i < m; ++i) wv[i] = p[i] - K * v[i];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j)
        a(k + 1 + i, k + 1 + j) -= v[i] * std::conj(wv[j]) + wv[i] * std::conj(v[j]);
    a(k + 1, k) = alpha;
    a(k, k + 1) = std::conj(alpha);
    for (int i = 1; i < m; ++i) { a(k + 1 + i, k) = 0; a(k, k + 1 + i) = 0; }
    // Q <- Q H on columns k+1..n-1
    for (int r = 0; r < n; ++r) {
      C s = 0;
      for (int j = 0; j < m; ++j) s += q(r, k + 1 + j) * v[j];
      s *= tau;
      for (int j = 0; j < m; ++j) q(r, k + 1 + j) -= s * std::conj(v[j]);
    }
  }
  // real symmetric tridiagonal via diagonal phases: T = D Tr D^H
  std::vector<double> d(n), e(n, 0.0);
  std::vector<C> delta(n, C(1.0));
  for (int k = 0; k < n; ++k) d[k] = a(k, k).real();
  for (int k = 0; k + 1 < n; ++k) {
    C ek = a(k + 1, k);
    double m = std::abs(ek);
    e[k] = m;
    delta[k + 1] = m > 0 ? delta[k] * ek / m : delta[k];
  }
  // implicit QL on (d, e), accumulating rotations into Zr
  std::vector<double> Zr(n * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) Zr[i * (size_t)n + i] = 1.0;
  const double eps = std::numeric_limits<double>::epsilon();
  for (int l = 0; l < n; ++l) {
    int iter = 0, m;
    do {
      for (m = l; m < n - 1; ++m) {
        double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= eps * dd) break;
      }
      if (m != l) {
        if (iter++ == 200) throw Error(FC_ENUMERIC, "herm_eig: QL iteration did not converge");
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = std::hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
        double s = 1.0, c = 1.0, pp = 0.0;
        int i;
        bool early = false;
        for (i = m - 1; i >= l; --i) {
          double f = s * e[i], b = c * e[i];
          r = std::hypot(f, g);
          e[i + 1] = r;
          if (r == 0.0) { d[i + 1] -= pp; e[m] = 0.0; early = true; break; }
          s = f / r; c = g / r;
          g = d[i + 1] - pp;
          r = (d[i] - g) * s + 2.0 * c * b;
          pp = s * r;
          d[i + 1] = g + pp;
          g = c * r - b;
          for (int k = 0; k < n; ++k) {
            double fz = Zr[k * (size_t)n + i + 1];
            Zr[k * (size_t)n + i + 1] = s * Zr[k * (size_t)n + i] + c * fz;
            Zr[k * (size_t)n + i] = c * Zr[k * (size_t)n + i] - s * fz;
          }
        }
        if (early) continue;
        d[l] -= pp; e[l] = g; e[m] = 0.0;
      }
    } while (m != l);
  }
  // eigenvectors X = Q D Zr, ascending order
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return d[x] < d[y]; });
  w.assign(n, 0.0);
  std::vector<z> out(n * (size_t)n);
  for (int c = 0; c < n; ++c) {
    int src = order[c];
    w[c] = d[src];
    for (int r = 0; r < n; ++r) {
      C s = 0;
      for (int k = 0; k < n; ++k) s += q(r, k) * delta[k] * Zr[k * (size_t)n + src];
      out[r * (size_t)n + c] = toz(s);
    }
  }
  Az.swap(out);
}

// ---- general complex eigenproblem ----------------------------------------------------------
void gen_eig(int n, const std::vector<z>& Az, std::vector<z>& wout, std::vector<z>& VR) {
  std::vector<C> H(n * (size_t)n), Q(n * (size_t)n, C(0));
  for (size_t i = 0; i < H.size(); ++i) H[i] = toc(Az[i]);
  for (int i = 0; i < n; ++i) Q[i * (size_t)n + i] = 1.0;
  auto h = [&](int i, int j) -> C& { return H[i * (size_t)n + j]; };
  auto q = [&](int i, int j) -> C& { return Q[i * (size_t)n + j]; };
  double anorm = 0;
  for (auto& x : H) anorm = std::max(anorm, std::abs(x));
  // Hessenberg reduction
  std::vector<C> v(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double nx = 0;
    for (int i = 0; i < m; ++i) nx += std::norm(h(k + 1 + i, k));
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    C x0 = h(k + 1, k);
    C phase = std::abs(x0) > 0 ? x0 / std::abs(x0) : C(1.0);
    C alpha = -phase * nx;
    for (int i = 0; i < m; ++i) v[i] = h(k + 1 + i, k);
    v[0] -= alpha;
    double vn2 = 0;
    for (int i = 0; i < m; ++i) vn2 += std::norm(v[i]);
    if (vn2 == 0.0) continue;
    const double tau = 2.0 / vn2;
    for (int c = k; c < n; ++c) {  // H <- P H (rows k+1..)
      C s = 0;
      for (int i = 0; i < m; ++i) s += std::conj(v[i]) * h(k + 1 + i, c);
      s *= tau;
      for (int i = 0; i < m; ++i) h(k + 1 + i, c) -= v[i] * s;
    }
    for (int r = 0; r < n; ++r) {  // H <- H P (cols k+1..)
      C s = 0;
      for (int j = 0; j < m; ++j) s += h(r, k + 1 + j) * v[j];
      s *= tau;
      for (int j = 0; j < m; ++j) h(r, k + 1 + j) -= s * std::conj(v[j]);
    }
    for (int r = 0; r < n; ++r) {  // Q <- Q P
      C s = 0;
      for (int j = 0; j < m; ++j) s += q(r, k + 1 + j) * v[j];
      s *= tau;
      for (int j = 0; j < m; ++j) q(r, k + 1 + j) -= s * std::conj(v[j]);
    }
    for (int i = 1; i < m; ++i) h(k + 1 + i, k) = 0;
  }
  // complex Schur form by single-shift implicit QR
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1, iter = 0, total = 0;
  while (hi > 0) {
    int l = hi;
    while (l > 0) {
      double s = std::abs(h(l, l)) + std::abs(h(l - 1, l - 1));
      if (s == 0.0) s = anorm;
      if (std::abs(h(l, l - 1)) <= eps * s) { h(l, l - 1) = 0; break; }
      --l;
    }
    if (l == hi) { --hi; iter = 0; continue; }
    if (++total > 100 * n + 1000) throw Error(FC_ENUMERIC, "gen_eig: QR iteration did not converge");
    ++iter;
    C a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
    C mu;
    if (iter % 11 == 10) {
      mu = d + C(std::abs(c), 0.0) * 0.75;  // exceptional shift
    } else {
      C half = 0.5 * (a - d);
      C disc = std::sqrt(half * half + b * c);
      C m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    C x = h(l, l) - mu, y = h(l + 1, l);
    for (int k = l; k < hi; ++k) {
      if (k > l) { x = h(k, k - 1); y = h(k + 1, k - 1); }
      double r = std::sqrt(std::norm(x) + std::norm(y));
      double cc;
      C s;
      if (r == 0.0) { cc = 1.0; s = 0.0; }
      else if (std::abs(x) == 0.0) { cc = 0.0; s = std::conj(y) / r; }
      else { cc = std::abs(x) / r; s = (x / std::abs(x)) * std::conj(y) / r; }
      // rows k, k+1 <- G rows
      for (int col = std::max(l, k - 1); col < n; ++col) {
        C u = h(k, col), w = h(k + 1, col);
        h(k, col) = cc * u + s * w;
        h(k + 1, col) = -std::conj(s) * u + cc * w;
      }
      if (k > l) h(k + 1, k - 1) = 0;
      // cols k, k+1 <- cols G^H
      const int rmax = std::min(k + 2, hi);
      for (int row = 0; row <= rmax; ++row) {
        C u = h(row, k), w = h(row, k + 1);
        h(row, k) = cc * u + std::conj(s) * w;
        h(row, k + 1) = -s * u + cc * w;
      }
      for (int row = 0; row < n; ++row) {
        C u = q(row, k), w = q(row, k + 1);
        q(row, k) = cc * u + std::conj(s) * w;
        q(row, k + 1) = -s * u + cc * w;
      }
    }
  }
  // eigenvectors of the triangular factor, then back to the original basis
  wout.resize(n);
  VR.assign(n * (size_t)n, make_double2(0, 0));
  const double small = std::max(anorm, 1e-300) * eps;
  std::vector<C> y(n);
  for (int k = 0; k < n; ++k) {
    C lam = h(k, k);
    wout[k] = toz(lam);
    std::fill(y.begin(), y.end(), C(0));
    y[k] = 1.0;
    for (int j = k - 1; j >= 0; --j) {
      C s = 0;
      for (int l2 = j + 1; l2 <= k; ++l2) s += h(j, l2) * y[l2];
      C den = h(j, j) - lam;
      if (std::abs(den) < small) den = small;
      y[j] = -s / den;
    }
    double nrm = 0;
    std::vector<C> xv(n, C(0));
    for (int r = 0; r < n; ++r) {
      C s = 0;
      for (int l2 = 0; l2 <= k; ++l2) s += q(r, l2) * y[l2];
      xv[r] = s;
      nrm += std::norm(s);
    }
    nrm = std::sqrt(nrm);
    for (int r = 0; r < n; ++r) VR[r * (size_t)n + k] = toz(xv[r] / nrm);
  }
}

// ---- small dense linear solve (partial pivoting) -------------------------------------------
bool lin_solve(int n, std::vector<z> Az, std::vector<z>& bz) {
  std::vector<C> A(n * (size_t)n), b(n);
  for (size_t i = 0; i < A.size(); ++i) A[i] = toc(Az[i]);
  for (int i = 0; i < n; ++i) b[i] = toc(bz[i]);
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(A[i * n + k]) > std::abs(A[piv * n + k])) piv = i;
    if (std::abs(A[piv * n + k]) == 0.0) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      C f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    C s = b[i];
    for (int j = i + 1; j < n; ++j) s -= A[i * n + j] * b[j];
    b[i] = s / A[i * n + i];
  }
  for (int i = 0; i < n; ++i) bz[i] = toz(b[i]);
  return true;
}

double cond_herm(int n, const std::vector<z>& A) {
  std::vector<z> a = A;
  std::vector<double> w;
  herm_eig(n, a, w);
  double mx = 0, mn = std::numeric_limits<double>::infinity();
  for (double x : w) { mx = std::max(mx, std::fabs(x)); mn = std::min(mn, std::fabs(x)); }
  return mn == 0.0 ? std::numeric_limits<double>::infinity() : mx / mn;
}

}  // namespace fc

extern "C" int fc_host_zheev(int n, double* A, double* w) {
  try {
    if (n < 0 || (n > 0 && (!A || !w))) return FC_EARG;
    std::vector<fc::z> a(n * (size_t)n);
    for (size_t i = 0; i < a.size(); ++i) a[i] = make_double2(A[2 * i], A[2 * i + 1]);
    std::vector<double> ww;
    fc::herm_eig(n, a, ww);
    for (size_t i = 0; i < a.size(); ++i) { A[2 * i] = a[i].x; A[2 * i + 1] = a[i].y; }
    for (int i = 0; i < n; ++i) w[i] = ww[i];
    return FC_OK;
  } catch (const fc::Error& e) {
    return e.code;
  } catch (...) {
    return FC_ENUMERIC;
  }
}

extern "C" int fc_host_zgeev(int n, const double* A, double* w, double* VR) {
  try {
    if (n < 0 || (n > 0 && (!A || !w || !VR))) return FC_EARG;
    std::vector<fc::z> a(n * (size_t)n), ww, vr;
    for (size_t i = 0; i < a.size(); ++i) a[i] = make_double2(A[2 * i], A[2 * i + 1]);
    fc::gen_eig(n, a, ww, vr);
    for (int i = 0; i < n; ++i) { w[2 * i] = ww[i].x; w[2 * i + 1] = ww[i].y; }
    for (size_t i = 0; i < vr.size(); ++i) { VR[2 * i] = vr[i].x; VR[2 * i + 1] = vr[i].y; }
    return FC_OK;
  } catch (const fc::Error& e) {
    return e.code;
  } catch (...) {
    return FC_ENUMERIC;
  }
}
