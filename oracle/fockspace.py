"""Brute-force second quantisation on tiny spinor spaces (test infrastructure).

Everything here is built from the operator definitions alone, with no use of
the working CCSD or IP-EOM equations, so that it can pin them:

* Fock space of n <= 12 spinors, basis = occupation bit strings, Jordan-Wigner
  signs (a_p picks up (-1)^(number of occupied spinors q < p)).
* H = sum_pq h_pq a+_p a_q + 1/2 sum_pqrs (pr|qs) a+_p a+_q a_s a_r with the
  Mulliken integrals of Eq. 21 formed directly from the Cholesky vectors, and
  h_pq = delta_pq eps_p - sum_k <pk||qk>, the one-body part that makes the
  Fock operator of the reference determinant diagonal with entries eps_p.
* Cluster operator T = sum t_i^a a+_a a_i + 1/4 sum t_ij^ab a+_a a+_b a_j a_i
  (Eq. 12), H-bar = e^-T H e^T (exact: T is nilpotent).
* IP operator R = sum r_i a_i + sum_{i<j,b} r_ij^b a+_b a_j a_i (Eq. 17).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


class FockSpace:
    def __init__(self, n):
        if n > 12:
            raise ValueError("brute force limited to n <= 12 spinors")
        self.n = n
        self.dim = 1 << n
        states = np.arange(self.dim)
        self.ann = []
        for p in range(n):
            occ = (states >> p) & 1
            below = np.array([bin(s & ((1 << p) - 1)).count("1") for s in states])
            src = states[occ == 1]
            dst = src ^ (1 << p)
            sign = np.where(below[occ == 1] % 2 == 0, 1.0, -1.0)
            self.ann.append(sp.csr_matrix((sign.astype(np.complex128), (dst, src)), shape=(self.dim, self.dim)))
        self.cre = [a.getH().tocsr() for a in self.ann]

    def a(self, p):
        return self.ann[p]

    def ad(self, p):
        return self.cre[p]

    def det(self, occupied):
        """State vector of the determinant a+_{p1} a+_{p2} ... |vac> with p1 < p2 < ... (sign +1)."""
        vec = np.zeros(self.dim, dtype=np.complex128)
        vec[sum(1 << p for p in occupied)] = 1.0
        return vec

    def number(self):
        return np.array([bin(s).count("1") for s in range(self.dim)])


def hamiltonian(fs: FockSpace, eps, L):
    """Second-quantised H (dense) from spinor energies and Cholesky vectors."""
    n = fs.n
    L = np.asarray(L, dtype=np.complex128)
    J = np.einsum("Ppr,Pqs->prqs", L, L)                      # (pr|qs)
    anti = J.transpose(0, 2, 1, 3) - J.transpose(0, 2, 3, 1)  # <pq||rs> = (pr|qs) - (ps|qr)
    h = np.diag(np.asarray(eps, dtype=np.complex128)).copy()
    # h_pq = eps_p delta_pq - sum_k <pk||qk>, k over the occupied spinors of the reference
    return h, J, anti


def build_h(fs: FockSpace, eps, L, o):
    n = fs.n
    h, J, anti = hamiltonian(fs, eps, L)
    h = h - np.einsum("pkqk->pq", anti[:, :o, :, :o])
    E = [[(fs.ad(p) @ fs.a(q)).tocsr() for q in range(n)] for p in range(n)]
    H = sp.csr_matrix((fs.dim, fs.dim), dtype=np.complex128)
    for p in range(n):
        for q in range(n):
            if h[p, q] != 0:
                H = H + h[p, q] * E[p][q]
    # 1/2 sum (pr|qs) a+_p a+_q a_s a_r = 1/2 sum (pr|qs) (E_pr E_qs - delta_qr E_ps)
    for P in range(L.shape[0]):
        Lam = sp.csr_matrix((fs.dim, fs.dim), dtype=np.complex128)
        for p in range(n):
            for r in range(n):
                if L[P, p, r] != 0:
                    Lam = Lam + L[P, p, r] * E[p][r]
        H = H + 0.5 * (Lam @ Lam)
    K = np.einsum("pqqs->ps", J)
    for p in range(n):
        for s in range(n):
            if K[p, s] != 0:
                H = H - 0.5 * K[p, s] * E[p][s]
    return H.toarray()


def cluster_operator(fs: FockSpace, t1, t2, o):
    v = t1.shape[1]
    T = sp.csr_matrix((fs.dim, fs.dim), dtype=np.complex128)
    for i in range(o):
        for a in range(v):
            if t1[i, a] != 0:
                T = T + t1[i, a] * (fs.ad(o + a) @ fs.a(i))
    for i in range(o):
        for j in range(i + 1, o):
            for a in range(v):
                for b in range(a + 1, v):
                    if t2[i, j, a, b] != 0:
                        T = T + t2[i, j, a, b] * (fs.ad(o + a) @ fs.ad(o + b) @ fs.a(j) @ fs.a(i))
    return T.toarray()


def expm_nilpotent(T, sign=1.0):
    out = np.eye(T.shape[0], dtype=np.complex128)
    term = out.copy()
    for k in range(1, 64):
        term = (sign / k) * (term @ T)
        if not np.any(term):
            break
        out = out + term
    return out


def hbar(fs, H, T):
    return expm_nilpotent(T, -1.0) @ H @ expm_nilpotent(T, 1.0)


def reference(fs, o):
    return fs.det(range(o))


def projections(fs, Hb, o, v):
    """(E, Omega1, Omega2): <Phi0|Hb|Phi0>, <Phi_i^a|Hb|Phi0>, <Phi_ij^ab|Hb|Phi0>.

    |Phi_i^a> = a+_a a_i |Phi0>,  |Phi_ij^ab> = a+_a a+_b a_j a_i |Phi0>.
    """
    phi0 = reference(fs, o)
    hv = Hb @ phi0
    E = np.vdot(phi0, hv)
    w1 = np.zeros((o, v), dtype=np.complex128)
    w2 = np.zeros((o, o, v, v), dtype=np.complex128)
    for i in range(o):
        for a in range(v):
            s = fs.ad(o + a) @ (fs.a(i) @ phi0)
            w1[i, a] = np.vdot(s, hv)
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    if i == j or a == b:
                        continue
                    s = fs.ad(o + a) @ (fs.ad(o + b) @ (fs.a(j) @ (fs.a(i) @ phi0)))
                    w2[i, j, a, b] = np.vdot(s, hv)
    return E, w1, w2


def ip_basis(fs, o, v):
    """Basis of the IP space: a_i|Phi0> (i), then a+_b a_j a_i|Phi0> for i<j, b (b fastest)."""
    phi0 = reference(fs, o)
    vecs = [fs.a(i) @ phi0 for i in range(o)]
    for i in range(o):
        for j in range(i + 1, o):
            for b in range(v):
                vecs.append(fs.ad(o + b) @ (fs.a(j) @ (fs.a(i) @ phi0)))
    return np.array(vecs)


def ip_sigma(fs, Hb, o, v, r1, r2):
    """<K|[H-bar, R]|Phi0> for the IP basis states K (1h then 2h1p, packed i<j)."""
    phi0 = reference(fs, o)
    R = sp.csr_matrix((fs.dim, fs.dim), dtype=np.complex128)
    for i in range(o):
        R = R + r1[i] * fs.a(i)
    for i in range(o):
        for j in range(i + 1, o):
            for b in range(v):
                R = R + r2[i, j, b] * (fs.ad(o + b) @ fs.a(j) @ fs.a(i))
    R = R.toarray()
    vec = Hb @ (R @ phi0) - R @ (Hb @ phi0)
    return ip_basis(fs, o, v).conj() @ vec


def sector_eigenvalues(fs, H, nelec):
    idx = np.where(fs.number() == nelec)[0]
    return np.linalg.eigvals(H[np.ix_(idx, idx)])
