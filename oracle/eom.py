"""IP-EOM-CCSD in FP64 (test infrastructure).

Eq. 16-18: the ionised states are R_k |Psi_cc> with R_k = sum_i r_i a_i +
sum_{i<j,b} r_ij^b a+_b a_j a_i (Eq. 17), and omega_k are the eigenvalues of
H-bar restricted to the 1h + 2h1p space (Eq. 18).  H-bar = e^-T H e^T enters
through its one- and two-body blocks with at most two virtual indices, built
once from the converged amplitudes (Sec. 3); one three-body piece appears as
X_e = 1/2 sum_mnf <mn||ef> r_mn^f.

Vector layout (shared with the library's documented ABI): r_i for i = 0..o-1,
then r_ij^b for i<j in lexicographic order with b fastest.  r_ji^b = -r_ij^b.

The sigma equations are pinned by the Fock-space brute force
(<K|[H-bar, R]|Phi0> for random T and R).
"""
from __future__ import annotations

import numpy as np

from .ccsd import taus
from .integrals import Blocks

ein = lambda *a: np.einsum(*a, optimize=True)


class Hbar:
    """F-bar and W-bar blocks of H-bar with at most two virtual indices."""

    def __init__(self, g: Blocks, eps, t1, t2):
        o, v = t1.shape
        eo, ev = np.asarray(eps[:o]), np.asarray(eps[o:])
        _, tau = taus(t1, t2)
        self.o, self.v = o, v
        self.Fmi = np.diag(eo).astype(np.complex128) + ein("ne,mnie->mi", t1, g.ooov) \
            + 0.5 * ein("inef,mnef->mi", tau, g.oovv)
        self.Fae = np.diag(ev).astype(np.complex128) + ein("mf,amef->ae", t1, g.vovv) \
            - 0.5 * ein("mnaf,mnef->ae", tau, g.oovv)
        self.Fme = ein("nf,mnef->me", t1, g.oovv)
        x = ein("je,mnie->mnij", t1, g.ooov)
        self.Wmnij = g.oooo + x - x.transpose(0, 1, 3, 2) + 0.5 * ein("ijef,mnef->mnij", tau, g.oovv)
        self.Wmnie = g.ooov + ein("if,mnfe->mnie", t1, g.oovv)
        self.Wmbej = (g.ovvo + ein("jf,mbef->mbej", t1, g.ovvv) - ein("nb,mnej->mbej", t1, g.oovo)
                      - ein("jnfb,mnef->mbej", t2 + ein("jf,nb->jnfb", t1, t1), g.oovv))
        # W_mbij = <mb||ij> - F_me t_ij^be - t_n^b W_mnij + 1/2 <mb||ef> tau_ij^ef
        #          + P(ij) <mn||ie> t_jn^be + P(ij) t_i^e (<mb||ej> - t_nj^bf <mn||ef>)
        W = g.ovoo - ein("me,ijbe->mbij", self.Fme, t2) - ein("nb,mnij->mbij", t1, self.Wmnij) \
            + 0.5 * ein("mbef,ijef->mbij", g.ovvv, tau)
        x = ein("mnie,jnbe->mbij", g.ooov, t2) \
            + ein("ie,mbej->mbij", t1, g.ovvo - ein("njbf,mnef->mbej", t2, g.oovv))
        self.Wmbij = W + x - x.transpose(0, 1, 3, 2)
        self.oovv = g.oovv
        self.t2 = t2

    def diagonal(self):
        """Diagonal of the 1h + 2h1p matrix: -F_ii; F_bb - F_ii - F_jj (i<j)."""
        o, v = self.o, self.v
        fo, fv = np.diag(self.Fmi), np.diag(self.Fae)
        iu, ju = np.triu_indices(o, 1)
        d2 = fv[None, :] - fo[iu][:, None] - fo[ju][:, None]
        return np.concatenate([-fo, d2.ravel()])


def dim(o, v):
    return o + o * (o - 1) // 2 * v


def unpack(vec, o, v):
    iu, ju = np.triu_indices(o, 1)
    r1 = vec[:o]
    r2 = np.zeros((o, o, v), dtype=np.complex128)
    x = vec[o:].reshape(len(iu), v)
    r2[iu, ju] = x
    r2[ju, iu] = -x
    return r1, r2


def pack(r1, r2):
    o = r1.shape[0]
    iu, ju = np.triu_indices(o, 1)
    return np.concatenate([r1, r2[iu, ju].ravel()])


def sigma_full(h: Hbar, r1, r2):
    """sigma = H-bar R on the 1h + 2h1p space, unpacked arrays r1[i], r2[i, j, b]."""
    s1 = -ein("mi,m->i", h.Fmi, r1) + ein("me,ime->i", h.Fme, r2) - 0.5 * ein("mnie,mne->i", h.Wmnie, r2)
    s2 = -ein("maij,m->ija", h.Wmbij, r1) + ein("ae,ije->ija", h.Fae, r2)
    x = ein("mi,mja->ija", h.Fmi, r2)
    s2 -= x - x.transpose(1, 0, 2)
    s2 += 0.5 * ein("mnij,mna->ija", h.Wmnij, r2)
    x = ein("maej,ime->ija", h.Wmbej, r2)
    s2 += x - x.transpose(1, 0, 2)
    X = 0.5 * ein("mnef,mnf->e", h.oovv, r2)
    s2 += ein("e,ijae->ija", X, h.t2)
    return s1, s2


def sigma(h: Hbar, vec):
    """sigma for a packed vector (or a (k, dim) block of them)."""
    vec = np.asarray(vec, dtype=np.complex128)
    if vec.ndim == 2:
        return np.array([sigma(h, x) for x in vec])
    r1, r2 = unpack(vec, h.o, h.v)
    s1, s2 = sigma_full(h, r1, r2)
    return pack(s1, s2)


def dense_matrix(h: Hbar):
    n = dim(h.o, h.v)
    M = np.zeros((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for k in range(n):
        e[:] = 0
        e[k] = 1
        M[:, k] = sigma(h, e)
    return M


def lowest_roots(w, k):
    order = np.lexsort((w.imag, w.real))
    return w[order[:k]], order[:k]


def dense_roots(h: Hbar, k):
    """Exact lowest-k (by real part) eigenvalues of the explicit IP-EOM matrix."""
    M = dense_matrix(h)
    w, V = np.linalg.eig(M)
    wk, idx = lowest_roots(w, k)
    return wk, V[:, idx]


def sigma_left(h: Hbar, vec):
    """Left sigma: the row vector(s) l times the IP-EOM matrix, (L H-bar) restricted to the 1h + 2h1p
    space (Eq. 19-20: <Phi0| L_k H-bar = omega_k <Phi0| L_k).  Plain definition through the dense
    matrix, whose columns are pinned by the Fock-space brute force."""
    vec = np.asarray(vec, dtype=np.complex128)
    return vec @ dense_matrix(h)


def left_right_roots(h: Hbar, k):
    """Lowest-k roots with right vectors (columns of R) and left vectors (rows of L) normalised to
    the biorthogonality of Eq. 19, sum_x L[k, x] R[x, l] = delta_kl (a bilinear product: <Phi0|L_k
    R_l|Phi0> pairs l^i with r_i and l_b^ij with r_ij^b, no complex conjugation)."""
    M = dense_matrix(h)
    w, V = np.linalg.eig(M)
    Vinv = np.linalg.inv(V)              # rows: left eigenvectors, Vinv V = 1
    wk, idx = lowest_roots(w, k)
    return wk, V[:, idx], Vinv[idx, :]


def one_hole_weight(L, R, o):
    """Share of the biorthonormal product carried by the 1h part, sum_i l^i r_i, per root."""
    return np.einsum("ki,ik->k", L[:, :o], R[:o, :])


def davidson(h: Hbar, k, r_tol=1e-9, w_tol=1e-10, max_iter=200, max_sub=None, nguess=None, verbose=False):
    """Non-Hermitian Davidson for the k eigenvalues of lowest real part.

    Readings taken (the paper names the method only): 2k unit guesses at the
    smallest real diagonal entries; subspace matrix G = V^H (H-bar V) with
    orthonormal V; Ritz pairs of lowest real part; correction
    (H-bar x - theta x) / (theta - diag); Gram-Schmidt twice; collapse to the
    current 2k Ritz vectors when the subspace exceeds 20k.
    """
    n = dim(h.o, h.v)
    nguess = nguess or min(n, 2 * k)
    max_sub = max_sub or min(n, max(20 * k, nguess + k))
    diag = h.diagonal()
    order = np.argsort(diag.real, kind="stable")[:nguess]
    V = np.zeros((nguess, n), dtype=np.complex128)
    V[np.arange(nguess), order] = 1.0
    S = sigma(h, V)
    theta_old = None
    for it in range(1, max_iter + 1):
        G = V.conj() @ S.T
        w, Y = np.linalg.eig(G)
        wk, idx = lowest_roots(w, k)
        Yk = Y[:, idx]
        X = Yk.T @ V                    # Ritz vectors (k, n)
        Rs = Yk.T @ S - wk[:, None] * X
        rn = np.linalg.norm(Rs, axis=1)
        dw = np.inf if theta_old is None else np.max(np.abs(wk - theta_old))
        if verbose:
            print(it, wk.real, rn.max())
        if rn.max() < r_tol and dw < w_tol:
            return wk, X, it
        theta_old = wk
        new = []
        for j in range(k):
            if rn[j] < r_tol:
                continue
            den = wk[j] - diag
            den = np.where(np.abs(den) < 1e-8, 1e-8, den)
            new.append(Rs[j] / den)
        if V.shape[0] + len(new) > max_sub:
            keep = min(len(w), 2 * k)
            _, idx2 = lowest_roots(w, keep)
            Yc = Y[:, idx2]
            Q, _ = np.linalg.qr((Yc.T @ V).T)
            V = Q.T.copy()
            S = sigma(h, V)
        added = []
        for x in new:
            for _ in range(2):
                x = x - V.conj() @ x @ V if V.size else x
                for y in added:
                    x = x - np.vdot(y, x) * y
            nrm = np.linalg.norm(x)
            if nrm > 1e-10:
                added.append(x / nrm)
        if not added:
            return wk, X, it
        A = np.array(added)
        V = np.vstack([V, A])
        S = np.vstack([S, sigma(h, A)])
    return wk, X, max_iter
