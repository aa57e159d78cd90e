"""CCSD amplitude equations in FP64 (test infrastructure).

The paper states the CCSD projections (Eq. 13-15) and defers the working
equations to the textbook literature.  This file writes them in the
spin-orbital Stanton-Gauss intermediate form with complex-correct index
placement: creation-side indices in the bra of <pq||rs>, annihilation-side
indices in the ket.  The Fock operator is diagonal (f_pq = delta_pq eps_p), so
f_ov = 0.  Amplitudes: t1[i, a] = t_i^a, t2[i, j, a, b] = t_ij^ab.

The residuals returned are Omega = <Phi_S| e^-T H e^T |Phi0> for the given
(not necessarily converged) amplitudes; the brute-force Fock-space check in
tests/test_oracle_fockspace.py pins them.
"""
from __future__ import annotations

import numpy as np

from .integrals import Blocks

ein = lambda *a: np.einsum(*a, optimize=True)


def denominators(eps, o):
    eo, ev = eps[:o], eps[o:]
    d1 = eo[:, None] - ev[None, :]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return d1, d2


def taus(t1, t2):
    """tau~ = t2 + 1/2 (t_i^a t_j^b - t_i^b t_j^a);  tau = t2 + t_i^a t_j^b - t_i^b t_j^a."""
    x = ein("ia,jb->ijab", t1, t1)
    x = x - x.transpose(0, 1, 3, 2)
    return t2 + 0.5 * x, t2 + x


def energy(g: Blocks, t1, t2):
    """E_corr = 1/4 sum <ij||ab> t_ij^ab + 1/2 sum <ij||ab> t_i^a t_j^b (Eq. 15 minus E_ref)."""
    return 0.25 * ein("ijab,ijab->", g.oovv, t2) + 0.5 * ein("ijab,ia,jb->", g.oovv, t1, t1)


def intermediates(g: Blocks, t1, t2):
    """F_ae, F_mi, F_me, W_mnij, W_mbej of the CCSD equations (W_abef is used row by row)."""
    taut, tau = taus(t1, t2)
    Fae = ein("mf,mafe->ae", t1, g.ovvv) - 0.5 * ein("mnaf,mnef->ae", taut, g.oovv)
    Fmi = ein("ne,mnie->mi", t1, g.ooov) + 0.5 * ein("inef,mnef->mi", taut, g.oovv)
    Fme = ein("nf,mnef->me", t1, g.oovv)
    x = ein("je,mnie->mnij", t1, g.ooov)
    Wmnij = g.oooo + x - x.transpose(0, 1, 3, 2) + 0.25 * ein("ijef,mnef->mnij", tau, g.oovv)
    Wmbej = (g.ovvo + ein("jf,mbef->mbej", t1, g.ovvv) - ein("nb,mnej->mbej", t1, g.oovo)
             - ein("jnfb,mnef->mbej", 0.5 * t2 + ein("jf,nb->jnfb", t1, t1), g.oovv))
    return Fae, Fmi, Fme, Wmnij, Wmbej


def ladder(g: Blocks, t1, t2, rows=None):
    """1/2 sum_ef tau_ij^ef W_abef, with
    W_abef = <ab||ef> - P(ab) sum_m t_m^b <am||ef> + 1/4 sum_mn tau_mn^ab <mn||ef>.

    W_abef is formed one leading virtual index a at a time; the <ab||ef> part
    is rebuilt from the Cholesky vectors each call (Eq. 23).  `rows` limits
    the loop to some values of a (used only to time a sample).
    """
    _, tau = taus(t1, t2)
    o, v = t1.shape
    out = np.zeros((o, o, v, v), dtype=np.complex128)
    has_t1 = bool(np.any(t1))
    for a in (range(v) if rows is None else rows):
        W = g.vvvv_row(a)                                              # <ab||ef>, (b,e,f)
        if has_t1:
            # - P(ab) sum_m t_m^b <am||ef> = - sum_m t_m^b <am||ef> + sum_m t_m^a <bm||ef>
            W -= ein("mb,mef->bef", t1, g.vovv[a])
            W += ein("m,bmef->bef", t1[:, a], g.vovv)
        W += 0.25 * ein("mnb,mnef->bef", tau[:, :, a, :], g.oovv)
        out[:, :, a, :] = 0.5 * ein("ijef,bef->ijb", tau, W)
    return out


def residuals(g: Blocks, eps, t1, t2, rows=None):
    """Omega1 = RHS1 - D1 t1 and Omega2 = RHS2 - D2 t2 (Stanton-Gauss form).

    With `rows` (values of the virtual index a) the ladder is evaluated for those rows only, so
    Omega2[:, :, a, :] is exact for a in rows and incomplete elsewhere (a sampled check at sizes
    where the full ladder loop is too slow)."""
    o = g.o
    d1, d2 = denominators(eps, o)
    Fae, Fmi, Fme, Wmnij, Wmbej = intermediates(g, t1, t2)
    _, tau = taus(t1, t2)

    r1 = (ein("ie,ae->ia", t1, Fae) - ein("ma,mi->ia", t1, Fmi) + ein("imae,me->ia", t2, Fme)
          - ein("nf,naif->ia", t1, g.ovov) - 0.5 * ein("imef,maef->ia", t2, g.ovvv)
          - 0.5 * ein("mnae,nmei->ia", t2, g.oovo))

    r2 = g.vvoo.transpose(2, 3, 0, 1).copy()                          # <ab||ij> as [i,j,a,b]
    x = ein("ijae,be->ijab", t2, Fae - 0.5 * ein("mb,me->be", t1, Fme))
    r2 += x - x.transpose(0, 1, 3, 2)
    x = ein("imab,mj->ijab", t2, Fmi + 0.5 * ein("je,me->mj", t1, Fme))
    r2 -= x - x.transpose(1, 0, 2, 3)
    r2 += 0.5 * ein("mnab,mnij->ijab", tau, Wmnij)
    r2 += ladder(g, t1, t2, rows=rows)
    x = ein("imae,mbej->ijab", t2, Wmbej) - ein("ie,ma,mbej->ijab", t1, t1, g.ovvo)
    r2 += x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
    x = ein("ie,abej->ijab", t1, g.vvvo)
    r2 += x - x.transpose(1, 0, 2, 3)
    x = ein("ma,mbij->ijab", t1, g.ovoo)
    r2 -= x - x.transpose(0, 1, 3, 2)

    return r1 - d1 * t1, r2 - d2 * t2


def pack_t2(t2):
    o, v = t2.shape[0], t2.shape[2]
    iu, ju = np.triu_indices(o, 1)
    au, bu = np.triu_indices(v, 1)
    return t2[iu, ju][:, au, bu]


class DIIS:
    """Complex Pulay extrapolation on error vectors e_k = t_{k+1} - t_k (FP64).

    Reading taken: error vectors over (T1, unique T2), at most `size` vectors,
    coefficients from [B 1; 1^T 0][c; lam] = [0; 1] with B_kl = <e_k|e_l>
    (B scaled by its largest diagonal entry); while that system's condition
    number exceeds 1e12 the oldest vector is dropped.
    """

    def __init__(self, size=8):
        self.size = size
        self.vecs, self.errs = [], []

    def push(self, vec, err):
        self.vecs.append(vec.copy())
        self.errs.append(err.copy())
        if len(self.vecs) > self.size:
            self.vecs.pop(0)
            self.errs.pop(0)

    def extrapolate(self):
        while len(self.vecs) >= 2:
            m = len(self.vecs)
            B = np.zeros((m + 1, m + 1), dtype=np.complex128)
            for k in range(m):
                for l in range(m):
                    B[k, l] = np.vdot(self.errs[k], self.errs[l])
            scale = max(abs(B[k, k]) for k in range(m))
            if scale == 0.0:
                break
            B[:m, :m] /= scale
            B[m, :m] = 1.0
            B[:m, m] = 1.0
            rhs = np.zeros(m + 1, dtype=np.complex128)
            rhs[m] = 1.0
            if np.linalg.cond(B) < 1e12:
                c = np.linalg.solve(B, rhs)[:m]
                return sum(ck * vk for ck, vk in zip(c, self.vecs))
            self.vecs.pop(0)                      # ill-conditioned: drop the oldest vector
            self.errs.pop(0)
        return self.vecs[-1]


def _flatten(t1, t2):
    return np.concatenate([t1.ravel(), t2.ravel()])


def _unflatten(x, o, v):
    return x[:o * v].reshape(o, v), x[o * v:].reshape(o, o, v, v)


def solve(L, eps, o, e_tol=1e-10, r_tol=1e-9, max_iter=200, diis_size=8, verbose=False, t_init=None):
    """Iterate t <- t + Omega / D with DIIS until |dE| < e_tol and RMS(Omega) < r_tol.

    Starts from t = 0, so the first iterate is the MP2 amplitude set.
    Returns (E_corr (complex), t1, t2, iterations, converged).
    """
    g = Blocks(L, o)
    v = g.v
    eps = np.asarray(eps, dtype=np.float64)
    d1, d2 = denominators(eps, o)
    if t_init is None:
        t1 = np.zeros((o, v), dtype=np.complex128)
        t2 = np.zeros((o, o, v, v), dtype=np.complex128)
    else:
        t1, t2 = (np.array(x, dtype=np.complex128) for x in t_init)
    e_old = energy(g, t1, t2)
    diis = DIIS(diis_size)
    for it in range(1, max_iter + 1):
        r1, r2 = residuals(g, eps, t1, t2)
        rms = np.sqrt((np.vdot(r1, r1).real + np.vdot(pack_t2(r2), pack_t2(r2)).real)
                      / (r1.size + pack_t2(r2).size)) if (r1.size + pack_t2(r2).size) else 0.0
        n1, n2 = t1 + r1 / d1, t2 + r2 / d2
        if diis_size > 1:
            diis.push(_flatten(n1, n2), _flatten(n1 - t1, n2 - t2))
            n1, n2 = _unflatten(diis.extrapolate(), o, v)
        t1, t2 = n1, n2
        e = energy(g, t1, t2)
        if verbose:
            print(f"iter {it:3d}  E = {e.real:+.12f} {e.imag:+.2e}i  dE = {abs(e - e_old):.2e}  rms = {rms:.2e}")
        if abs(e - e_old) < e_tol and rms < r_tol:
            return e, t1, t2, it, True
        e_old = e
    return e, t1, t2, max_iter, False


def mp2_energy(L, eps, o):
    """E_MP2 = 1/4 sum |<ab||ij>|^2 / D_ij^ab (the first Jacobi iterate's energy from t = 0)."""
    g = Blocks(L, o)
    _, d2 = denominators(eps, o)
    t2 = g.vvoo.transpose(2, 3, 0, 1) / d2
    return energy(g, np.zeros((o, g.v), dtype=np.complex128), t2)
