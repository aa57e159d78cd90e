"""MP2 frozen natural spinors in FP64 (test infrastructure), Eq. 24-28.

Readings taken where the paper is terse:
* Eq. 24's denominator eps_ij^ac is eps_i + eps_j - eps_a - eps_c; with
  t_ij^ab = <ab||ij> / eps_ij^ab the density is D_ab = 1/2 sum_ijc t_ij^ac conj(t_ij^bc)
  (Hermitian, positive semi-definite).
* Eq. 25: eigenvalues sorted descending; a natural spinor is kept when its
  occupation is strictly above the threshold.
* Eq. 26: F_vv is the canonical diag(eps_v).
* Eq. 28 prints U = Z~ V~, which does not compose (V~ is v x v', Z~ is
  v' x v'); the transformation taken is U = V~ Z~ (v x v').
* Only virtual spinors are rotated; occupied spinors stay canonical.
"""
from __future__ import annotations

import numpy as np

from .integrals import antisym


def mp2_amplitudes(L, eps, o):
    n = L.shape[1]
    O, V = slice(0, o), slice(o, n)
    eo, ev = eps[:o], eps[o:]
    d2 = eo[:, None, None, None] + eo[None, :, None, None] - ev[None, None, :, None] - ev[None, None, None, :]
    return antisym(np.asarray(L, np.complex128), V, V, O, O).transpose(2, 3, 0, 1) / d2


def vv_density(L, eps, o):
    """D_ab = 1/2 sum_ijc t_ij^ac conj(t_ij^bc) (Eq. 24)."""
    t = mp2_amplitudes(L, eps, o)
    return 0.5 * np.einsum("ijac,ijbc->ab", t, t.conj(), optimize=True)


def natural_spinors(L, eps, o, thresh):
    """Eq. 25-28: returns (U (v x v'), eps_vir_new (v'), occupations (v, descending))."""
    D = vv_density(L, eps, o)
    n_occ, V = np.linalg.eigh(D)
    order = np.argsort(-n_occ, kind="stable")
    n_occ, V = n_occ[order], V[:, order]
    keep = n_occ > thresh
    Vt = V[:, keep]
    F = Vt.conj().T @ np.diag(eps[o:]) @ Vt
    e_new, Z = np.linalg.eigh(F)
    U = Vt @ Z
    return U, e_new, n_occ


def transform(L, eps, o, U, e_new):
    """Rotate the virtual spinors by U: L_ov U, U^H L_vo, U^H L_vv U; eps_v <- e_new."""
    L = np.asarray(L, np.complex128)
    vp = U.shape[1]
    n2 = o + vp
    out = np.zeros((L.shape[0], n2, n2), dtype=np.complex128)
    O, V = slice(0, o), slice(o, L.shape[1])
    out[:, :o, :o] = L[:, O, O]
    out[:, :o, o:] = L[:, O, V] @ U
    out[:, o:, :o] = U.conj().T @ L[:, V, O]
    out[:, o:, o:] = U.conj().T @ L[:, V, V] @ U
    return out, np.concatenate([eps[:o], e_new])


def truncate(L, eps, o, thresh):
    """Full FNS step: (L', eps', v', occupations, U)."""
    U, e_new, n_occ = natural_spinors(L, eps, o, thresh)
    L2, eps2 = transform(L, eps, o, U, e_new)
    return L2, eps2, U.shape[1], n_occ, U
