"""Single-step pivoted Cholesky of AO integrals and the 2-component MO transform
(test infrastructure), Eq. 21-22.

Readings taken: the pivot is the largest remaining diagonal element (lowest
composite index on ties); vectors are added while that element is not below
the threshold, i.e. the loop stops as soon as max diagonal < tau.  The AO
vectors are real (Eq. 8 makes the two-electron operator spin-free), and for
two-component spinors with coefficients C = [C_alpha; C_beta] the spinor-basis
vectors are L^P = C_alpha^H L^P_AO C_alpha + C_beta^H L^P_AO C_beta (Hermitian).
"""
from __future__ import annotations

import numpy as np


def pivoted_cholesky(M, tau, max_vec=None, with_pivots=False):
    """Return (Lvec (nvec, m), residual diagonal) with M ~= Lvec^T Lvec; with_pivots adds the
    pivot index of each vector.  max_vec caps the number of vectors (the loop then ends early
    with the diagonal still above tau)."""
    M = np.asarray(M, dtype=np.float64)
    m = M.shape[0]
    cap = m if max_vec is None else min(m, max_vec)
    d = np.diag(M).copy()
    vecs, pivots = [], []
    while len(vecs) < cap:
        p = int(np.argmax(d))          # first index among equal maxima
        if d[p] < tau:
            break
        col = M[:, p].copy()
        for l in vecs:
            col -= l * l[p]
        l = col / np.sqrt(d[p])
        vecs.append(l)
        pivots.append(p)
        d = d - l * l
        d[p] = 0.0
    Lvec = np.array(vecs) if vecs else np.zeros((0, m))
    if with_pivots:
        return Lvec, d, np.array(pivots, dtype=np.int64)
    return Lvec, d


def ao_to_spinor(Lao, C, nao):
    """L^P_pq = sum_{mu nu} C*_{mu p} L^P_{mu nu} C_{nu q} over both spin blocks (Eq. 22)."""
    Lao = np.asarray(Lao, dtype=np.float64).reshape(-1, nao, nao)
    Ca, Cb = C[:nao], C[nao:]
    return (np.einsum("mp,Pmn,nq->Ppq", Ca.conj(), Lao, Ca, optimize=True)
            + np.einsum("mp,Pmn,nq->Ppq", Cb.conj(), Lao, Cb, optimize=True))
