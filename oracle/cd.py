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


def pivoted_cholesky(M, tau):
    """Return (Lvec (nvec, m), residual diagonal) with M ~= Lvec^T Lvec."""
    M = np.asarray(M, dtype=np.float64)
    m = M.shape[0]
    d = np.diag(M).copy()
    vecs = []
    while True:
        p = int(np.argmax(d)) if m else 0
        if m == 0 or d[p] < tau:
            break
        col = M[:, p].copy()
        for l in vecs:
            col -= l * l[p]
        l = col / np.sqrt(d[p])
        vecs.append(l)
        d = d - l * l
        d[p] = 0.0
        if len(vecs) == m:
            break
    return (np.array(vecs) if vecs else np.zeros((0, m))), d


def ao_to_spinor(Lao, C, nao):
    """L^P_pq = sum_{mu nu} C*_{mu p} L^P_{mu nu} C_{nu q} over both spin blocks (Eq. 22)."""
    Lao = np.asarray(Lao, dtype=np.float64).reshape(-1, nao, nao)
    Ca, Cb = C[:nao], C[nao:]
    return (np.einsum("mp,Pmn,nq->Ppq", Ca.conj(), Lao, Ca, optimize=True)
            + np.einsum("mp,Pmn,nq->Ppq", Cb.conj(), Lao, Cb, optimize=True))
