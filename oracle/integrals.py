"""Antisymmetrised two-electron integrals from Cholesky vectors (test infrastructure).

Eq. 21: (pr|qs) = sum_P L^P_pr L^P_qs  (Mulliken order, bra spinor p conjugated).
Eq. 23: <pq||rs> = sum_P (L^P_pr L^P_qs - L^P_ps L^P_qr).

Spinor index convention: 0..o-1 occupied, o..n-1 virtual.
"""
from __future__ import annotations

import numpy as np


def mulliken(L, s1, s2, s3, s4):
    """(pq|rs) block for index slices: sum_P L^P_pq L^P_rs (Eq. 21)."""
    return np.einsum("Ppq,Prs->pqrs", L[:, s1, s2], L[:, s3, s4], optimize=True)


def antisym(L, s1, s2, s3, s4):
    """<pq||rs> block: sum_P L^P_pr L^P_qs - L^P_ps L^P_qr (Eq. 23)."""
    a = np.einsum("Ppr,Pqs->pqrs", L[:, s1, s3], L[:, s2, s4], optimize=True)
    b = np.einsum("Pps,Pqr->pqrs", L[:, s1, s4], L[:, s2, s3], optimize=True)
    return a - b


def full_antisym(L):
    """All of <pq||rs> (tiny systems only)."""
    s = slice(0, L.shape[1])
    return antisym(L, s, s, s, s)


class Blocks:
    """The integral blocks the CCSD and IP-EOM equations use, each built on first use.

    Blocks with at most two virtual indices are the ones the paper stores
    (Sec. 3); the three-virtual blocks here are plain full arrays (the
    oracle only runs on sizes where they fit) and the four-virtual block is
    produced one leading index at a time by `vvvv_row`.
    """

    _SLICES = {
        "oooo": "OOOO", "ooov": "OOOV", "oovo": "OOVO", "oovv": "OOVV", "ovov": "OVOV",
        "ovvo": "OVVO", "ovoo": "OVOO", "vvoo": "VVOO", "ovvv": "OVVV", "vovv": "VOVV",
        "vvvo": "VVVO",
    }

    def __init__(self, L, o):
        self.L = np.asarray(L, dtype=np.complex128)
        self.o = o
        self.n = self.L.shape[1]
        self.v = self.n - o
        self.O, self.V = slice(0, o), slice(o, self.n)

    def __getattr__(self, name):
        kinds = Blocks._SLICES.get(name)
        if kinds is None:
            raise AttributeError(name)
        sl = [self.O if k == "O" else self.V for k in kinds]
        block = antisym(self.L, *sl)
        setattr(self, name, block)
        return block

    def vvvv_row(self, a):
        """<ab||ef> for a fixed first virtual index a: shape (v, v, v) over (b, e, f)."""
        V = self.V
        La = self.L[:, self.o + a, V]            # L^P_{a e}
        Lvv = self.L[:, V, V]
        x = np.einsum("Pe,Pbf->bef", La, Lvv, optimize=True)
        y = np.einsum("Pf,Pbe->bef", La, Lvv, optimize=True)
        return x - y
