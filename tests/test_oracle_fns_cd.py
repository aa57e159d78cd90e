"""Pins of the oracle's Cholesky (Eq. 21-22) and frozen-natural-spinor (Eq. 24-28) steps.

P5: the pivoted Cholesky residual is positive semi-definite, so every entry of M - L^T L is bounded
by the largest remaining diagonal (< tau); as tau -> 0 the vector count equals rank(M) and the
spinor-basis integrals rebuilt from the vectors equal the explicit four-index transform.
P6: D_vv is Hermitian positive semi-definite with trace 1/2 sum |t|^2.
P7: with nothing truncated, FNS is a unitary rotation of the virtuals: energies and IPs unchanged.
"""
import numpy as np
import pytest

from paper_2506_06805_amd import synth
from oracle import ccsd, cd, eom, fns, integrals


@pytest.mark.parametrize("tau", [1e-1, 1e-3, 1e-6])
def test_p5_cd_error_bound(tau):
    nao = 6
    M = synth.make_ao_eri(nao, 30, seed=1)
    Lv, d = cd.pivoted_cholesky(M, tau)
    R = M - Lv.T @ Lv
    assert np.abs(R).max() <= np.max(d) + 1e-12
    assert np.max(d) < tau
    assert np.linalg.eigvalsh(R).min() > -1e-10


def test_p5_cd_exact_limit_matches_four_index_transform():
    nao, rank, n, o = 5, 12, 6, 2
    M = synth.make_ao_eri(nao, rank, seed=2)
    Lv, _ = cd.pivoted_cholesky(M, 1e-12)
    assert Lv.shape[0] == np.linalg.matrix_rank(M, tol=1e-9)
    C = synth.make_spinor_coefficients(nao, n, seed=3)
    L = cd.ao_to_spinor(Lv, C, nao)
    for P in range(L.shape[0]):
        assert np.abs(L[P] - L[P].conj().T).max() < 1e-12
    # explicit transform: (pq|rs) = sum D^pq_{mu nu} M_{mu nu, ka la} D^rs_{ka la},
    # D^pq_{mu nu} = sum_sigma conj(C_{mu sigma, p}) C_{nu sigma, q}
    Dm = np.einsum("mp,nq->pqmn", C[:nao].conj(), C[:nao]) + np.einsum("mp,nq->pqmn", C[nao:].conj(), C[nao:])
    Dm = Dm.reshape(n, n, nao * nao)
    mull = np.einsum("pqx,xy,rsy->pqrs", Dm, M, Dm)
    s = slice(0, n)
    assert np.abs(integrals.mulliken(L, s, s, s, s) - mull).max() < 1e-10
    anti = mull.transpose(0, 2, 1, 3) - mull.transpose(0, 2, 3, 1)
    assert np.abs(integrals.full_antisym(L) - anti).max() < 1e-10


def test_p5_cd_pivot_order_diagonal_matrix():
    # a diagonal M is its own Cholesky factor: vectors sqrt(m_pp) e_p, pivots in descending order
    # of the diagonal, the lowest index first among equal entries; max_vec stops early
    vals = np.array([3.0, 1.0, 4.0, 1.5, 9.0, 2.6, 4.0])
    Lv, d, piv = cd.pivoted_cholesky(np.diag(vals), 1e-12, with_pivots=True)
    assert list(piv) == [4, 2, 6, 0, 5, 3, 1]
    assert np.allclose(Lv, np.sqrt(vals)[piv, None] * np.eye(7)[piv], atol=0, rtol=1e-15)
    assert np.abs(d).max() == 0.0
    Lv2, d2, piv2 = cd.pivoted_cholesky(np.diag(vals), 1e-12, max_vec=2, with_pivots=True)
    assert list(piv2) == [4, 2] and np.array_equal(Lv2, Lv[:2])
    assert d2.max() == 4.0
    _, _, piv3 = cd.pivoted_cholesky(np.diag(vals), 2.0, with_pivots=True)
    assert list(piv3) == [4, 2, 6, 0, 5]


def test_p5_cd_full_rank_is_permuted_cholesky():
    # positive definite M, tau -> 0: M[piv][:, piv] = G G^T with G lower triangular, G = L[:, piv]^T
    rng = np.random.default_rng(4)
    A = rng.standard_normal((9, 9))
    M = A @ A.T + 0.1 * np.eye(9)
    Lv, _, piv = cd.pivoted_cholesky(M, 1e-14, with_pivots=True)
    assert sorted(piv) == list(range(9))
    G = Lv[:, piv].T
    assert np.abs(np.triu(G, 1)).max() < 1e-12    # earlier pivots vanish in later vectors
    assert np.abs(G - np.linalg.cholesky(M[np.ix_(piv, piv)])).max() < 1e-12


def test_p6_density_properties():
    inst = synth.make_instance(4, 9, 15, seed=5, kappa=0.6)
    D = fns.vv_density(inst.L, inst.eps, inst.o)
    t = fns.mp2_amplitudes(inst.L, inst.eps, inst.o)
    assert np.abs(D - D.conj().T).max() < 1e-15
    assert np.linalg.eigvalsh(D).min() > -1e-15
    assert abs(np.trace(D) - 0.5 * np.sum(np.abs(t) ** 2)) < 1e-14


def test_p7_untruncated_fns_equals_canonical():
    inst = synth.make_instance(4, 10, 16, seed=7, kappa=0.5)
    L2, eps2, vp, occ, U = fns.truncate(inst.L, inst.eps, inst.o, 0.0)
    assert vp == inst.v
    assert np.abs(U.conj().T @ U - np.eye(vp)).max() < 1e-13
    assert np.all(np.diff(occ) <= 0)
    e0, t1, t2, _, _ = ccsd.solve(inst.L, inst.eps, inst.o)
    e1, s1, s2, _, _ = ccsd.solve(L2, eps2, inst.o)
    assert abs(e0 - e1) < 1e-9
    w0, _ = eom.dense_roots(eom.Hbar(integrals.Blocks(inst.L, inst.o), inst.eps, t1, t2), 6)
    w1, _ = eom.dense_roots(eom.Hbar(integrals.Blocks(L2, inst.o), eps2, s1, s2), 6)
    assert np.abs(w0 - w1).max() < 1e-9
    # the semicanonical virtual block is diagonal: F^NS Z = Z eps (Eq. 27)
    assert np.all(np.diff(eps2[inst.o:]) >= 0)


def test_fns_truncation_structured_variant():
    inst = synth.make_instance(4, 24, 30, seed=8, kappa=0.5, fns_gamma=6.0)
    L2, eps2, vp, occ, U = fns.truncate(inst.L, inst.eps, inst.o, 1e-5)
    assert 0 < vp < inst.v
    assert vp == int(np.sum(occ > 1e-5))
    for P in range(L2.shape[0]):
        assert np.abs(L2[P] - L2[P].conj().T).max() < 1e-13
    assert np.abs(U.conj().T @ U - np.eye(vp)).max() < 1e-12
