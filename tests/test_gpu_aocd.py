"""The step in front of the hot path on the GPU: pivoted Cholesky of the AO supermatrix (Eq. 21)
and the two-component transform to the spinor basis (Eq. 22), against the FP64 oracle.

* small supermatrices (one, several and ragged 64-index workgroups): the same pivots, vectors to
  1e-12, the cap on the vector count;
* a 14400 x 14400 supermatrix (nao = 120): the first 40 vectors and pivots against the oracle on
  the same matrix, and at the end the residual bounds that hold for any pivoted Cholesky;
* the transform: whole results at small sizes, sampled vectors at nao = 120, n = 200;
* the whole chain AO supermatrix -> vectors -> spinor basis -> CCSD energy against the oracle's.
"""
import numpy as np
import pytest

from paper_2506_06805_amd import synth
from oracle import ccsd, cd

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(x):
    return x.detach().cpu().numpy()


@pytest.mark.parametrize("nao,rank,tau", [(5, 12, 1e-8), (8, 40, 1e-6), (12, 100, 1e-5), (12, 100, 1e-1)])
def test_cd_parity_small(gpu_ctx, nao, rank, tau):
    from paper_2506_06805_amd import fnscc
    M = synth.make_ao_eri(nao, rank, seed=nao + rank)
    Lr, dr, pr = cd.pivoted_cholesky(M, tau, with_pivots=True)
    L, piv = fnscc.cd_ao_pivoted(gpu_ctx, _dev(M), tau, M.shape[0])
    assert list(piv) == list(pr)
    L = _host(L)
    assert np.abs(L - Lr).max() < 1e-12 * np.abs(Lr).max()
    assert np.abs(M - L.T @ L).max() <= max(dr.max(), 0) + 1e-12 * np.abs(M).max()


def test_cd_cap(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    M = synth.make_ao_eri(8, 40, seed=3)
    Lr, _, pr = cd.pivoted_cholesky(M, 1e-10, max_vec=7, with_pivots=True)
    with pytest.raises(fnscc.FcError) as e:
        fnscc.cd_ao_pivoted(gpu_ctx, _dev(M), 1e-10, 7)
    assert e.value.code == fnscc.FC_ENOCONV
    L, piv = fnscc.cd_ao_pivoted(gpu_ctx, _dev(M), 1e-10, 7, allow_cap=True)
    assert list(piv) == list(pr)
    assert np.abs(_host(L) - Lr).max() < 1e-12 * np.abs(Lr).max()


def test_cd_large_supermatrix(gpu_ctx):
    import torch
    from paper_2506_06805_amd import fnscc
    nao, rank, tau = 120, 1200, 1e-6
    w, X = synth.make_ao_eri_factors(nao, rank, seed=11)
    Xd = _dev(X)
    M = synth.symmetrize_eri((Xd.T * _dev(w)) @ Xd, nao)
    del Xd
    m = nao * nao
    L, piv = fnscc.cd_ao_pivoted(gpu_ctx, M, tau, 4000)
    nvec = L.shape[0]
    assert 0 < nvec <= min(rank, nao * (nao + 1) // 2)
    assert len(set(piv.tolist())) == nvec
    # the oracle's first 40 steps on the same matrix
    Mh = _host(M)
    Lr, _, pr = cd.pivoted_cholesky(Mh, tau, max_vec=40, with_pivots=True)
    assert list(piv[:40]) == list(pr)
    assert np.abs(_host(L[:40]) - Lr).max() < 1e-11 * np.abs(Lr).max()
    del Mh, Lr
    # residual: diagonal below tau, and |R_xy| <= sqrt(R_xx R_yy) on sampled rows
    d = torch.diagonal(M) - (L * L).sum(0)
    dmax = float(d.max())
    assert dmax < tau and float(d.min()) > -1e-9
    rows = torch.from_numpy(np.random.default_rng(2).choice(m, 64, replace=False)).cuda()
    R = M[rows] - L[:, rows].T @ L
    assert float(R.abs().max()) <= tau + 1e-9


@pytest.mark.parametrize("nao,n,nvec", [(4, 6, 3), (10, 14, 30), (70, 90, 20)])
def test_ao_to_spinor_parity(gpu_ctx, nao, n, nvec):
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(nao)
    A = rng.standard_normal((nvec, nao, nao))
    Lao = (A + A.transpose(0, 2, 1)).reshape(nvec, nao * nao)
    Cs = synth.make_spinor_coefficients(nao, n, seed=n)
    out = _host(fnscc.ao_to_spinor(gpu_ctx, _dev(Lao), _dev(Cs), nao))
    ref = cd.ao_to_spinor(Lao, Cs, nao)
    assert np.abs(out - ref).max() < 1e-12 * np.abs(ref).max()


def test_ao_to_spinor_sampled_at_scale(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    nao, n, nvec = 120, 200, 1500
    rng = np.random.default_rng(5)
    A = rng.standard_normal((nvec, nao, nao))
    Lao = (A + A.transpose(0, 2, 1)).reshape(nvec, nao * nao)
    Cs = synth.make_spinor_coefficients(nao, n, seed=6)
    out = fnscc.ao_to_spinor(gpu_ctx, _dev(Lao), _dev(Cs), nao)
    for P in (0, 777, nvec - 1):
        ref = cd.ao_to_spinor(Lao[P:P + 1], Cs, nao)[0]
        got = _host(out[P])
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max(), P
        assert np.abs(got - got.conj().T).max() < 1e-12 * np.abs(ref).max(), P


def test_chain_ao_to_ccsd_energy(gpu_ctx):
    # supermatrix -> vectors -> spinor basis -> CCSD, every step on the GPU, against the oracle chain
    from paper_2506_06805_amd import fnscc
    nao, n, o, s = 6, 10, 4, 0.2
    M = synth.make_ao_eri(nao, 30, seed=1) * (s * s)
    Cs = synth.make_spinor_coefficients(nao, n, seed=3)
    rng = np.random.default_rng(8)
    eps = np.concatenate([np.sort(rng.uniform(-3, -0.3, o)), np.sort(rng.uniform(0.05, 6, n - o))])
    Lr, _ = cd.pivoted_cholesky(M, 1e-10)
    e_ref, _, _, _, conv = ccsd.solve(cd.ao_to_spinor(Lr, Cs, nao), eps, o)
    assert conv
    Lao, _ = fnscc.cd_ao_pivoted(gpu_ctx, _dev(M), 1e-10, M.shape[0])
    Lmo = fnscc.ao_to_spinor(gpu_ctx, Lao, _dev(Cs), nao)
    ints = fnscc.cd_integrals(gpu_ctx, eps, Lmo, o)
    e, _, _ = fnscc.ccsd_solve(gpu_ctx, ints)
    assert abs(e - e_ref) < 1e-10
