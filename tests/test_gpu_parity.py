"""GPU hot path vs the FP64 CPU oracle, through the C ABI.

Sizes are chosen so the oracle finishes in seconds while the GPU GEMMs span several 64 x 64 tiles
with ragged tails (v = 70 > 64, o*v not a multiple of 64).
"""
import numpy as np
import pytest

from paper_2506_06805_amd import synth
from oracle import ccsd, eom, integrals

pytestmark = pytest.mark.gpu

TOL_TERM = 1e-11     # relative, one residual / sigma evaluation in FP64
TOL_E = 1e-8         # Eh, converged energies and IPs


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _host(x):
    return x.detach().cpu().numpy()


def _rand_amps(o, v, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    t1 = (rng.standard_normal((o, v)) + 1j * rng.standard_normal((o, v))) * scale
    t2 = (rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v))) * scale
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    return t1, t2


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SHAPES = [(4, 10, 20), (9, 70, 45), (3, 5, 7)]


@pytest.mark.parametrize("o,v,N", SHAPES)
def test_residual_parity_random_t(gpu_ctx, o, v, N):
    from paper_2506_06805_amd import fnscc
    inst = synth.make_instance(o, v, N, seed=11 + o, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    t1, t2 = _rand_amps(o, v, 3)
    r1, r2 = fnscc.ccsd_residual(gpu_ctx, ints, _dev(t1), _dev(t2))
    g = integrals.Blocks(inst.L, o)
    w1, w2 = ccsd.residuals(g, inst.eps, t1, t2)
    assert _rel(_host(r1), w1) < TOL_TERM
    assert _rel(_host(r2), w2) < TOL_TERM


@pytest.mark.parametrize("o,v,N", SHAPES)
def test_ladder_parity(gpu_ctx, o, v, N):
    from paper_2506_06805_amd import fnscc
    inst = synth.make_instance(o, v, N, seed=21 + v, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    _, tau = _rand_amps(o, v, 5)
    R = _host(fnscc.ladder(gpu_ctx, ints, _dev(tau)))
    V = slice(o, o + v)
    vvvv = integrals.antisym(inst.L.astype(np.complex128), V, V, V, V)
    ref = 0.5 * np.einsum("ijef,abef->ijab", tau, vvvv, optimize=True)
    assert _rel(R, ref) < TOL_TERM


@pytest.mark.parametrize("o,v,N", SHAPES)
def test_sigma_parity_random_t(gpu_ctx, o, v, N):
    from paper_2506_06805_amd import fnscc
    inst = synth.make_instance(o, v, N, seed=31 + o, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    t1, t2 = _rand_amps(o, v, 7)
    amps = fnscc.amps_create(gpu_ctx, ints, _dev(t1), _dev(t2))
    g = integrals.Blocks(inst.L, o)
    h = eom.Hbar(g, inst.eps, t1, t2)
    rng = np.random.default_rng(9)
    dim = eom.dim(o, v)
    R = rng.standard_normal((3, dim)) + 1j * rng.standard_normal((3, dim))
    S = _host(fnscc.ipeom_sigma(gpu_ctx, ints, amps, _dev(R)))
    ref = eom.sigma(h, R)
    assert _rel(S, ref) < TOL_TERM


def test_sigma_parity_large_block(gpu_ctx):
    # 40 trial vectors at o = 12: the ring product has k o = 480 rows, so both grouped launches run
    # on the direct-to-LDS three-product tile; right and left products against the oracle
    from paper_2506_06805_amd import fnscc
    o, v, N, k = 12, 24, 60, 40
    inst = synth.make_instance(o, v, N, seed=83, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    t1, t2 = _rand_amps(o, v, 8)
    amps = fnscc.amps_create(gpu_ctx, ints, _dev(t1), _dev(t2))
    h = eom.Hbar(integrals.Blocks(inst.L, o), inst.eps, t1, t2)
    rng = np.random.default_rng(10)
    dim = eom.dim(o, v)
    R = rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))
    assert _rel(_host(fnscc.ipeom_sigma(gpu_ctx, ints, amps, _dev(R))), eom.sigma(h, R)) < TOL_TERM
    assert _rel(_host(fnscc.ipeom_sigma_left(gpu_ctx, ints, amps, _dev(R))), eom.sigma_left(h, R)) < TOL_TERM


def test_solve_parity_small(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    o, v, N, k = 6, 20, 60, 4
    inst = synth.make_instance(o, v, N, seed=77, kappa=synth.kappa_for(v, N))
    e_ref, t1, t2, _, conv = ccsd.solve(inst.L, inst.eps, o)
    assert conv
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    e, it, amps = fnscc.ccsd_solve(gpu_ctx, ints)
    assert abs(e - e_ref) < TOL_E
    g = integrals.Blocks(inst.L, o)
    w_ref, _ = eom.dense_roots(eom.Hbar(g, inst.eps, t1, t2), k)
    w, its = fnscc.ipeom_davidson(gpu_ctx, ints, amps, k)
    assert np.abs(w - w_ref).max() < TOL_E
