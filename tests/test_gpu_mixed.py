"""Split-precision ladder and Cholesky assembly (hi/lo BF16 or FP16 on MFMA, FP32 accumulation).

Bounds: a split operand keeps ~16 (BF16) or ~22 (FP16) significant bits and each product drops only
lo*lo, so one ladder evaluation carries a relative error of order 1e-5 (BF16) or 1e-7 (FP16) of its
largest entry; the converged IPs must stay within 1e-5 Eh of the FP64 oracle.
"""
import numpy as np
import pytest

from paper_2506_06805_amd import synth
from oracle import ccsd, eom, integrals

pytestmark = pytest.mark.gpu

LADDER_TOL = {"split-bf16": 2e-4, "split-fp16": 2e-6}


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _tau(o, v, seed):
    rng = np.random.default_rng(seed)
    t = (rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v))) * 0.05
    t = t - t.transpose(1, 0, 2, 3)
    return t - t.transpose(0, 1, 3, 2)


@pytest.mark.parametrize("prec", ["split-bf16", "split-fp16"])
@pytest.mark.parametrize("o,v,N", [(4, 10, 20), (9, 70, 45), (5, 131, 40)])
def test_split_ladder_error_bound(gpu_ctx, prec, o, v, N):
    from paper_2506_06805_amd import fnscc
    inst = synth.make_instance(o, v, N, seed=51 + v, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    tau = _tau(o, v, 3)
    R64 = fnscc.ladder(gpu_ctx, ints, _dev(tau), precision="fp64").cpu().numpy()
    Rs = fnscc.ladder(gpu_ctx, ints, _dev(tau), precision=prec).cpu().numpy()
    V = slice(o, o + v)
    ref = 0.5 * np.einsum("ijef,abef->ijab", tau, integrals.antisym(inst.L, V, V, V, V), optimize=True)
    scale = np.abs(ref).max()
    assert np.abs(R64 - ref).max() < 1e-12 * scale
    err = np.abs(Rs - ref).max() / scale
    assert err < LADDER_TOL[prec], err
    assert err > 1e-15        # the split path really ran


@pytest.mark.parametrize("prec", ["split-bf16", "split-fp16"])
def test_split_assembly_integrals(gpu_ctx, prec):
    """Stored integrals assembled in split precision reproduce the FP64 residual at random T."""
    from paper_2506_06805_amd import fnscc
    o, v, N = 6, 40, 60
    inst = synth.make_instance(o, v, N, seed=61, kappa=0.5)
    i64 = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o, precision="fp64")
    isp = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o, precision=prec)
    rng = np.random.default_rng(2)
    t1 = _dev((rng.standard_normal((o, v)) + 0j) * 0.01)
    t2 = _dev(_tau(o, v, 4) * 0.2)
    a1, a2 = fnscc.ccsd_residual(gpu_ctx, i64, t1, t2)
    b1, b2 = fnscc.ccsd_residual(gpu_ctx, isp, t1, t2)
    s = max(a1.abs().max().item(), a2.abs().max().item())
    err = max((a1 - b1).abs().max().item(), (a2 - b2).abs().max().item()) / s
    assert 0 < err < LADDER_TOL[prec]


@pytest.mark.parametrize("prec", ["split-bf16", "split-fp16"])
def test_mixed_residual_error(gpu_ctx, prec):
    # split ladder + FP32 arithmetic for every other product of the residual
    from paper_2506_06805_amd import fnscc
    o, v, N = 6, 40, 50
    inst = synth.make_instance(o, v, N, seed=61, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    rng = np.random.default_rng(4)
    t1 = (rng.standard_normal((o, v)) + 1j * rng.standard_normal((o, v))) * 0.02
    t2 = _tau(o, v, 5) * 0.5
    w1, w2 = ccsd.residuals(integrals.Blocks(inst.L, o), inst.eps, t1, t2)
    r1, r2 = fnscc.ccsd_residual(gpu_ctx, ints, _dev(t1), _dev(t2), precision=prec)
    for a, b in ((r1, w1), (r2, w2)):
        rel = np.abs(a.cpu().numpy() - b).max() / np.abs(b).max()
        assert rel < LADDER_TOL[prec], rel


# o=8, v=32, N=120, 4 roots (the smallest benchmark workload): the whole oracle solve against the
# plain FP64 path (1e-8 Eh on E_corr and every IP) and against the split precisions (1e-5 Eh on
# every IP, with the energy error they carry)
SOLVE_TOL = {"fp64": (1e-8, 1e-8), "split-bf16": (1e-5, 1e-4), "split-fp16": (1e-5, 1e-4)}


@pytest.fixture(scope="module")
def c1_oracle():
    wl = synth.WORKLOADS["o8v32n120"]
    o, v, N, k = wl["o"], wl["v"], wl["ncd"], wl["roots"]
    inst = synth.make_instance(o, v, N, seed=wl["seed"], kappa=synth.kappa_for(v, N))
    e_ref, t1, t2, _, conv = ccsd.solve(inst.L, inst.eps, o)
    assert conv
    w_ref, _ = eom.dense_roots(eom.Hbar(integrals.Blocks(inst.L, o), inst.eps, t1, t2), k)
    return inst, k, e_ref, w_ref


@pytest.mark.parametrize("prec", ["fp64", "split-bf16", "split-fp16"])
def test_solve_against_oracle_o8v32(gpu_ctx, c1_oracle, prec):
    from paper_2506_06805_amd import fnscc
    inst, k, e_ref, w_ref = c1_oracle
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, inst.o, precision=prec)
    e, _, amps = fnscc.ccsd_solve(gpu_ctx, ints, precision=prec)
    w, _ = fnscc.ipeom_davidson(gpu_ctx, ints, amps, k)
    tol_w, tol_e = SOLVE_TOL[prec]
    assert np.abs(w - w_ref).max() < tol_w, (prec, np.abs(w - w_ref).max())
    assert abs(e - e_ref) < tol_e, (prec, abs(e - e_ref))
