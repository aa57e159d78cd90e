"""GEMM autotuning and the chunked ladder paths: results must not depend on tile choices or on how
the (a,b) pairs are chunked."""
import os

import numpy as np
import pytest

from oracle import ccsd, integrals
from paper_2506_06805_amd import synth

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def _tau(o, v, seed):
    rng = np.random.default_rng(seed)
    t = (rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v))) * 0.05
    t = t - t.transpose(1, 0, 2, 3)
    return t - t.transpose(0, 1, 3, 2)


def _ladder_ref(inst, tau):
    o, v = inst.o, inst.v
    V = slice(o, o + v)
    return 0.5 * np.einsum("ijef,abef->ijab", tau, integrals.antisym(inst.L, V, V, V, V), optimize=True)


@pytest.mark.parametrize("o,v,N", [(3, 65, 20), (4, 129, 16)])
@pytest.mark.parametrize("budget_gb", ["8", "0.0004"])
def test_ladder_chunking(gpu_ctx, o, v, N, budget_gb, monkeypatch):
    from paper_2506_06805_amd import fnscc
    monkeypatch.setenv("FNSCC_LADDER_BUDGET_GB", budget_gb)
    inst = synth.make_instance(o, v, N, seed=5 + v, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    tau = _tau(o, v, 1)
    ref = _ladder_ref(inst, tau)
    for prec, tol in (("fp64", 1e-11), ("split-bf16", 2e-4), ("split-fp16", 2e-6)):
        R = fnscc.ladder(gpu_ctx, ints, _dev(tau), precision=prec).cpu().numpy()
        assert np.abs(R - ref).max() / np.abs(ref).max() < tol, prec


def test_split_ladder_on_the_96_wide_contraction_tile(gpu_ctx):
    # o = 24 gives 276 occupied pairs, a width that the 128 x 96 split tile pads much less than the
    # 128 x 128 one, so the contraction runs on it (its staging covers 128 rows per pass and must not
    # store the 32 past the tile); the lo planes' contribution must survive at the FP16 bound
    from paper_2506_06805_amd import fnscc
    o, v, N = 24, 12, 20
    inst = synth.make_instance(o, v, N, seed=41, kappa=0.6)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    tau = _tau(o, v, 4)
    ref = _ladder_ref(inst, tau)
    for prec, tol in (("split-bf16", 2e-4), ("split-fp16", 2e-6)):
        for _ in range(3):
            R = fnscc.ladder(gpu_ctx, ints, _dev(tau), precision=prec).cpu().numpy()
            assert np.abs(R - ref).max() / np.abs(ref).max() < tol, prec


@pytest.mark.parametrize("cfg", [2, 8, 9, 10])
def test_ladder_with_forced_tiles(cfg):
    # the FP64 ladder's assembly and contraction products, ladder-layout epilogue included, on the
    # register-staged 128 x 128 tile (2), the direct-to-LDS 128 x 128 tile (8) and the
    # direct-to-LDS 128 x 64 tiles with Gauss's three products (9, 10)
    from paper_2506_06805_amd import fnscc
    o, v, N = 4, 129, 16
    inst = synth.make_instance(o, v, N, seed=5 + v, kappa=0.6)
    tau = _tau(o, v, 1)
    ref = _ladder_ref(inst, tau)
    ctx = fnscc.Context(0)
    try:
        ctx.set_gemm_config(cfg)
        ints = fnscc.cd_integrals(ctx, inst.eps, inst.L, o)
        R = fnscc.ladder(ctx, ints, _dev(tau), precision="fp64").cpu().numpy()
        assert np.abs(R - ref).max() / np.abs(ref).max() < 1e-11
    finally:
        ctx.close()


def test_autotune_keeps_results_and_roundtrips(gpu_ctx, tmp_path):
    from paper_2506_06805_amd import fnscc
    o, v, N = 7, 90, 60
    inst = synth.make_instance(o, v, N, seed=17, kappa=0.5)
    rng = np.random.default_rng(3)
    t1 = (rng.standard_normal((o, v)) + 1j * rng.standard_normal((o, v))) * 0.02
    t2 = _tau(o, v, 2) * 0.3
    ref1, ref2 = ccsd.residuals(integrals.Blocks(inst.L, o), inst.eps, t1, t2)
    ctx = fnscc.Context(0)
    try:
        ctx.set_autotune(True)
        ints = fnscc.cd_integrals(ctx, inst.eps, inst.L, o)
        r1, r2 = fnscc.ccsd_residual(ctx, ints, _dev(t1), _dev(t2))
        assert ctx.autotune_size() > 5
        for a, b in ((r1, ref1), (r2, ref2)):
            a = a.cpu().numpy()
            assert np.abs(a - b).max() / np.abs(b).max() < 1e-11
        path = tmp_path / "tune.txt"
        ctx.autotune_save(path)
        ctx2 = fnscc.Context(0)
        ctx2.autotune_load(path)
        assert ctx2.autotune_size() == ctx.autotune_size()
        ctx2.close()
    finally:
        ctx.close()


@pytest.mark.parametrize("cfg", [0, 2])
def test_split_ladder_staging(cfg):
    # the split ladder's assembly (ladder-layout epilogue, triangular launches) and contraction with
    # the 128-wide tiles staged through registers (0) or straight into LDS (2): the same bits, and
    # within the split's bound of the oracle ladder
    from paper_2506_06805_amd import fnscc
    o, v, N = 6, 70, 200
    inst = synth.make_instance(o, v, N, seed=77, kappa=0.6)
    tau = _tau(o, v, 6)
    ref = _ladder_ref(inst, tau)
    ctxs = [fnscc.Context(0), fnscc.Context(0)]
    try:
        ctxs[1].set_split_config(cfg)
        for prec, tol in (("split-bf16", 2e-4), ("split-fp16", 2e-6)):
            R = []
            for ctx in ctxs:
                ints = fnscc.cd_integrals(ctx, inst.eps, inst.L, o)
                R.append(fnscc.ladder(ctx, ints, _dev(tau), precision=prec).cpu().numpy())
            assert np.abs(R[1] - ref).max() / np.abs(ref).max() < tol, prec
            assert np.array_equal(R[0], R[1]), prec
    finally:
        for ctx in ctxs:
            ctx.close()
