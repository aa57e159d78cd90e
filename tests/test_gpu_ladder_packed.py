"""The ladder on packed amplitudes (fc_ladder_packed) and complex64 Cholesky vectors.

* The packed entry point computes exactly what the full one does: R[i<j][a<b] equals the unique
  entries of the full-layout ladder bit for bit, in every precision, with and without T1
  dressing, at shapes whose virtual count is not a multiple of the 32-wide (e, f) blocks.
* complex64 vectors are kept in complex64 on the device (the split precisions read them directly);
  the result equals that of the same vectors widened to complex128 on the host.
* the packed ladder against the oracle's ladder rows (Eq. 21, 23) at 1e-11 in FP64.
"""
import numpy as np
import pytest

from paper_2506_06805_amd import synth

pytestmark = pytest.mark.gpu

SHAPES = [(4, 37, 30), (6, 70, 45)]


def _tau(o, v, seed):
    rng = np.random.default_rng(seed)
    t = 1e-2 * (rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v)))
    t = t - t.transpose(1, 0, 2, 3)
    return t - t.transpose(0, 1, 3, 2)


def _pack(x):
    o, v = x.shape[0], x.shape[2]
    iu, ju = np.triu_indices(o, 1)
    au, bu = np.triu_indices(v, 1)
    return np.ascontiguousarray(x[iu, ju][:, au, bu])


@pytest.mark.parametrize("o,v,N", SHAPES)
@pytest.mark.parametrize("prec", ["fp64", "split-bf16", "split-fp16"])
@pytest.mark.parametrize("dressed", [False, True])
def test_packed_ladder_equals_full(gpu_ctx, o, v, N, prec, dressed):
    import torch

    from paper_2506_06805_amd import fnscc
    inst = synth.make_instance(o, v, N, seed=o + v, kappa=0.5)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o, precision=prec)
    tau = _tau(o, v, 3)
    rng = np.random.default_rng(4)
    t1 = 1e-2 * (rng.standard_normal((o, v)) + 1j * rng.standard_normal((o, v))) if dressed else None
    dt1 = torch.from_numpy(t1).cuda() if dressed else None
    full = fnscc.ladder(gpu_ctx, ints, torch.from_numpy(tau).cuda(), dt1, precision=prec).cpu().numpy()
    packed = fnscc.ladder_packed(gpu_ctx, ints, torch.from_numpy(_pack(tau)).cuda(), dt1, precision=prec).cpu().numpy()
    assert np.array_equal(packed, _pack(full))


@pytest.mark.parametrize("prec", ["fp64", "split-bf16", "split-fp16"])
def test_complex64_vectors_match_their_widening(gpu_ctx, prec):
    import torch

    from paper_2506_06805_amd import fnscc
    o, v, N = 5, 45, 40
    inst = synth.make_instance(o, v, N, seed=9, kappa=0.5, dtype=np.complex64)
    tau = _pack(_tau(o, v, 5))
    rng = np.random.default_rng(6)
    t1 = torch.from_numpy(1e-2 * (rng.standard_normal((o, v)) + 1j * rng.standard_normal((o, v)))).cuda()
    out = []
    for L in (torch.from_numpy(inst.L).cuda(), inst.L.astype(np.complex128)):
        ints = fnscc.cd_integrals(gpu_ctx, inst.eps, L, o, precision=prec)
        out.append(fnscc.ladder_packed(gpu_ctx, ints, torch.from_numpy(tau).cuda(), t1, precision=prec).cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_packed_ladder_against_oracle_rows(gpu_ctx):
    import torch

    from oracle import integrals
    from paper_2506_06805_amd import fnscc
    o, v, N = 4, 37, 30
    inst = synth.make_instance(o, v, N, seed=12, kappa=0.5)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    tau = _tau(o, v, 7)
    R = fnscc.ladder_packed(gpu_ctx, ints, torch.from_numpy(_pack(tau)).cuda()).cpu().numpy()
    g = integrals.Blocks(inst.L, o)
    Lv = g.L[:, o:, o:]
    iu, ju = np.triu_indices(o, 1)
    for a in (0, 18, 35):
        x = np.einsum("Pe,Pbf->bef", Lv[:, a, :], Lv, optimize=True)
        ref = 0.5 * np.einsum("ijef,bef->ijb", tau, x - x.transpose(0, 2, 1), optimize=True)[iu, ju]
        for b in range(a + 1, v):
            col = a * (2 * v - a - 1) // 2 + (b - a - 1)
            err = np.abs(R[:, col] - ref[:, b]).max() / np.abs(ref).max()
            assert err < 1e-11, (a, b, err)


def test_device_generator_recipe(gpu_ctx):
    # the device-drawn vectors follow the recipe: Hermitian per P, complex64, decaying scale
    import torch
    o, v, N = 3, 29, 200
    eps, L = synth.make_instance_device(o, v, N, seed=4, kappa=0.7)
    assert L.dtype == torch.complex64 and tuple(L.shape) == (N, o + v, o + v)
    assert torch.equal(L, L.transpose(1, 2).conj())
    host = synth.make_instance(o, v, N, seed=4, kappa=0.7)
    assert np.array_equal(eps, host.eps)
    # off-diagonal entries: variance (kappa 0.3 exp(-4P/N))^2 / 2 per complex entry
    rms = torch.sqrt(torch.mean(torch.abs(L[:, 0, 1:]).double() ** 2, dim=1)).cpu().numpy()
    want = 0.7 * 0.3 * np.exp(-4.0 * np.arange(N) / N) / np.sqrt(2.0)
    assert np.abs(np.log(rms[:50].mean() / want[:50].mean())) < 0.1
    assert np.abs(np.log(rms[-50:].mean() / want[-50:].mean())) < 0.1
