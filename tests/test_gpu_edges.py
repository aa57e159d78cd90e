"""Edge cases of the C ABI on the GPU.

* empty sizes (no occupied spinors, no Cholesky vectors) and root counts outside [1, dim] are
  refused with FC_EARG;
* a sigma call on zero vectors does nothing;
* asking for every root (nroots = dim) returns the whole spectrum of the oracle's dense matrix;
* the degenerate instance without two-electron interaction (L = 0): E_corr = 0 and the IPs are
  the eigenvalues of the then diagonal IP-EOM-CCSD matrix, -eps_i (1h) and
  eps_a - eps_i - eps_j (2h1p), exactly;
* complex64 Cholesky vectors, from host or device memory, solve bit for bit like their exact
  complex128 widening.
"""
import numpy as np
import pytest

from paper_2506_06805_amd import synth
from oracle import ccsd, eom, integrals

pytestmark = pytest.mark.gpu


def test_empty_sizes_are_refused(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    inst = synth.make_instance(4, 10, 20, seed=1, kappa=0.3)
    for o, L in ((0, inst.L), (4, inst.L[:0])):
        with pytest.raises(fnscc.FcError) as e:
            fnscc.cd_integrals(gpu_ctx, inst.eps, L, o)
        assert e.value.code == fnscc.FC_EARG


def test_root_count_out_of_range_is_refused(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    o, v = 3, 4
    inst = synth.make_instance(o, v, 10, seed=2, kappa=0.3)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    _, _, amps = fnscc.ccsd_solve(gpu_ctx, ints)
    dim = o + o * (o - 1) // 2 * v
    for k in (0, dim + 1):
        with pytest.raises(fnscc.FcError) as e:
            fnscc.ipeom_davidson(gpu_ctx, ints, amps, k)
        assert e.value.code == fnscc.FC_EARG


def test_sigma_on_no_vectors_is_a_no_op(gpu_ctx):
    import torch
    from paper_2506_06805_amd import fnscc
    o, v = 3, 5
    inst = synth.make_instance(o, v, 12, seed=3, kappa=0.3)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    _, _, amps = fnscc.ccsd_solve(gpu_ctx, ints)
    dim = o + o * (o - 1) // 2 * v
    R = torch.zeros((0, dim), dtype=torch.complex128, device="cuda")
    S = fnscc.ipeom_sigma(gpu_ctx, ints, amps, R)
    assert S.shape == (0, dim)


def test_all_roots_equal_dense_spectrum(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    o, v, N = 2, 3, 8
    inst = synth.make_instance(o, v, N, seed=4, kappa=0.4)
    e_ref, t1, t2, _, conv = ccsd.solve(inst.L, inst.eps, o)
    assert conv
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, inst.L, o)
    e, _, amps = fnscc.ccsd_solve(gpu_ctx, ints)
    assert abs(e - e_ref) < 1e-8
    dim = o + o * (o - 1) // 2 * v
    w_ref, _ = eom.dense_roots(eom.Hbar(integrals.Blocks(inst.L, o), inst.eps, t1, t2), dim)
    w, _ = fnscc.ipeom_davidson(gpu_ctx, ints, amps, dim)
    assert np.abs(np.sort_complex(w) - np.sort_complex(w_ref)).max() < 1e-8


def test_no_two_electron_interaction(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    o, v, N = 4, 6, 10
    inst = synth.make_instance(o, v, N, seed=5, kappa=0.3)
    L = np.zeros_like(inst.L)
    ints = fnscc.cd_integrals(gpu_ctx, inst.eps, L, o)
    e, _, amps = fnscc.ccsd_solve(gpu_ctx, ints)
    assert abs(e) == 0.0
    eo, ev = inst.eps[:o], inst.eps[o:]
    levels = [-eo[i] for i in range(o)]
    levels += [ev[a] - eo[i] - eo[j] for i in range(o) for j in range(i + 1, o) for a in range(v)]
    k = 8
    w, _ = fnscc.ipeom_davidson(gpu_ctx, ints, amps, k)
    assert np.abs(w.imag).max() < 1e-12
    assert np.abs(w.real - np.sort(levels)[:k]).max() < 1e-10


def test_complex64_vectors_equal_their_complex128_upcast(gpu_ctx):
    # complex64 Cholesky vectors (host or device) are widened exactly when staged, so the solve
    # matches the one on the same values given as complex128, bit for bit
    import torch
    from paper_2506_06805_amd import fnscc
    o, v, N = 4, 14, 30
    inst = synth.make_instance(o, v, N, seed=6, kappa=synth.kappa_for(v, N))
    L64 = inst.L.astype(np.complex64)
    ref = fnscc.cd_integrals(gpu_ctx, inst.eps, L64.astype(np.complex128), o)
    e_ref, _, _ = fnscc.ccsd_solve(gpu_ctx, ref)
    for L in (L64, torch.from_numpy(L64).to("cuda")):
        ints = fnscc.cd_integrals(gpu_ctx, inst.eps, L, o)
        e, _, _ = fnscc.ccsd_solve(gpu_ctx, ints)
        assert e == e_ref
