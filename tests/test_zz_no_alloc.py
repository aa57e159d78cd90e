"""The allocation-free complex product (fc_zgemm_noalloc) against the allocating one (fc_zgemm).

Shapes with few output tiles and long K, so that the split-K partial sums live in the fixed
per-device workspace; two calls in a row, the second smaller, so that leftover contents of the
first cannot leak into the second.  With autotuning off both entry points pick the same tiles and
split, so the results agree bit for bit; both are also checked against a host FP64 product."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CASES = [  # M, N, K, opA, opB
    (200, 136, 24000, "N", "T"),
    (64, 40, 9000, "C", "N"),
]


def _operands(M, N, K, opA, opB, seed):
    rng = np.random.default_rng(seed)

    def cplx(*shape):
        return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)

    A = cplx(K, M) if opA in "TC" else cplx(M, K)
    B = cplx(N, K) if opB in "TC" else cplx(K, N)
    C0 = cplx(M, N)
    return A, B, C0


def _op(X, op):
    return {"N": X, "T": X.T, "C": X.conj().T, "R": X.conj()}[op]


@pytest.mark.parametrize("fp32", [False, True])
def test_noalloc_product_matches_allocating_product(gpu_ctx, fp32):
    import torch

    from paper_2506_06805_amd import fnscc
    alpha, beta = 0.75 - 0.5j, 0.25 + 1.0j
    for n, (M, N, K, opA, opB) in enumerate(CASES):
        A, B, C0 = _operands(M, N, K, opA, opB, seed=11 + n)
        dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        ref = fnscc.zgemm(gpu_ctx, opA, opB, dA, dB, alpha, beta, C=torch.from_numpy(C0).cuda(), fp32=fp32)
        out = fnscc.zgemm(gpu_ctx, opA, opB, dA, dB, alpha, beta, C=torch.from_numpy(C0).cuda(), fp32=fp32,
                          noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (M, N, K, fp32)
        host = alpha * (_op(A, opA) @ _op(B, opB)) + beta * C0
        scale = np.abs(A).max() * np.abs(B).max() * K
        err = np.abs(out.cpu().numpy() - host).max() / scale
        assert err < (4 * 2.0**-24 if fp32 else 1e-14), (M, N, K, fp32, err)


def test_noalloc_product_without_split(gpu_ctx):
    # a product that fills the chip with tiles takes no split and no workspace
    import torch

    from paper_2506_06805_amd import fnscc
    A, B, C0 = _operands(512, 384, 96, "N", "N", seed=5)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = fnscc.zgemm(gpu_ctx, "N", "N", dA, dB, 1.0, 0.0, C=torch.from_numpy(C0).cuda())
    out = fnscc.zgemm(gpu_ctx, "N", "N", dA, dB, 1.0, 0.0, C=torch.from_numpy(C0).cuda(), noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(out, ref)
