"""The FP64 complex GEMM behind every contraction: all operand layouts, ragged tiles, split K."""
import itertools

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

OPS = "NTCR"


def _op(X, op):
    return {"N": X, "T": X.T, "C": X.conj().T, "R": X.conj()}[op]


def _rand(shape, rng):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


# shapes reach the default tile configurations: 64 x 64 with 8- and 16-element K slices, with and
# without split K, and 32 x 32 (tiny output, long K, many splits); 128 x 128 and 128 x 96 (FP32)
# in the tests below and in the solver tests
@pytest.mark.parametrize("M,N,K", [(70, 133, 37), (1, 300, 2000), (129, 65, 8), (256, 256, 513),
                                   (1100, 260, 200), (24, 20, 3000), (70, 90, 2100)])
def test_zgemm_layouts(gpu_ctx, M, N, K):
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(M + N + K)
    alpha, beta = 0.7 - 0.2j, -0.3 + 0.9j
    for opA, opB in itertools.product(OPS, OPS):
        A = _rand((K, M) if opA in "TC" else (M, K), rng)
        B = _rand((N, K) if opB in "TC" else (K, N), rng)
        C0 = _rand((M, N), rng)
        ref = alpha * (_op(A, opA) @ _op(B, opB)) + beta * C0
        C = torch.from_numpy(C0.copy()).cuda()
        fnscc.zgemm(gpu_ctx, opA, opB, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), alpha, beta, C)
        err = np.abs(C.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (opA, opB, err)


def test_zgemm_deterministic(gpu_ctx):
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(1)
    A = torch.from_numpy(_rand((3, 50000), rng)).cuda()
    B = torch.from_numpy(_rand((50000, 5), rng)).cuda()
    c1 = fnscc.zgemm(gpu_ctx, "N", "N", A, B).cpu().numpy()
    c2 = fnscc.zgemm(gpu_ctx, "N", "N", A, B).cpu().numpy()
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("M,N,K", [(70, 133, 37), (3, 200, 5000), (256, 256, 513), (1100, 260, 200),
                                   (24, 20, 3000)])
def test_zgemm_fp32_arithmetic(gpu_ctx, M, N, K):
    # FP32 products and sums on FP64 data: error of order 2^-24 sqrt(K) of sum |a||b|
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(K)
    for opA, opB in (("N", "N"), ("T", "C"), ("R", "T"), ("C", "N")):
        A = _rand((K, M) if opA in "TC" else (M, K), rng)
        B = _rand((N, K) if opB in "TC" else (K, N), rng)
        ref = _op(A, opA) @ _op(B, opB)
        scale = np.abs(_op(A, opA)) @ np.abs(_op(B, opB))
        C = fnscc.zgemm(gpu_ctx, opA, opB, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), fp32=True)
        err = (np.abs(C.cpu().numpy() - ref) / scale).max()
        assert err < 4 * 2.0 ** -24 * np.sqrt(K), (opA, opB, err)
        # and it is not FP64 arithmetic in disguise
        assert err > 2.0 ** -40


# the tiles staged by direct-to-LDS loads (configuration 8: 128 x 128, four real products per
# complex one; 9 and 10: 128 x 64, Gauss's three, K slices of 8 and 16) against the register-staged 128 x 128 tile
# (configuration 2) and numpy: every operand layout, ragged rows, columns and K
# (elements outside the product are fetched as zeros), split K (140 x 200, K = 3000), and a single
# K slice (K = 5: the FP32 128 x 128 tile's two-slice pipeline with nothing past its first slice)
@pytest.mark.parametrize("M,N,K", [(300, 257, 37), (129, 130, 9), (256, 384, 520), (140, 200, 3000), (130, 140, 5)])
def test_zgemm_direct_to_lds_tile(M, N, K):
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(7 * M + N + K)
    alpha, beta = 0.4 + 0.3j, 0.8 - 0.1j
    ctx = fnscc.Context(0)
    try:
        for opA, opB in itertools.product(OPS, OPS):
            A = _rand((K, M) if opA in "TC" else (M, K), rng)
            B = _rand((N, K) if opB in "TC" else (K, N), rng)
            C0 = _rand((M, N), rng)
            ref = alpha * (_op(A, opA) @ _op(B, opB)) + beta * C0
            out, raw, raw32 = {}, {}, {}
            dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
            for cfg in (2, 8, 9, 10):
                ctx.set_gemm_config(cfg)
                C = torch.from_numpy(C0.copy()).cuda()
                fnscc.zgemm(ctx, opA, opB, dA, dB, alpha, beta, C)
                out[cfg] = C.cpu().numpy()
                raw[cfg] = fnscc.zgemm(ctx, opA, opB, dA, dB).cpu().numpy()
                raw32[cfg] = fnscc.zgemm(ctx, opA, opB, dA, dB, fp32=True).cpu().numpy()
            # FP32 arithmetic: every tile rounds the operands to FP32 the same way and sums the
            # same three products in the same order (same split-K counts at these shapes)
            for cfg in (8, 9, 10):
                assert np.array_equal(raw32[cfg], raw32[2]), (cfg, opA, opB, np.abs(raw32[cfg] - raw32[2]).max())
            for cfg in (8, 9, 10):
                err = np.abs(out[cfg] - ref).max() / np.abs(ref).max()
                assert err < 1e-13, (cfg, opA, opB, err)
            # configuration 8 sums the same products in the same order as the register-staged tile
            # (the alpha/beta epilogue may fuse its multiply-adds differently in the two kernels)
            assert np.array_equal(raw[8], raw[2]), (opA, opB, np.abs(raw[8] - raw[2]).max())
            # configurations 9 and 10 (Gauss's three real products, K slices of 8 and 16): error
            # bounded like the four-product form's up to a small factor,
            # |error| <~ K eps (|ar| + |ai|)(|br| + |bi|)
            scale = (np.abs(_op(A, opA).real) + np.abs(_op(A, opA).imag)) @ \
                    (np.abs(_op(B, opB).real) + np.abs(_op(B, opB).imag))
            for cfg in (9, 10):
                e3 = (np.abs(raw[cfg] - _op(A, opA) @ _op(B, opB)) / scale).max()
                assert e3 < 4 * K * 2.0 ** -53, (cfg, opA, opB, e3)
    finally:
        ctx.close()


def test_gemm_config_override_is_validated(gpu_ctx):
    from paper_2506_06805_amd import fnscc
    n = fnscc.Context.gemm_num_configs()
    assert n >= 9
    with pytest.raises(RuntimeError):
        gpu_ctx.set_gemm_config(n)
    with pytest.raises(RuntimeError):
        gpu_ctx.set_gemm_config(-2)
    gpu_ctx.set_gemm_config(-1)


@pytest.mark.parametrize("prec,unit", [("split-bf16", 2.0 ** -16), ("split-fp16", 2.0 ** -22)])
def test_zgemm_split_precisions(gpu_ctx, prec, unit):
    # hi/lo split products: error within a few units of the split's precision of sum |a||b|
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(11)
    M, N, K = 150, 140, 300
    for opA, opB in (("N", "T"), ("R", "C"), ("N", "C")):
        A, B = _rand((M, K), rng), _rand((N, K), rng)
        ref = _op(A, opA) @ _op(B, opB)
        scale = np.abs(A) @ np.abs(B).T
        C = fnscc.zgemm(gpu_ctx, opA, opB, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), precision=prec)
        err = (np.abs(C.cpu().numpy() - ref) / scale).max()
        assert err < 8 * unit, (opA, opB, err)
    # A stored K x M ('T'): not contraction-contiguous, refused by the library
    with pytest.raises(fnscc.FcError) as e:
        fnscc.zgemm(gpu_ctx, "T", "T", torch.from_numpy(A.T.copy()).cuda(), torch.from_numpy(B).cuda(), precision=prec)
    assert e.value.code == fnscc.FC_EUNSUPPORTED


def test_fp16_split_scales_each_k_batch(gpu_ctx):
    # Columns k < 256 carry O(1) entries on the first half of the rows, columns k >= 256 entries of
    # 2^-30 on the second half (Cholesky vectors decay over their index).  With one scale per
    # operand the small entries would fall into FP16's subnormal range (2^-30 x 2^13 = 2^-17) and keep
    # a few bits; with one power-of-two scale per 128 columns they keep the split's full precision.
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(12)
    M, N, K, h = 96, 80, 512, 256
    A, B = np.zeros((M, K), complex), np.zeros((N, K), complex)
    A[:M // 2, :h], B[:N // 2, :h] = _rand((M // 2, h), rng), _rand((N // 2, h), rng)
    A[M // 2:, h:], B[N // 2:, h:] = _rand((M - M // 2, K - h), rng) * 2.0 ** -30, _rand((N - N // 2, K - h), rng) * 2.0 ** -30
    ref = A @ B.T
    scale = np.abs(A) @ np.abs(B).T
    C = fnscc.zgemm(gpu_ctx, "N", "T", torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                    precision="split-fp16").cpu().numpy()
    for rows, cols in ((slice(0, M // 2), slice(0, N // 2)), (slice(M // 2, M), slice(N // 2, N))):
        err = (np.abs(C[rows, cols] - ref[rows, cols]) / scale[rows, cols]).max()
        assert err < 8 * 2.0 ** -22, err
    # the blocks that share no nonzero column are exactly zero
    assert not C[:M // 2, N // 2:].any() and not C[M // 2:, :N // 2].any()


@pytest.mark.parametrize("M,N,K", [(96, 100, 20), (300, 257, 37), (129, 130, 64), (256, 384, 96), (140, 200, 3000),
                                   (260, 270, 520)])
def test_split_direct_to_lds_tile(M, N, K):
    # the split product staged straight into LDS (three A buffers, two B buffers; K slices 1, 2, 3
    # and many, ragged tiles, split-K on the long contraction) against the register-staged tile: the
    # same MFMAs per accumulator in the same order, so the same bits; FP16 with its per-K-batch
    # scales crossing batch boundaries
    import torch
    from paper_2506_06805_amd import fnscc
    rng = np.random.default_rng(M + N + K)
    A, B = _rand((M, K), rng), _rand((N, K), rng)
    dA, dB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    ref = A @ B.T
    scale = np.abs(A) @ np.abs(B).T
    ctx = fnscc.Context(0)
    try:
        assert fnscc.Context.split_num_configs() == 3
        for prec, unit in (("split-bf16", 2.0 ** -16), ("split-fp16", 2.0 ** -22)):
            out = {}
            for cfg in (0, 2):
                ctx.set_split_config(cfg)
                out[cfg] = fnscc.zgemm(ctx, "N", "T", dA, dB, precision=prec).cpu().numpy()
            assert np.array_equal(out[0], out[2]), prec
            assert (np.abs(out[2] - ref) / scale).max() < 8 * unit, prec
        ctx.set_split_config(-1)
        with pytest.raises(fnscc.FcError):
            ctx.set_split_config(3)
    finally:
        ctx.close()
