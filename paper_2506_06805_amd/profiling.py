"""Profiling helpers.

`python -m paper_2506_06805_amd.profiling copy --mib 1024` runs one device-to-device copy of a known
size, the reference dispatch used to scale the FETCH_SIZE / WRITE_SIZE hardware counters into HBM
bytes (a copy of S bytes must read S and write S bytes).

`python -m paper_2506_06805_amd.profiling gemm` times the library's complex GEMM on the shapes the
hot path uses, next to torch's complex128 matmul.
"""
from __future__ import annotations

import argparse
import json


def copy_probe(mib: int) -> None:
    import torch

    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n * 4}))


# (name, M, N, K, opA, opB): square, the ladder assembly at v=160 with 64 and 32 virtuals per block,
# the sigma ring product of a 6-vector block at o=24 v=200, and ladder contractions at o=24 and o=40
GEMM_SHAPES = [("square4096", 4096, 4096, 4096, "N", "N"), ("assembly_T64", 10240, 10240, 500, "N", "T"),
               ("assembly_T32", 5120, 5120, 500, "N", "T"), ("ring_sigma", 144, 4800, 4800, "N", "N"),
               ("contraction_o24", 12720, 276, 12720, "N", "T"), ("contraction_o40", 8000, 780, 20000, "N", "T")]


def gemm_probe(reps: int) -> None:
    """TFLOP/s of the library's complex GEMM (FP64 and FP32 arithmetic) on the listed shapes, next
    to torch's complex128 matmul on the same operands (a vendor-library reference point)."""
    import torch

    from . import fnscc

    ctx = fnscc.Context(0)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    for name, M, N, K, oa, ob in GEMM_SHAPES:
        A = torch.randn(M, K, dtype=torch.complex128, device="cuda")
        B = torch.randn(K, N, dtype=torch.complex128, device="cuda") if ob == "N" else \
            torch.randn(N, K, dtype=torch.complex128, device="cuda")
        C = torch.empty(M, N, dtype=torch.complex128, device="cuda")
        Bn = B if ob == "N" else B.t().contiguous()
        fl = 8.0 * M * N * K
        res = {"shape": name, "M": M, "N": N, "K": K}
        res["fp64_tflops"] = fl / timed(lambda: fnscc.zgemm(ctx, oa, ob, A, B, C=C)) / 1e9
        res["fp32_tflops"] = fl / timed(lambda: fnscc.zgemm(ctx, oa, ob, A, B, C=C, fp32=True)) / 1e9
        res["torch_complex128_tflops"] = fl / timed(lambda: torch.matmul(A, Bn, out=C)) / 1e9
        print(json.dumps({k: (round(x, 1) if isinstance(x, float) else x) for k, x in res.items()}), flush=True)
        del A, B, C, Bn


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    g = sub.add_parser("gemm")
    g.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    if args.cmd == "copy":
        copy_probe(args.mib)
    elif args.cmd == "gemm":
        gemm_probe(args.reps)


if __name__ == "__main__":
    main()
