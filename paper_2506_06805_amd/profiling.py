"""Profiling helpers.

`python -m paper_2506_06805_amd.profiling copy --mib 1024` runs one device-to-device copy of a known
size, the reference dispatch used to scale the FETCH_SIZE / WRITE_SIZE hardware counters into HBM
bytes (a copy of S bytes must read S and write S bytes).

`python -m paper_2506_06805_amd.profiling gemm` times the library's complex GEMM on the shapes the
hot path uses, next to torch's complex128 matmul.

`python -m paper_2506_06805_amd.profiling split-gemm` times the hi/lo split products (BF16 and FP16)
with the 128-wide tiles staged through registers and straight into LDS.

`python -m paper_2506_06805_amd.profiling fns-presets` runs the paper's frozen-natural-spinor presets
against the untruncated solve on the FNS-structured generator.

`python -m paper_2506_06805_amd.profiling ao-cd` times the pivoted Cholesky of a synthetic AO
supermatrix and the two-component transform of its vectors on the device.

`python -m paper_2506_06805_amd.profiling sigma` times the right and left IP-EOM sigma products for
blocks of k trial vectors against the FP64 matrix-core peak.

`python -m paper_2506_06805_amd.profiling learned-curve` trains the learned T2 update on growing
sets of generated instances and reports what it gains over plain Jacobi + DIIS on the benchmark
workloads.
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
               ("contraction_o24", 12720, 276, 12720, "N", "T"), ("contraction_o40", 8000, 780, 20000, "N", "T"),
               ("ring_o24v160", 3840, 3840, 3840, "N", "N"), ("fmi_o24v160", 24, 24, 614400, "N", "T"),
               ("fae_o24v160", 160, 160, 92160, "N", "N")]


def gemm_probe(reps: int, tune: bool = False, save: str = "", cfg: int = -1, shapes: str = "",
               fp64_only: bool = False, fp32_only: bool = False) -> None:
    """TFLOP/s of the library's complex GEMM (FP64 and FP32 arithmetic) on the listed shapes, next
    to torch's complex128 matmul on the same operands (a vendor-library reference point).  With
    `tune` the library's autotuner times every tile configuration first and keeps the fastest.
    `shapes` (comma-separated names) restricts the shapes; `fp64_only` / `fp32_only` time the FP64
    or the FP32-arithmetic products alone (clean programs for counter runs)."""
    import torch

    from . import fnscc

    ctx = fnscc.Context(0)
    if tune:
        ctx.set_autotune(True)
    if cfg >= 0:
        ctx.set_gemm_config(cfg)

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

    keep = set(shapes.split(",")) if shapes else None
    for name, M, N, K, oa, ob in GEMM_SHAPES:
        if keep is not None and name not in keep:
            continue
        A = torch.randn(M, K, dtype=torch.complex128, device="cuda")
        B = torch.randn(K, N, dtype=torch.complex128, device="cuda") if ob == "N" else \
            torch.randn(N, K, dtype=torch.complex128, device="cuda")
        C = torch.empty(M, N, dtype=torch.complex128, device="cuda")
        Bn = B if ob == "N" else B.t().contiguous()
        fl = 8.0 * M * N * K
        res = {"shape": name, "M": M, "N": N, "K": K}
        if not fp32_only:
            res["fp64_tflops"] = fl / timed(lambda: fnscc.zgemm(ctx, oa, ob, A, B, C=C)) / 1e9
        if not fp64_only:
            res["fp32_tflops"] = fl / timed(lambda: fnscc.zgemm(ctx, oa, ob, A, B, C=C, fp32=True)) / 1e9
        if not (fp64_only or fp32_only):
            res["torch_complex128_tflops"] = fl / timed(lambda: torch.matmul(A, Bn, out=C)) / 1e9
        print(json.dumps({k: (round(x, 1) if isinstance(x, float) else x) for k, x in res.items()}), flush=True)
        del A, B, C, Bn
    if tune and save:
        ctx.autotune_save(save)


# The paper's thresholds (Sec. 4.1): natural-spinor occupation and Cholesky threshold per preset.
FNS_PRESETS = [("LOOSE", 1e-4, 1e-3), ("NORMAL", 10 ** -4.5, 1e-4), ("TIGHT", 1e-5, 1e-5)]


def split_gemm_probe(reps: int) -> None:
    """C = A B^T on complex128 operands through the split precisions: the whole call (splitting
    both operands into hi/lo planes, the product, the FP64 output), timed with hipEvents on the
    current stream, for each staging of the 128-wide tiles (0 registers, 2 direct-to-LDS)."""
    import torch

    from . import fnscc
    ctx = fnscc.Context(0)
    shapes = [("assembly_T64", 10240, 10240, 512), ("square4096", 4096, 4096, 4096),
              ("contraction_o40", 8000, 780, 20000), ("contraction_o24", 12720, 276, 12720)]
    for name, m, n, k in shapes:
        A = torch.randn(m, k, dtype=torch.complex128, device="cuda")
        B = torch.randn(n, k, dtype=torch.complex128, device="cuda")
        C = torch.empty(m, n, dtype=torch.complex128, device="cuda")
        row = {"shape": name, "M": m, "N": n, "K": k}
        for prec in ("split-bf16", "split-fp16"):
            for cfg in (0, 2):
                ctx.set_split_config(cfg)
                fnscc.zgemm(ctx, "N", "T", A, B, C=C, precision=prec)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    fnscc.zgemm(ctx, "N", "T", A, B, C=C, precision=prec)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                row[f"{prec}_cfg{cfg}_ms"] = round(ms, 3)
                row[f"{prec}_cfg{cfg}_tflops"] = round(8.0 * m * n * k / (ms * 1e-3) / 1e12, 1)
        print(json.dumps(row), flush=True)
        del A, B, C
    ctx.set_split_config(-1)
    ctx.close()


def fns_presets(o: int, v: int, ncd: int, gamma: float, roots: int, seed: int) -> None:
    """Time-to-IPs and IP error of the frozen-natural-spinor presets against the untruncated solve
    on the FNS-structured generator.  The Cholesky threshold of each preset has no counterpart here:
    the vectors arrive in the spinor basis, so every preset uses all ncd of them."""
    import time

    import numpy as np
    import torch

    from . import fnscc, synth

    ctx = fnscc.Context(0)
    inst = synth.make_instance(o, v, ncd, seed=seed, kappa=synth.kappa_for(v, ncd), fns_gamma=gamma)
    L = torch.from_numpy(inst.L).cuda()

    def solve(thresh):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ints = fnscc.cd_integrals(ctx, inst.eps, L, o)
        vk, occ = v, None
        if thresh is not None:
            ints, occ = fnscc.fns_truncate(ctx, ints, thresh)
            vk = ints.v
        e, it, amps = fnscc.ccsd_solve(ctx, ints)
        w, _ = fnscc.ipeom_davidson(ctx, ints, amps, roots)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, vk, e, np.sort_complex(np.asarray(w)), it

    solve(None)                      # warm-up
    t_ref, _, e_ref, w_ref, it_ref = solve(None)
    print(json.dumps({"preset": "none", "v_kept": v, "time_to_ips_s": round(t_ref, 3), "ccsd_iters": it_ref,
                      "e_corr": [e_ref.real, e_ref.imag], "ips": [round(float(x.real), 8) for x in w_ref]}),
          flush=True)
    for name, fns_thr, cd_thr in FNS_PRESETS:
        t, vk, e, w, it = solve(fns_thr)
        print(json.dumps({"preset": name, "fns_threshold": fns_thr, "cd_threshold": cd_thr, "v_kept": vk,
                          "time_to_ips_s": round(t, 3), "speedup": round(t_ref / t, 2), "ccsd_iters": it,
                          "abs_dE": abs(e - e_ref), "max_abs_dIP": float(np.abs(w - w_ref).max()),
                          "max_abs_dIP_eV": float(np.abs(w - w_ref).max() * 27.211386)}), flush=True)


def ao_cd(nao: int, rank: int, n: int, tau: float, reps: int, seed: int) -> None:
    """Pivoted Cholesky (Eq. 21) of an nao^2 x nao^2 synthetic supermatrix and the transform
    (Eq. 22) of its vectors to n spinors.  Algorithmic bytes of the Cholesky: step j reads the j
    earlier vectors and the pivot row of M, reads and writes the diagonal and writes the new
    vector, (j + 4) m doubles.  Algorithmic flops of the transform: 2 nvec nao^2 (2n) real
    multiply-adds of the real AO vectors with the complex coefficients (4 flop each as complex
    products with one real factor) and 8 nvec n^2 (2 nao) for the complex products."""
    import time

    import numpy as np
    import torch

    from . import fnscc, synth

    ctx = fnscc.Context(0)
    m = nao * nao
    w, X = synth.make_ao_eri_factors(nao, rank, seed)
    Xd = torch.from_numpy(X).cuda()
    M = synth.symmetrize_eri((Xd.T * torch.from_numpy(w).cuda()) @ Xd, nao)
    del Xd
    Cs = torch.from_numpy(synth.make_spinor_coefficients(nao, n, seed + 1)).cuda()

    def timed(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, out

    fnscc.cd_ao_pivoted(ctx, M, tau, 4 * rank)       # warm-up
    tcd = []
    for _ in range(reps):
        t, (L, piv) = timed(lambda: fnscc.cd_ao_pivoted(ctx, M, tau, 4 * rank))
        tcd.append(t)
    nvec = L.shape[0]
    cd_bytes = 8.0 * m * sum(j + 4 for j in range(nvec))
    fnscc.ao_to_spinor(ctx, L, Cs, nao)              # warm-up
    ttr = []
    for _ in range(reps):
        t, Lmo = timed(lambda: fnscc.ao_to_spinor(ctx, L, Cs, nao))
        ttr.append(t)
    tr_flop = 4.0 * nvec * nao * nao * 2 * n + 8.0 * nvec * n * n * 2 * nao
    t_cd, t_tr = min(tcd), min(ttr)
    print(json.dumps({"nao": nao, "m": m, "rank": rank, "tau": tau, "nvec": nvec, "n_spinors": n,
                      "cd_s": round(t_cd, 5), "cd_algorithmic_bytes": cd_bytes,
                      "cd_GBps": round(cd_bytes / t_cd / 1e9, 1), "cd_frac_of_hbm": round(cd_bytes / t_cd / 8e12, 3),
                      "transform_s": round(t_tr, 5), "transform_flop": tr_flop,
                      "transform_TFLOPs": round(tr_flop / t_tr / 1e12, 2),
                      "transform_frac_of_fp64_peak": round(tr_flop / t_tr / 78.6e12, 3),
                      "max_abs_imag_diag": float(torch.diagonal(Lmo, dim1=1, dim2=2).imag.abs().max())}),
          flush=True)


def sigma_flops(o: int, v: int, k: int) -> float:
    """Algorithmic flops of one sigma product for k vectors (8 per complex multiply-add): the 1h
    block R B1, the ring product over the unpacked r_im^e, X_e, F_ae, the pair mixing and
    [r_m | X_e] B2 (the left product has the same shapes transposed)."""
    no = o * (o - 1) // 2
    dim = o + no * v
    return 8.0 * k * (dim * o + o ** 3 * v ** 2 + 2 * no * v * v + no * no * v + (o + v) * no * v)


def sigma_probe(o: int, v: int, ncd: int, ks, reps: int, seed: int) -> None:
    import time

    import numpy as np
    import torch

    from . import fnscc, synth

    ctx = fnscc.Context(0)
    inst = synth.make_instance(o, v, ncd, seed=seed, kappa=synth.kappa_for(v, ncd))
    ints = fnscc.cd_integrals(ctx, inst.eps, torch.from_numpy(inst.L).cuda(), o)
    _, _, amps = fnscc.ccsd_solve(ctx, ints)
    dim = o + o * (o - 1) // 2 * v
    rng = np.random.default_rng(seed)
    for k in ks:
        R = torch.from_numpy(rng.standard_normal((k, dim)) + 1j * rng.standard_normal((k, dim))).cuda()
        for name, fn in (("right", fnscc.ipeom_sigma), ("left", fnscc.ipeom_sigma_left)):
            fn(ctx, ints, amps, R)                     # operators built, warm-up
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                fn(ctx, ints, amps, R)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            t = min(ts)
            f = sigma_flops(o, v, k)
            print(json.dumps({"sigma": name, "o": o, "v": v, "k": k, "ms": round(t * 1e3, 3), "flop": f,
                              "TFLOPs": round(f / t / 1e12, 2), "frac_of_fp64_peak": round(f / t / 78.6e12, 3)}),
                  flush=True)


def learned_curve(sizes, seed: int, per_iter_max: int, epochs: int, diis: int) -> None:
    """Iterations and time-to-IPs with the learned update against plain Jacobi + DIIS(diis), for
    networks trained on `sizes` generated instances (learn.training_instances: o 6-16, v 30-80,
    N = 4 v, seeds 100 seed + k), on o=24 v=160 N=500 and on the FNS-structured o=40 v=600 N=1800
    workload at the threshold 1e-5, in FP64 and split-BF16."""
    import sys
    import time

    import numpy as np
    import torch

    from . import fnscc, learn, synth

    ctx = fnscc.Context(0)

    def log(msg):
        print(f"[learned-curve] {msg}", file=sys.stderr, flush=True)

    evals = []
    for name, wl, gamma, thr in (("o24v160n500", synth.WORKLOADS["o24v160n500"], None, None),
                                 ("o40v600n1800 FNS 1e-5 structured", synth.WORKLOADS["o40v600n1800"], 6.0, 1e-5)):
        o, v, N = wl["o"], wl["v"], wl["ncd"]
        inst = synth.make_instance(o, v, N, seed=wl["seed"], kappa=synth.kappa_for(v, N), fns_gamma=gamma,
                                   dtype=np.complex64 if gamma else np.complex128)
        evals.append((name, inst, torch.from_numpy(inst.L).cuda(), thr, wl["roots"]))

    def solve(ev, prec, mlp):
        name, inst, L, thr, roots = ev
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ints = fnscc.cd_integrals(ctx, inst.eps, L, inst.o, precision=prec)
        if thr is not None:
            ints, _ = fnscc.fns_truncate(ctx, ints, thr)
        kw = {"mlp": mlp} if mlp is not None else {}
        e, it, amps = fnscc.ccsd_solve(ctx, ints, precision=prec, diis_dim=diis, **kw)
        w, _ = fnscc.ipeom_davidson(ctx, ints, amps, roots)
        torch.cuda.synchronize()
        return it, time.perf_counter() - t0, e, np.sort_complex(np.asarray(w))

    base = {}
    for ev in evals:
        for prec in ("fp64", "split-bf16"):
            solve(ev, prec, None)   # warm-up
            base[(ev[0], prec)] = solve(ev, prec, None)
            it, t, e, _ = base[(ev[0], prec)]
            print(json.dumps({"train_instances": 0, "workload": ev[0], "precision": prec, "diis": diis,
                              "ccsd_iters": it, "time_to_ips_s": round(t, 4)}), flush=True)
    for n in sizes:
        per_iter = max(32, min(per_iter_max, per_iter_max * 64 // max(n, 1)))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        data = learn.collect(ctx, learn.training_instances(n, seed), per_iter=per_iter, seed=seed, log=log)
        t_col = time.perf_counter() - t0
        net, hist = learn.train(ctx, data, epochs=epochs, batch=2048, lr=2e-3, seed=1)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0 - t_col
        log(f"{n} instances: {int(data[0].shape[0])} samples, collected in {t_col:.1f} s, trained in {t_train:.1f} s")
        for ev in evals:
            for prec in ("fp64", "split-bf16"):
                it, t, e, w = solve(ev, prec, net)
                it0, t0_, e0, w0 = base[(ev[0], prec)]
                print(json.dumps({"train_instances": n, "samples": int(data[0].shape[0]), "per_iter": per_iter,
                                  "collect_s": round(t_col, 1), "train_s": round(t_train, 1),
                                  "loss_first": hist[0], "loss_last": hist[-1], "workload": ev[0],
                                  "precision": prec, "diis": diis, "ccsd_iters": it, "plain_iters": it0,
                                  "time_to_ips_s": round(t, 4), "speedup_vs_plain": round(t0_ / t, 3),
                                  "max_abs_dIP_vs_plain": float(np.abs(w - w0).max()),
                                  "abs_dE_vs_plain": abs(e - e0)}), flush=True)
        del data, net


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    g = sub.add_parser("gemm")
    g.add_argument("--reps", type=int, default=5)
    g.add_argument("--tune", action="store_true")
    g.add_argument("--save", type=str, default="", help="with --tune: write the tuned table to this file")
    g.add_argument("--cfg", type=int, default=-1, help="force this tile configuration where it fits")
    g.add_argument("--shapes", type=str, default="", help="comma-separated shape names (default: all)")
    g.add_argument("--fp64-only", action="store_true", help="time the FP64 products alone")
    g.add_argument("--fp32-only", action="store_true", help="time the FP32-arithmetic products alone")
    sg = sub.add_parser("split-gemm")
    sg.add_argument("--reps", type=int, default=5)
    f = sub.add_parser("fns-presets")
    f.add_argument("--o", type=int, default=24)
    f.add_argument("--v", type=int, default=300)
    f.add_argument("--ncd", type=int, default=900)
    f.add_argument("--gamma", type=float, default=6.0)
    f.add_argument("--roots", type=int, default=8)
    f.add_argument("--seed", type=int, default=5000)
    a = sub.add_parser("ao-cd")
    a.add_argument("--nao", type=int, default=200)
    a.add_argument("--rank", type=int, default=1000)
    a.add_argument("--n", type=int, default=300)
    a.add_argument("--tau", type=float, default=1e-6)
    a.add_argument("--reps", type=int, default=3)
    a.add_argument("--seed", type=int, default=6000)
    q = sub.add_parser("sigma")
    q.add_argument("--o", type=int, default=24)
    q.add_argument("--v", type=int, default=160)
    q.add_argument("--ncd", type=int, default=500)
    q.add_argument("--ks", type=str, default="1,8,16,32")
    q.add_argument("--reps", type=int, default=5)
    q.add_argument("--seed", type=int, default=1001)
    lc = sub.add_parser("learned-curve")
    lc.add_argument("--sizes", type=str, default="16,128,512,2000")
    lc.add_argument("--seed", type=int, default=1000)
    lc.add_argument("--per-iter", type=int, default=1024)
    lc.add_argument("--epochs", type=int, default=12)
    lc.add_argument("--diis", type=int, default=10)
    args = ap.parse_args()
    if args.cmd == "copy":
        copy_probe(args.mib)
    elif args.cmd == "gemm":
        gemm_probe(args.reps, args.tune, args.save, args.cfg, args.shapes, args.fp64_only, args.fp32_only)
    elif args.cmd == "split-gemm":
        split_gemm_probe(args.reps)
    elif args.cmd == "fns-presets":
        fns_presets(args.o, args.v, args.ncd, args.gamma, args.roots, args.seed)
    elif args.cmd == "sigma":
        sigma_probe(args.o, args.v, args.ncd, [int(x) for x in args.ks.split(",")], args.reps, args.seed)
    elif args.cmd == "ao-cd":
        ao_cd(args.nao, args.rank, args.n, args.tau, args.reps, args.seed)
    elif args.cmd == "learned-curve":
        learned_curve([int(x) for x in args.sizes.split(",")], args.seed, args.per_iter, args.epochs, args.diis)


if __name__ == "__main__":
    main()
