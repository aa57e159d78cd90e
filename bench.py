"""Time-to-IPs and ladder throughput of the CD IP-EOM-CCSD hot path on one MI355X.

One step = the whole hot path on one synthetic instance with its inputs already in HBM:
cd_integrals (Cholesky staging + stored-integral assembly) -> ccsd_solve (Jacobi + DIIS to
|dE| < 1e-10, RMS residual < 1e-9) -> ipeom_davidson (lowest roots) -> IPs on the host.

Prints one JSON line.  `value` is the time-to-IPs in seconds of the benchmarked path (lower is
better).  The `roofline` object reports the particle-particle ladder, the dominant kernel: its
algorithmic flops per evaluation, F = 4 N v^3 (v-1) + o(o-1) v^2 (v-1)^2, divided by the mean
duration of a ladder evaluation measured with hipEvents on the library's stream over the timed
region.  `cpu_baseline` times the FP64 NumPy oracle on the host cores on a bounded sample of the
same workload and scales it to a time-to-IPs estimate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6, "split-bf16": 2516.6, "split-fp16": 2516.6}   # TFLOP/s, MI355X dense MFMA

# HBM bytes per ladder evaluation: rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, on
# `bench.py --ladder-only --steps 2 --warmup 0 --precision <p>`, summed over the ladder's kernels
# (from its first fill on) and scaled by what each counter reads for a 1 GiB device copy (FETCH
# x2.0, WRITE x1.0): FP64 33.13 GB fetched + 9.09 GB written; split-BF16 16.70 + 5.00 GB.  Only
# for the kernels and workload they were measured on.
LADDER_TRAFFIC_BYTES = {("o24v160n500", "fp64"): 41.90e9, ("o24v160n500", "split-bf16"): 21.59e9}
TRAFFIC_SOURCE = ("profile constant, not counted in this run: rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE "
                  "summed over the ladder kernels of the same kernel version and workload "
                  "(profiles/ladder_o24v160n500.md), each scaled by its reading for a 1 GiB copy")


def host_cpu():
    """CPU model, physical cores and logical CPUs of this host (from /proc/cpuinfo), and the BLAS
    threads the oracle runs with (OMP_NUM_THREADS, else every logical CPU)."""
    model, phys = "unknown", set()
    try:
        with open("/proc/cpuinfo") as f:
            cur = {}
            for line in f:
                if ":" in line:
                    k, v = (x.strip() for x in line.split(":", 1))
                    cur[k] = v
                    if k == "model name":
                        model = v
                elif cur:
                    phys.add((cur.get("physical id", "0"), cur.get("core id", cur.get("processor"))))
                    cur = {}
            if cur:
                phys.add((cur.get("physical id", "0"), cur.get("core id", cur.get("processor"))))
    except OSError:
        pass
    logical = os.cpu_count() or 1
    threads = int(os.environ.get("OMP_NUM_THREADS") or logical)
    return {"threads": threads, "cpu_model": model, "physical_cores": len(phys) or None, "logical_cpus": logical}


def _cpu_line(value, sample):
    h = host_cpu()
    return {"value": value, "unit": "s", "cores": h["threads"], "kind": "oracle", "sample": sample,
            "cpu_model": h["cpu_model"], "host_physical_cores": h["physical_cores"],
            "host_logical_cpus": h["logical_cpus"]}


# FP64 ladder rate measured at o=40, v=600, N=1800 (bench.py --ladder-only --workload o40v600n1800
# --precision fp64): the basis of the extrapolated FP64 time at shapes where an FP64 ladder would
# take tens of minutes
FP64_LADDER_RATE = 68.9e12


def ladder_flops(o, v, N):
    return 4.0 * N * v ** 3 * (v - 1) + o * (o - 1) * v ** 2 * (v - 1) ** 2


def run_gpu(args, inst, wl, precision, mlp=None, ctx=None):
    import torch

    from paper_2506_06805_amd import fnscc

    torch.cuda.set_device(0)
    ctx = ctx or fnscc.Context(0)
    # host-resident vectors: cd_integrals copies them over PCIe inside the timed region
    L_dev = inst.L if args.host_inputs else torch.from_numpy(inst.L).to("cuda")
    o, v, N, k = inst.o, inst.v, inst.ncd, wl["roots"]
    extra = {"mlp": mlp} if mlp is not None else {}

    last = {}

    def step():
        ints = fnscc.cd_integrals(ctx, inst.eps, L_dev, o, precision=precision)
        if args.fns is not None:   # frozen natural spinors inside the timed step, as in the method
            ints, _ = fnscc.fns_truncate(ctx, ints, args.fns)
        e, it, amps = fnscc.ccsd_solve(ctx, ints, precision=precision, **extra)
        w, its = fnscc.ipeom_davidson(ctx, ints, amps, k)
        last.update(ints=ints, amps=amps, v_kept=ints.v)
        return e, it, w, its

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(2)            # hipEvents around ladder evaluations only (no synchronisation)
    ctx.take_timings()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = []
    for s in range(args.steps):
        out.append(step())
        print(f"[bench] step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.take_timings()
    ctx.set_timing(0)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    n_lad = tm.get("ladder_events", 0.0)
    lad_ms = tm.get("ladder_event_ms", 0.0) / max(n_lad, 1.0)
    e, it, w, its = out[-1]
    return dict(ms_per_step=ms_per_step, ladder_ms=lad_ms, ladder_calls=n_lad, e=e, iters=it, w=w,
                eom_iters=its, **last)


def left_vectors(ctx, r, k):
    """Left eigenvectors and one-hole weights (Eq. 19-20) of the timed solve's last step, timed on
    their own: they are not part of time-to-IPs."""
    import torch

    from paper_2506_06805_amd import fnscc

    w, _, R = fnscc.ipeom_davidson(ctx, r["ints"], r["amps"], k, want_vectors=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wl, its, L, wt = fnscc.ipeom_left(ctx, r["ints"], r["amps"], k, R)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    bi = float(np.abs(L.cpu().numpy() @ R.cpu().numpy().T - np.eye(k)).max())
    return {"seconds": t1 - t0, "davidson_iters": its, "max_abs_dw_vs_right": float(np.abs(wl - w).max()),
            "max_abs_biorthonormality_error": bi, "one_hole_weights": [float(x) for x in np.real(wt)]}


def train_update_network(ctx, count=16, seed=1000):
    """The learned T2 update, trained on the GPU from plain-solver trajectories of small synthetic
    instances (uneven-batch generator, o in 6..16, v in 30..80); returns (network, seconds, info)."""
    import torch

    from paper_2506_06805_amd import learn

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    data = learn.collect(ctx, learn.training_instances(count, seed), per_iter=1024, seed=seed)
    net, hist = learn.train(ctx, data, epochs=12, batch=2048, lr=2e-3, seed=1)
    torch.cuda.synchronize()
    return net, time.perf_counter() - t0, {"instances": count, "samples": int(data[0].shape[0]),
                                           "epochs": 12, "loss_first": hist[0], "loss_last": hist[-1]}


def run_ladder_only(args, inst, wl):
    """Ladder evaluations alone (random tau, T1-dressed vectors), timed with hipEvents.

    Workloads drawn on the device (o=40, v=1698, N=4000) keep their complex64 vectors in complex64
    and run the ladder on packed amplitudes (tau and R over i<j, a<b): their full-layout complex128
    o^2 v^2 arrays would take 74 GB each."""
    import torch

    from paper_2506_06805_amd import fnscc, synth

    ctx = fnscc.Context(0)
    o, v, N = wl["o"], wl["v"], wl["ncd"]
    torch.cuda.reset_peak_memory_stats()
    t_setup = time.perf_counter()
    if wl.get("device"):
        eps, L = synth.make_instance_device(o, v, N, seed=wl["seed"], kappa=synth.kappa_for(v, N))
        ints = fnscc.cd_integrals(ctx, eps, L, o, precision=args.precision)
        del L
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    else:
        ints = fnscc.cd_integrals(ctx, inst.eps, torch.from_numpy(inst.L).to("cuda"), o, precision=args.precision)
    packed = bool(wl.get("device")) or args.packed
    g = torch.Generator(device="cuda").manual_seed(0)
    if packed:
        no, nv = o * (o - 1) // 2, v * (v - 1) // 2
        tau = torch.randn((no, nv), dtype=torch.complex128, device="cuda", generator=g).mul_(1e-2)
    else:
        gc = torch.Generator(device="cpu").manual_seed(0)
        tau = 1e-2 * torch.randn((o, o, v, v), dtype=torch.complex128, generator=gc)
        tau = (tau - tau.transpose(0, 1)) - (tau - tau.transpose(0, 1)).transpose(2, 3)
        tau = tau.contiguous().to("cuda")
    t1 = torch.randn((o, v), dtype=torch.complex128, device="cuda", generator=g).mul_(1e-2)
    R = torch.empty_like(tau)

    def run():
        if packed:
            fnscc.ladder_packed(ctx, ints, tau, t1, precision=args.precision, out=R)
        else:
            fnscc.ladder(ctx, ints, tau, t1, precision=args.precision, out=R)

    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    for _ in range(args.warmup):
        run()
    torch.cuda.synchronize()
    ctx.set_timing(2)
    ctx.take_timings()
    t0 = time.perf_counter()
    for s in range(args.steps):
        run()
        print(f"[bench] ladder {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1_ = time.perf_counter()
    tm = ctx.take_timings()
    n = max(tm.get("ladder_events", 0.0), 1.0)
    props = torch.cuda.get_device_properties(0)
    mem = {"peak_allocated_GB": torch.cuda.max_memory_allocated() / 1e9,
           "peak_reserved_GB": torch.cuda.max_memory_reserved() / 1e9,
           "device_total_GB": props.total_memory / 1e9,
           "L_vv_GB": v * v * N * (8 if wl.get("device") else 16) / 1e9,
           "split_planes_GB": 8.0 * v * v * N / 1e9 if args.precision != "fp64" else 0.0,
           "tau_GB": tau.numel() * 16 / 1e9, "R_GB": R.numel() * 16 / 1e9,
           "amplitude_layout": "packed i<j, a<b" if packed else "full o x o x v x v"}
    return dict(ms_per_step=(t1_ - t0) * 1000.0 / args.steps, ladder_ms=tm.get("ladder_event_ms", 0.0) / n,
                ladder_calls=n, memory=mem, setup_s=t_setup)


def run_batch(args, bw):
    """Uneven instances: CCSD per instance, then one batched Davidson over all of them.

    Also times the EOM stage of the same converged amplitudes one instance at a time (the
    comparison for the batched, graph-replayed sigma launches)."""
    import torch

    from paper_2506_06805_amd import fnscc, synth

    torch.cuda.set_device(0)
    ctx = fnscc.Context(0)
    if args.autotune:
        ctx.set_autotune(True)
    insts = synth.make_batch(bw["count"], bw["seed"])
    L_dev = [torch.from_numpy(x.L).to("cuda") for x in insts]
    k = bw["roots"]

    def step():
        ints, amps, es, its = [], [], [], []
        for inst, Ld in zip(insts, L_dev):
            I = fnscc.cd_integrals(ctx, inst.eps, Ld, inst.o, precision=args.precision)
            e, it, a = fnscc.ccsd_solve(ctx, I, precision=args.precision)
            ints.append(I); amps.append(a); es.append(e); its.append(it)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        w, eits = fnscc.ipeom_davidson(ctx, ints, amps, [k] * len(ints))
        torch.cuda.synchronize()
        return dict(ints=ints, amps=amps, e=es, iters=its, w=w, eom_iters=eits, t_eom=time.perf_counter() - tc)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_timing(2)
    ctx.take_timings()
    t0 = time.perf_counter()
    out = None
    t_eom = 0.0
    for s in range(args.steps):
        out = step()
        t_eom += out["t_eom"]
        print(f"[bench] step {s + 1}/{args.steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.take_timings()
    ctx.set_timing(0)
    # EOM stage again on the last step's amplitudes (H-bar and sigma operators now cached in the
    # handles): all instances in one batched Davidson, then one instance at a time
    tq = time.perf_counter()
    fnscc.ipeom_davidson(ctx, out["ints"], out["amps"], [k] * len(out["ints"]))
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - tq
    tq = time.perf_counter()
    for I, a in zip(out["ints"], out["amps"]):
        fnscc.ipeom_davidson(ctx, I, a, k)
    torch.cuda.synchronize()
    t_single = time.perf_counter() - tq
    F = sum(ladder_flops(x.o, x.v, x.ncd) * it for x, it in zip(insts, out["iters"]))
    lad_s = tm.get("ladder_event_ms", 0.0) * 1e-3 / args.steps
    return dict(ms_per_step=(t1 - t0) * 1000.0 / args.steps, eom_s=t_eom / args.steps, eom_single_s=t_single,
                eom_batched_s=t_batched,
                ladder_flop=F, ladder_s=lad_s, ladder_calls=tm.get("ladder_events", 0.0) / args.steps,
                insts=insts, **{kk: out[kk] for kk in ("e", "iters", "w", "eom_iters")})


def batch_cpu_baseline(insts, iters, sample=4, rows=4):
    """The oracle on `sample` instances of the batch (spread over the size range), scaled to all."""
    order = sorted(range(len(insts)), key=lambda i: insts[i].o ** 2 * insts[i].v ** 4)
    pick = [order[int(round(j * (len(order) - 1) / max(sample - 1, 1)))] for j in range(sample)]
    per = []
    for i in pick:
        x = insts[i]
        b = cpu_baseline(x, None, iters[i], rows=rows, other_terms=False)
        per.append(b["value"] / (x.o ** 2 * x.v ** 4 + x.ncd * x.v ** 4))
    scale = float(np.median(per))
    est = sum(scale * (x.o ** 2 * x.v ** 4 + x.ncd * x.v ** 4) for x in insts)
    return _cpu_line(est, (f"oracle lower bound (stored blocks + sampled ladder rows) on instances {pick}, "
                           f"scaled to the batch by the o^2 v^4 + N v^4 ladder cost; other terms and EOM not included"))


def cpu_baseline(inst, wl, iters, rows=8, other_terms=True):
    """The FP64 oracle on a bounded sample of the same workload, scaled to a time-to-IPs figure.

    Workloads with o^2 v^4 <= 1e10 (o=8, v=32) run whole: the oracle's CCSD solve and the dense
    IP-EOM-CCSD eigenvalues.  Larger ones: the stored integral blocks (<= 2 virtual indices) once,
    and `rows` of the v rows of the oracle's particle-particle ladder loop; the estimate is
    blocks + iterations x (ladder rows x v / rows + one residual without the ladder).  The EOM
    stage is left out, so it is a lower bound on the oracle's time-to-IPs.
    """
    from oracle import ccsd, eom, integrals

    o, v = inst.o, inst.v
    if wl is not None and o * o * v ** 4 <= 1e10:
        # small enough for the whole oracle time-to-IPs: CCSD, then the dense IP-EOM eigenproblem
        t0 = time.perf_counter()
        _, t1, t2, _, _ = ccsd.solve(inst.L, inst.eps, o)
        eom.dense_roots(eom.Hbar(integrals.Blocks(inst.L, o), inst.eps, t1, t2), wl["roots"])
        t_all = time.perf_counter() - t0
        return _cpu_line(t_all, "the whole workload: oracle CCSD solve and dense IP-EOM-CCSD eigenvalues")
    g = integrals.Blocks(inst.L, o)
    t0 = time.perf_counter()
    for name in ("oooo", "ooov", "oovv", "ovvo"):
        getattr(g, name)
    t_blocks = time.perf_counter() - t0
    rng = np.random.default_rng(0)
    t2 = 1e-3 * (rng.standard_normal((o, o, v, v)) + 1j * rng.standard_normal((o, o, v, v)))
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    t1 = np.zeros((o, v), dtype=np.complex128)
    rows = min(rows, v)
    t0 = time.perf_counter()
    ccsd.ladder(g, t1, t2, rows=range(rows))
    t_rows = time.perf_counter() - t0
    t_ladder = t_rows * v / rows
    if not other_terms:
        est = t_blocks + iters * t_ladder
        return _cpu_line(est, (f"stored integral blocks {t_blocks:.1f} s + oracle ladder on {rows} of {v} rows "
                               f"{t_rows:.1f} s, scaled to {t_ladder:.1f} s per iteration x {iters} CCSD iterations; "
                               "other residual terms and the EOM stage not included (lower bound)"))
    # every other term of one residual: the residual with an empty ladder row set, twice; the first
    # call also forms the three-virtual blocks, a one-time cost of the solve
    t0 = time.perf_counter()
    ccsd.residuals(g, inst.eps, t1, t2, rows=[])
    t_first = time.perf_counter() - t0
    t0 = time.perf_counter()
    ccsd.residuals(g, inst.eps, t1, t2, rows=[])
    t_rest = time.perf_counter() - t0
    t_once = t_blocks + max(0.0, t_first - t_rest)
    est = t_once + iters * (t_ladder + t_rest)
    return _cpu_line(est, (f"integral blocks {t_once:.1f} s once + per CCSD iteration the oracle ladder "
                           f"({rows} of {v} rows in {t_rows:.1f} s, scaled to {t_ladder:.1f} s) and the other "
                           f"residual terms ({t_rest:.1f} s), x {iters} iterations; the EOM stage not included "
                           "(lower bound)"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="o24v160n500")
    ap.add_argument("--precision", default="fp64", choices=sorted(PEAK))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ladder-only", action="store_true",
                    help="time ladder evaluations alone (profiling aid; not the time-to-IPs metric)")
    ap.add_argument("--no-left", dest="left", action="store_false",
                    help="skip the left eigenvectors and one-hole weights of the benchmarked instance")
    ap.add_argument("--no-compare", dest="compare", action="store_false",
                    help="skip the FP64 + learned, split-BF16 and split-BF16 + learned runs on the same instance")
    ap.add_argument("--host-inputs", action="store_true",
                    help="pass the Cholesky vectors from host memory (PCIe-inclusive time-to-IPs; not the metric)")
    ap.add_argument("--no-host-inputs", dest="host_compare", action="store_false",
                    help="skip the extra steps that time the same solve from host-resident vectors")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune GEMM tiles during the warmup steps (cached for the timed steps)")
    ap.add_argument("--fns", type=float, default=None,
                    help="frozen-natural-spinor occupation threshold applied inside each step (Eq. 24-28)")
    ap.add_argument("--fns-gamma", type=float, default=6.0,
                    help="decay of the FNS-structured generator used with --fns")
    ap.add_argument("--c64", action="store_true", help="complex64 Cholesky vectors (FP64 arithmetic)")
    ap.add_argument("--packed", action="store_true",
                    help="with --ladder-only: the ladder on packed amplitudes (fc_ladder_packed)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: the benchmark measures a single MI355X; --gpus must be 1"}))
        sys.exit(2)

    from paper_2506_06805_amd import synth

    if args.workload in synth.BATCHES:
        bw = synth.BATCHES[args.workload]
        r = run_batch(args, bw)
        achieved = r["ladder_flop"] / r["ladder_s"] / 1e12 if r["ladder_s"] > 0 else 0.0
        peak = PEAK[args.precision]
        line = {
            "metric": "time-to-IPs (s) + ladder TFLOP/s",
            "value": r["ms_per_step"] / 1000.0,
            "unit": "s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": r["ms_per_step"],
            "higher_is_better": False,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "c64 input / f64 compute" if args.precision == "fp64" else f"c64 input / {args.precision} ladder",
            "data": "synthetic",
            "config": {"workload": (f"{bw['count']} uneven CCSD + IP-EOM-CCSD instances, o~U{{6..24}}, v~U{{30..200}}, "
                                    f"N_CD=4v, complex64 Cholesky vectors, {bw['roots']} roots each, one batched Davidson"),
                       "precision": args.precision},
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                         "frac": achieved / peak, "traffic": None,
                         "kernel": "particle-particle ladder, all instances and CCSD iterations of one step",
                         "flop_per_step": r["ladder_flop"], "ladder_s_per_step": r["ladder_s"],
                         "launches": r["ladder_calls"]},
            "result": {"eom_s": r["eom_s"], "eom_cached_batched_s": r["eom_batched_s"],
                       "eom_cached_one_at_a_time_s": r["eom_single_s"],
                       "ccsd_iters": [int(x) for x in r["iters"]], "eom_iters": [int(x) for x in r["eom_iters"]],
                       "lowest_ip": float(np.min(np.real(r["w"])))},
        }
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = batch_cpu_baseline(r["insts"], r["iters"])
        print(json.dumps(line), flush=True)
        return

    wl = synth.WORKLOADS[args.workload]
    o, v, N = wl["o"], wl["v"], wl["ncd"]
    kappa = synth.kappa_for(v, N)
    F = ladder_flops(o, v, N)
    if wl.get("device") and not args.ladder_only:
        print(json.dumps({"error": f"{args.workload}: only --ladder-only runs at this shape (the CCSD residual's "
                                   "other terms still use full o^2 v^2 intermediates, 74 GB each)"}))
        sys.exit(2)
    inst = None
    if not wl.get("device"):
        inst = synth.make_instance(o, v, N, seed=wl["seed"], kappa=kappa,
                                   dtype=np.complex64 if args.c64 else np.complex128,
                                   fns_gamma=args.fns_gamma if args.fns is not None else None)
    if args.ladder_only:
        r = run_ladder_only(args, inst, wl)
        achieved = F / (r["ladder_ms"] * 1e-3) / 1e12
        line = {"metric": "ladder TFLOP/s (algorithmic)", "value": achieved, "unit": "TFLOP/s",
                "ms_per_launch": r["ladder_ms"], "launches": r["ladder_calls"],
                "flop_per_launch": F, "precision": args.precision,
                "frac": achieved / PEAK[args.precision],
                "config": {"workload": f"ladder o={o} v={v} N_CD={N}"
                           + (", complex64 vectors drawn on the device, packed tau and R" if wl.get("device") else ""),
                           "kappa": kappa},
                "memory": r["memory"], "setup_s": r["setup_s"]}
        if args.precision != "fp64":
            line["fp64_extrapolated_s"] = {
                "value": F / FP64_LADDER_RATE, "note": ("extrapolated, not measured: this ladder's flops at the FP64 "
                                                        f"ladder rate measured at o=40 v=600 N=1800 "
                                                        f"({FP64_LADDER_RATE / 1e12:.1f} TFLOP/s)")}
        print(json.dumps(line), flush=True)
        return
    from paper_2506_06805_amd import fnscc

    ctx = fnscc.Context(0)
    r = run_gpu(args, inst, wl, args.precision, ctx=ctx)
    vk = r.pop("v_kept", v)
    F = ladder_flops(o, vk, N)     # the ladder runs over the kept virtual spinors
    achieved = F / (r["ladder_ms"] * 1e-3) / 1e12 if r["ladder_ms"] > 0 else 0.0
    peak = PEAK[args.precision]
    dim = o + o * (o - 1) // 2 * vk
    traffic = None if (args.fns is not None or args.c64) else LADDER_TRAFFIC_BYTES.get((args.workload, args.precision))
    line = {
        "metric": "time-to-IPs (s) + ladder TFLOP/s",
        "value": r["ms_per_step"] / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "c128/f64", "split-bf16": "c128 + split-bf16 ladder", "split-fp16": "c128 + split-fp16 ladder"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"CCSD + IP-EOM-CCSD o={o} v={v} N_CD={N} {'complex64' if args.c64 else 'complex128'}, "
                               f"{wl['roots']} roots, kappa={kappa:.4f}"
                               + (f", FNS threshold {args.fns:g} on the generator with decay {args.fns_gamma:g}: "
                                  f"v'={vk}" if args.fns is not None else ""),
                   "precision": args.precision, "eom_dim": dim,
                   "inputs": "host memory (PCIe-inclusive)" if args.host_inputs else "HBM"},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": traffic,
                     "traffic_source": (TRAFFIC_SOURCE if traffic is not None else
                                        "no counter profile of this kernel version on this workload"),
                     "kernel": "particle-particle ladder (assembly GEMM + contraction GEMM per ab tile)",
                     "flop_per_launch": F, "ms_per_launch": r["ladder_ms"], "launches": r["ladder_calls"]},
        "result": {"e_corr": [r["e"].real, r["e"].imag], "ccsd_iters": r["iters"], "eom_iters": r["eom_iters"],
                   "ips": [float(x) for x in np.real(r["w"])]},
    }
    if args.host_compare and not args.host_inputs and args.steps > 0:
        # the same step with the Cholesky vectors handed over from host memory (cd_integrals copies
        # them over PCIe inside the timed region): the PCIe-inclusive figure, never `value`
        import copy
        ah = copy.copy(args)
        ah.host_inputs, ah.warmup, ah.steps = True, 0, min(2, args.steps)
        rh = run_gpu(ah, inst, wl, args.precision, ctx=ctx)
        line["host_inputs"] = {"time_to_ips_s": rh["ms_per_step"] / 1000.0, "steps": ah.steps,
                               "delta_vs_hbm_s": (rh["ms_per_step"] - r["ms_per_step"]) / 1000.0,
                               "bytes_over_pcie": int(inst.L.nbytes)}
    if args.left:
        line["left_vectors"] = left_vectors(ctx, r, wl["roots"])
    r.pop("ints", None)
    r.pop("amps", None)
    if args.compare and args.precision == "fp64":
        # the same instance with the learned update on the FP64 path, through the split-BF16 path,
        # and through the split-BF16 path with the learned update
        w64 = np.sort_complex(np.asarray(r["w"]))
        cmp = {}
        net, t_train, info = train_update_network(ctx)
        for name, prec, mlp in (("fp64+learned", "fp64", net), ("split-bf16", "split-bf16", None),
                                ("split-bf16+learned", "split-bf16", net)):
            rm = run_gpu(args, inst, wl, prec, mlp=mlp, ctx=ctx)
            wm = np.sort_complex(np.asarray(rm["w"]))
            lad = F / (rm["ladder_ms"] * 1e-3) / 1e12 if rm["ladder_ms"] > 0 else 0.0
            cmp[name] = {"time_to_ips_s": rm["ms_per_step"] / 1000.0,
                         "speedup_vs_fp64": r["ms_per_step"] / rm["ms_per_step"],
                         "max_abs_dIP_vs_fp64": float(np.abs(wm - w64).max()),
                         "abs_dE_vs_fp64": float(abs(rm["e"] - r["e"])),
                         "ccsd_iters": rm["iters"],
                         "ladder_tflops": lad, f"ladder_frac_of_{'fp64' if prec == 'fp64' else 'bf16'}_peak":
                         lad / PEAK[prec], "ladder_ms": rm["ladder_ms"]}
        for name in ("fp64+learned", "split-bf16+learned"):
            cmp[name]["training_s"] = t_train
        cmp["split-bf16+learned"]["training"] = info
        line["compare"] = cmp
    if not args.no_cpu_baseline and args.fns is None:   # the oracle baseline covers untruncated solves
        line["cpu_baseline"] = cpu_baseline(inst, wl, r["iters"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
