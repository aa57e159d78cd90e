"""Training of the learned T2 update from plain-solver trajectories (argument marshalling only;
sampling, forward, backward and Adam all run in the HIP library).

collect(): for each instance, a plain Jacobi + DIIS solve gives the converged doubles t*; the same
deterministic solve is repeated and, at every iterate t_k, `per_iter` amplitudes are sampled with
their features (which use the previous iterate's residual), the dressed Jacobi step
q = Omega / (D - (F_aa + F_bb - F_ii - F_jj)) and target correction r = (t* - t_k) - q.  Samples
that are not finite or whose step exceeds `qmax` are dropped.
train(): Adam on minibatches of those samples.
"""
from __future__ import annotations

import numpy as np

from . import fnscc, synth


def collect(ctx, instances, per_iter=2048, seed=1, max_iter=40, qmax=1.0, log=None):
    torch = ctx.torch
    chunks = []
    for n, inst in enumerate(instances):
        if log and n % 100 == 0:
            log(f"collect: instance {n} of {len(instances)}")
        ints = fnscc.cd_integrals(ctx, inst.eps, inst.L, inst.o)
        _, _, amps = fnscc.ccsd_solve(ctx, ints)
        _, t2s = amps.read()
        o, v = inst.o, inst.v
        dev = f"cuda:{ctx.device}"
        nit = max_iter
        X = torch.zeros((nit * per_iter, 4), dtype=torch.float32, device=dev)
        q = torch.zeros((nit * per_iter, 2), dtype=torch.float32, device=dev)
        r = torch.zeros((nit * per_iter, 2), dtype=torch.float32, device=dev)
        prev = [None]

        def on_iter(it, p1, p2, _user, ints=ints, t2s=t2s, X=X, q=q, r=r, n=n, prev=prev, o=o, v=v):
            if it > nit:
                return
            fnscc.learn_samples(ctx, ints, p1, p2, t2s, per_iter, seed * 1000003 + n * 1009 + it,
                                out=(X, q, r), offset=(it - 1) * per_iter, prev=prev[0])
            prev[0] = (fnscc.device_copy(ctx, p1, (o, v)), fnscc.device_copy(ctx, p2, (o, o, v, v)))

        fnscc.ccsd_solve(ctx, ints, allow_noconv=True, max_iter=nit, on_iter=on_iter)
        finite = torch.isfinite(X).all(1) & torch.isfinite(q).all(1) & torch.isfinite(r).all(1)
        keep = (q.abs().sum(1) > 0) & finite & (q.abs().max(1).values < qmax) & (r.abs().max(1).values < qmax)
        chunks.append((X[keep], q[keep], r[keep]))
    return tuple(torch.cat([c[k] for c in chunks]) for k in range(3))


def describe(data):
    """Sample count and magnitude summary (for logs)."""
    X, q, r = data
    return {"n": int(X.shape[0]), "max|X|": float(X.abs().max()), "max|q|": float(q.abs().max()),
            "max|r|": float(r.abs().max())}


def train(ctx, data, epochs=20, batch=4096, lr=2e-3, seed=0, mlp=None, log=None):
    torch = ctx.torch
    X, q, r = data
    mlp = mlp or fnscc.Mlp(ctx, seed=seed)
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        tot, nb = 0.0, 0
        for s in range(0, n - batch + 1, batch):
            idx = perm[s:s + batch]
            loss = mlp.train_step(X[idx].contiguous(), q[idx].contiguous(), r[idx].contiguous(), lr)
            if not np.isfinite(loss):
                raise FloatingPointError(f"training loss not finite at epoch {ep + 1}, batch {nb}: {describe(data)}")
            tot += loss
            nb += 1
        hist.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep + 1}: loss {hist[-1]:.4f}")
    return mlp, hist


def training_instances(count, seed, o_range=(6, 16), v_range=(30, 80)):
    """Small instances from the uneven-batch generator (N = 4 v), each with its coupling scale;
    instance k is drawn with seed 100 seed + k (seed >= 1000 keeps them apart from every
    benchmark and test instance)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        o = int(rng.integers(o_range[0], o_range[1] + 1))
        v = int(rng.integers(v_range[0], v_range[1] + 1))
        N = 4 * v
        out.append(synth.make_instance(o, v, N, seed=seed * 100 + k, kappa=synth.kappa_for(v, N)))
    return out
