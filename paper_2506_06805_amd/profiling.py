"""Profiling helpers.

`python -m paper_2506_06805_amd.profiling copy --mib 1024` runs one device-to-device copy of a known
size, the reference dispatch used to scale the FETCH_SIZE / WRITE_SIZE hardware counters into HBM
bytes (a copy of S bytes must read S and write S bytes).
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


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    args = ap.parse_args()
    if args.cmd == "copy":
        copy_probe(args.mib)


if __name__ == "__main__":
    main()
