"""Preservation time per slice, VATE (asynchronous timestamps, two blocks per
slice) against VDRE (distance recorders, the whole pool every slice), the
comparison of the paper's Sec. 5 (its PT column and PT speed-up), on one GPU.

Setting as in Sec. 5: window k = k' = 300 slices, g = 1024, pools of 2^23 to
2^32 counters, 10-bit ATs against 9-bit DRs packed exactly (the paper's
sizes; --containers uses 16-bit containers for both).  Each slice ingests 1M
random packets; PT is the time of the advance step (clock + preservation or
full-pool maintenance), measured with HIP events around an empty ingest
call, which performs exactly that step.

    python -m paper_1812_00282_amd.pt_compare [--pools 23,26,28,30,32] [--containers]

Prints one JSON line per pool size.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from .sketch import Config, Sketch


def measure(c: int, w: int, k: int = 300, g: int = 1024, slices: int = 24, packets: int = 1_000_000,
            counter: int = 0, device="cuda") -> float:
    sk = Sketch(Config(c, w, k, g, seed_a=1, seed_b=2, counter=counter), device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(c)
    empty = torch.empty((0, 2), dtype=torch.int32, device=device)
    times = []
    for t in range(slices):
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        sk.ingest(empty)            # advance + preserve (VATE) / maintain (VDRE)
        ev1.record()
        pairs = torch.randint(-2**31, 2**31, (packets, 2), generator=gen, device=device,
                              dtype=torch.int64).to(torch.int32)
        sk.ingest(pairs)
        sk.close_slice()
        if t >= 4:
            times.append((ev0, ev1))
    torch.cuda.synchronize()
    ms = float(np.median([a.elapsed_time(b) for a, b in times]))
    del sk
    torch.cuda.empty_cache()
    return ms


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--pools", default="23,26,28,30,32")
    ap.add_argument("--containers", action="store_true", help="16-bit containers for both")
    args = ap.parse_args()
    k = 300
    w_at, w_dr = (16, 16) if args.containers else ((2 * k).bit_length(), k.bit_length())
    for c in [int(x) for x in args.pools.split(",")]:
        vate = measure(c, w_at, k, counter=0)
        vdre = measure(c, w_dr, k, counter=1)
        print(json.dumps({"log2_counters": c, "k": k, "g": 1024, "vate_bits": w_at, "vdre_bits": w_dr,
                          "vate_pt_ms": vate, "vdre_pt_ms": vdre, "pt_speedup": vdre / vate}), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
