"""Merge quality / cost trade-off: candidate count K and beam width W.

Sec. 4.2 studies how the number of candidates kept per subgraph trades
solution quality against merge cost (the leaf count 2K^M grows with K). Here
the plain method runs once per workload with top-16 candidates; the merge is
then repeated for every K (the first K of each subgraph's list, i.e. its K
most probable canonical bitstrings) and every beam width W, timing each
merge on the device and recording the merged cut.

Run: python -m paper_2603_26232_amd.sweep --out DIR [--workload NAME ...]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import time

import numpy as np
import torch

from . import synth, _abi
from .batch import _ptr, _stream
from .partition import partition_equal, partition_chain
from .solve import Solver, SolveConfig

WORKLOADS = {
    "plain400": lambda: (synth.erdos_renyi(400, 0.05, 0), None, 20, False),
    "ragged2000": lambda: (synth.erdos_renyi(2000, 0.01, 0), (14, 26), None, True),
    "learned16000": lambda: (synth.erdos_renyi(16000, 0.001, 0), (20, 24), None, True),
}


def build(name):
    g, ragged, N, skip = WORKLOADS[name]()
    part = partition_chain(g.num_vertices, synth.ragged_sizes(1, ragged[0], ragged[1], g.num_vertices)) \
        if ragged else partition_equal(g.num_vertices, N)
    return g, part, skip


def time_merge(g, part, cand, K, W, reps=3):
    """Median device time (ms) of one beam merge and its cut."""
    dev = cand.device
    nw = (g.num_vertices + 31) // 32
    mb = _abi.qaoa_merge_workspace_bytes(g.num_vertices, part.M, g.num_edges, K, W)
    ws = torch.empty(mb, dtype=torch.uint8, device=dev)
    best = torch.zeros(nw, dtype=torch.int32, device=dev)
    cut = torch.zeros(1, dtype=torch.int64, device=dev)
    s = _stream(None)
    times = []
    for _ in range(reps):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        _abi.qaoa_merge_beam(g.num_vertices, part.M, part.start, part.size, g.num_edges, g.u, g.v, g.w, K,
                             _ptr(cand), W, _ptr(ws), mb, _ptr(best), _ptr(cut), s)
        ev[1].record()
        torch.cuda.synchronize()
        times.append(ev[0].elapsed_time(ev[1]))
    return float(np.median(times)), int(cut.item())


def sweep(name, Ks, Ws, iters=50, log=print):
    g, part, skip = build(name)
    kmax = max(Ks)
    S = Solver(g, part, SolveConfig(p=3, iters=iters, k=kmax, beam=max(Ws)), skip_edgeless=skip)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.run()
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    r = S.result()
    cand_all = S.idx.view(part.M, kmax)
    log(f"sweep: {name}: {g}, {part.M} subgraphs, plain solve {t_solve:.3f} s, cut {r.cut} (K={kmax}, "
        f"W={max(Ws)})")
    rows = []
    for K in Ks:
        cand = cand_all[:, :K].contiguous()
        for W in Ws:
            ms, cut = time_merge(g, part, cand, K, W)
            rows.append({"K": K, "W": W, "cut": cut, "merge_ms": ms,
                         "exact": bool(math.log2(W) >= 1 + (part.M - 1) * math.log2(K))})
            log(f"sweep: {name} K={K:3d} W={W:5d} cut {cut} merge {ms:.3f} ms")
    S.close()
    return {"workload": name, "vertices": g.num_vertices, "edges": g.num_edges, "subgraphs": part.M,
            "plain_solve_s": t_solve, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--workload", nargs="+", default=["plain400", "ragged2000", "learned16000"],
                    choices=list(WORKLOADS))
    ap.add_argument("--K", type=int, nargs="+", default=[1, 2, 4, 8, 16])
    ap.add_argument("--W", type=int, nargs="+", default=[1, 16, 64, 256, 1024, 4096, 8192])
    ap.add_argument("--tuning", default="default",
                    help="group-split table to apply: 'default' (the package's), 'none', or a path")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    log = lambda *a: print(*a, flush=True)
    if args.tuning != "none":
        from . import autotune
        autotune.apply(autotune.DEFAULT_TABLE if args.tuning == "default" else args.tuning)
    res = [sweep(w, args.K, args.W, log=log) for w in args.workload]
    with open(os.path.join(args.out, "merge_sweep.json"), "w") as f:
        json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
