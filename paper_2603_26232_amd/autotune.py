"""Autotuner for the strided qubit groups of the tile passes.

A subgraph with n > 13 qubits is simulated in group 0 (qubits 0..10 and the
top qubit, which acts on the stored half-state as the complement; 4096-
amplitude tiles of two mirrored blocks) plus strided groups of at most 8 of
the qubits 11..n-2, one HBM pass per group and layer. How the n - 12 strided
qubits are split decides each pass's register layout chain, how many register
bits are real qubits and how long the contiguous rows of a strided tile are
(2^(12 - size) amplitudes). Every split gives the same state; the tuner times the
candidate splits (fewest groups, every ordered composition of n - 12 into
parts of at most 8) on a batch of random graphs with n qubits, one optimiser
evaluation (forward pass + adjoint sweep) or one forward evaluation per
repetition, and keeps the fastest. The table is saved as JSON and applied
with `apply()` before batches are created.

Run: python -m paper_2603_26232_amd.autotune --n 21 22 ... --out FILE
"""
from __future__ import annotations

import argparse
import itertools
import json
import os

import numpy as np
import torch

from . import synth, _abi
from .batch import QaoaBatch

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_gfx950.json")


def candidates(n: int, max_parts: int = 3):
    """Ordered compositions of n - 12 into the fewest parts of size 1..8."""
    R = n - 12
    if n <= 13:  # whole-state kernel, no strided groups
        return []
    parts = -(-R // 8)
    if parts > max_parts:
        return []
    out = []
    for comp in itertools.product(range(1, 9), repeat=parts):
        if sum(comp) == R:
            out.append(list(comp))
    return out


def default_split(n: int):
    R = n - 12
    G1 = -(-R // 8)
    return [R // G1 + (1 if g < R % G1 else 0) for g in range(G1)]


def time_split(n, split, p=3, gradient=True, amps=1 << 24, reps=5, seed=0):
    """Device milliseconds per evaluation and per 2^20 amplitudes."""
    B = max(1, amps >> n)
    edges = []
    for b in range(B):
        g = synth.erdos_renyi(n, 0.15, seed + b)
        edges.append((g.u, g.v, g.w))
    gamma, beta = synth.uniform_angles(seed + 999, p, batch=B)
    _abi.qaoa_tune_group_split(n, split)
    try:
        bt = QaoaBatch([n] * B, edges, max_p=p, max_k=8, gradient=gradient)
    finally:
        _abi.qaoa_tune_group_split(n, None)
    g = torch.as_tensor(gamma, device="cuda")
    b = torch.as_tensor(beta, device="cuda")

    def once():
        if gradient:
            bt.expectation_grad(g, b)
        else:
            bt.apply_layers(g, b)
            bt.expectation()

    once()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        once()
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / reps
    bt.close()
    return ms, ms / (B * (1 << n) / (1 << 20))


def tune(ns, p=3, gradient=True, log=print):
    table = {}
    for n in ns:
        cands = candidates(n)
        if len(cands) <= 1:
            continue
        res = []
        for sp in cands:
            ms, per = time_split(n, sp, p=p, gradient=gradient)
            res.append((per, sp, ms))
            log(f"autotune: n={n} split {sp}: {ms:.3f} ms per evaluation ({per:.4f} ms per 2^20 amplitudes)")
        res.sort(key=lambda r: r[0])
        best = res[0]
        dflt = next(r for r in res if r[1] == default_split(n))
        table[str(n)] = {"split": best[1], "ms_per_mamp": best[0], "default_split": dflt[1],
                         "default_ms_per_mamp": dflt[0],
                         "all": [{"split": r[1], "ms_per_mamp": r[0]} for r in res]}
        log(f"autotune: n={n}: best {best[1]} ({best[0]:.4f}), default {dflt[1]} ({dflt[0]:.4f})")
    return table


def apply(path: str = DEFAULT_TABLE) -> dict:
    """Load a tuning table and set it in the library; returns {n: split}."""
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    out = {}
    for n, e in data.get("entries", {}).items():
        _abi.qaoa_tune_group_split(int(n), e["split"])
        out[int(n)] = e["split"]
    return out


def reset(ns=range(14, 31)):
    for n in ns:
        _abi.qaoa_tune_group_split(n, None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=list(range(21, 31)))
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--forward-only", action="store_true")
    ap.add_argument("--out", default=DEFAULT_TABLE)
    args = ap.parse_args()
    log = lambda *a: print(*a, flush=True)
    table = tune(args.n, p=args.p, gradient=not args.forward_only, log=log)
    dev = torch.cuda.get_device_properties(0)
    with open(args.out, "w") as f:
        json.dump({"device": dev.name, "arch": getattr(dev, "gcnArchName", ""), "p": args.p,
                   "gradient": not args.forward_only, "entries": table}, f, indent=1)
    log(f"autotune: wrote {args.out}")


if __name__ == "__main__":
    main()
