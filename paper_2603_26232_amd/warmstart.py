"""Learned warm start vs cold start of the plain method.

Protocol:
  * training data: plain-method runs (cold ramp, T_max Adam steps) on fresh
    seeded Erdos-Renyi graphs partitioned into ragged 14..26-vertex chains;
    every subgraph with at least one edge contributes (features, canonical
    optimised angles);
  * the predictor is trained on the GPU by libparaqaoa's MLP and Adam kernels;
  * evaluation on a target workload: a cold plain run to T_max gives the
    reference E*_b; iterations-to-converge of a run is the first step t with
    E_b(t) >= E*_b - 1e-3 max(1, |E_b|_edges); the merged cut of the cold run
    after `plain_iters` steps is compared with the merged cut of the warm run
    after `warm_iters` steps (the plain optimiser always runs; the predictor
    only supplies its starting point).

Run: python -m paper_2603_26232_amd.warmstart --out DIR [options]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import numpy as np
import torch

from . import synth
from .learned import AnglePredictor, LearnedStart, canonical_angles, features
from .partition import partition_chain, partition_equal
from .solve import Solver, SolveConfig, cold_start
from .batch import _ptr, _stream
from . import _abi


def run_with_history(S: Solver, gamma0, beta0, iters: int, start=None, lr=None):
    """Adam steps from the given angles (or from a learned.LearnedStart's
    start, with its per-subgraph cold-start fallback); returns E at the start
    of every step and after the last ([iters + 1, B] numpy) and leaves the
    angles in S."""
    if start is not None:
        start.start()
    else:
        S.set_angles(gamma0, beta0)
    hist = torch.zeros((iters + 1, S.B), dtype=torch.float64, device=S.device)
    cfg = S.cfg
    P = S.B * cfg.p
    s = _stream(None)
    th, gr = _ptr(S.theta), _ptr(S.grad)
    for t in range(iters):
        _abi.qaoa_expectation_grad(S.batch.handle, cfg.p, th, th + 8 * P, _ptr(S.E), gr, gr + 8 * P, s)
        hist[t].copy_(S.E)
        _abi.qaoa_adam_step(2 * P, th, gr, _ptr(S.m), _ptr(S.v), _ptr(S.step), cfg.lr if lr is None else lr,
                            cfg.beta1, cfg.beta2, cfg.eps, 1, s)
    _abi.qaoa_apply_layers(S.batch.handle, cfg.p, th, th + 8 * P, s)
    _abi.qaoa_expectation(S.batch.handle, _ptr(S.E), s)
    hist[iters].copy_(S.E)
    return hist.cpu().numpy()


def iterations_to_converge(hist, E_star, n_edges, tol=1e-3):
    """First t with E(t) >= E* - tol max(1, |E|); len(hist) if never."""
    thr = E_star - tol * np.maximum(1.0, n_edges)
    ok = hist >= thr[None, :]
    first = np.where(ok.any(0), ok.argmax(0), hist.shape[0])
    return first


def ragged_graph(seed, nV, p_edge, lo, hi):
    g = synth.erdos_renyi(nV, p_edge, seed)
    part = partition_chain(nV, synth.ragged_sizes(seed + 1, lo, hi, nV))
    return g, part


def collect(seeds, nV=2000, p_edge=0.01, lo=14, hi=26, p=3, T=200, log=print):
    X, Y = [], []
    for seed in seeds:
        g, part = ragged_graph(seed, nV, p_edge, lo, hi)
        S = Solver(g, part, SolveConfig(p=p, iters=T, k=16, beam=64), skip_edgeless=True)
        g0, b0 = cold_start(p, S.B)
        t0 = time.perf_counter()
        run_with_history(S, g0, b0, T)
        torch.cuda.synchronize()
        th = S.theta.cpu().numpy()
        gam = th[:S.B * p].reshape(S.B, p)
        bet = th[S.B * p:].reshape(S.B, p)
        cg, cb = canonical_angles(gam, bet)
        n_act = 0
        for b in range(S.B):
            u, v, w = S.sub_edges[b]
            if len(u) == 0:
                continue
            X.append(features(int(part.size[b]), u, v))
            Y.append(np.concatenate([cg[b], cb[b]]))
            n_act += 1
        log(f"warmstart: seed {seed}: {part.M} subgraphs, {n_act} with edges, {T} steps in "
            f"{time.perf_counter() - t0:.1f} s")
        S.close()
        del S
        torch.cuda.empty_cache()
    return np.array(X, np.float32), np.array(Y, np.float32)


def compare(model: AnglePredictor, g, part, p=3, T_max=200, plain_iters=50, warm_iters=(0, 5, 10, 20, 50),
            k=16, beam=4096, log=print):
    """Cold vs warm on one workload; returns a dict of the protocol's numbers."""
    cfg = SolveConfig(p=p, iters=plain_iters, k=k, beam=beam)
    S = Solver(g, part, cfg, skip_edgeless=True)
    nE = np.array([len(e[0]) for e in S.sub_edges])
    act = nE > 0
    g0, b0 = cold_start(p, S.B)
    # reference: long cold run
    t0 = time.perf_counter()
    hist_cold = run_with_history(S, g0, b0, T_max)
    torch.cuda.synchronize()
    t_ref = time.perf_counter() - t0
    E_star = hist_cold[-1]
    it_cold = iterations_to_converge(hist_cold, E_star, nE)
    # plain method at its own budget: time the whole solve (optimise + finish)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.run(iters=plain_iters)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    r_plain = S.result()
    # warm start: predicted angles on the device, each subgraph falling back
    # to the cold start where that start's <C> is larger
    LS = LearnedStart(S, model)
    hist_warm = run_with_history(S, None, None, T_max, start=LS, lr=cfg.warm_lr)
    it_warm = iterations_to_converge(hist_warm, E_star, nE)
    out = {"subgraphs": int(S.B), "with_edges": int(act.sum()), "T_max": T_max,
           "plain_iters": plain_iters, "plain_cut": r_plain.cut, "plain_solve_s": t_plain,
           "plain_sum_E": float(r_plain.energies[act].sum()),
           "reference_run_s": t_ref,
           "iters_to_converge_cold": {"mean": float(it_cold[act].mean()), "median": float(np.median(it_cold[act]))},
           "iters_to_converge_warm": {"mean": float(it_warm[act].mean()), "median": float(np.median(it_warm[act]))},
           "E_sum_cold_final": float(E_star[act].sum()), "E_sum_warm_at0": float(hist_warm[0][act].sum()),
           "E_sum_cold_at0": float(hist_cold[0][act].sum()), "warm": []}
    for wi in warm_iters:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.run_learned(LS, wi)
        torch.cuda.synchronize()
        t_w = time.perf_counter() - t0
        r = S.result()
        out["warm"].append({"iters": wi, "cut": r.cut, "solve_s": t_w, "cut_ratio_vs_plain": r.cut / r_plain.cut,
                            "sum_E": float(r.energies[act].sum())})
        log(f"warmstart: warm start + {wi} steps: cut {r.cut} (plain {r_plain.cut} after {plain_iters}), "
            f"sum E {out['warm'][-1]['sum_E']:.3f} (plain {out['plain_sum_E']:.3f}), {t_w:.3f} s vs {t_plain:.3f} s")
    S.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--train-seeds", type=int, nargs=2, default=[100, 110])
    ap.add_argument("--train-T", type=int, default=200)
    ap.add_argument("--fit-steps", type=int, default=4000)
    ap.add_argument("--model", default=None, help="load a trained model (.npz) instead of training")
    ap.add_argument("--eval", choices=["c3", "c5", "both", "none"], default="both")
    ap.add_argument("--T-max", type=int, default=200)
    ap.add_argument("--tuning", default="default",
                    help="group-split table to apply: 'default' (the package's), 'none', or a path")
    args = ap.parse_args()
    os.makedirs(args.out, exist_ok=True)
    log = lambda *a: print(*a, flush=True)
    if args.tuning != "none":
        from . import autotune
        autotune.apply(autotune.DEFAULT_TABLE if args.tuning == "default" else args.tuning)
    p = 3
    model = AnglePredictor(p, seed=0)
    result = {}
    if args.model:
        model = AnglePredictor.from_file(args.model)
    else:
        X, Y = collect(range(*args.train_seeds), T=args.train_T, log=log)
        log(f"warmstart: training set {X.shape[0]} subgraphs")
        t0 = time.perf_counter()
        loss = model.fit(X, Y, steps=args.fit_steps, lr=1e-3)
        log(f"warmstart: fit {args.fit_steps} steps in {time.perf_counter() - t0:.1f} s, loss "
            f"{loss[0]:.4f} -> {loss[-1]:.4f}")
        np.savez(os.path.join(args.out, "angle_mlp.npz"), **model.state())
        result["train"] = {"samples": int(X.shape[0]), "loss_first": float(loss[0]), "loss_last": float(loss[-1])}
    if args.eval in ("c3", "both"):
        g, part = ragged_graph(0, 2000, 0.01, 14, 26)
        result["c3"] = compare(model, g, part, T_max=args.T_max, log=log)
        log(json.dumps(result["c3"]))
    if args.eval in ("c5", "both"):
        g, part = ragged_graph(0, 16000, 0.001, 20, 24)
        result["c5"] = compare(model, g, part, T_max=args.T_max, log=log)
        log(json.dumps(result["c5"]))
    with open(os.path.join(args.out, "warmstart.json"), "w") as f:
        json.dump(result, f, indent=1)


if __name__ == "__main__":
    main()
