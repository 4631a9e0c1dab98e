#!/usr/bin/env python3
"""Benchmark of the ParaQAOA hot path on one MI355X.

Default workload (ragged2000): one step = one whole plain-method solve of a
2000-vertex graph: batch build with integer cut tables, 50 Adam steps of every
subgraph's angles on exact adjoint gradients, the final state and <C>, top-16
extraction, the level-wise beam merge (W = 4096) and the integer CutVal of the
winner. Erdos-Renyi G(2000, 0.01), seed 0, unit weights, partitioned into a
chain of ragged subgraphs of 14..26 vertices (sizes from stream seed 1);
edgeless subgraphs are not simulated (closed form); QAOA depth p = 3.
Consecutive solves are pipelined: a solve's merge and CutVal run on a second
stream while the next solve starts (--no-overlap runs them in line); the timed
region still ends when every solve's merge has finished. The subgraphs'
qubit-group classes run concurrently on the library's side streams
(--serial-classes: in order), except in the steps that carry kernel events
(the profiled warm-up step and the last tenth of the timed steps), which run
them serially so that no other kernel overlaps the timed launches; the line
also times both modes apart (solve.plain_classes).

The same line carries the learned-warm-start solve of the same graph: the
angle predictor (committed weights, trained on plain-method runs of other
seeds) gives every subgraph its starting angles on the device, each subgraph
falls back to the plain method's cold start where that start has the larger
<C>, then 5 Adam steps (step size 0.02) and the same finish. Both solve times (pipelined, and
the latency of one solve run alone with its merge in line) and both merged cuts
are reported.

Other workloads (--workload):
  plain400     the same plain solve on G(400, 0.05), seed 0, 21 subgraphs of
               20 vertices (equal partition, stride 19).
  learned16000 the plain and the learned-warm-start solves of G(16000, 0.001),
               seed 0, chained into ragged subgraphs of 20..24 vertices
               (sizes from stream seed 1; 764 subgraphs, 148 with edges).
  precision26  one forward evaluation (all layers + <C>) of 32 random 3-regular
               graphs on 26 vertices, p = 4, angles U(0, pi); --mixer picks the
               mixer precision mode.

value = amplitude updates per second of the plain solves: per forward
evaluation every layer applies n RX gates and one diagonal phase to each
amplitude, U = sum_b p (n_b + 1) 2^n_b over simulated subgraphs; an optimiser
step is a forward evaluation plus the adjoint sweep over two states (3 U),
and the final evaluation adds U.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QAOA amp-updates/s + HBM GB/s; 2k-vertex solve time, learned vs plain angles"
PASSES = [f"fwd_{k}_g{g}" for k in ("first", "single", "mid", "last") for g in range(4)] + \
    [f"bwd_{k}_g{g}" for k in ("fused", "single", "mid", "last", "single_nopsi", "mid_nopsi") for g in range(4)]
KERNELS = PASSES + ["small", "cut_tables", "angle_prep", "reduce", "reduce_adam", "topk", "maxcut", "adam", "merge",
                    "mlp_forward", "warm_angles", "keep_better"]
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _record(path, kernel):
    """The RECORD line of `kernel` in a committed profile summary, if that
    summary was taken on the current kernel source; else None."""
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("RECORD "):
            r = json.loads(line[len("RECORD "):])
            if r.get("kernel") == kernel:
                rec = r
    if not rec:
        return None
    src = os.path.join(ROOT, "paper_2603_26232_amd", "csrc", rec.get("source", "sim.hip"))
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    if sha != rec.get("source_sha256"):
        return None
    return rec


def traffic_record(kernel, workload):
    """Measured HBM traffic per launch of `kernel` (FETCH_SIZE + WRITE_SIZE)."""
    return _record(os.path.join(ROOT, "profiles", f"pmc_passes_{workload}.txt"), kernel)


def valu_record(kernel, workload):
    """Measured wave-wide VALU instructions per launch of `kernel` (SQ_INSTS_VALU)."""
    return _record(os.path.join(ROOT, "profiles", f"pmc_valu_{workload}.txt"), kernel)


# wave-wide VALU instruction issue peak: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles
# per wave-wide FP32 instruction (16 lanes per cycle; no packed FP32)
VALU_PEAK = 256 * 4 * 2.4e9 / 4


def amp_updates(sizes, p):
    return sum(p * (int(n) + 1) * (1 << int(n)) for n in sizes)


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo, as lscpu shows it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_solves(run, n, sync_each=False):
    """Seconds per solve of `n` calls of run() (after a device sync); with
    sync_each, the median of single solves each waited for (latency)."""
    import torch
    torch.cuda.synchronize()
    if sync_each:
        ts = []
        for _ in range(n):
            t0 = time.perf_counter()
            run()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[len(ts) // 2]
    t0 = time.perf_counter()
    for _ in range(n):
        run()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / n


def workload_solve(args, name):
    """plain400 / ragged2000 / learned16000: the plain-method solve as one
    step; the ragged workloads also time the learned-warm-start solve of the
    same graph."""
    import numpy as np
    import torch
    from paper_2603_26232_amd import synth
    from paper_2603_26232_amd.partition import partition_equal, partition_chain
    from paper_2603_26232_amd.solve import Solver, SolveConfig, cold_start

    if name == "plain400":
        g = synth.erdos_renyi(400, 0.05, 0)
        part = partition_equal(400, 20)
        skip = False
        desc = "plain-method solve, G(400,0.05) seed 0, 21 subgraphs x 20 qubits, p=3, 50 Adam steps, top-16, " \
               "beam 4096, CutVal"
    elif name == "learned16000":
        g = synth.erdos_renyi(16000, 0.001, 0)
        part = partition_chain(16000, synth.ragged_sizes(1, 20, 24, 16000))
        skip = True
        desc = "16k-vertex solve: G(16000,0.001) seed 0, ragged chain of 20..24-qubit subgraphs, edgeless " \
               "skipped, p=3, top-16, beam 4096, CutVal; plain = cold start + 50 Adam steps, learned = " \
               f"predicted start (cold-start fallback per subgraph) + {args.warm_iters} Adam steps at step size " \
               f"{args.warm_lr}"
    else:
        g = synth.erdos_renyi(2000, 0.01, 0)
        part = partition_chain(2000, synth.ragged_sizes(1, 14, 26, 2000))
        skip = True
        desc = "2k-vertex solve: G(2000,0.01) seed 0, ragged chain of 14..26-qubit subgraphs, edgeless " \
               "skipped, p=3, top-16, beam 4096, CutVal; plain = cold start + 50 Adam steps, learned = " \
               f"predicted start (cold-start fallback per subgraph) + {args.warm_iters} Adam steps at step size " \
               f"{args.warm_lr}"
    cfg = SolveConfig(p=3, iters=50, k=16, beam=4096)
    log(f"bench: graph {g}, {part.M} subgraphs of sizes {min(part.size)}..{max(part.size)}, p={cfg.p}, "
        f"iters={cfg.iters}, k={cfg.k}, W={cfg.beam}")
    conc = not args.serial_classes
    S = Solver(g, part, cfg, skip_edgeless=skip, gradient_memory=args.gradient_memory, concurrent_classes=conc)
    from paper_2603_26232_amd import _abi

    def classes(concurrent):
        """Qubit-group classes on concurrent side streams or in serial order,
        from the next batch build (every step starts with one) on."""
        if concurrent:
            S.batch.flags |= _abi.QAOA_FLAG_CONCURRENT_CLASSES
        else:
            S.batch.flags &= ~_abi.QAOA_FLAG_CONCURRENT_CLASSES

    ckpt = _abi.qaoa_gradient_checkpoints(S.batch.handle)
    nE = np.array([len(e[0]) for e in S.sub_edges])
    act = nE > 0
    sim = [int(n) for n, e in zip(part.size, nE) if not (skip and e == 0)]
    U = amp_updates(sim, cfg.p)
    overlap = not args.no_overlap

    LS = None
    if name in ("ragged2000", "learned16000") and not args.no_learned:
        from paper_2603_26232_amd.learned import AnglePredictor, LearnedStart
        model = AnglePredictor.from_file(args.predictor)
        LS = LearnedStart(S, model)
        log(f"bench: angle predictor {os.path.basename(args.predictor)} ({model.npar} parameters)")

    def step():
        S.rebuild()
        S.run(overlap=overlap)

    def learned_step(ov=overlap):
        S.rebuild()
        S.run_learned(LS, args.warm_iters, overlap=ov, lr=args.warm_lr)

    def plain_alone():
        S.rebuild()
        S.run(overlap=False)

    def graph_step():
        S.rebuild()
        S.run(graph=True, overlap=overlap)

    def result():
        r = S.result()
        return {"cut": r.cut, "sum_E_with_edges": round(float(np.sum(r.energies[act])), 6)}

    def summary():
        return {"solve": result()}

    n_cmp = max(3, args.steps // 2)

    def graph_compare(plain_s, ref):
        """The same plain solves with the 50 Adam steps replayed from one
        captured HIP graph (captured by the first, untimed solve)."""
        log(f"bench: plain solves with the {cfg.iters}-step Adam loop in one HIP graph, {n_cmp} timed")
        c0 = time.perf_counter()
        graph_step()
        torch.cuda.synchronize()
        first = time.perf_counter() - c0
        gs = time_solves(graph_step, n_cmp)
        r = result()
        log(f"bench: graph replay {gs:.4f} s/solve (eager {plain_s:.4f}), first solve with capture {first:.2f} s")
        return {"seconds": round(gs, 4), "eager_seconds": round(plain_s, 4), "speedup_vs_eager": round(plain_s / gs, 4),
                "first_solve_with_capture_seconds": round(first, 3), "same_result_as_eager": r == ref}

    def classes_compare():
        """Plain solves with the classes concurrent, then in serial order (each
        mode's first solve untimed); the results must be identical."""
        log(f"bench: plain solves with concurrent and with serial classes, {n_cmp} timed each")
        res = {}
        try:
            for mode in (True, False):
                classes(mode)
                step()
                res[mode] = (time_solves(step, n_cmp), result())
        finally:
            classes(conc)
        c, s_ = res[True][0], res[False][0]
        log(f"bench: classes concurrent {c:.4f} s/solve, serial {s_:.4f} s/solve")
        return {"concurrent_seconds": round(c, 4), "serial_seconds": round(s_, 4),
                "concurrent_speedup": round(s_ / c, 4), "same_result": res[True][1] == res[False][1]}

    def extra(plain_s):
        """After the timed plain solves: their result, the plain solves with
        the Adam loop replayed from a HIP graph, with the classes concurrent
        and serial, the learned solves timed the same way, and the latency of
        one solve of each kind."""
        out = {"plain": dict(result(), seconds=round(plain_s, 4), adam_steps=cfg.iters, adam_lr=cfg.lr)}
        if not args.no_graph_compare:
            out["plain_graph_replay"] = graph_compare(plain_s, result())
        if not args.no_classes_compare:
            out["plain_classes"] = classes_compare()
        if LS is None:
            return {"solve": out}
        log(f"bench: learned-warm-start solves ({args.warm_iters} Adam steps), {args.steps} timed")
        learned_step()
        learned_s = time_solves(learned_step, args.steps)
        out["learned"] = dict(result(), seconds=round(learned_s, 4), adam_steps=args.warm_iters,
                              adam_lr=args.warm_lr)
        log(f"bench: latency of single solves (merge in line), {args.latency_solves} of each")
        out["plain"]["latency_seconds"] = round(time_solves(plain_alone, args.latency_solves, True), 4)
        out["learned"]["latency_seconds"] = round(time_solves(lambda: learned_step(False), args.latency_solves,
                                                              True), 4)
        out["learned_vs_plain"] = {"speedup": round(plain_s / learned_s, 3),
                                   "sum_E_ratio": round(out["learned"]["sum_E_with_edges"] /
                                                        out["plain"]["sum_E_with_edges"], 5),
                                   "latency_speedup": round(out["plain"]["latency_seconds"] /
                                                            out["learned"]["latency_seconds"], 3),
                                   "cut_ratio": round(out["learned"]["cut"] / out["plain"]["cut"], 4)}
        log(f"bench: plain {plain_s:.3f} s/solve cut {out['plain']['cut']}; learned {learned_s:.3f} s/solve "
            f"cut {out['learned']['cut']}")
        return {"solve": out}

    def cpu_baseline():
        import oracle
        # bounded sample: every subgraph (plain400) or every 2nd (ragged2000)
        # or 6th (learned16000, all of 20 qubits or more) simulated subgraph of
        # at most 22 qubits, T Adam steps with the final evaluation; then a
        # quarter of it on one thread
        every = 6 if name == "learned16000" else 2
        idx = list(range(part.M)) if name == "plain400" else \
            [b for b in range(part.M) if not (skip and nE[b] == 0) and part.size[b] <= 22][::every]
        which = "all" if name == "plain400" else f"every {every}th simulated one of at most 22 qubits".replace(
            "2th", "2nd")
        T = args.cpu_iters

        def timed(ids, T):
            sizes = [int(part.size[b]) for b in ids]
            edges = [S.sub_edges[b] for b in ids]
            g0, b0 = cold_start(cfg.p, len(ids))
            c0 = time.perf_counter()
            oracle.solve_batch(sizes, edges, g0, b0, T, cfg.k, lr=cfg.lr)
            c1 = time.perf_counter()
            return (3 * T + 1) * amp_updates(sizes, cfg.p) / (c1 - c0), c1 - c0

        threads = oracle.num_threads()
        log(f"bench: CPU baseline: FP64 oracle, {len(idx)} subgraphs x ({T} Adam steps + final evaluation), "
            f"{threads} threads")
        val, sec = timed(idx, T)
        one = idx[::4]
        T1 = max(1, T // 3)
        log(f"bench: CPU baseline: {len(one)} subgraphs x ({T1} Adam steps + final evaluation), 1 thread")
        oracle.set_num_threads(1)
        try:
            val1, sec1 = timed(one, T1)
        finally:
            oracle.set_num_threads(threads)
        return {"value": val, "unit": "amp-updates/s", "cores": threads, "kind": "oracle",
                "seconds": round(sec, 2), "cpu_model": cpu_model(),
                "sample": f"{len(idx)} subgraphs ({which}) of this workload, {T} Adam steps with adjoint "
                          f"gradients + final evaluation and top-{cfg.k} (FP64)",
                "one_thread": {"value": val1, "unit": "amp-updates/s", "cores": 1, "seconds": round(sec1, 2),
                               "sample": f"every 4th subgraph of that sample ({len(one)}), {T1} Adam steps + "
                                         f"final evaluation"}}

    config = {"workload": desc, "merge_overlaps_next_solve": overlap,
              "classes": ("concurrent on side streams, serial in the last tenth of the timed steps (the steps "
                          "that carry the dominant kernel's events) and in the profiled warm-up step") if conc
              else "serial",
              "gradient_memory": ("forward checkpoints" if ckpt else "in place") + f" ({args.gradient_memory})",
              "vertices": g.num_vertices, "edges": g.num_edges,
              "subgraphs": part.M, "simulated_subgraphs": len(sim),
              "qubits": [int(min(part.size)), int(max(part.size))],
              "p": cfg.p, "adam_steps": cfg.iters, "k": cfg.k, "beam": cfg.beam}
    if LS is not None:
        config["learned_adam_steps"] = args.warm_iters
        config["predictor"] = os.path.basename(args.predictor)
    return dict(step=step, updates=(3 * cfg.iters + 1) * U, config=config, summary=summary, extra=extra,
                cpu_baseline=cpu_baseline, close=S.close, dtype="fp32", classes=classes, concurrent=conc)


def workload_precision(args):
    """precision26: one forward evaluation per step."""
    import numpy as np
    import torch
    from paper_2603_26232_amd import synth
    from paper_2603_26232_amd.batch import QaoaBatch

    graphs = [synth.random_regular3(26, s) for s in range(32)]
    edges = [(gr.u, gr.v, gr.w) for gr in graphs]
    ang = [synth.uniform_angles(2000 + s, 4) for s in range(32)]
    gamma = np.concatenate([a[0] for a in ang])
    beta = np.concatenate([a[1] for a in ang])
    bt = QaoaBatch([26] * 32, edges, max_p=4, max_k=8, mixer=args.mixer)
    g = torch.as_tensor(gamma, device="cuda")
    b = torch.as_tensor(beta, device="cuda")
    E = torch.empty(32, dtype=torch.float64, device="cuda")
    U = amp_updates([26] * 32, 4)

    def step():
        bt.apply_layers(g, b)
        bt.expectation(E)

    def summary():
        return {"sum_E": float(E.sum())}

    def cpu_baseline():
        import oracle
        sizes, sub = [26] * 2, edges[:2]
        log("bench: CPU baseline: FP64 oracle, 2 of the 32 subgraphs, one forward evaluation each")
        c0 = time.perf_counter()
        oracle.eval_batch(sizes, sub, gamma[:2], beta[:2])
        c1 = time.perf_counter()
        return {"value": amp_updates(sizes, 4) / (c1 - c0), "unit": "amp-updates/s",
                "cores": oracle.num_threads(), "kind": "oracle", "seconds": round(c1 - c0, 2), "cpu_model": cpu_model(),
                "sample": "2 of the 32 subgraphs (26 qubits, p = 4), one FP64 forward evaluation with <C>"}

    dtype = {"valu": "fp32", "mfma_f32": "fp32", "mfma_bf16x3": "bf16x3 (mixer block)",
             "mfma_bf16x4": "bf16x4 (mixer block)"}[args.mixer]
    config = {"workload": "forward evaluation, 32 random 3-regular graphs x 26 qubits, p=4, angles U(0,pi)",
              "mixer": args.mixer, "subgraphs": 32, "qubits": 26, "p": 4}
    return dict(step=step, updates=U, config=config, summary=summary, cpu_baseline=cpu_baseline,
                close=bt.close, dtype=dtype)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["ragged2000", "learned16000", "plain400", "precision26"],
                    default="ragged2000")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run each solve's merge on the main stream instead of overlapping it with the next solve")
    ap.add_argument("--mixer", choices=["valu", "mfma_f32", "mfma_bf16x3", "mfma_bf16x4"], default="valu",
                    help="mixer precision mode (precision26 only)")
    ap.add_argument("--cpu-iters", type=int, default=12, help="Adam steps in the CPU-baseline sample")
    ap.add_argument("--no-learned", action="store_true",
                    help="ragged workloads: skip the learned-warm-start solves")
    ap.add_argument("--warm-iters", type=int, default=5, help="Adam steps of a learned-warm-start solve")
    ap.add_argument("--warm-lr", type=float, default=0.02, help="Adam step size of a learned-warm-start solve")
    ap.add_argument("--predictor", default=None, help="trained angle predictor (.npz); default: the package's")
    ap.add_argument("--latency-solves", type=int, default=3, help="single solves timed alone, per kind")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph-compare", action="store_true",
                    help="solve workloads: skip the plain solves with the Adam loop replayed from a HIP graph")
    ap.add_argument("--gradient-memory", choices=["auto", "checkpoints", "inplace"], default="auto",
                    help="forward checkpoints, one psi rebuilt in place, or the library's choice by size")
    ap.add_argument("--serial-classes", action="store_true",
                    help="solve workloads: run the qubit-group classes in serial order throughout (default: "
                         "concurrently on side streams, except in the profiled steps)")
    ap.add_argument("--no-classes-compare", action="store_true",
                    help="solve workloads: skip the plain solves timed with concurrent and with serial classes")
    ap.add_argument("--tuning", default="default",
                    help="group-split tuning table (JSON from paper_2603_26232_amd.autotune); 'default' = the "
                         "package's table if present, 'none' = untuned")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy (counter calibration, copy bandwidth)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); the hot path "
              "shards by subgraph with no communication until the merge, which this box cannot show.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_26232_amd import _abi
    if args.predictor is None:
        from paper_2603_26232_amd.learned import DEFAULT_MODEL
        args.predictor = DEFAULT_MODEL

    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    torch.cuda.set_device(0)
    if args.copy_probe:
        # one untimed copy, then three timed ones: four copies in all
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(3):
            dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / 3
        log(f"bench: copy probe: {n} bytes read + {n} written per copy, {ms:.3f} ms per copy, "
            f"{2 * n / (ms * 1e-3) / 1e9:.1f} GB/s")
        return

    from paper_2603_26232_amd import autotune
    tuned = {} if args.tuning == "none" else autotune.apply(
        autotune.DEFAULT_TABLE if args.tuning == "default" else args.tuning)
    if tuned:
        log(f"bench: tuned group splits {tuned}")
    W = workload_precision(args) if args.workload == "precision26" else workload_solve(args, args.workload)
    W["config"]["tuned_group_splits"] = {str(k): v for k, v in tuned.items()}
    step = W["step"]

    def read_profile():
        kern = {}
        for k in KERNELS:
            n, ms, by = _abi.qaoa_profile_read(k)
            if n:
                kern[k] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / n, "algo_bytes": by}
        return kern

    # warm-up; the last warm-up step is timed kernel by kernel (every launch
    # bracketed by events) to find the kernel with the largest share
    # with concurrent classes, the steps that carry kernel events (the
    # profiled warm-up step, the last tenth of the timed steps) run the
    # classes serially: overlapping launches would stretch each kernel's
    # event-timed duration
    classes = W.get("classes", lambda concurrent: None)
    conc = W.get("concurrent", False)
    kern = {}
    for i in range(args.warmup):
        if i == args.warmup - 1:
            classes(False)
            _abi.qaoa_profile_select(None)
            _abi.qaoa_profile_enable(1)
        step()
    torch.cuda.synchronize()
    if args.warmup:
        kern = read_profile()
        _abi.qaoa_profile_enable(0)
    # without a warm-up the last timed step times every kernel instead
    dom = max(kern, key=lambda k: kern[k]["total_ms"]) if kern else None
    log(f"bench: {args.warmup} warmup steps done; timing {args.steps} steps (kernel events on "
        f"{dom or 'every kernel'} in the last)")
    # timed region: events only around the dominant kernel's launches, and
    # only in the last tenth of the steps (each event pair leaves a gap of a
    # few microseconds around the launch, ~3 % of a step when on every step);
    # until then no kernel is selected (selecting needs no host wait)
    nprof = max(1, args.steps // 10)
    _abi.qaoa_profile_select("-")
    _abi.qaoa_profile_enable(1)
    classes(conc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        if i == args.steps - nprof:
            classes(False)
            _abi.qaoa_profile_select(dom)
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    classes(conc)
    timed = read_profile()
    _abi.qaoa_profile_enable(0)
    _abi.qaoa_profile_select(None)
    if dom is None:
        dom = max(timed, key=lambda k: timed[k]["total_ms"])
    elapsed = t1 - t0
    ms_step = 1e3 * elapsed / args.steps
    value = W["updates"] * args.steps / elapsed
    log(f"bench: {ms_step:.3f} ms/step, {value:.4e} amp-updates/s")
    log("bench: kernels of the profiled warm-up step:")
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["total_ms"]):
        gbs = v["algo_bytes"] / (v["total_ms"] * 1e-3) / 1e9 if v["total_ms"] > 0 else 0.0
        log(f"  {k:11s} {v['launches']:6d} launches  avg {v['avg_us']:9.2f} us  {gbs:8.1f} GB/s algorithmic")

    d = timed[dom]
    log(f"bench: timed region: {dom} {d['launches']} launches, avg {d['avg_us']:.2f} us")
    achieved = d["algo_bytes"] / (d["total_ms"] * 1e-3) / 1e9
    tr = traffic_record(dom, args.workload) if args.mixer == "valu" else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "algo_bytes_per_launch": d["algo_bytes"] / d["launches"], "avg_launch_us": round(d["avg_us"], 2),
                "traffic": (None if tr is None else tr["hbm_bytes_per_launch"]),
                "measured_on": f"the last {nprof} of the {args.steps} timed steps" +
                               (", qubit-group classes serial" if conc else "")}
    vr = valu_record(dom, args.workload) if args.mixer == "valu" else None
    if vr is not None:
        # the same kernel seen from the vector units: measured VALU issue rate
        va = vr["valu_insts_per_launch"] / (d["avg_us"] * 1e-6)
        roofline["alu"] = {"achieved": round(va / 1e9, 1), "peak": round(VALU_PEAK / 1e9, 1),
                           "unit": "G VALU wave-instructions/s", "frac": round(va / VALU_PEAK, 4),
                           "valu_insts_per_launch": vr["valu_insts_per_launch"]}

    out = {
        "metric": METRIC, "value": value, "unit": "amp-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": W["dtype"], "data": "synthetic", "config": W["config"],
        "roofline": roofline,
    }
    out.update(W["summary"]())
    out["kernels_warmup_step"] = {k: {"launches": v["launches"], "avg_us": round(v["avg_us"], 2),
                                      "algo_GBs": round(v["algo_bytes"] / (v["total_ms"] * 1e-3) / 1e9, 1)
                                      if v["total_ms"] else 0} for k, v in kern.items()}
    if "extra" in W:
        out.update(W["extra"](ms_step / 1e3))
    W["close"]()
    if not args.no_cpu_baseline:
        cb = W["cpu_baseline"]()
        out["cpu_baseline"] = cb
        log(f"bench: CPU baseline {cb['value']:.4e} amp-updates/s in {cb['seconds']} s on {cb['cores']} threads")
        if "one_thread" in cb:
            log(f"bench: CPU baseline {cb['one_thread']['value']:.4e} amp-updates/s on 1 thread")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
