"""The plain ParaQAOA method on one GPU (paper Sec. 3, Fig. 3 stages 1-3):
partition (host), batched QAOA with on-device angle optimisation, top-k,
level-wise merge and integer cut evaluation. Every numeric step runs in
libparaqaoa's HIP kernels; this module only orders the calls and owns the
torch tensors that hold device memory."""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _abi
from .batch import QaoaBatch, _ptr, _stream
from .partition import Partition, bucket_edges


@dataclass
class SolveConfig:
    p: int = 3
    iters: int = 50            # Adam steps per subgraph
    k: int = 16                # top-k per subgraph
    beam: int = 4096           # merge beam width W
    lr: float = 0.05
    # Adam step size of learned-warm-start solves: their start is close to an
    # optimum, where steps of 0.05 (the size of Adam's first bias-corrected
    # steps) overshoot; 0.02 was chosen on the predictor's training graphs
    warm_lr: float = 0.02
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


def cold_start(p: int, B: int):
    """Linear-ramp angles gamma_l = (pi/2)(l - 1/2)/p, beta_l = (pi/4)(1 - (l - 1/2)/p)
    for every subgraph (our reading: the paper gives no initialisation)."""
    f = (np.arange(p) + 0.5) / p
    g = np.tile(0.5 * math.pi * f, (B, 1))
    b = np.tile(0.25 * math.pi * (1.0 - f), (B, 1))
    return g, b


@dataclass
class SolveResult:
    cut: int
    assignment: np.ndarray          # uint8 per vertex
    energies: np.ndarray            # final <C> per subgraph
    gamma: np.ndarray
    beta: np.ndarray
    cand: np.ndarray                # uint32 [M, k]
    timings: dict = field(default_factory=dict)


class Solver:
    """Holds the device buffers of one graph so repeated solves allocate
    nothing new (the bench times `run`)."""

    def __init__(self, graph, part: Partition, cfg: SolveConfig, device="cuda", skip_edgeless=False,
                 gradient_memory="auto", concurrent_classes=False):
        self.g = graph
        self.part = part
        self.cfg = cfg
        self.device = torch.device(device)
        self.sub_edges, self.inter = bucket_edges(part, graph.u, graph.v, graph.w)
        self.B = part.M
        dev = self.device
        self.batch = QaoaBatch(part.size, self.sub_edges, max_p=cfg.p, max_k=cfg.k, gradient=True,
                               skip_edgeless=skip_edgeless, device=dev, gradient_memory=gradient_memory,
                               concurrent_classes=concurrent_classes)
        P = self.B * cfg.p
        self.theta = torch.zeros(2 * P, dtype=torch.float64, device=dev)   # [gamma | beta]
        self._theta_host = torch.zeros(2 * P, dtype=torch.float64, pin_memory=dev.type == "cuda")
        self._theta_copied = None  # event after the last copy out of _theta_host
        self.grad = torch.zeros(2 * P, dtype=torch.float64, device=dev)    # [dgamma | dbeta]
        self.m = torch.zeros(2 * P, dtype=torch.float64, device=dev)
        self.v = torch.zeros(2 * P, dtype=torch.float64, device=dev)
        self.step = torch.zeros(1, dtype=torch.int32, device=dev)
        self.E = torch.zeros(self.B, dtype=torch.float64, device=dev)
        self.idx = torch.zeros(self.B * cfg.k, dtype=torch.int32, device=dev)
        self.prob = torch.zeros(self.B * cfg.k, dtype=torch.float32, device=dev)
        # full graph on the device for the final CutVal
        self.du = torch.as_tensor(graph.u, device=dev)
        self.dv = torch.as_tensor(graph.v, device=dev)
        self.dw = torch.as_tensor(graph.w, device=dev)
        self.nw = (graph.num_vertices + 31) // 32
        self.best = torch.zeros(self.nw, dtype=torch.int32, device=dev)
        self.best_cut = torch.zeros(1, dtype=torch.int64, device=dev)
        self.eval_cut = torch.zeros(1, dtype=torch.int64, device=dev)
        mb = _abi.qaoa_merge_workspace_bytes(graph.num_vertices, part.M, graph.num_edges, cfg.k, cfg.beam)
        self.merge_ws = torch.empty(mb, dtype=torch.uint8, device=dev)
        # overlapped finish: a second merge slot, its stream and slot events
        self._slot1 = None
        self._side = None
        self._slot_free = [None, None]
        self._next_slot = 0
        self._last_slot = 0

    def rebuild(self, stream=None):
        """Re-create the batch on its existing workspace: validates the
        subgraphs again, uploads the edge lists and rebuilds every cut table
        (the batch-build step of the hot path)."""
        bt = self.batch
        from .partition import batch_arrays
        nq, off, u, v, w = batch_arrays(self.part.size, self.sub_edges)
        _abi.qaoa_batch_destroy(bt.handle)
        bt.handle = 0
        bt.handle = _abi.qaoa_batch_create(bt.B, nq, off, u, v, w, bt.max_p, bt.max_k, bt.flags,
                                           _ptr(bt.workspace), bt.workspace.numel(), _stream(stream))

    def set_angles(self, gamma, beta):
        P = self.B * self.cfg.p
        host = np.concatenate([np.asarray(gamma, dtype=np.float64).reshape(-1),
                               np.asarray(beta, dtype=np.float64).reshape(-1)])
        assert host.size == 2 * P
        # persistent pinned staging + asynchronous copy: the host waits only
        # for the previous copy out of the staging buffer (allocating or
        # freeing pinned memory here would wait for the whole device)
        if self._theta_copied is not None:
            self._theta_copied.synchronize()
        self._theta_host.numpy()[:] = host
        self.theta.copy_(self._theta_host, non_blocking=True)
        if self._theta_copied is None:
            self._theta_copied = torch.cuda.Event()
        self._theta_copied.record()
        self.m.zero_()
        self.v.zero_()
        self.step.zero_()

    def optimise(self, iters: int, stream=None, lr=None):
        """`iters` Adam ascent steps on every subgraph's <C>, one library call
        (no host sync); lr defaults to the configuration's."""
        cfg = self.cfg
        _abi.qaoa_optimize(self.batch.handle, cfg.p, iters, _ptr(self.theta), _ptr(self.m), _ptr(self.v),
                           _ptr(self.step), cfg.lr if lr is None else lr, cfg.beta1, cfg.beta2, cfg.eps,
                           _ptr(self.E), _stream(stream))

    def optimise_separate(self, iters: int, stream=None):
        """The same steps as separate gradient and Adam calls (reference for
        the fused path)."""
        cfg = self.cfg
        P = self.B * cfg.p
        s = _stream(stream)
        th, gr = _ptr(self.theta), _ptr(self.grad)
        for _ in range(iters):
            _abi.qaoa_expectation_grad(self.batch.handle, cfg.p, th, th + 8 * P, _ptr(self.E), gr, gr + 8 * P, s)
            _abi.qaoa_adam_step(2 * P, th, gr, _ptr(self.m), _ptr(self.v), _ptr(self.step), cfg.lr, cfg.beta1,
                                cfg.beta2, cfg.eps, 1, s)

    def _steps(self, n: int, s: int):
        cfg = self.cfg
        _abi.qaoa_optimize(self.batch.handle, cfg.p, n, _ptr(self.theta), _ptr(self.m), _ptr(self.v),
                           _ptr(self.step), cfg.lr, cfg.beta1, cfg.beta2, cfg.eps, _ptr(self.E), s)

    def optimise_graph(self, iters: int, chunk: int = None):
        """Same as `optimise`, replaying captured HIP graphs of `chunk` Adam
        steps each (default: all `iters` steps in one graph; every step is the
        angle tables, the gradient passes and the fused reduction + Adam). The
        step counter lives on the device, so each replay continues where the
        last one stopped. A graph is captured on first use of its step count
        and kept with the solver (it holds this batch's buffers)."""
        chunk = iters if chunk is None else max(1, min(chunk, iters))
        if getattr(self, "_graphs", None) is None:
            self._graphs = {}
        done = 0
        while done < iters:
            n = min(chunk, iters - done)
            g = self._graphs.get(n)
            if g is None:
                # the captured kernels reference only the workspace (whose
                # layout a rebuild of the same batch reproduces) and this
                # solver's buffers
                cap = torch.cuda.Stream()
                cap.wait_stream(torch.cuda.current_stream())
                g = torch.cuda.CUDAGraph()
                with torch.cuda.graph(g, stream=cap):
                    self._steps(n, int(cap.cuda_stream))
                torch.cuda.current_stream().wait_stream(cap)
                self._graphs[n] = g
            g.replay()
            done += n

    def _merge_slot(self, k):
        """Buffers of merge slot k: (idx, prob, merge_ws, best, best_cut, eval_cut)."""
        if k == 0:
            return self.idx, self.prob, self.merge_ws, self.best, self.best_cut, self.eval_cut
        if self._slot1 is None:
            self._slot1 = tuple(torch.empty_like(t) for t in self._merge_slot(0))
        return self._slot1

    def finish(self, stream=None, overlap=False):
        """Final state, expectation, top-k, merge and CutVal (device only).

        overlap: run the merge and CutVal on a second stream (default
        priority) so that they overlap whatever the caller enqueues next on
        `stream` (the next solve); the two merge slots alternate, and a slot's
        top-k waits until the merge that last read it has finished."""
        cfg = self.cfg
        P = self.B * cfg.p
        main = stream if stream is not None else torch.cuda.current_stream()
        s = int(main.cuda_stream)
        k = self._next_slot if overlap else 0
        idx, prob, mws, best, best_cut, eval_cut = self._merge_slot(k)
        if overlap and self._slot_free[k] is not None:
            main.wait_event(self._slot_free[k])
        th = _ptr(self.theta)
        _abi.qaoa_apply_layers(self.batch.handle, cfg.p, th, th + 8 * P, s)
        _abi.qaoa_expectation(self.batch.handle, _ptr(self.E), s)
        _abi.qaoa_topk(self.batch.handle, cfg.k, _ptr(idx), _ptr(prob), s)
        ms = s
        if overlap:
            if self._side is None:
                self._side = torch.cuda.Stream()
            ready = torch.cuda.Event()
            ready.record(main)
            self._side.wait_event(ready)
            ms = int(self._side.cuda_stream)
        g = self.g
        _abi.qaoa_merge_beam(g.num_vertices, self.part.M, self.part.start, self.part.size, g.num_edges, g.u, g.v,
                             g.w, cfg.k, _ptr(idx), cfg.beam, _ptr(mws), mws.numel(), _ptr(best), _ptr(best_cut), ms)
        _abi.maxcut_eval(g.num_vertices, g.num_edges, _ptr(self.du), _ptr(self.dv), _ptr(self.dw), 1, _ptr(best),
                         _ptr(eval_cut), ms)
        if overlap:
            done = torch.cuda.Event()
            done.record(self._side)
            self._slot_free[k] = done
            self._next_slot ^= 1
        self._last_slot = k

    def run(self, gamma0=None, beta0=None, iters=None, stream=None, graph=False, overlap=False, graph_chunk=None):
        if gamma0 is None:
            gamma0, beta0 = cold_start(self.cfg.p, self.B)
        self.set_angles(gamma0, beta0)
        n = self.cfg.iters if iters is None else iters
        if graph:
            self.optimise_graph(n, graph_chunk)
        else:
            self.optimise(n, stream)
        self.finish(stream, overlap=overlap)

    def run_learned(self, start, iters: int, stream=None, overlap=False, lr=None):
        """A learned-warm-start solve: `start` (a learned.LearnedStart of this
        solver) enqueues the predicted angles, with each subgraph falling back
        to the cold start where that start's <C> is larger; then `iters` Adam
        steps (step size lr, default the configuration's warm_lr) and the same finish
        as the plain method (device only)."""
        start.start(stream)
        if iters > 0:
            self.optimise(iters, stream, lr=self.cfg.warm_lr if lr is None else lr)
        self.finish(stream, overlap=overlap)

    def result(self) -> SolveResult:
        """The last finished solve's outputs (waits for the device)."""
        torch.cuda.synchronize()
        idx, _, _, best, best_cut, eval_cut = self._merge_slot(self._last_slot)
        P = self.B * self.cfg.p
        th = self.theta.cpu().numpy()
        words = best.cpu().numpy().view(np.uint32)
        nV = self.g.num_vertices
        x = ((words[np.arange(nV) // 32] >> (np.arange(nV) % 32).astype(np.uint32)) & 1).astype(np.uint8)
        cut = int(eval_cut.cpu()[0])
        assert cut == int(best_cut.cpu()[0]), "merge score and CutVal disagree"
        return SolveResult(cut=cut, assignment=x, energies=self.E.cpu().numpy(),
                           gamma=th[:P].reshape(self.B, -1), beta=th[P:].reshape(self.B, -1),
                           cand=idx.cpu().numpy().view(np.uint32).reshape(self.B, -1))

    def close(self):
        self._graphs = None
        self.batch.close()


def merge_beam(graph, part: Partition, cand: torch.Tensor, K: int, W: int, stream=None):
    """GPU beam merge of candidates cand (int32/uint32 [M, K] on the device);
    returns (best_words int32 tensor, best_cut int64 tensor)."""
    dev = cand.device
    nw = (graph.num_vertices + 31) // 32
    mb = _abi.qaoa_merge_workspace_bytes(graph.num_vertices, part.M, graph.num_edges, K, W)
    ws = torch.empty(mb, dtype=torch.uint8, device=dev)
    best = torch.zeros(nw, dtype=torch.int32, device=dev)
    cut = torch.zeros(1, dtype=torch.int64, device=dev)
    _abi.qaoa_merge_beam(graph.num_vertices, part.M, part.start, part.size, graph.num_edges, graph.u, graph.v,
                         graph.w, K, _ptr(cand), W, _ptr(ws), mb, _ptr(best), _ptr(cut), _stream(stream))
    return best, cut, ws


def maxcut_eval(graph_dev, num_vertices, assign: torch.Tensor, stream=None):
    """CutVal of each row of `assign` (int32 [A, ceil(V/32)] device)."""
    du, dv, dw = graph_dev
    A = assign.shape[0]
    out = torch.empty(A, dtype=torch.int64, device=assign.device)
    _abi.maxcut_eval(num_vertices, du.numel(), _ptr(du), _ptr(dv), _ptr(dw), A, _ptr(assign), _ptr(out),
                     _stream(stream))
    return out
