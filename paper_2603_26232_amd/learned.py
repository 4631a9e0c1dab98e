"""Learned warm start of the angle optimisation (not a step of the paper;
Sec. 2.2 notes that initialisation affects solution quality and iteration
count). An MLP maps per-subgraph features to depth-p angles; it is trained on
angles that the plain method itself optimised, with libparaqaoa's forward,
backward and Adam kernels on the GPU, and it only supplies the starting
point: the plain optimiser still runs and judges the result.

Features (18 for the default shape): a 16-bin histogram of intra-subgraph
vertex degrees (bins 0..14 and >= 15) divided by n, the edge density
|E_i| / C(n, 2) and n / 26.

Targets are canonical representatives of the optimised angles under the
ansatz's exact symmetries for integer cut values: beta_l -> beta_l + pi/2
(X on every qubit commutes with both operators), gamma_l -> gamma_l + 2 pi
(integer C(z)), and (gamma, beta) -> (-gamma, -beta) (complex conjugation).
"""
from __future__ import annotations

import math
import os

import numpy as np
import torch

from . import _abi
from .batch import _ptr, _stream

N_BINS = 16
N_FEATURES = N_BINS + 2
HIDDEN = 128


def features(n: int, u, v) -> np.ndarray:
    """Feature vector of one subgraph with n vertices and local edges (u, v)."""
    deg = np.bincount(np.concatenate([np.asarray(u), np.asarray(v)]).astype(np.int64), minlength=n)[:n]
    hist = np.bincount(np.minimum(deg, N_BINS - 1), minlength=N_BINS).astype(np.float64) / n
    dens = len(u) / (n * (n - 1) / 2) if n > 1 else 0.0
    return np.concatenate([hist, [dens, n / 26.0]]).astype(np.float32)


def canonical_angles(gamma, beta):
    """Canonical form of [.., p] angle arrays: beta in (-pi/4, pi/4], gamma in
    (-pi, pi], and gamma_1 >= 0 (else all signs flipped)."""
    g = np.asarray(gamma, dtype=np.float64).copy()
    b = np.asarray(beta, dtype=np.float64).copy()
    b = b - (math.pi / 2) * np.ceil((b - math.pi / 4) / (math.pi / 2))
    g = g - (2 * math.pi) * np.ceil((g - math.pi) / (2 * math.pi))
    flip = g[..., :1] < 0
    g = np.where(flip, -g, g)
    b = np.where(flip, -b, b)
    # the sign flip can move beta = pi/4 to -pi/4 and gamma = pi to -pi
    b = np.where(np.isclose(b, -math.pi / 4), math.pi / 4, b)
    g = np.where(np.isclose(g, -math.pi), math.pi, g)
    return g, b


class AnglePredictor:
    """MLP (in -> 128 -> 128 -> 2p) with FP64 master weights on the GPU."""

    def __init__(self, p: int, seed: int = 0, device="cuda", in_dim: int = N_FEATURES, hidden: int = HIDDEN):
        self.p = p
        self.in_dim, self.hidden, self.out = in_dim, hidden, 2 * p
        self.device = torch.device(device)
        self.npar = _abi.qaoa_mlp_num_params(self.in_dim, self.hidden, self.out)
        rng = np.random.default_rng(seed)
        parts = []
        for fan_in, fan_out in [(in_dim, hidden), (hidden, hidden), (hidden, self.out)]:
            parts.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), fan_in * fan_out))  # He init, W[out][in]
            parts.append(np.zeros(fan_out))
        self.params = torch.as_tensor(np.concatenate(parts), device=self.device)
        assert self.params.numel() == self.npar
        # feature / target standardisation (plain host arithmetic on the
        # training set, applied before the kernels)
        self.x_mu = np.zeros(in_dim, np.float32)
        self.x_sd = np.ones(in_dim, np.float32)
        self.y_mu = np.zeros(self.out, np.float32)
        self.y_sd = np.ones(self.out, np.float32)

    def _fwd(self, X: torch.Tensor, stream=None):
        B = X.shape[0]
        Y = torch.empty((B, self.out), dtype=torch.float32, device=self.device)
        A = torch.empty((B, 2 * self.hidden), dtype=torch.float32, device=self.device)
        _abi.qaoa_mlp_forward(B, self.in_dim, self.hidden, self.out, _ptr(self.params), _ptr(X), _ptr(Y), _ptr(A),
                              _stream(stream))
        return Y, A

    def fit(self, X, Y, steps=3000, lr=1e-3, batch=None, seed=0, log_every=0):
        """Adam on the mean-squared error of standardised targets; returns
        the loss history (every step's full-batch or mini-batch loss)."""
        X = np.asarray(X, np.float32)
        Y = np.asarray(Y, np.float32)
        self.x_mu, self.x_sd = X.mean(0), X.std(0) + 1e-6
        self.y_mu, self.y_sd = Y.mean(0), Y.std(0) + 1e-6
        Xs = torch.as_tensor((X - self.x_mu) / self.x_sd, device=self.device)
        Ys = torch.as_tensor((Y - self.y_mu) / self.y_sd, device=self.device)
        N = Xs.shape[0]
        B = N if batch is None else min(batch, N)
        grad = torch.zeros(self.npar, dtype=torch.float64, device=self.device)
        m = torch.zeros_like(grad)
        v = torch.zeros_like(grad)
        step = torch.zeros(1, dtype=torch.int32, device=self.device)
        loss = torch.zeros(steps, dtype=torch.float64, device=self.device)
        sb = _abi.qaoa_mlp_scratch_bytes(B, self.in_dim, self.hidden, self.out)
        scratch = torch.empty(sb, dtype=torch.uint8, device=self.device)
        rng = np.random.default_rng(seed)
        s = _stream(None)
        for t in range(steps):
            if B < N:
                idx = torch.as_tensor(rng.choice(N, B, replace=False), device=self.device)
                xb, yb = Xs[idx].contiguous(), Ys[idx].contiguous()
            else:
                xb, yb = Xs, Ys
            yp, act = self._fwd(xb)
            _abi.qaoa_mlp_backward(B, self.in_dim, self.hidden, self.out, _ptr(self.params), _ptr(xb), _ptr(yp),
                                   _ptr(act), _ptr(yb), _ptr(scratch), sb, _ptr(grad), _ptr(loss) + 8 * t, s)
            _abi.qaoa_adam_step(self.npar, _ptr(self.params), _ptr(grad), _ptr(m), _ptr(v), _ptr(step), lr, 0.9,
                                0.999, 1e-8, 0, s)
        return loss.cpu().numpy()

    def predict(self, X):
        """Angles (gamma [B, p], beta [B, p]) for feature rows X."""
        X = np.asarray(X, np.float32)
        Xs = torch.as_tensor((X - self.x_mu) / self.x_sd, device=self.device)
        Y, _ = self._fwd(Xs)
        Y = Y.cpu().numpy() * self.y_sd + self.y_mu
        return Y[:, :self.p].astype(np.float64), Y[:, self.p:].astype(np.float64)

    def state(self) -> dict:
        return {"params": self.params.cpu().numpy(), "x_mu": self.x_mu, "x_sd": self.x_sd, "y_mu": self.y_mu,
                "y_sd": self.y_sd, "p": self.p}

    def load(self, st: dict):
        self.params = torch.as_tensor(st["params"], device=self.device)
        self.x_mu, self.x_sd, self.y_mu, self.y_sd = st["x_mu"], st["x_sd"], st["y_mu"], st["y_sd"]

    @classmethod
    def from_file(cls, path: str, device="cuda") -> "AnglePredictor":
        """A trained predictor saved from `state()` with numpy.savez (plain
        arrays only; loaded without pickle)."""
        with np.load(path, allow_pickle=False) as z:
            st = {k: z[k] for k in z.files}
        p = int(st["p"])
        n_in = int(st["x_mu"].shape[0])
        m = cls(p, device=device, in_dim=n_in, hidden=_hidden_width(n_in, 2 * p, int(st["params"].shape[0])))
        m.load(st)
        return m


def _hidden_width(n_in: int, out: int, count: int) -> int:
    """Hidden width H of an n_in -> H -> H -> out network with `count`
    parameters: H (n_in + 1) + H (H + 1) + out (H + 1) = count."""
    b = n_in + 2 + out
    H = int(round((-b + math.sqrt(b * b + 4 * (count - out))) / 2))
    if H * (n_in + 1) + H * (H + 1) + out * (H + 1) != count:
        raise ValueError(f"{count} parameters do not form an {n_in} -> H -> H -> {out} network")
    return H


DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "angle_mlp_p3.npz")


class LearnedStart:
    """Learned warm start of one Solver's batch, on the device.

    Built once per graph (input preparation, like the partition): the
    standardised feature rows of every subgraph, the predictor's parameters
    and target standardisation, and buffers for the two candidate starts.
    `start()` only enqueues work: the predictor's forward pass, its outputs
    turned into angles, <C> at the predicted and at the cold-start angles,
    and per subgraph the start with the larger <C> (the plain method's
    start remains the fallback)."""

    def __init__(self, solver, model: AnglePredictor):
        from .solve import cold_start
        S = solver
        assert model.p == S.cfg.p, f"predictor depth {model.p} != solve depth {S.cfg.p}"
        self.S, self.model = S, model
        dev = S.device
        F = np.stack([features(int(S.part.size[b]), S.sub_edges[b][0], S.sub_edges[b][1]) for b in range(S.B)])
        self.X = torch.as_tensor(((F - model.x_mu) / model.x_sd).astype(np.float32), device=dev)
        self.mu = torch.as_tensor(np.asarray(model.y_mu, np.float32), device=dev)
        self.sd = torch.as_tensor(np.asarray(model.y_sd, np.float32), device=dev)
        self.Y = torch.empty((S.B, model.out), dtype=torch.float32, device=dev)
        self.act = torch.empty((S.B, 2 * model.hidden), dtype=torch.float32, device=dev)
        g0, b0 = cold_start(S.cfg.p, S.B)
        self.theta_cold = torch.as_tensor(np.concatenate([g0.reshape(-1), b0.reshape(-1)]), device=dev)
        self.theta_alt = torch.empty_like(self.theta_cold)
        self.E_alt = torch.empty(S.B, dtype=torch.float64, device=dev)

    def start(self, stream=None):
        S, m = self.S, self.model
        p, B = S.cfg.p, S.B
        P = B * p
        st = _stream(stream)
        h = S.batch.handle
        self.theta_alt.copy_(self.theta_cold)
        ta = _ptr(self.theta_alt)
        _abi.qaoa_apply_layers(h, p, ta, ta + 8 * P, st)
        _abi.qaoa_expectation(h, _ptr(self.E_alt), st)
        _abi.qaoa_mlp_forward(B, m.in_dim, m.hidden, m.out, _ptr(m.params), _ptr(self.X), _ptr(self.Y),
                              _ptr(self.act), st)
        th = _ptr(S.theta)
        _abi.qaoa_warm_angles(B, p, _ptr(self.Y), _ptr(self.mu), _ptr(self.sd), th, st)
        _abi.qaoa_apply_layers(h, p, th, th + 8 * P, st)
        _abi.qaoa_expectation(h, _ptr(S.E), st)
        _abi.qaoa_keep_better(B, p, _ptr(self.E_alt), ta, _ptr(S.E), th, st)
        S.m.zero_()
        S.v.zero_()
        S.step.zero_()
