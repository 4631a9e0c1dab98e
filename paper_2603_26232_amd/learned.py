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
