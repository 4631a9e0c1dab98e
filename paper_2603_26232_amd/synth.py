"""Seeded synthetic inputs shared by the GPU path, the tests and the bench.

This module holds no arithmetic of the method itself: it only draws random
numbers and turns them into graphs, subgraph size sequences and angle vectors.
Everything random that the method consumes is produced here and passed in as
an input, so the HIP path and the FP64 oracle see identical data.

Random stream: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014). Output i (i = 0, 1, ...) of the
stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), so any element
can be computed independently (counter-based); u01 = (x >> 11) * 2^-53.

Workload shapes follow the paper's evaluation (Section 4.1): Erdos-Renyi
graphs G(n, p) with unit weights and integer seeds. The instances are our
own draws, not the paper's NetworkX instances.
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 of the SplitMix64 stream for `seed`."""
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def u01(seed: int, start: int, count: int) -> np.ndarray:
    """Uniform doubles in [0, 1) from the stream (53 random bits each)."""
    return (splitmix64(seed, start, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Graph:
    """Undirected weighted graph as a COO edge list with u < v (int32)."""

    def __init__(self, num_vertices: int, u, v, w=None):
        self.num_vertices = int(num_vertices)
        self.u = np.ascontiguousarray(u, dtype=np.int32)
        self.v = np.ascontiguousarray(v, dtype=np.int32)
        if w is None:
            w = np.ones(self.u.shape[0], dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.int32)
        assert self.u.shape == self.v.shape == self.w.shape

    @property
    def num_edges(self) -> int:
        return int(self.u.shape[0])

    def __repr__(self) -> str:
        return f"Graph(|V|={self.num_vertices}, |E|={self.num_edges})"


def erdos_renyi(n: int, p: float, seed: int, chunk: int = 1 << 24) -> Graph:
    """G(n, p): one draw per vertex pair u < v in row-major pair order; the
    edge exists iff its uniform draw is below p. Unit weights."""
    us, vs = [], []
    # pairs of row u are (u, u+1) .. (u, n-1); their stream offset is the number
    # of pairs in the rows before u.
    row_start = np.zeros(n + 1, dtype=np.int64)
    if n > 1:
        row_len = np.arange(n - 1, -1, -1, dtype=np.int64)  # n-1, n-2, ..., 0
        row_start[1:] = np.cumsum(row_len)
    total = int(row_start[-1])
    pos = 0
    while pos < total:
        cnt = min(chunk, total - pos)
        draws = u01(seed, pos, cnt)
        hit = np.nonzero(draws < p)[0].astype(np.int64) + pos
        if hit.size:
            u = np.searchsorted(row_start, hit, side="right") - 1
            v = u + 1 + (hit - row_start[u])
            us.append(u.astype(np.int32))
            vs.append(v.astype(np.int32))
        pos += cnt
    if us:
        return Graph(n, np.concatenate(us), np.concatenate(vs))
    return Graph(n, np.zeros(0, np.int32), np.zeros(0, np.int32))


def random_regular3(n: int, seed: int, max_tries: int = 100000) -> Graph:
    """Random 3-regular graph by the pairing (configuration) model: 3n points
    shuffled by Fisher-Yates, consecutive points paired; an attempt with a
    self-loop or a repeated edge is discarded and the stream continues."""
    assert n % 2 == 0 and n >= 4
    npts = 3 * n
    pos = 0
    for _ in range(max_tries):
        pts = np.repeat(np.arange(n, dtype=np.int64), 3)
        r = u01(seed, pos, npts - 1)
        pos += npts - 1
        for k, i in enumerate(range(npts - 1, 0, -1)):
            j = int(r[k] * (i + 1))
            pts[i], pts[j] = pts[j], pts[i]
        a = pts[0::2]
        b = pts[1::2]
        if np.any(a == b):
            continue
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        key = lo * n + hi
        if np.unique(key).size != key.size:
            continue
        order = np.argsort(key, kind="stable")
        return Graph(n, lo[order], hi[order])
    raise RuntimeError("random_regular3: no simple pairing found")


def random_weights(num_edges: int, seed: int, lo: int = 1, hi: int = 9) -> np.ndarray:
    """Integer edge weights uniform in [lo, hi] (for weighted test cases)."""
    x = splitmix64(seed, 0, num_edges)
    return (np.uint64(lo) + x % np.uint64(hi - lo + 1)).astype(np.int32)


def ragged_sizes(seed: int, lo: int, hi: int, count: int) -> np.ndarray:
    """`count` subgraph sizes n_i = lo + (x_i mod (hi - lo + 1)) from the
    stream with seed `seed` (the graph seed plus one by convention)."""
    x = splitmix64(seed, 0, count)
    return (np.uint64(lo) + x % np.uint64(hi - lo + 1)).astype(np.int32)


def uniform_angles(seed: int, p: int, batch: int = 1, lo: float = 0.0, hi: float = math.pi):
    """Angles gamma, beta ~ U(lo, hi), each [batch, p] float64. Stream order:
    for each batch row, gamma_1..gamma_p then beta_1..beta_p."""
    r = u01(seed, 0, 2 * p * batch).reshape(batch, 2, p)
    a = lo + (hi - lo) * r
    return np.ascontiguousarray(a[:, 0, :]), np.ascontiguousarray(a[:, 1, :])

