"""Host-side input preparation: the graph partition of the paper's Alg. 1
(Sec. 3.2, Connectivity-Preserving Partitioning) and one-pass edge bucketing.

Reading of Alg. 1 used here: subgraph i is the contiguous vertex range
[start_i, start_i + size_i); the next range starts at the last vertex of the
previous one, so adjacent subgraphs share exactly one vertex (constraint 1 of
Sec. 3.2.1) and every size is at most N (constraint 2). With equal sizes the
stride is N - 1 and M = ceil((|V| - 1)/(N - 1)); the last range is clipped at
|V|. (Alg. 1 as printed gives the last subgraph the whole remainder, which
can exceed N; this reading keeps every subgraph within the solver size.)

GetSubgraph of Alg. 1 scans all of E once per subgraph; here one pass over E
assigns each edge to the subgraph holding both endpoints (unique, since two
ranges share at most one vertex) or to the inter-partition list. The result
is the same edge sets.
"""
from __future__ import annotations

import numpy as np


class Partition:
    """Chain partition of a graph: ranges plus per-subgraph local edge lists."""

    def __init__(self, num_vertices, start, size):
        self.num_vertices = int(num_vertices)
        self.start = np.ascontiguousarray(start, dtype=np.int32)
        self.size = np.ascontiguousarray(size, dtype=np.int32)

    @property
    def M(self) -> int:
        return int(self.start.shape[0])


def partition_equal(num_vertices: int, N: int) -> Partition:
    """Ranges of size N with stride N - 1 (the last one clipped)."""
    if N < 2:
        raise ValueError("subgraph size N must be >= 2")
    if num_vertices <= N:
        return Partition(num_vertices, [0], [num_vertices])
    M = -(-(num_vertices - 1) // (N - 1))
    start = np.arange(M, dtype=np.int64) * (N - 1)
    end = np.minimum(start + N, num_vertices)
    return Partition(num_vertices, start, end - start)


def partition_chain(num_vertices: int, sizes) -> Partition:
    """Ranges with the given sizes in order, sharing one vertex, until the
    chain reaches num_vertices (the last range clipped)."""
    start, size = [], []
    s = 0
    for n in np.asarray(sizes, dtype=np.int64):
        n = int(n)
        if n < 2:
            raise ValueError("subgraph sizes must be >= 2")
        start.append(s)
        if s + n >= num_vertices:
            size.append(num_vertices - s)
            return Partition(num_vertices, start, size)
        size.append(n)
        s += n - 1
    raise ValueError("sizes do not cover the graph")


def bucket_edges(part: Partition, u, v, w=None):
    """One pass over E: for each subgraph its induced edges in local ids, and
    the inter-partition edges. Returns (list of (lu, lv, lw), inter (u, v, w))."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    w = np.ones_like(u) if w is None else np.asarray(w, dtype=np.int64)
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    # the last range starting at or before lo is the only one that can hold
    # both endpoints (lo is its first or an inner vertex; any earlier range
    # ends at or before lo)
    starts = part.start.astype(np.int64)
    ends = starts + part.size.astype(np.int64)
    i = np.searchsorted(starts, lo, side="right") - 1
    owner = np.where(hi < ends[i], i, -1)
    subs = []
    order = np.argsort(owner, kind="stable")
    own_sorted = owner[order]
    bounds = np.searchsorted(own_sorted, np.arange(-1, part.M + 1))
    for k in range(part.M):
        sel = order[bounds[k + 1]:bounds[k + 2]]
        s = starts[k]
        subs.append(((u[sel] - s).astype(np.int32), (v[sel] - s).astype(np.int32),
                     w[sel].astype(np.int32)))
    inter_sel = order[bounds[0]:bounds[1]]
    inter = (u[inter_sel].astype(np.int32), v[inter_sel].astype(np.int32), w[inter_sel].astype(np.int32))
    return subs, inter


def batch_arrays(sizes, sub_edges):
    """Flatten per-subgraph edge lists into the (num_qubits, edge_offsets,
    u, v, w) arrays of the batch ABI."""
    nq = np.ascontiguousarray(sizes, dtype=np.int32)
    off = np.zeros(len(sub_edges) + 1, dtype=np.int64)
    for i, (a, _, _) in enumerate(sub_edges):
        off[i + 1] = off[i] + len(a)
    cat = lambda k: (np.concatenate([e[k] for e in sub_edges]).astype(np.int32)
                     if off[-1] > 0 else np.zeros(0, np.int32))
    return nq, off, cat(0), cat(1), cat(2)
