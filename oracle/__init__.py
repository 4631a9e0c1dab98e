"""FP64 CPU oracle for the ParaQAOA hot path (test infrastructure).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The product library never calls into it. The functions
here are thin numpy/ctypes wrappers around `oracle.c`; each one names the
passage of the paper it follows.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

UINT32_MAX = 0xFFFFFFFF


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (portable -O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    """The loaded oracle library. PQ_ORACLE_LIB names a prebuilt copy to load
    instead (the sanitizer build of the test-suite); else oracle.c is built
    here if needed."""
    global _lib
    if _lib is None:
        path = os.environ.get("PQ_ORACLE_LIB")
        if not path:
            path = build()
        _lib = ct.CDLL(path)
        _declare(_lib)
    return _lib


_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_c128p = np.ctypeslib.ndpointer(dtype=np.complex128, flags="C_CONTIGUOUS")


def _declare(L):
    L.or_num_threads.restype = ct.c_int
    L.or_set_num_threads.restype = None
    L.or_set_num_threads.argtypes = [ct.c_int]
    L.or_cutval.restype = ct.c_int64
    L.or_cutval.argtypes = [ct.c_int64, _i32p, _i32p, ct.c_void_p, _u8p]
    L.or_cutval_packed.restype = None
    L.or_cutval_packed.argtypes = [ct.c_int64, ct.c_int32, ct.c_int64, _i32p, _i32p, ct.c_void_p,
                                   _u32p, _i64p]
    L.or_bruteforce_maxcut.restype = ct.c_int64
    L.or_bruteforce_maxcut.argtypes = [ct.c_int32, ct.c_int64, _i32p, _i32p, ct.c_void_p, _u8p]
    L.or_cut_table.restype = None
    L.or_cut_table.argtypes = [ct.c_int32, ct.c_int64, _i32p, _i32p, ct.c_void_p, _i64p]
    L.or_qaoa_state.restype = None
    L.or_qaoa_state.argtypes = [ct.c_int32, _i64p, ct.c_int32, _f64p, _f64p, _c128p]
    L.or_qaoa_unapply.restype = None
    L.or_qaoa_unapply.argtypes = [ct.c_int32, _i64p, ct.c_int32, _f64p, _f64p, _c128p]
    L.or_expectation.restype = ct.c_double
    L.or_expectation.argtypes = [ct.c_int32, _c128p, _i64p]
    L.or_topk.restype = ct.c_int32
    L.or_topk.argtypes = [ct.c_int32, _c128p, ct.c_int32, ct.c_int32, ct.c_uint32, _u32p, _f64p]
    L.or_tie_rank.restype = ct.c_uint64
    L.or_tie_rank.argtypes = [ct.c_uint64, ct.c_int32]
    L.or_free_mask.restype = ct.c_uint32
    L.or_free_mask.argtypes = [ct.c_int32, ct.c_int64, _i32p, _i32p, ct.c_void_p]
    L.or_gradient.restype = None
    L.or_gradient.argtypes = [ct.c_int32, _i64p, ct.c_int32, _f64p, _f64p, ct.c_void_p, _f64p, _f64p]
    L.or_cold_start.restype = None
    L.or_cold_start.argtypes = [ct.c_int32, _f64p, _f64p]
    L.or_adam_solve.restype = None
    L.or_adam_solve.argtypes = [ct.c_int32, _i64p, ct.c_int32, ct.c_int32, ct.c_double, ct.c_double,
                                ct.c_double, ct.c_double, _f64p, _f64p, ct.c_void_p]
    L.or_adam_update.restype = None
    L.or_adam_update.argtypes = [ct.c_int64, _f64p, _f64p, _f64p, _f64p, ct.c_int32, ct.c_double,
                                 ct.c_double, ct.c_double, ct.c_double, ct.c_double]
    L.or_eval_batch.restype = None
    L.or_eval_batch.argtypes = [ct.c_int32, _i32p, _i64p, _i32p, _i32p, ct.c_void_p, ct.c_int32,
                                _f64p, _f64p, _f64p, ct.c_int32, ct.c_int32, _u32p, _f64p]
    L.or_solve_batch.restype = None
    L.or_solve_batch.argtypes = [ct.c_int32, _i32p, _i64p, _i32p, _i32p, ct.c_void_p, ct.c_int32,
                                 ct.c_int32, ct.c_double, ct.c_double, ct.c_double, ct.c_double,
                                 _f64p, _f64p, _f64p, ct.c_int32, ct.c_int32, _u32p, _f64p]
    L.or_partition_equal.restype = ct.c_int32
    L.or_partition_equal.argtypes = [ct.c_int32, ct.c_int32, _i32p, _i32p]
    L.or_partition_chain.restype = ct.c_int32
    L.or_partition_chain.argtypes = [ct.c_int32, ct.c_int32, _i32p, _i32p, _i32p]
    L.or_mlp_num_params.restype = ct.c_int64
    L.or_mlp_num_params.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32]
    L.or_mlp_forward.restype = None
    L.or_mlp_forward.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, _f64p, _f64p, _f64p]
    L.or_mlp_loss_grad.restype = ct.c_double
    L.or_mlp_loss_grad.argtypes = [ct.c_int32, ct.c_int32, ct.c_int32, ct.c_int32, _f64p, _f64p, _f64p, _f64p]
    L.or_merge.restype = ct.c_int64
    L.or_merge.argtypes = [ct.c_int32, ct.c_int32, _i32p, _i32p, ct.c_int64, _i32p, _i32p,
                           ct.c_void_p, ct.c_int32, _u32p, ct.c_int64, _u8p, _i32p,
                           ct.POINTER(ct.c_double)]


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _wptr(w):
    if w is None:
        return None, None
    w = _i32(w)
    return w, w.ctypes.data_as(ct.c_void_p)


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    """Threads of the OpenMP loops from now on (1 = a single core)."""
    lib().or_set_num_threads(int(n))


# --- Sec. 2.1 -------------------------------------------------------------
def cutval(u, v, w, x) -> int:
    """CutVal of assignment x (0/1 per vertex) over edges (u, v, w)."""
    u, v = _i32(u), _i32(v)
    w, wp = _wptr(w)
    return int(lib().or_cutval(u.shape[0], u, v, wp, np.ascontiguousarray(x, dtype=np.uint8)))


def cutval_packed(num_vertices, u, v, w, words) -> np.ndarray:
    """CutVal of each bit-packed assignment row (vertex t = word t/32, bit t%32)."""
    u, v = _i32(u), _i32(v)
    w, wp = _wptr(w)
    words = np.ascontiguousarray(words, dtype=np.uint32)
    A = words.shape[0]
    out = np.zeros(A, dtype=np.int64)
    lib().or_cutval_packed(A, num_vertices, u.shape[0], u, v, wp, words.reshape(-1), out)
    return out


def bruteforce_maxcut(num_vertices, u, v, w=None):
    """Exhaustive optimum (vertex 0 fixed to side 0); returns (cut, x)."""
    u, v = _i32(u), _i32(v)
    w, wp = _wptr(w)
    x = np.zeros(num_vertices, dtype=np.uint8)
    c = lib().or_bruteforce_maxcut(num_vertices, u.shape[0], u, v, wp, x)
    return int(c), x


# --- Sec. 2.2 -------------------------------------------------------------
def cut_table(n, u, v, w=None) -> np.ndarray:
    """Diagonal of H_C: C(z) for z < 2^n (int64)."""
    u, v = _i32(u), _i32(v)
    w, wp = _wptr(w)
    out = np.zeros(1 << n, dtype=np.int64)
    lib().or_cut_table(n, u.shape[0], u, v, wp, out)
    return out


def qaoa_state(n, C, gamma, beta) -> np.ndarray:
    """QAOA ansatz state (complex128, 2^n) for angle vectors gamma, beta."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    psi = np.zeros(1 << n, dtype=np.complex128)
    lib().or_qaoa_state(n, np.ascontiguousarray(C, dtype=np.int64), gamma.shape[0], gamma, beta, psi)
    return psi


def qaoa_unapply(n, C, gamma, beta, psi) -> np.ndarray:
    """Apply the inverse of the ansatz circuit to psi (returns a new array)."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    out = np.array(psi, dtype=np.complex128, copy=True)
    lib().or_qaoa_unapply(n, np.ascontiguousarray(C, dtype=np.int64), gamma.shape[0], gamma, beta, out)
    return out


def expectation(n, psi, C) -> float:
    """<psi|H_C|psi> with a pairwise sum."""
    return float(lib().or_expectation(n, np.ascontiguousarray(psi, dtype=np.complex128),
                                      np.ascontiguousarray(C, dtype=np.int64)))


def free_mask(n, u, v, w=None) -> int:
    """Vertices without an edge of positive weight inside the subgraph (bit j
    = local vertex j): the state is exactly invariant under flipping them."""
    u, v = _i32(u), _i32(v)
    wa, wp = _wptr(w)
    return int(lib().or_free_mask(n, u.shape[0], u, v, wp))


def tie_rank(x, m) -> int:
    """Rank of index x inside a tie group of 2^m strings (or_topk's order)."""
    return int(lib().or_tie_rank(int(x), int(m)))


def topk(n, psi, k, canonical=True, free=0):
    """Top-k by probability (Sec. 3.3.2) with the tie order of or_topk (tie
    groups from the free-vertex mask `free`, see free_mask); returns
    (idx uint32[k], prob float64[k], k_eff)."""
    idx = np.zeros(k, dtype=np.uint32)
    prob = np.zeros(k, dtype=np.float64)
    ke = lib().or_topk(n, np.ascontiguousarray(psi, dtype=np.complex128), k, int(canonical), int(free), idx, prob)
    return idx, prob, int(ke)


def gradient(n, C, gamma, beta):
    """(E, dE/dgamma, dE/dbeta) by the adjoint sweep."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    beta = np.ascontiguousarray(beta, dtype=np.float64)
    p = gamma.shape[0]
    E = np.zeros(1, dtype=np.float64)
    dg = np.zeros(p, dtype=np.float64)
    db = np.zeros(p, dtype=np.float64)
    lib().or_gradient(n, np.ascontiguousarray(C, dtype=np.int64), p, gamma, beta,
                      E.ctypes.data_as(ct.c_void_p), dg, db)
    return float(E[0]), dg, db


def cold_start(p):
    g = np.zeros(p, dtype=np.float64)
    b = np.zeros(p, dtype=np.float64)
    lib().or_cold_start(p, g, b)
    return g, b


def adam_solve(n, C_table, gamma, beta, T, lr=0.05, b1=0.9, b2=0.999, eps=1e-8):
    """Adam ascent on E for T steps; returns (gamma, beta, E_hist[T+1])."""
    g = np.array(gamma, dtype=np.float64, copy=True)
    b = np.array(beta, dtype=np.float64, copy=True)
    hist = np.zeros(T + 1, dtype=np.float64)
    lib().or_adam_solve(n, np.ascontiguousarray(C_table, dtype=np.int64), g.shape[0], T, lr, b1, b2,
                        eps, g, b, hist.ctypes.data_as(ct.c_void_p))
    return g, b, hist


def adam_update(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8, maximise=True):
    """One Adam step in place on float64 arrays."""
    lib().or_adam_update(theta.size, theta, np.ascontiguousarray(grad, dtype=np.float64), m, v, t,
                         lr, b1, b2, eps, 1.0 if maximise else -1.0)


# --- batches ----------------------------------------------------------------
def _batch_arrays(sub_n, sub_edges):
    nq = _i32(sub_n)
    eoff = np.zeros(len(sub_edges) + 1, dtype=np.int64)
    us, vs, ws = [], [], []
    for i, (u, v, w) in enumerate(sub_edges):
        eoff[i + 1] = eoff[i] + len(u)
        us.append(_i32(u))
        vs.append(_i32(v))
        ws.append(_i32(w))
    cat = (lambda a: np.concatenate(a) if a else np.zeros(0, np.int32))
    return nq, eoff, _i32(cat(us)), _i32(cat(vs)), _i32(cat(ws))


def eval_batch(sub_n, sub_edges, gamma, beta, k=0, canonical=True):
    """E_b and top-k for every subgraph at fixed angles ([B, p] arrays)."""
    nq, eoff, u, v, w = _batch_arrays(sub_n, sub_edges)
    B = nq.shape[0]
    gamma = np.ascontiguousarray(gamma, dtype=np.float64).reshape(B, -1)
    beta = np.ascontiguousarray(beta, dtype=np.float64).reshape(B, -1)
    p = gamma.shape[1]
    E = np.zeros(B, dtype=np.float64)
    idx = np.zeros(max(B * k, 1), dtype=np.uint32)
    prob = np.zeros(max(B * k, 1), dtype=np.float64)
    lib().or_eval_batch(B, nq, eoff, u, v, w.ctypes.data_as(ct.c_void_p), p, gamma.reshape(-1),
                        beta.reshape(-1), E, k, int(canonical), idx, prob)
    return E, idx[:B * k].reshape(B, k), prob[:B * k].reshape(B, k)


def solve_batch(sub_n, sub_edges, gamma0, beta0, T, k, lr=0.05, b1=0.9, b2=0.999, eps=1e-8,
                canonical=True):
    """Plain method per subgraph: Adam for T steps, then E and top-k."""
    nq, eoff, u, v, w = _batch_arrays(sub_n, sub_edges)
    B = nq.shape[0]
    g = np.array(gamma0, dtype=np.float64, copy=True).reshape(B, -1)
    b = np.array(beta0, dtype=np.float64, copy=True).reshape(B, -1)
    p = g.shape[1]
    E = np.zeros(B, dtype=np.float64)
    idx = np.zeros(max(B * k, 1), dtype=np.uint32)
    prob = np.zeros(max(B * k, 1), dtype=np.float64)
    gf, bf = g.reshape(-1).copy(), b.reshape(-1).copy()
    lib().or_solve_batch(B, nq, eoff, u, v, w.ctypes.data_as(ct.c_void_p), p, T, lr, b1, b2, eps,
                         gf, bf, E, k, int(canonical), idx, prob)
    return gf.reshape(B, p), bf.reshape(B, p), E, idx[:B * k].reshape(B, k), prob[:B * k].reshape(B, k)


# --- Sec. 3.2, Alg. 1 ---------------------------------------------------------
def partition_equal(num_vertices, N):
    start = np.zeros(num_vertices + 1, dtype=np.int32)
    size = np.zeros(num_vertices + 1, dtype=np.int32)
    M = lib().or_partition_equal(num_vertices, N, start, size)
    return start[:M].copy(), size[:M].copy()


def partition_chain(num_vertices, sizes):
    sizes = _i32(sizes)
    start = np.zeros(sizes.shape[0], dtype=np.int32)
    size = np.zeros(sizes.shape[0], dtype=np.int32)
    M = lib().or_partition_chain(num_vertices, sizes.shape[0], sizes, start, size)
    if M < 0:
        raise ValueError("not enough sizes to cover the graph")
    return start[:M].copy(), size[:M].copy()


def induced_edges(u, v, w, start, size):
    """GetSubgraph of Alg. 1: edges with both endpoints in [start, start+size),
    as local ids (a scan over all of E, as the algorithm is written)."""
    u, v = np.asarray(u), np.asarray(v)
    w = np.ones_like(u) if w is None else np.asarray(w)
    out_u, out_v, out_w = [], [], []
    for e in range(u.shape[0]):
        if start <= u[e] < start + size and start <= v[e] < start + size:
            out_u.append(u[e] - start)
            out_v.append(v[e] - start)
            out_w.append(w[e])
    return _i32(out_u), _i32(out_v), _i32(out_w)


# --- Sec. 3.4, Alg. 2 ---------------------------------------------------------
def merge(num_vertices, start, size, u, v, w, cand, W=0):
    """Merge of candidate sets (exhaustive when W <= 0, else a beam of width
    W). cand is [M, K] uint32 with UINT32_MAX padding. Returns
    (best_cut, best_x uint8[nV], digits int32[M], leaves)."""
    start, size = _i32(start), _i32(size)
    u, v = _i32(u), _i32(v)
    w, wp = _wptr(w)
    cand = np.ascontiguousarray(cand, dtype=np.uint32)
    M, K = cand.shape
    x = np.zeros(num_vertices, dtype=np.uint8)
    digits = np.zeros(M, dtype=np.int32)
    leaves = ct.c_double(0.0)
    best = lib().or_merge(num_vertices, M, start, size, u.shape[0], u, v, wp, K,
                          cand.reshape(-1), int(W), x, digits, ct.byref(leaves))
    if best < 0:
        raise ValueError("invalid merge input")
    return int(best), x, digits, leaves.value


# --- angle predictor (learned warm start) ------------------------------------
def mlp_num_params(in_dim, hidden, out_dim) -> int:
    return int(lib().or_mlp_num_params(in_dim, hidden, out_dim))


def mlp_forward(params, X, hidden, out_dim):
    """FP64 MLP forward: X [B, in] -> Y [B, out]."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    B, in_dim = X.shape
    Y = np.zeros((B, out_dim), dtype=np.float64)
    lib().or_mlp_forward(B, in_dim, hidden, out_dim, np.ascontiguousarray(params, dtype=np.float64),
                         X.reshape(-1), Y.reshape(-1))
    return Y


def mlp_loss_grad(params, X, T, hidden):
    """(mean squared error, gradient) of the MLP on (X, T)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    B, in_dim = X.shape
    out_dim = T.shape[1]
    G = np.zeros(mlp_num_params(in_dim, hidden, out_dim), dtype=np.float64)
    loss = lib().or_mlp_loss_grad(B, in_dim, hidden, out_dim, np.ascontiguousarray(params, dtype=np.float64),
                                  X.reshape(-1), T.reshape(-1), G)
    return float(loss), G
