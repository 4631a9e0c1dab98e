"""ctypes binding of libparaqaoa (include/paraqaoa.h), same names as the C ABI.

Argument marshalling only: device pointers and streams are plain integers
(torch's data_ptr() and cuda_stream), host arrays are numpy arrays. A
non-OK status raises QaoaError with the library's message. The library must
have been built (paper_2603_26232_amd.build); there is no fallback.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparaqaoa.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "paraqaoa.h")

QAOA_FLAG_GRADIENT = 0x1
QAOA_FLAG_TOPK_RAW = 0x2
QAOA_FLAG_SKIP_EDGELESS = 0x4
QAOA_FLAG_MIXER_MFMA_F32 = 0x8
QAOA_FLAG_MIXER_MFMA_BF16X3 = 0x10
QAOA_FLAG_MIXER_MFMA_BF16X4 = 0x20
QAOA_FLAG_GRADIENT_INPLACE = 0x40
QAOA_FLAG_GRADIENT_CHECKPOINTS = 0x80
QAOA_FLAG_CONCURRENT_CLASSES = 0x100
QAOA_MAX_QUBITS = 30
QAOA_MAX_DEPTH = 32
QAOA_MAX_K = 64
QAOA_MAX_WEIGHT_SUM = 2047
QAOA_MAX_BEAM = 8192

STATUS = {0: "QAOA_OK", 1: "QAOA_ERR_INVALID_ARG", 2: "QAOA_ERR_OUT_OF_RANGE",
          3: "QAOA_ERR_WORKSPACE_TOO_SMALL", 4: "QAOA_ERR_HIP", 5: "QAOA_ERR_STATE",
          6: "QAOA_ERR_NOT_SUPPORTED"}


class QaoaError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        super().__init__(f"{fn}: {STATUS.get(status, status)}: {detail}")
        self.status = status
        self.detail = detail


_lib = None

_vp = ct.c_void_p
_i32 = ct.c_int32
_i64 = ct.c_int64
_u32 = ct.c_uint32
_f64 = ct.c_double
_st = ct.c_int  # qaoa_status_t


def lib() -> ct.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ct.CDLL(LIB_PATH)
        sig = {
            "qaoa_workspace_bytes": [_i32, _vp, _vp, _vp, _i32, _i32, _u32, _vp],
            "qaoa_batch_create": [_i32, _vp, _vp, _vp, _vp, _vp, _i32, _i32, _u32, _vp, ct.c_size_t, _vp, _vp],
            "qaoa_batch_destroy": [_vp],
            "qaoa_apply_layers": [_vp, _i32, _vp, _vp, _vp],
            "qaoa_expectation": [_vp, _vp, _vp],
            "qaoa_topk": [_vp, _i32, _vp, _vp, _vp],
            "qaoa_expectation_grad": [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp],
            "qaoa_adam_step": [_i32, _vp, _vp, _vp, _vp, _vp, _f64, _f64, _f64, _f64, _i32, _vp],
            "qaoa_optimize": [_vp, _i32, _i32, _vp, _vp, _vp, _vp, _f64, _f64, _f64, _f64, _vp, _vp],
            "maxcut_eval": [_i32, _i64, _vp, _vp, _vp, _i64, _vp, _vp, _vp],
            "qaoa_merge_workspace_bytes": [_i32, _i32, _i64, _i32, _i32, _vp],
            "qaoa_merge_beam": [_i32, _i32, _vp, _vp, _i64, _vp, _vp, _vp, _i32, _vp, _i32, _vp,
                                ct.c_size_t, _vp, _vp, _vp],
            "qaoa_mlp_num_params": [_i32, _i32, _i32, _vp],
            "qaoa_mlp_scratch_bytes": [_i32, _i32, _i32, _i32, _vp],
            "qaoa_mlp_forward": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp],
            "qaoa_mlp_backward": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, ct.c_size_t, _vp, _vp, _vp],
            "qaoa_mlp_backward_noalloc": [_i32, _i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp],
            "qaoa_warm_angles": [_i32, _i32, _vp, _vp, _vp, _vp, _vp],
            "qaoa_keep_better": [_i32, _i32, _vp, _vp, _vp, _vp, _vp],
            "qaoa_state_offset": [_vp, _i32, _vp],
            "qaoa_gradient_checkpoints": [_vp, _vp],
            "qaoa_profile_enable": [_i32],
            "qaoa_profile_read": [ct.c_char_p, _vp, _vp, _vp],
            "qaoa_profile_select": [ct.c_char_p],
            "qaoa_tune_group_split": [_i32, _i32, _vp],
        }
        for name, args in sig.items():
            if not hasattr(L, name):
                continue
            f = getattr(L, name)
            f.argtypes = args
            f.restype = _st
        L.qaoa_status_string.argtypes = [_st]
        L.qaoa_status_string.restype = ct.c_char_p
        L.qaoa_last_error.argtypes = []
        L.qaoa_last_error.restype = ct.c_char_p
        _lib = L
    return _lib


def _call(name: str, *args) -> None:
    L = lib()
    s = getattr(L, name)(*args)
    if s != 0:
        raise QaoaError(name, s, (L.qaoa_last_error() or b"").decode())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_vp)


def _ai32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


def _ai64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int64)


def header_functions() -> list:
    """Function names declared in include/paraqaoa.h."""
    import re
    txt = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"^\s*(?:qaoa_status_t|const char\*)\s+(\w+)\s*\(", txt, re.M)))


# --------------------------------------------------------------------------- ABI
def qaoa_status_string(status: int) -> str:
    return lib().qaoa_status_string(status).decode()


def qaoa_last_error() -> str:
    return (lib().qaoa_last_error() or b"").decode()


def qaoa_workspace_bytes(B, num_qubits, edge_offsets, edge_w, max_p, max_k, flags) -> int:
    nq, eo, w = _ai32(num_qubits), _ai64(edge_offsets), _ai32(edge_w)
    out = ct.c_size_t(0)
    _call("qaoa_workspace_bytes", B, _np_ptr(nq), _np_ptr(eo), _np_ptr(w), max_p, max_k, flags,
          ct.byref(out))
    return int(out.value)


def qaoa_batch_create(B, num_qubits, edge_offsets, edge_u, edge_v, edge_w, max_p, max_k, flags,
                      d_workspace: int, workspace_bytes: int, stream: int) -> int:
    nq, eo = _ai32(num_qubits), _ai64(edge_offsets)
    u, v, w = _ai32(edge_u), _ai32(edge_v), _ai32(edge_w)
    h = _vp(0)
    _call("qaoa_batch_create", B, _np_ptr(nq), _np_ptr(eo), _np_ptr(u), _np_ptr(v), _np_ptr(w),
          max_p, max_k, flags, _vp(d_workspace), workspace_bytes, _vp(stream), ct.byref(h))
    return int(h.value)


def qaoa_batch_destroy(h: int) -> None:
    _call("qaoa_batch_destroy", _vp(h))


def qaoa_apply_layers(h: int, p: int, d_gamma: int, d_beta: int, stream: int) -> None:
    _call("qaoa_apply_layers", _vp(h), p, _vp(d_gamma), _vp(d_beta), _vp(stream))


def qaoa_expectation(h: int, d_out: int, stream: int) -> None:
    _call("qaoa_expectation", _vp(h), _vp(d_out), _vp(stream))


def qaoa_topk(h: int, k: int, d_idx: int, d_prob: int, stream: int) -> None:
    _call("qaoa_topk", _vp(h), k, _vp(d_idx), _vp(d_prob), _vp(stream))


def qaoa_expectation_grad(h: int, p: int, d_gamma: int, d_beta: int, d_E: int, d_dgamma: int,
                          d_dbeta: int, stream: int) -> None:
    _call("qaoa_expectation_grad", _vp(h), p, _vp(d_gamma), _vp(d_beta), _vp(d_E), _vp(d_dgamma),
          _vp(d_dbeta), _vp(stream))


def qaoa_adam_step(count: int, d_theta: int, d_grad: int, d_m: int, d_v: int, d_step: int, lr: float,
                   beta1: float, beta2: float, eps: float, maximise: int, stream: int) -> None:
    _call("qaoa_adam_step", count, _vp(d_theta), _vp(d_grad), _vp(d_m), _vp(d_v), _vp(d_step), lr,
          beta1, beta2, eps, maximise, _vp(stream))


def qaoa_optimize(h: int, p: int, iters: int, d_theta: int, d_m: int, d_v: int, d_step: int, lr: float,
                  beta1: float, beta2: float, eps: float, d_E: int, stream: int) -> None:
    _call("qaoa_optimize", _vp(h), p, iters, _vp(d_theta), _vp(d_m), _vp(d_v), _vp(d_step), lr, beta1, beta2, eps,
          _vp(d_E), _vp(stream))


def maxcut_eval(num_vertices: int, num_edges: int, d_u: int, d_v: int, d_w, num_assign: int,
                d_assign: int, d_cut: int, stream: int) -> None:
    _call("maxcut_eval", num_vertices, num_edges, _vp(d_u), _vp(d_v), _vp(d_w or 0), num_assign,
          _vp(d_assign), _vp(d_cut), _vp(stream))


def qaoa_merge_workspace_bytes(num_vertices, M, num_edges, K, W) -> int:
    out = ct.c_size_t(0)
    _call("qaoa_merge_workspace_bytes", num_vertices, M, num_edges, K, W, ct.byref(out))
    return int(out.value)


def qaoa_merge_beam(num_vertices, M, h_start, h_size, num_edges, h_u, h_v, h_w, K, d_cand: int, W,
                    d_workspace: int, workspace_bytes: int, d_best_assign: int, d_best_cut: int,
                    stream: int) -> None:
    st, sz = _ai32(h_start), _ai32(h_size)
    u, v, w = _ai32(h_u), _ai32(h_v), _ai32(h_w)
    _call("qaoa_merge_beam", num_vertices, M, _np_ptr(st), _np_ptr(sz), num_edges, _np_ptr(u),
          _np_ptr(v), _np_ptr(w), K, _vp(d_cand), W, _vp(d_workspace), workspace_bytes,
          _vp(d_best_assign), _vp(d_best_cut), _vp(stream))


def qaoa_mlp_num_params(in_dim: int, hidden: int, out_dim: int) -> int:
    out = ct.c_int64(0)
    _call("qaoa_mlp_num_params", in_dim, hidden, out_dim, ct.byref(out))
    return int(out.value)


def qaoa_mlp_scratch_bytes(batch: int, in_dim: int, hidden: int, out_dim: int) -> int:
    out = ct.c_size_t(0)
    _call("qaoa_mlp_scratch_bytes", batch, in_dim, hidden, out_dim, ct.byref(out))
    return int(out.value)


def qaoa_mlp_forward(batch, in_dim, hidden, out_dim, d_params, d_x, d_y, d_act, stream) -> None:
    _call("qaoa_mlp_forward", batch, in_dim, hidden, out_dim, _vp(d_params), _vp(d_x), _vp(d_y), _vp(d_act),
          _vp(stream))


def qaoa_mlp_backward(batch, in_dim, hidden, out_dim, d_params, d_x, d_y, d_act, d_target, d_scratch,
                      scratch_bytes, d_grad, d_loss, stream) -> None:
    _call("qaoa_mlp_backward", batch, in_dim, hidden, out_dim, _vp(d_params), _vp(d_x), _vp(d_y), _vp(d_act),
          _vp(d_target), _vp(d_scratch), scratch_bytes, _vp(d_grad), _vp(d_loss), _vp(stream))


def qaoa_warm_angles(B: int, p: int, d_y: int, d_mu: int, d_sd: int, d_theta: int, stream: int) -> None:
    _call("qaoa_warm_angles", B, p, _vp(d_y), _vp(d_mu), _vp(d_sd), _vp(d_theta), _vp(stream))


def qaoa_keep_better(B: int, p: int, d_E_alt: int, d_theta_alt: int, d_E: int, d_theta: int, stream: int) -> None:
    _call("qaoa_keep_better", B, p, _vp(d_E_alt), _vp(d_theta_alt), _vp(d_E), _vp(d_theta), _vp(stream))


def qaoa_mlp_backward_noalloc(batch, in_dim, hidden, out_dim, d_params, d_x, d_y, d_act, d_target, d_grad,
                              d_loss, stream) -> None:
    _call("qaoa_mlp_backward_noalloc", batch, in_dim, hidden, out_dim, _vp(d_params), _vp(d_x), _vp(d_y),
          _vp(d_act), _vp(d_target), _vp(d_grad), _vp(d_loss), _vp(stream))


def qaoa_gradient_checkpoints(h: int) -> bool:
    out = ct.c_int32(0)
    _call("qaoa_gradient_checkpoints", _vp(h), ct.byref(out))
    return bool(out.value)


def qaoa_state_offset(h: int, b: int) -> int:
    out = ct.c_size_t(0)
    _call("qaoa_state_offset", _vp(h), b, ct.byref(out))
    return int(out.value)


def qaoa_profile_enable(on: int) -> None:
    _call("qaoa_profile_enable", int(on))


def qaoa_tune_group_split(n: int, sizes) -> None:
    """Strided group sizes for n-qubit subgraphs of batches created from now
    on (empty / None = default split)."""
    arr = np.ascontiguousarray(sizes if sizes else [0], dtype=np.int32)
    _call("qaoa_tune_group_split", int(n), len(sizes) if sizes else 0, arr.ctypes.data_as(ct.c_void_p))


def qaoa_profile_select(kernel) -> None:
    """Time only `kernel` (None = every kernel)."""
    _call("qaoa_profile_select", None if kernel is None else kernel.encode())


def qaoa_profile_read(kernel: str):
    """(launches, total_ms, algorithmic_bytes) of a kernel since profiling began."""
    n = ct.c_int64(0)
    ms = ct.c_double(0.0)
    by = ct.c_double(0.0)
    _call("qaoa_profile_read", kernel.encode(), ct.byref(n), ct.byref(ms), ct.byref(by))
    return int(n.value), float(ms.value), float(by.value)
