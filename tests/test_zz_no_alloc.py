"""qaoa_mlp_backward_noalloc (scratch held by the library) against
qaoa_mlp_backward (caller's scratch): identical loss and gradient on two calls
in a row, the second with a smaller batch, and the size limit."""
import numpy as np
import pytest
import torch

from paper_2603_26232_amd import _abi

pytestmark = pytest.mark.gpu


def _ptr(t):
    return int(t.data_ptr())


def _case(B, in_dim, H, out, seed):
    rng = np.random.default_rng(seed)
    npar = _abi.qaoa_mlp_num_params(in_dim, H, out)
    dev = "cuda"
    P = torch.as_tensor(rng.normal(0, 1.0 / np.sqrt(max(in_dim, H)), npar), device=dev)
    X = torch.as_tensor(rng.normal(0, 1, (B, in_dim)).astype(np.float32), device=dev)
    T = torch.as_tensor(rng.normal(0, 1, (B, out)).astype(np.float32), device=dev)
    Y = torch.empty((B, out), dtype=torch.float32, device=dev)
    A = torch.empty((B, 2 * H), dtype=torch.float32, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    _abi.qaoa_mlp_forward(B, in_dim, H, out, _ptr(P), _ptr(X), _ptr(Y), _ptr(A), s)
    return P, X, T, Y, A, npar


def test_noalloc_backward_matches_workspace_backward():
    s = torch.cuda.current_stream().cuda_stream
    shapes = [(5000, 18, 128, 6), (37, 18, 128, 6)]  # the second call is smaller
    for i, (B, in_dim, H, out) in enumerate(shapes):
        print(f"no-alloc MLP backward: call {i}, batch {B}", flush=True)
        P, X, T, Y, A, npar = _case(B, in_dim, H, out, 100 + i)
        sb = _abi.qaoa_mlp_scratch_bytes(B, in_dim, H, out)
        S = torch.empty(sb, dtype=torch.uint8, device="cuda")
        G_ref = torch.full((npar,), np.nan, dtype=torch.float64, device="cuda")
        L_ref = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        _abi.qaoa_mlp_backward(B, in_dim, H, out, _ptr(P), _ptr(X), _ptr(Y), _ptr(A), _ptr(T), _ptr(S), sb,
                               _ptr(G_ref), _ptr(L_ref), s)
        G = torch.full((npar,), np.nan, dtype=torch.float64, device="cuda")
        L = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
        _abi.qaoa_mlp_backward_noalloc(B, in_dim, H, out, _ptr(P), _ptr(X), _ptr(Y), _ptr(A), _ptr(T), _ptr(G),
                                       _ptr(L), s)
        torch.cuda.synchronize()
        assert torch.equal(G, G_ref) and torch.equal(L, L_ref), i
        assert bool(torch.isfinite(G).all())


def test_noalloc_backward_rejects_a_batch_beyond_its_scratch():
    with pytest.raises(_abi.QaoaError) as ei:
        _abi.qaoa_mlp_backward_noalloc(9000, 18, 128, 6, 8, 8, 8, 8, 8, 8, 8, 0)
    assert ei.value.status == 2
