"""GPU parity of the angle predictor's forward/backward kernels and of the
Adam step against the FP64 oracle.

Tolerances: forward outputs |dy| <= 1e-4 max(1, |y|) (FP32 sums of <= 128
terms of O(1) values); gradient |dg| <= 1e-4 max(1, max |g|) and loss
relative 1e-5."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_26232_amd import _abi

pytestmark = pytest.mark.gpu


def _ptr(t):
    return int(t.data_ptr())


@pytest.mark.parametrize("B,in_dim,H,out", [(1, 18, 128, 6), (37, 18, 128, 6), (300, 5, 64, 3), (8, 64, 256, 64)])
def test_mlp_forward_backward(B, in_dim, H, out):
    rng = np.random.default_rng(B + H)
    npar = _abi.qaoa_mlp_num_params(in_dim, H, out)
    assert npar == oracle.mlp_num_params(in_dim, H, out)
    P = rng.normal(0, 1.0 / np.sqrt(max(in_dim, H)), npar)
    X = rng.normal(0, 1, (B, in_dim)).astype(np.float32)
    T = rng.normal(0, 1, (B, out)).astype(np.float32)
    dev = "cuda"
    dP = torch.as_tensor(P, device=dev)
    dX = torch.as_tensor(X, device=dev)
    dT = torch.as_tensor(T, device=dev)
    dY = torch.empty((B, out), dtype=torch.float32, device=dev)
    dA = torch.empty((B, 2 * H), dtype=torch.float32, device=dev)
    sb = _abi.qaoa_mlp_scratch_bytes(B, in_dim, H, out)
    dS = torch.empty(sb, dtype=torch.uint8, device=dev)
    dG = torch.empty(npar, dtype=torch.float64, device=dev)
    dL = torch.empty(1, dtype=torch.float64, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    _abi.qaoa_mlp_forward(B, in_dim, H, out, _ptr(dP), _ptr(dX), _ptr(dY), _ptr(dA), s)
    _abi.qaoa_mlp_backward(B, in_dim, H, out, _ptr(dP), _ptr(dX), _ptr(dY), _ptr(dA), _ptr(dT), _ptr(dS), sb,
                           _ptr(dG), _ptr(dL), s)
    torch.cuda.synchronize()
    Y_ref = oracle.mlp_forward(P, X.astype(np.float64), H, out)
    loss_ref, G_ref = oracle.mlp_loss_grad(P, X.astype(np.float64), T.astype(np.float64), H)
    Y = dY.cpu().numpy()
    assert np.max(np.abs(Y - Y_ref) / np.maximum(1, np.abs(Y_ref))) <= 1e-4
    assert abs(float(dL.cpu()[0]) - loss_ref) <= 1e-5 * max(1.0, loss_ref)
    G = dG.cpu().numpy()
    assert np.max(np.abs(G - G_ref)) <= 1e-4 * max(1.0, float(np.abs(G_ref).max()))


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(5)
    n = 3000
    theta = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    dth = torch.as_tensor(theta.copy(), device="cuda")
    dm = torch.zeros(n, dtype=torch.float64, device="cuda")
    dv = torch.zeros(n, dtype=torch.float64, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    for t in range(1, 6):
        g = rng.normal(size=n)
        dg = torch.as_tensor(g, device="cuda")
        for maximise in (1,):
            _abi.qaoa_adam_step(n, _ptr(dth), _ptr(dg), _ptr(dm), _ptr(dv), _ptr(step), 0.01, 0.9, 0.999, 1e-8,
                                maximise, s)
        oracle.adam_update(theta, g, m, v, t, 0.01, maximise=True)
    torch.cuda.synchronize()
    assert int(step.cpu()[0]) == 5
    assert np.max(np.abs(dth.cpu().numpy() - theta)) <= 1e-12


@pytest.mark.parametrize("B,p", [(1, 1), (104, 3), (777, 4)])
def test_warm_angles_and_fallback(B, p):
    """qaoa_warm_angles maps the predictor's standardised outputs to the
    [gamma | beta] angle layout with y * sd + mu rounded in FP32 (bit-exact vs
    numpy's float32 arithmetic); qaoa_keep_better takes, per subgraph, the
    alternative's angles and <C> exactly where its <C> is strictly larger."""
    rng = np.random.default_rng(B * 31 + p)
    Y = rng.normal(size=(B, 2 * p)).astype(np.float32)
    mu = rng.normal(size=2 * p).astype(np.float32)
    sd = rng.uniform(0.1, 2.0, 2 * p).astype(np.float32)
    dY, dmu, dsd = (torch.as_tensor(a, device="cuda") for a in (Y, mu, sd))
    th = torch.full((2 * B * p,), np.nan, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    _abi.qaoa_warm_angles(B, p, _ptr(dY), _ptr(dmu), _ptr(dsd), _ptr(th), s)
    A = (Y * sd + mu).astype(np.float64)  # numpy float32: product, then sum, each rounded
    ref = np.concatenate([A[:, :p].reshape(-1), A[:, p:].reshape(-1)])
    torch.cuda.synchronize()
    assert np.array_equal(th.cpu().numpy(), ref)
    # fallback: ties keep the current start
    E = rng.integers(0, 4, B).astype(np.float64)
    E_alt = rng.integers(0, 4, B).astype(np.float64)
    th_alt = rng.normal(size=2 * B * p)
    dE, dEa, dta = (torch.as_tensor(a.copy(), device="cuda") for a in (E, E_alt, th_alt))
    _abi.qaoa_keep_better(B, p, _ptr(dEa), _ptr(dta), _ptr(dE), _ptr(th), s)
    torch.cuda.synchronize()
    take = E_alt > E
    exp_th = ref.copy().reshape(2, B, p)
    exp_th[:, take, :] = th_alt.reshape(2, B, p)[:, take, :]
    assert np.array_equal(th.cpu().numpy(), exp_th.reshape(-1))
    assert np.array_equal(dE.cpu().numpy(), np.where(take, E_alt, E))
