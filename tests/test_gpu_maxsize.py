"""The largest subgraph the library takes (30 qubits: 2^29 stored amplitudes,
4 GiB per state) against results that hold at any size, since the FP64 oracle
cannot hold such states:

* <C> at p = 1 on a 3-regular graph against the closed form of Wang et al.
  (Phys. Rev. A 97, 022304), and the adjoint gradient against that closed
  form's derivatives (FP64 central differences of the formula);
* beta = 0: every amplitude is 2^(-n/2) e^(-i C(z) sum gamma), on sampled z,
  with 2-byte cut tables (weight sum above 255);
* the state's norm;
* top-16: the returned probabilities are those of the state at the returned
  indices, in order, and no other canonical index is more probable than the
  16th (the ordering of equal probabilities is not unique, section 3.3.2).
"""
import math

import numpy as np
import pytest
import torch

from paper_2603_26232_amd import synth
from paper_2603_26232_amd.batch import QaoaBatch, idx_to_uint32

pytestmark = pytest.mark.gpu

N = 30


def _p1_closed_form(u, v, n, gam, bet):
    adj = [set() for _ in range(n)]
    for a, b in zip(u, v):
        adj[a].add(b)
        adj[b].add(a)
    e = 0.0
    for a, b in zip(u, v):
        f = len(adj[a] & adj[b])
        du, dv = len(adj[a]) - 1, len(adj[b]) - 1
        e += (0.5 + 0.25 * math.sin(4 * bet) * math.sin(gam) * (math.cos(gam) ** du + math.cos(gam) ** dv)
              - 0.25 * math.sin(2 * bet) ** 2 * math.cos(gam) ** (du + dv - 2 * f) * (1 - math.cos(2 * gam) ** f))
    return e


def _norm(bt):
    """sum |psi|^2 of the whole state, from the stored half (whose amplitudes
    are scaled by sqrt(2)), in FP64 over chunks."""
    red = bt.reduced_state(0)
    tot = 0.0
    chunk = 1 << 26
    for i in range(0, red.numel(), chunk):
        c = red[i:i + chunk]
        tot += float((c.real.double() ** 2 + c.imag.double() ** 2).sum())
    return tot


def test_p1_energy_gradient_norm_at_30_qubits():
    g = synth.random_regular3(N, 5)
    gam, bet = 0.61, 0.37
    bt = QaoaBatch([N], [(g.u, g.v, g.w)], max_p=1, max_k=16, gradient=True)
    print(f"maxsize: n={N}, {g.num_edges} edges, p=1", flush=True)
    bt.apply_layers(np.array([[gam]]), np.array([[bet]]))
    E = float(bt.expectation().cpu()[0])
    ref = _p1_closed_form(g.u, g.v, N, gam, bet)
    assert abs(E - ref) <= 1e-5 * max(1.0, abs(ref)), (E, ref)
    # the stored half holds the whole state's norm (scaled by sqrt(2))
    assert abs(_norm(bt) - 1.0) <= 1e-5
    red = bt.reduced_state(0)
    half = 1 << (N - 1)

    def amp(z):
        # full index z -> stored index (top bit clear), value / sqrt(2)
        zr = torch.where(z >= half, ((1 << N) - 1) ^ z, z)
        return red[zr.to(red.device)] / math.sqrt(2.0)
    # top-16 against the state itself
    idx, prob = bt.topk(16)
    z = torch.as_tensor(idx_to_uint32(idx).astype(np.int64)).view(-1)
    pr_sel = amp(z).abs().double() ** 2
    assert torch.allclose(pr_sel.cpu(), prob.view(-1).double().cpu(), rtol=1e-6, atol=0.0)
    p_all = prob.view(-1).double().cpu().numpy()
    assert np.all(np.diff(p_all) <= 0.0)
    assert np.all(z.numpy() % 2 == 0)  # canonical: bit 0 clear
    kth = float(p_all[-1])
    # probabilities of all stored amplitudes of canonical full indices: a
    # stored index r (top bit clear) is canonical itself when its bit 0 is
    # clear, else through its complement (whose bit 0 is then clear)
    above = 0
    chunk = 1 << 26
    for i in range(0, red.numel(), chunk):
        c = red[i:i + chunk]
        pr = (c.real.float() ** 2 + c.imag.float() ** 2) * 0.5
        above += int((pr > kth * (1.0 + 1e-6)).sum())
    # each stored index stands for one canonical full index, so at most 15
    # may be strictly more probable than the 16th returned
    assert above <= 15, above
    # adjoint gradient against the closed form's derivatives
    Eg, dg, db = bt.expectation_grad(np.array([[gam]]), np.array([[bet]]))
    h = 1e-5
    g_ref = (_p1_closed_form(g.u, g.v, N, gam + h, bet) - _p1_closed_form(g.u, g.v, N, gam - h, bet)) / (2 * h)
    b_ref = (_p1_closed_form(g.u, g.v, N, gam, bet + h) - _p1_closed_form(g.u, g.v, N, gam, bet - h)) / (2 * h)
    scale = max(1.0, abs(g_ref), abs(b_ref))
    assert abs(float(Eg.cpu()[0]) - ref) <= 1e-5 * max(1.0, abs(ref))
    assert abs(float(dg.cpu()[0, 0]) - g_ref) <= 1e-4 * scale, (float(dg.cpu()[0, 0]), g_ref)
    assert abs(float(db.cpu()[0, 0]) - b_ref) <= 1e-4 * scale, (float(db.cpu()[0, 0]), b_ref)
    bt.close()


def test_beta_zero_wide_tables_at_30_qubits():
    # weights 5..12 on ~70 edges: weight sum above 255, so 2-byte cut tables
    g = synth.erdos_renyi(N, 0.16, 9)
    w = synth.random_weights(g.num_edges, 19, 5, 12)
    while w.sum() > 2047:
        w = np.maximum(1, w // 2).astype(np.int32)
    assert w.sum() > 255
    gam = np.array([[0.4, -0.9]])
    bt = QaoaBatch([N], [(g.u, g.v, w)], max_p=2, max_k=4)
    bt.apply_layers(gam, np.zeros((1, 2)))
    red = bt.reduced_state(0)
    zs = np.random.default_rng(3).integers(0, 1 << (N - 1), 8192)
    cut = np.zeros(zs.shape, np.int64)
    for a, b, ww in zip(g.u, g.v, w):
        cut += np.where(((zs >> a) ^ (zs >> b)) & 1, int(ww), 0)
    ref = math.sqrt(2.0) * 2.0 ** (-N / 2) * np.exp(-1j * cut * gam.sum())
    got = red[torch.as_tensor(zs, device=red.device)].cpu().numpy().astype(np.complex128)
    assert np.max(np.abs(got - ref)) <= 1e-6 * math.sqrt(2.0) * 2.0 ** (-N / 2) * 10
    assert abs(_norm(bt) - 1.0) <= 1e-5
    bt.close()
