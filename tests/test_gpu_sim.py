"""GPU parity of the batched simulation against the FP64 oracle.

Tolerances (from the FP32-amplitude / FP64-accumulation design):
  amplitudes  max |psi_gpu - psi_oracle| <= 1e-5 (global phase included),
              and the whole error vector's 2-norm <= 1e-5 (psi has norm 1;
              FP32 rounding over p(n+1) gate layers stays near 1e-6)
  <C>         |dE| <= 1e-5 * max(1, |E_oracle|)
  gradient    |dg| <= 1e-4 * max(1, max |g_oracle|)
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2603_26232_amd import synth
from paper_2603_26232_amd.batch import QaoaBatch, idx_to_uint32

pytestmark = pytest.mark.gpu

AMP_TOL = 1e-5
L2_TOL = 1e-5
E_TOL = 1e-5
G_TOL = 1e-4


def _subgraphs(sizes, seed, p_edge=0.4, weighted=False):
    out = []
    for i, n in enumerate(sizes):
        if n >= 2:
            g = synth.erdos_renyi(n, p_edge, seed + i)
            w = synth.random_weights(g.num_edges, seed + 50 + i, 1, 5) if weighted else g.w
            # keep the weight sum inside the phase-table limit
            while w.sum() > 2047:
                w = np.maximum(1, w // 2).astype(np.int32)
            out.append((g.u, g.v, w))
        else:
            out.append((np.zeros(0, np.int32),) * 3)
    return out


def _check_states(bt, sizes, edges, gamma, beta):
    E = bt.expectation().cpu().numpy()
    torch.cuda.synchronize()
    for b, n in enumerate(sizes):
        u, v, w = edges[b]
        C = oracle.cut_table(n, u, v, w)
        ref = oracle.qaoa_state(n, C, gamma[b], beta[b])
        got = bt.state(b).cpu().numpy().astype(np.complex128)
        err = np.abs(got - ref)
        assert err.max() <= AMP_TOL, f"b={b} n={n} max amp err {err.max():.2e}"
        assert np.sqrt((err ** 2).sum()) <= L2_TOL, f"b={b} n={n} l2 err {np.sqrt((err**2).sum()):.2e}"
        e_ref = oracle.expectation(n, ref, C)
        assert abs(E[b] - e_ref) <= E_TOL * max(1.0, abs(e_ref)), (b, n, E[b], e_ref)


@pytest.mark.parametrize("sizes,p,seed,weighted", [
    ([12], 2, 0, False),                    # the single-subgraph parity case (n = 12, p = 2)
    ([1, 2, 3, 5, 11], 3, 1, True),         # small-n whole-state kernel, ragged
    ([13, 14, 15, 16], 2, 2, False),        # one strided group of 1..4 qubits
    ([17, 20], 3, 3, True),                 # strided group of 5 and 8 qubits
    ([21, 22], 1, 4, False),                # two strided groups
    ([12, 13, 20, 21, 5], 4, 5, True),      # every class in one batch
])
def test_states_and_expectation(sizes, p, seed, weighted):
    edges = _subgraphs(sizes, 100 + seed, weighted=weighted)
    gamma, beta = synth.uniform_angles(1000 + seed, p, batch=len(sizes))
    bt = QaoaBatch(sizes, edges, max_p=p, max_k=8)
    bt.apply_layers(gamma, beta)
    _check_states(bt, sizes, edges, gamma, beta)
    bt.close()


def test_zero_angles_give_half_the_edges():
    sizes = [4, 12, 16, 23]
    edges = _subgraphs(sizes, 7, p_edge=0.5, weighted=True)
    bt = QaoaBatch(sizes, edges, max_p=2, max_k=4)
    z = np.zeros((len(sizes), 2))
    bt.apply_layers(z, z)
    E = bt.expectation().cpu().numpy()
    for b in range(len(sizes)):
        assert abs(E[b] - edges[b][2].sum() / 2) <= 1e-6 * max(1, edges[b][2].sum())
        st = bt.state(b).cpu().numpy()
        assert np.max(np.abs(st - 2.0 ** (-sizes[b] / 2))) <= 1e-6
    bt.close()


def test_beta_zero_closed_form_at_24_qubits():
    # beta = 0: psi(z) = 2^{-n/2} exp(-i C(z) sum gamma), checked on samples
    n = 24
    g = synth.erdos_renyi(n, 0.3, 11)
    C = oracle.cut_table(n, g.u, g.v)
    gam = np.array([[0.4, -0.9, 1.3]])
    bt = QaoaBatch([n], [(g.u, g.v, g.w)], max_p=3, max_k=4)
    bt.apply_layers(gam, np.zeros((1, 3)))
    st = bt.state(0).cpu().numpy()
    zs = np.random.default_rng(0).integers(0, 1 << n, 4096)
    ref = 2.0 ** (-n / 2) * np.exp(-1j * C[zs] * gam.sum())
    assert np.max(np.abs(st[zs] - ref)) <= 1e-6
    bt.close()


def test_p1_closed_form_on_3_regular_26_qubits():
    # a full-size subgraph (26 qubits, 2^26 amplitudes); p = 1 expectation of a
    # triangle-free-or-not unweighted graph has the closed form of Wang et al.
    n = 26
    g = synth.random_regular3(n, 3)
    gam, bet = 0.61, 0.37
    bt = QaoaBatch([n], [(g.u, g.v, g.w)], max_p=1, max_k=4)
    bt.apply_layers(np.array([[gam]]), np.array([[bet]]))
    E = float(bt.expectation().cpu()[0])
    adj = [set() for _ in range(n)]
    for a, b in zip(g.u, g.v):
        adj[a].add(b)
        adj[b].add(a)
    ref = 0.0
    for a, b in zip(g.u, g.v):
        f = len(adj[a] & adj[b])
        du, dv = len(adj[a]) - 1, len(adj[b]) - 1
        ref += (0.5 + 0.25 * math.sin(4 * bet) * math.sin(gam) * (math.cos(gam) ** du + math.cos(gam) ** dv)
                - 0.25 * math.sin(2 * bet) ** 2 * math.cos(gam) ** (du + dv - 2 * f) * (1 - math.cos(2 * gam) ** f))
    assert abs(E - ref) <= E_TOL * max(1.0, abs(ref))
    # norm and complement symmetry hold at any size
    st = bt.state(0)
    pr = (st.real.double() ** 2 + st.imag.double() ** 2)
    assert abs(float(pr.sum()) - 1.0) <= 1e-5
    zs = torch.randint(0, 1 << n, (8192,), device=st.device)
    comp = ((1 << n) - 1) ^ zs
    assert float((pr[zs] - pr[comp]).abs().max()) <= 1e-12
    bt.close()


def test_determinism():
    sizes = [20, 14, 9]
    edges = _subgraphs(sizes, 31)
    gamma, beta = synth.uniform_angles(77, 3, batch=3)
    bt = QaoaBatch(sizes, edges, max_p=3, max_k=8, gradient=True)
    outs = []
    for _ in range(2):
        bt.apply_layers(gamma, beta)
        E = bt.expectation().clone()
        idx, prob = bt.topk(8)
        st = bt.state(0).clone()
        Eg, dg, db = bt.expectation_grad(gamma, beta)
        outs.append((E, idx.clone(), prob.clone(), st, Eg.clone(), dg.clone(), db.clone()))
    torch.cuda.synchronize()
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    bt.close()


def _tie_group(z, n, free, canonical):
    """(representative, index inside the group, m) of z's tie group, as the
    oracle's top-k defines them (free vertices and the complement move)."""
    full = (1 << n) - 1
    fm = free & ~1 if canonical else free
    halves = 2 if ((free & 1 if canonical else 1) and free != full) else 1
    m = bin(fm).count("1") + (1 if halves == 2 else 0)
    rep, half = z & ~fm, 0
    if halves == 2:
        r2 = (((~z) & full) ^ (1 if canonical else 0)) & ~fm
        if r2 < rep:
            rep, half = r2, 1
    x, t = 0, 0
    for j in range(n):
        if fm >> j & 1:
            x |= ((z >> j) & 1) << t
            t += 1
    return rep, ((x << 1) | half) if halves == 2 else x, m


def _accept_topk(got_idx, got_prob, psi, k, canonical=True, free=0, eps=1e-5):
    """Tolerance-aware acceptance of a GPU top-k list against the FP64 state:
    distinct (canonical) indices, every pick within 2*delta of the oracle's
    k-th probability, adjacent pairs in oracle order unless within 2*delta;
    each tie group (free-vertex mask `free`) appears as one contiguous block
    of its strings in the oracle's rank order 0, 1, 2, ...; and when no two
    different groups come within 2*delta of each other at the list's
    boundaries, the list equals the oracle's."""
    n_amp = psi.shape[0]
    n = n_amp.bit_length() - 1
    pr = np.abs(psi) ** 2
    delta = eps * (2 * np.abs(psi).max() + eps)
    n_cand = n_amp // 2 if canonical else n_amp
    k_eff = min(k, n_cand)
    k2 = min(n_cand, k + 64)
    oi, op, _ = oracle.topk(n, psi, k2, canonical, free)
    oi = oi.astype(np.int64)
    kth = pr[oi[k_eff - 1]]
    gi = got_idx[:k_eff].astype(np.int64)
    assert np.all(got_idx[k_eff:] == 0xFFFFFFFF) and np.all(got_prob[k_eff:] == -1.0)
    assert len(set(gi.tolist())) == k_eff
    if canonical:
        assert np.all(gi % 2 == 0)
    assert np.all(pr[gi] >= kth - 2 * delta)
    for a, b in zip(gi[:-1], gi[1:]):
        assert pr[a] > pr[b] - 2 * delta or (abs(pr[a] - pr[b]) <= 2 * delta)
    assert np.all(np.abs(got_prob[:k_eff] - pr[gi]) <= 2 * delta)
    # groups: contiguous blocks in rank order
    seen, cur, nxt = set(), None, 0
    for z in gi.tolist():
        rep, x, m = _tie_group(z, n, free, canonical)
        if rep != cur:
            assert rep not in seen, "a tie group appears in two blocks"
            seen.add(rep)
            cur, nxt = rep, 0
        assert oracle.tie_rank(x, m) == nxt, (z, rep, x, m, nxt)
        nxt += 1
    # clear boundaries between the groups that fill the list (and the next
    # one): identical lists
    full = (1 << n) - 1
    fm = free & ~1 if canonical else free
    halves = 2 if ((free & 1 if canonical else 1) and free != full) else 1
    z = np.arange(0, n_amp, 2 if canonical else 1, dtype=np.int64)
    keep = (z & fm) == 0
    if halves == 2:
        keep &= z <= ((((~z) & full) ^ (1 if canonical else 0)) & ~fm)
    reps = z[keep]
    reps = reps[np.lexsort((reps, -pr[reps]))]
    size = 1 << (bin(fm).count("1") + (1 if halves == 2 else 0))
    need = min(len(reps), -(-k_eff // size) + 1)
    gaps = np.abs(np.diff(pr[reps[:need]]))
    if gaps.size == 0 or gaps.min() > 2 * delta:
        assert np.array_equal(gi, oi[:k_eff])


@pytest.mark.parametrize("sizes,k,raw,p_edge", [([12], 8, False, 0.4), ([3, 5, 13, 20], 16, False, 0.4),
                                                ([14, 21], 16, True, 0.4), ([2, 4], 64, False, 0.4),
                                                ([14, 21, 9, 17], 16, False, 0.08), ([15, 20, 6], 40, True, 0.06)])
def test_topk(sizes, k, raw, p_edge):
    """Sparse cases have free vertices: their strings come in tie groups."""
    edges = _subgraphs(sizes, 40 + k, p_edge=p_edge)
    p = 3
    gamma, beta = synth.uniform_angles(500 + k, p, batch=len(sizes))
    bt = QaoaBatch(sizes, edges, max_p=p, max_k=k, raw_topk=raw)
    bt.apply_layers(gamma, beta)
    idx, prob = bt.topk(k)
    gi = idx_to_uint32(idx)
    gp = prob.cpu().numpy()
    for b, n in enumerate(sizes):
        u, v, w = edges[b]
        C = oracle.cut_table(n, u, v, w)
        psi = oracle.qaoa_state(n, C, gamma[b], beta[b])
        _accept_topk(gi[b], gp[b], psi, k, canonical=not raw, free=oracle.free_mask(n, u, v, w))
    bt.close()


@pytest.mark.parametrize("memory", ["checkpoints", "inplace"])
@pytest.mark.parametrize("sizes,p,seed", [([6], 1, 0), ([12], 2, 1), ([13, 16], 3, 2), ([20], 3, 3),
                                          ([21, 12, 7], 2, 4), ([22], 3, 5), ([20, 21], 4, 6), ([16, 21], 1, 7)])
def test_gradient(sizes, p, seed, memory):
    """Both gradient memory modes: checkpoints of every forward pass (the
    adjoint sweep reads psi) and in place (the sweep rebuilds psi)."""
    edges = _subgraphs(sizes, 300 + seed, p_edge=0.3, weighted=seed % 2 == 1)
    gamma, beta = synth.uniform_angles(900 + seed, p, batch=len(sizes))
    bt = QaoaBatch(sizes, edges, max_p=p, max_k=4, gradient=True, gradient_memory=memory)
    from paper_2603_26232_amd import _abi
    assert _abi.qaoa_gradient_checkpoints(bt.handle) == (memory == "checkpoints")
    E, dg, db = bt.expectation_grad(gamma, beta)
    E, dg, db = E.cpu().numpy(), dg.cpu().numpy(), db.cpu().numpy()
    for b, n in enumerate(sizes):
        u, v, w = edges[b]
        C = oracle.cut_table(n, u, v, w)
        e_ref, g_ref, b_ref = oracle.gradient(n, C, gamma[b], beta[b])
        scale = max(1.0, float(np.abs(np.concatenate([g_ref, b_ref])).max()))
        assert abs(E[b] - e_ref) <= E_TOL * max(1.0, abs(e_ref))
        assert np.max(np.abs(dg[b] - g_ref)) <= G_TOL * scale, (n, dg[b], g_ref)
        assert np.max(np.abs(db[b] - b_ref)) <= G_TOL * scale, (n, db[b], b_ref)
    # the gradient call consumes the state: top-k needs a fresh apply
    with pytest.raises(Exception):
        bt.topk(4)
    bt.apply_layers(gamma, beta)
    bt.topk(4)
    bt.close()


def test_edgeless_subgraph_gradient_is_zero():
    sizes = [14, 5]
    edges = [(np.zeros(0, np.int32),) * 3] * 2
    gamma, beta = synth.uniform_angles(3, 2, batch=2)
    bt = QaoaBatch(sizes, edges, max_p=2, max_k=4, gradient=True)
    E, dg, db = bt.expectation_grad(gamma, beta)
    assert float(E.abs().max()) == 0.0 and float(dg.abs().max()) == 0.0 and float(db.abs().max()) == 0.0
    bt.close()


def test_skip_edgeless_matches_simulation():
    # edgeless subgraphs in closed form: E = 0, gradient 0, top-k = 0, 2, 4, ...
    sizes = [14, 9, 20, 12]
    edges = _subgraphs(sizes, 61)
    edges[1] = (np.zeros(0, np.int32),) * 3
    edges[2] = (np.zeros(0, np.int32),) * 3
    gamma, beta = synth.uniform_angles(62, 2, batch=len(sizes))
    ref = QaoaBatch(sizes, edges, max_p=2, max_k=8, gradient=True)
    skp = QaoaBatch(sizes, edges, max_p=2, max_k=8, gradient=True, skip_edgeless=True)
    out = []
    for bt in (ref, skp):
        bt.apply_layers(gamma, beta)
        E = bt.expectation().cpu().numpy()
        idx, prob = bt.topk(8)
        Eg, dg, db = bt.expectation_grad(gamma, beta)
        out.append((E, idx_to_uint32(idx), prob.cpu().numpy(), Eg.cpu().numpy(), dg.cpu().numpy(), db.cpu().numpy()))
    (E0, i0, p0, Eg0, dg0, db0), (E1, i1, p1, Eg1, dg1, db1) = out
    assert np.array_equal(E0, E1) and np.array_equal(Eg0, Eg1)
    assert np.array_equal(dg0, dg1) and np.array_equal(db0, db1)
    # subgraphs with edges: identical; edgeless ones: every vertex is free,
    # so simulated and closed form list the one tie group in the same rank
    # order (the oracle's, on the uniform state), with probability 2^-n
    for b in (0, 3):
        assert np.array_equal(i0[b], i1[b]) and np.array_equal(p0[b], p1[b])
    for b, n in ((1, 9), (2, 20)):
        uniform = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
        oi, _, _ = oracle.topk(n, uniform, 8, True, (1 << n) - 1)
        assert np.array_equal(i1[b], oi) and np.array_equal(i0[b], oi)
        assert np.all(p1[b] == np.float32(2.0 ** -n))
        assert np.allclose(p0[b], 2.0 ** -n, rtol=1e-5, atol=0)
    ref.close()
    skp.close()


@pytest.mark.parametrize("n,split", [(21, [1, 8]), (21, [8, 1]), (21, [3, 3, 3]), (22, [6, 4]), (26, [6, 8]),
                                     (26, [8, 6]), (16, [1, 1, 2])])
def test_tuned_group_splits(n, split):
    """Any split of the strided qubits into groups gives the same state."""
    from paper_2603_26232_amd import _abi
    edges = _subgraphs([n], 700 + n, p_edge=0.2)
    gamma, beta = synth.uniform_angles(7000 + n, 2, batch=1)
    _abi.qaoa_tune_group_split(n, split)
    try:
        bt = QaoaBatch([n], edges, max_p=2, max_k=8, gradient=True)
    finally:
        _abi.qaoa_tune_group_split(n, None)
    bt.apply_layers(gamma, beta)
    _check_states(bt, [n], edges, gamma, beta)
    if n > 22:  # the FP64 adjoint on one core takes too long beyond this
        bt.close()
        return
    E, dg, db = bt.expectation_grad(gamma, beta)
    u, v, w = edges[0]
    C = oracle.cut_table(n, u, v, w)
    e_ref, g_ref, b_ref = oracle.gradient(n, C, gamma[0], beta[0])
    scale = max(1.0, float(np.abs(np.concatenate([g_ref, b_ref])).max()))
    assert np.max(np.abs(dg.cpu().numpy()[0] - g_ref)) <= G_TOL * scale
    assert np.max(np.abs(db.cpu().numpy()[0] - b_ref)) <= G_TOL * scale
    bt.close()


def test_wide_cut_tables():
    """Weight sums above 255 use 2-byte cut tables (1 byte otherwise); both
    widths in one batch, tile path and whole-state path."""
    sizes = [16, 21, 10, 14]
    edges = []
    for i, n in enumerate(sizes):
        g = synth.erdos_renyi(n, 0.3, 900 + i)
        w = synth.random_weights(g.num_edges, 950 + i, 10, 20) if i % 2 == 0 else g.w
        while w.sum() > 2047:
            w = np.maximum(1, w // 2).astype(np.int32)
        edges.append((g.u, g.v, w))
    assert edges[0][2].sum() > 255 and edges[1][2].sum() <= 255
    gamma, beta = synth.uniform_angles(9000, 2, batch=len(sizes))
    bt = QaoaBatch(sizes, edges, max_p=2, max_k=8, gradient=True)
    bt.apply_layers(gamma, beta)
    _check_states(bt, sizes, edges, gamma, beta)
    E, dg, db = bt.expectation_grad(gamma, beta)
    for b, n in enumerate(sizes):
        u, v, w = edges[b]
        C = oracle.cut_table(n, u, v, w)
        e_ref, g_ref, b_ref = oracle.gradient(n, C, gamma[b], beta[b])
        scale = max(1.0, float(np.abs(np.concatenate([g_ref, b_ref])).max()))
        assert np.max(np.abs(dg.cpu().numpy()[b] - g_ref)) <= G_TOL * scale
        assert np.max(np.abs(db.cpu().numpy()[b] - b_ref)) <= G_TOL * scale
    bt.close()


def test_host_arrays_reusable_after_create(monkeypatch):
    """qaoa_batch_create stages its host arrays before returning: overwriting
    them right after the call, while the upload still waits behind earlier
    work on the stream, changes nothing."""
    from paper_2603_26232_amd import _abi
    busy_sizes = [24] * 4
    busy = QaoaBatch(busy_sizes, _subgraphs(busy_sizes, 7, p_edge=0.2), max_p=4, max_k=8)
    g4, b4 = synth.uniform_angles(99, 4, batch=4)
    busy.apply_layers(g4, b4)  # queued work ahead of the upload
    sizes = [14, 18]
    edges = _subgraphs(sizes, 321)
    gamma, beta = synth.uniform_angles(4321, 2, batch=len(sizes))
    orig = _abi.qaoa_batch_create

    def create_then_overwrite(B, nq, off, u, v, w, *rest):
        h = orig(B, nq, off, u, v, w, *rest)
        for a in (off, u, v, w):  # (the batch object keeps nq as its sizes)
            a[...] = -1
        return h

    monkeypatch.setattr(_abi, "qaoa_batch_create", create_then_overwrite)
    bt = QaoaBatch(sizes, edges, max_p=2, max_k=8)
    monkeypatch.undo()
    bt.apply_layers(gamma, beta)
    _check_states(bt, sizes, edges, gamma, beta)
    bt.close()
    busy.close()
