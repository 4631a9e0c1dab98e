"""Pins for the FP64 oracle: results the paper or the mathematics fixes
independently of the oracle's own loops (closed forms, symmetries, brute
force, dense matrix exponentials, values printed in the paper)."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2603_26232_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_examples.json")


def _edges(pairs):
    u = np.array([a for a, b in pairs], dtype=np.int32)
    v = np.array([b for a, b in pairs], dtype=np.int32)
    return u, v


def ring(n):
    return _edges([(i, (i + 1) % n) if i < (i + 1) % n else ((i + 1) % n, i) for i in range(n)])


def complete(n):
    return _edges([(a, b) for a in range(n) for b in range(a + 1, n)])


def bits_of(z, n):
    return np.array([(z >> j) & 1 for j in range(n)], dtype=np.uint8)


# ---------------------------------------------------------------- Sec. 2.1
def test_cutval_closed_forms():
    # K_n: the best bipartition is balanced, floor(n/2) * ceil(n/2)
    for n in range(2, 10):
        u, v = complete(n)
        best, x = oracle.bruteforce_maxcut(n, u, v)
        assert best == (n // 2) * ((n + 1) // 2)
        assert oracle.cutval(u, v, None, x) == best
    # bipartite graphs: every edge can be cut
    for n in (4, 6, 8, 10):  # even rings
        u, v = ring(n)
        assert oracle.bruteforce_maxcut(n, u, v)[0] == n
    u, v = _edges([(a, b) for a in range(3) for b in range(3, 7)])  # K_{3,4}
    assert oracle.bruteforce_maxcut(7, u, v)[0] == 12
    # odd ring: one edge must stay uncut
    u, v = ring(7)
    assert oracle.bruteforce_maxcut(7, u, v)[0] == 6


def test_cutval_complement_and_weights():
    g = synth.erdos_renyi(30, 0.3, 5)
    w = synth.random_weights(g.num_edges, 11)
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.integers(0, 2, 30).astype(np.uint8)
        c = oracle.cutval(g.u, g.v, w, x)
        assert c == oracle.cutval(g.u, g.v, w, 1 - x)
        # weight-linearity: doubling every weight doubles the cut
        assert oracle.cutval(g.u, g.v, 2 * w, x) == 2 * c


def test_cutval_packed_matches_unpacked():
    g = synth.erdos_renyi(70, 0.1, 3)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, 2, (5, 70)).astype(np.uint8)
    words = np.zeros((5, 3), dtype=np.uint32)
    for a in range(5):
        for t in range(70):
            words[a, t // 32] |= np.uint32(int(xs[a, t]) << (t % 32))
    got = oracle.cutval_packed(70, g.u, g.v, None, words)
    for a in range(5):
        assert got[a] == oracle.cutval(g.u, g.v, None, xs[a])


def test_golden_ar_example():
    gold = json.load(open(GOLDEN))
    ex = gold["approximation_ratio_example"]
    assert ex["cut_alg"] / ex["cut_opt"] == pytest.approx(ex["ar"])
    ex = gold["merge_concatenation_example"]
    assert ex["cut"] / ex["cut_opt"] == pytest.approx(0.75)


# ---------------------------------------------------------------- cut table
@pytest.mark.parametrize("n,p,seed", [(6, 0.5, 0), (9, 0.4, 1), (12, 0.5, 2)])
def test_cut_table_is_cutval_per_bitstring(n, p, seed):
    g = synth.erdos_renyi(n, p, seed)
    w = synth.random_weights(g.num_edges, seed + 7)
    C = oracle.cut_table(n, g.u, g.v, w)
    for z in range(0, 1 << n, max(1, (1 << n) // 97)):
        assert C[z] == oracle.cutval(g.u, g.v, w, bits_of(z, n))
    best, _ = oracle.bruteforce_maxcut(n, g.u, g.v, w)
    assert C.max() == best  # pin 1: max_z C(z) is the brute-force optimum
    # complement symmetry C(z) = C(~z)
    full = (1 << n) - 1
    z = np.arange(1 << n)
    assert np.array_equal(C, C[full ^ z])


# ---------------------------------------------------------------- Sec. 2.2
def _dense_qaoa(n, C, gamma, beta):
    """Independent construction: dense matrices, U_M = expm(-i beta sum_j X_j)
    built from Kronecker products, U_C = diag(exp(-i gamma C))."""
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    I2 = np.eye(2, dtype=np.complex128)
    HM = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for j in range(n):
        op = np.array([[1.0]], dtype=np.complex128)
        # qubit j is bit j of z, i.e. the j-th factor from the right
        for q in reversed(range(n)):
            op = np.kron(op, X if q == j else I2)
        HM += op
    psi = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
    for g_, b_ in zip(gamma, beta):
        psi = np.exp(-1j * g_ * C.astype(np.float64)) * psi
        psi = scipy.linalg.expm(-1j * b_ * HM) @ psi
    return psi


@pytest.mark.parametrize("n,p,seed", [(1, 1, 0), (2, 2, 1), (5, 3, 2), (7, 2, 3), (8, 4, 4)])
def test_state_matches_dense_matrix_exponential(n, p, seed):
    if n >= 2:
        g = synth.erdos_renyi(n, 0.6, seed)
        u, v, w = g.u, g.v, synth.random_weights(g.num_edges, seed)
    else:
        u = v = np.zeros(0, np.int32)
        w = None
    C = oracle.cut_table(n, u, v, w)
    gamma, beta = synth.uniform_angles(100 + seed, p)
    psi = oracle.qaoa_state(n, C, gamma[0], beta[0])
    ref = _dense_qaoa(n, C, gamma[0], beta[0])
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_zero_angles_give_uniform_superposition():
    g = synth.erdos_renyi(10, 0.5, 4)
    C = oracle.cut_table(10, g.u, g.v)
    psi = oracle.qaoa_state(10, C, [0.0, 0.0], [0.0, 0.0])
    assert np.max(np.abs(psi - 2.0 ** -5)) < 1e-15
    assert oracle.expectation(10, psi, C) == pytest.approx(g.num_edges / 2, abs=1e-12)
    w = synth.random_weights(g.num_edges, 9)
    Cw = oracle.cut_table(10, g.u, g.v, w)
    assert oracle.expectation(10, psi, Cw) == pytest.approx(w.sum() / 2, abs=1e-11)


def test_closed_forms_single_operator_kinds():
    n = 9
    g = synth.erdos_renyi(n, 0.5, 8)
    C = oracle.cut_table(n, g.u, g.v)
    gam = np.array([0.3, -1.1, 2.0])
    # beta = 0: only phases, psi(z) = 2^{-n/2} exp(-i C(z) sum gamma)
    psi = oracle.qaoa_state(n, C, gam, np.zeros(3))
    ref = 2.0 ** (-n / 2) * np.exp(-1j * C * gam.sum())
    assert np.max(np.abs(psi - ref)) < 1e-12
    # gamma = 0: |+> is an eigenvector of every X_j, psi = e^{-i n sum beta} |+>
    bet = np.array([0.7, 0.2, -0.4])
    psi = oracle.qaoa_state(n, C, np.zeros(3), bet)
    assert np.max(np.abs(psi - 2.0 ** (-n / 2) * np.exp(-1j * n * bet.sum()))) < 1e-12


def test_norm_and_symmetries():
    n = 10
    g = synth.erdos_renyi(n, 0.4, 21)
    w = synth.random_weights(g.num_edges, 3)
    C = oracle.cut_table(n, g.u, g.v, w)
    gam, bet = synth.uniform_angles(7, 3)
    gam, bet = gam[0], bet[0]
    psi = oracle.qaoa_state(n, C, gam, bet)
    pr = np.abs(psi) ** 2
    assert pr.sum() == pytest.approx(1.0, abs=1e-12)                     # pin 4
    full = (1 << n) - 1
    z = np.arange(1 << n)
    assert np.allclose(pr, pr[full ^ z], rtol=1e-12, atol=0)               # pin 7
    psi_neg = oracle.qaoa_state(n, C, -gam, -bet)
    assert np.max(np.abs(psi_neg - np.conj(psi))) < 1e-12                  # pin 8
    # pin 9: beta_l + pi/2 multiplies by -i X on every qubit; X^n commutes with
    # U_C (C(z) = C(~z)), so psi' = (-i)^n psi(~z) and pi is unchanged.
    bet2 = bet.copy()
    bet2[1] += math.pi / 2
    psi2 = oracle.qaoa_state(n, C, gam, bet2)
    assert np.max(np.abs(psi2 - (-1j) ** n * psi[full ^ z])) < 1e-12
    # pin 10: the inverse circuit returns |+>
    back = oracle.qaoa_unapply(n, C, gam, bet, psi)
    assert np.max(np.abs(back - 2.0 ** (-n / 2))) < 1e-12


def _p1_edge_expectation(gamma, beta, du, dv, f):
    """p = 1 expectation of one edge term [z_u != z_v] for unweighted graphs
    (Wang, Hadfield, Jiang, Rieffel, Phys. Rev. A 97, 022304 (2018)):
    d = degree - 1 at each endpoint, f = triangles through the edge."""
    return (0.5 + 0.25 * math.sin(4 * beta) * math.sin(gamma)
            * (math.cos(gamma) ** du + math.cos(gamma) ** dv)
            - 0.25 * math.sin(2 * beta) ** 2 * math.cos(gamma) ** (du + dv - 2 * f)
            * (1 - math.cos(2 * gamma) ** f))


def _p1_graph_expectation(n, u, v, gamma, beta):
    adj = [set() for _ in range(n)]
    for a, b in zip(u, v):
        adj[a].add(b)
        adj[b].add(a)
    tot = 0.0
    for a, b in zip(u, v):
        f = len(adj[a] & adj[b])
        tot += _p1_edge_expectation(gamma, beta, len(adj[a]) - 1, len(adj[b]) - 1, f)
    return tot


@pytest.mark.parametrize("seed", range(4))
def test_p1_closed_form(seed):
    n = 10
    g = synth.erdos_renyi(n, 0.45, 30 + seed)
    C = oracle.cut_table(n, g.u, g.v)
    gam, bet = synth.uniform_angles(40 + seed, 1, lo=-math.pi, hi=math.pi)
    psi = oracle.qaoa_state(n, C, gam[0], bet[0])
    E = oracle.expectation(n, psi, C)
    assert E == pytest.approx(_p1_graph_expectation(n, g.u, g.v, gam[0, 0], bet[0, 0]), abs=1e-12)


def test_k2_worked_example():
    # single edge at (gamma, beta) = (pi/2, pi/8): pi(01) = pi(10) = 1/2, E = 1,
    # canonical top-1 is z = 0b10 (bit 0 = 0)
    u, v = _edges([(0, 1)])
    C = oracle.cut_table(2, u, v)
    assert list(C) == [0, 1, 1, 0]
    psi = oracle.qaoa_state(2, C, [math.pi / 2], [math.pi / 8])
    pr = np.abs(psi) ** 2
    assert pr[1] == pytest.approx(0.5, abs=1e-15) and pr[2] == pytest.approx(0.5, abs=1e-15)
    assert oracle.expectation(2, psi, C) == pytest.approx(1.0, abs=1e-15)
    idx, prob, ke = oracle.topk(2, psi, 1, canonical=True)
    assert ke == 1 and idx[0] == 2


def test_edgeless_subgraph():
    n = 8
    C = oracle.cut_table(n, np.zeros(0, np.int32), np.zeros(0, np.int32))
    gam, bet = synth.uniform_angles(3, 3)
    psi = oracle.qaoa_state(n, C, gam[0], bet[0])
    assert np.allclose(np.abs(psi) ** 2, 2.0 ** -n, atol=1e-15)
    E, dg, db = oracle.gradient(n, C, gam[0], bet[0])
    assert E == 0.0 and np.all(dg == 0.0) and np.all(db == 0.0)
    idx, prob, ke = oracle.topk(n, psi, 4)
    # all probabilities tie, so the order is by index: 0, 2, 4, 6
    assert list(idx) == [0, 2, 4, 6]


# ---------------------------------------------------------------- top-k
def test_topk_against_full_sort():
    n = 9
    g = synth.erdos_renyi(n, 0.5, 77)
    C = oracle.cut_table(n, g.u, g.v)
    gam, bet = synth.uniform_angles(78, 2)
    psi = oracle.qaoa_state(n, C, gam[0], bet[0])
    pr = np.abs(psi) ** 2
    for canonical in (True, False):
        zs = [z for z in range(1 << n) if not (canonical and z & 1)]
        ranked = sorted(zs, key=lambda z: (-pr[z], z))
        for k in (1, 5, 16):
            idx, prob, ke = oracle.topk(n, psi, k, canonical)
            assert ke == k
            assert list(idx) == ranked[:k]
            assert np.allclose(prob, pr[ranked[:k]], rtol=1e-14, atol=0)
    # k larger than the canonical half: pad
    idx, prob, ke = oracle.topk(2, oracle.qaoa_state(2, oracle.cut_table(2, *_edges([(0, 1)])), [0.4], [0.3]), 4)
    assert ke == 2 and idx[2] == oracle.UINT32_MAX and prob[3] == -1.0


def test_free_vertices_leave_the_state_invariant():
    """A vertex without an edge inside the subgraph keeps its qubit in |+>:
    psi(z) = psi(z ^ 2^j) exactly for it, and not for the others."""
    n = 7
    u, v = _edges([(0, 2), (2, 5), (5, 0), (1, 5)])  # vertices 3, 4, 6 free
    w = np.array([2, 1, 3, 1], np.int32)
    assert oracle.free_mask(n, u, v, w) == (1 << 3) | (1 << 4) | (1 << 6)
    assert oracle.free_mask(n, u, v, np.array([2, 1, 3, 0], np.int32)) == (1 << 1) | (1 << 3) | (1 << 4) | (1 << 6)
    C = oracle.cut_table(n, u, v, w)
    gam, bet = synth.uniform_angles(41, 3)
    psi = oracle.qaoa_state(n, C, gam[0], bet[0])
    z = np.arange(1 << n)
    for j in range(n):
        d = np.max(np.abs(psi - psi[z ^ (1 << j)]))
        if j in (3, 4, 6):
            assert d <= 1e-15, j
        else:
            assert d > 1e-6, j


def test_tie_rank_is_a_bijection():
    for m in range(0, 15):
        ranks = [oracle.tie_rank(x, m) for x in range(1 << m)]
        assert sorted(ranks) == list(range(1 << m)), m


def _tie_groups(n, free, canonical):
    """Tie groups by closure: strings connected by flipping a free bit (not
    bit 0 in canonical mode) or by the complement (with bit 0 flipped back in
    canonical mode, allowed there only when vertex 0 is free)."""
    full = (1 << n) - 1
    cand = [z for z in range(1 << n) if not (canonical and z & 1)]
    moves = [1 << j for j in range(n) if free >> j & 1 and not (canonical and j == 0)]
    part = (lambda z: (~z & full) ^ 1) if canonical else (lambda z: ~z & full)
    part_ok = (free & 1) if canonical else True
    group = {}
    for z0 in cand:
        if z0 in group:
            continue
        orbit, todo = {z0}, [z0]
        while todo:
            z = todo.pop()
            nxt = [z ^ mv for mv in moves] + ([part(z)] if part_ok else [])
            for y in nxt:
                if y not in orbit:
                    orbit.add(y)
                    todo.append(y)
        for y in orbit:
            group[y] = frozenset(orbit)
    return cand, group


@pytest.mark.parametrize("canonical", [True, False])
@pytest.mark.parametrize("edges,n,seed", [([(0, 1)], 6, 1), ([(1, 2), (2, 4)], 7, 2), ([(0, 3)], 5, 3), ([], 5, 4),
                                          ([(0, 1), (1, 2), (2, 0), (3, 4)], 5, 5)])
def test_topk_ties_by_groups(edges, n, seed, canonical):
    """The top-k list runs through tie groups (found by closure) in order of
    their probability and then of their smallest member; inside a group it
    lists distinct members; a group is finished before the next starts."""
    u, v = _edges(edges)
    free = oracle.free_mask(n, u, v)
    C = oracle.cut_table(n, u, v)
    gam, bet = synth.uniform_angles(seed, 2)
    psi = oracle.qaoa_state(n, C, gam[0], bet[0])
    pr = np.abs(psi) ** 2
    cand, group = _tie_groups(n, free, canonical)
    # probabilities are constant on a group
    for z in cand:
        assert all(abs(pr[y] - pr[z]) <= 1e-15 for y in group[z])
    order = sorted(set(group[z] for z in cand), key=lambda gset: (-pr[min(gset)], min(gset)))
    k = min(24, len(cand))
    idx, prob, ke = oracle.topk(n, psi, k, canonical, free)
    assert ke == k and len(set(idx.tolist())) == k
    expect_groups, left = [], k
    for gset in order:
        if left <= 0:
            break
        expect_groups += [gset] * min(len(gset), left)
        left -= len(gset)
    for z, gset, p in zip(idx, expect_groups, prob):
        assert int(z) in gset and p == pytest.approx(pr[min(gset)], abs=1e-15)


def test_topk_tie_order_worked_example():
    """Hand-worked order inside a tie group (tests/golden/topk_tie_example.json)."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "topk_tie_example.json")))
    n = g["n"]
    u, v = _edges([tuple(e) for e in g["edges"]])
    C = oracle.cut_table(n, u, v)
    psi = oracle.qaoa_state(n, C, [math.pi / 2], [math.pi / 8])
    free = oracle.free_mask(n, u, v)
    idx, prob, ke = oracle.topk(n, psi, 4, False, free)
    assert list(idx) == g["top4_raw"] and np.allclose(prob, 1 / 32, atol=1e-15)
    idx, prob, ke = oracle.topk(n, psi, 4, True, free)
    assert list(idx) == g["top4_canonical"]


# ---------------------------------------------------------------- gradient
@pytest.mark.parametrize("n,p,seed", [(6, 1, 0), (8, 3, 1), (10, 2, 2), (7, 4, 3)])
def test_adjoint_gradient_matches_central_differences(n, p, seed):
    g = synth.erdos_renyi(n, 0.5, 50 + seed)
    w = synth.random_weights(g.num_edges, seed)
    C = oracle.cut_table(n, g.u, g.v, w)
    gam, bet = synth.uniform_angles(60 + seed, p)
    gam, bet = gam[0], bet[0]
    E, dg, db = oracle.gradient(n, C, gam, bet)
    assert E == pytest.approx(oracle.expectation(n, oracle.qaoa_state(n, C, gam, bet), C), abs=1e-12)
    h = 1e-5

    def f(gg, bb):
        return oracle.expectation(n, oracle.qaoa_state(n, C, gg, bb), C)

    scale = max(1.0, float(np.abs(np.concatenate([dg, db])).max()))
    for l in range(p):
        e = np.zeros(p)
        e[l] = h
        fd_g = (f(gam + e, bet) - f(gam - e, bet)) / (2 * h)
        fd_b = (f(gam, bet + e) - f(gam, bet - e)) / (2 * h)
        assert abs(dg[l] - fd_g) <= 1e-7 * scale
        assert abs(db[l] - fd_b) <= 1e-7 * scale


def test_p1_analytic_gradient():
    # differentiate the closed form of the p = 1 edge expectation numerically
    # with a tiny step in extended form, against the adjoint gradient
    n = 9
    g = synth.erdos_renyi(n, 0.5, 91)
    C = oracle.cut_table(n, g.u, g.v)
    gam, bet = 0.37, -0.61
    E, dg, db = oracle.gradient(n, C, np.array([gam]), np.array([bet]))
    h = 1e-6
    F = lambda a, b: _p1_graph_expectation(n, g.u, g.v, a, b)
    assert E == pytest.approx(F(gam, bet), abs=1e-12)
    assert dg[0] == pytest.approx((F(gam + h, bet) - F(gam - h, bet)) / (2 * h), abs=1e-8)
    assert db[0] == pytest.approx((F(gam, bet + h) - F(gam, bet - h)) / (2 * h), abs=1e-8)


def test_ring_optimiser_reaches_three_quarters():
    # p = 1 on a ring (2-regular, triangle-free): E/|E| = 1/2 + 1/4 sin4b sin2g,
    # maximum 3/4 at (pi/4, pi/8). Start away from it and let Adam climb.
    for n in (6, 9):
        u, v = ring(n)
        C = oracle.cut_table(n, u, v)
        g, b, hist = oracle.adam_solve(n, C, [0.5], [0.25], T=400, lr=0.02)
        assert hist[-1] / n == pytest.approx(0.75, abs=1e-6)
        assert math.sin(4 * b[0]) * math.sin(2 * g[0]) == pytest.approx(1.0, abs=1e-5)


def test_cold_start_ramp():
    g, b = oracle.cold_start(1)
    assert g[0] == pytest.approx(math.pi / 4) and b[0] == pytest.approx(math.pi / 8)
    g, b = oracle.cold_start(3)
    assert np.allclose(g, [math.pi / 12, math.pi / 4, 5 * math.pi / 12])
    assert np.allclose(b, [5 * math.pi / 24, math.pi / 8, math.pi / 24])


def test_adam_update_matches_definition():
    theta = np.array([0.1, -0.2])
    m = np.zeros(2)
    v = np.zeros(2)
    g1 = np.array([0.5, -2.0])
    oracle.adam_update(theta, g1, m, v, 1, lr=0.1)
    # first bias-corrected step is lr * sign(g) (up to eps)
    assert np.allclose(theta, [0.2, -0.3], atol=1e-7)


ADAM_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adam_worked_example.json")


@pytest.mark.parametrize("eps", [0.0, 0.5])
@pytest.mark.parametrize("maximise", [True, False])
def test_adam_update_worked_example(eps, maximise):
    # four steps of a sign-alternating gradient with b1 != b2, against the
    # moments and bias-corrected estimates worked out by hand in exact
    # rationals from Kingma and Ba (2015), Algorithm 1; a second parameter
    # sees -g/2 (moments scaled by -1/2 and 1/4)
    gold = json.load(open(ADAM_GOLDEN))
    c = {k: float(Fraction(x)) for k, x in gold["constants"].items()}
    fr = lambda key, t: float(Fraction(gold[key][t]))
    sgn = 1.0 if maximise else -1.0
    theta = np.array([0.25, -0.5])
    expect = theta.copy()
    m = np.zeros(2)
    v = np.zeros(2)
    for t in range(4):
        gt = fr("grad", t)
        oracle.adam_update(theta, np.array([gt, -gt / 2]), m, v, t + 1, lr=c["lr"], b1=c["b1"], b2=c["b2"], eps=eps,
                           maximise=maximise)
        assert m == pytest.approx([fr("m", t), -fr("m", t) / 2], abs=1e-15)
        assert v == pytest.approx([fr("v", t), fr("v", t) / 4], abs=1e-15)
        mh, vh = fr("mhat", t), fr("vhat", t)
        expect += sgn * c["lr"] * np.array([mh / (math.sqrt(vh) + eps), (-mh / 2) / (math.sqrt(vh / 4) + eps)])
        assert theta == pytest.approx(expect, abs=1e-14)
    if eps == 0.0:
        # the two parameters moved by opposite steps of equal size
        assert theta[0] - 0.25 == pytest.approx(-(theta[1] + 0.5), abs=1e-15)


def test_adam_solve_follows_adam_on_the_closed_form_gradient():
    # K2 at p = 1: E = 1/2 + 1/2 sin(4 beta) sin(gamma) (pin 5), so
    # dE/dgamma = 1/2 sin(4 beta) cos(gamma), dE/dbeta = 2 cos(4 beta) sin(gamma).
    # The optimiser's own Adam loop must equal Adam (pinned above) driven by
    # that closed-form gradient; with lr = 0.3 the trajectory overshoots, so
    # both gradient components change sign along the way.
    u, v = _edges([(0, 1)])
    C = oracle.cut_table(2, u, v)
    b1, b2, lr, T = 0.5, 0.75, 0.3, 6
    gam, bet, hist = oracle.adam_solve(2, C, [1.2], [0.55], T=T, lr=lr, b1=b1, b2=b2, eps=0.0)
    theta = np.array([1.2, 0.55])
    m = np.zeros(2)
    vv = np.zeros(2)
    signs = []
    closed = lambda g, b: 0.5 + 0.5 * math.sin(4 * b) * math.sin(g)
    for t in range(T):
        g, b = theta
        assert hist[t] == pytest.approx(closed(g, b), abs=1e-13)
        grad = np.array([0.5 * math.sin(4 * b) * math.cos(g), 2 * math.cos(4 * b) * math.sin(g)])
        signs.append(np.sign(grad))
        oracle.adam_update(theta, grad, m, vv, t + 1, lr=lr, b1=b1, b2=b2, eps=0.0)
    assert gam[0] == pytest.approx(theta[0], abs=1e-12) and bet[0] == pytest.approx(theta[1], abs=1e-12)
    assert hist[T] == pytest.approx(closed(*theta), abs=1e-13)
    signs = np.array(signs)
    assert np.all((signs > 0).any(0) & (signs < 0).any(0))


def _ragged_batch():
    sizes = [4, 6, 2, 5, 3, 7]
    edges = []
    for i, n in enumerate(sizes):
        g = synth.erdos_renyi(n, 0.6, 40 + i)
        edges.append((g.u, g.v, g.w))
    edges[4] = (np.zeros(0, np.int32),) * 3  # an edgeless subgraph
    assert len(edges[1][0]) > 0
    return sizes, edges


@pytest.mark.parametrize("canonical", [True, False])
def test_eval_batch_equals_per_subgraph_functions(canonical):
    sizes, edges = _ragged_batch()
    p, k = 2, 3
    gamma, beta = synth.uniform_angles(77, p, batch=len(sizes))
    E, idx, prob = oracle.eval_batch(sizes, edges, gamma, beta, k=k, canonical=canonical)
    for b, (n, (u, v, w)) in enumerate(zip(sizes, edges)):
        C = oracle.cut_table(n, u, v, w)
        psi = oracle.qaoa_state(n, C, gamma[b], beta[b])
        assert E[b] == oracle.expectation(n, psi, C)
        oi, op, ke = oracle.topk(n, psi, k, canonical=canonical, free=oracle.free_mask(n, u, v, w))
        assert np.array_equal(idx[b], oi) and np.array_equal(prob[b], op)


def test_solve_batch_equals_per_subgraph_functions():
    sizes, edges = _ragged_batch()
    p, T, k = 2, 5, 3
    g0, b0 = synth.uniform_angles(78, p, batch=len(sizes))
    gf, bf, E, idx, prob = oracle.solve_batch(sizes, edges, g0, b0, T, k, lr=0.07, b1=0.8, b2=0.95)
    for b, (n, (u, v, w)) in enumerate(zip(sizes, edges)):
        C = oracle.cut_table(n, u, v, w)
        g, be, hist = oracle.adam_solve(n, C, g0[b], b0[b], T, lr=0.07, b1=0.8, b2=0.95)
        assert np.array_equal(gf[b], g) and np.array_equal(bf[b], be)
        psi = oracle.qaoa_state(n, C, g, be)
        assert E[b] == oracle.expectation(n, psi, C) == hist[T]
        oi, op, ke = oracle.topk(n, psi, k, free=oracle.free_mask(n, u, v, w))
        assert np.array_equal(idx[b], oi) and np.array_equal(prob[b], op)
    # the edgeless subgraph never moves (its gradient is exactly 0)
    assert np.array_equal(gf[4], g0[4]) and np.array_equal(bf[4], b0[4]) and E[4] == 0.0


# ---------------------------------------------------------------- Alg. 1
@pytest.mark.parametrize("nV,N", [(400, 20), (401, 20), (20, 20), (12, 20), (1000, 26), (57, 5)])
def test_partition_equal_invariants(nV, N):
    start, size = oracle.partition_equal(nV, N)
    M = len(start)
    assert start[0] == 0 and start[-1] + size[-1] == nV
    assert np.all(size <= N) and np.all(size >= 2)
    for i in range(1, M):
        assert start[i] == start[i - 1] + size[i - 1] - 1   # exactly one shared vertex
    covered = set()
    for s, n in zip(start, size):
        covered |= set(range(s, s + n))
    assert covered == set(range(nV))
    for i in range(M):
        for j in range(i + 2, M):                              # non-adjacent share nothing
            assert start[i] + size[i] <= start[j]
    if nV > N:
        assert M == math.ceil((nV - 1) / (N - 1))


def test_partition_400_gives_21_subgraphs_of_20():
    start, size = oracle.partition_equal(400, 20)
    assert len(start) == 21 and np.all(size == 20)


def test_partition_chain_ragged():
    sizes = synth.ragged_sizes(1, 14, 26, 400)
    start, size = oracle.partition_chain(2000, sizes)
    assert start[-1] + size[-1] == 2000 and size[-1] >= 2
    assert np.array_equal(size[:-1], sizes[:len(size) - 1])
    for i in range(1, len(start)):
        assert start[i] == start[i - 1] + size[i - 1] - 1


def test_induced_edges_partition_edges_exactly_once():
    g = synth.erdos_renyi(60, 0.2, 2)
    start, size = oracle.partition_equal(60, 8)
    intra = 0
    for s, n in zip(start, size):
        u, v, w = oracle.induced_edges(g.u, g.v, g.w, s, n)
        assert np.all((u >= 0) & (u < n) & (v >= 0) & (v < n))
        intra += len(u)
    # single-vertex overlaps cannot share an edge, so intra sets are disjoint
    both_in_one = 0
    for a, b in zip(g.u, g.v):
        if any(s <= a < s + n and s <= b < s + n for s, n in zip(start, size)):
            both_in_one += 1
    assert intra == both_in_one


# ---------------------------------------------------------------- Alg. 2
def _merge_instance(seed, M, K, n_sub, p=0.3, raw=False):
    rng = np.random.default_rng(seed)
    nV = M * (n_sub - 1) + 1
    g = synth.erdos_renyi(nV, p, seed)
    start, size = oracle.partition_equal(nV, n_sub)
    assert len(start) == M
    cand = np.zeros((M, K), dtype=np.uint32)
    for i in range(M):
        pool = np.arange(0, 1 << size[i], 1 if raw else 2)
        cand[i] = rng.choice(pool, K, replace=False)
    return nV, g, start, size, cand


def _brute_merge(nV, g, start, size, cand):
    """Enumerate B_1 x ... x B_M with complements, keep only compatible
    tuples (shared vertex agrees), take the max cut, ties by traversal order."""
    M, K = cand.shape
    best, best_x, count = -1, None, 0
    members = []
    for i in range(M):
        lst = []
        for j in range(K):
            b = int(cand[i, j])
            lst.append(b)
            lst.append(b ^ ((1 << size[i]) - 1))
        members.append(lst)
    for combo in itertools.product(*members):
        x = np.full(nV, 255, dtype=np.int64)
        ok = True
        for i, b in enumerate(combo):
            for t in range(size[i]):
                bit = (b >> t) & 1
                if x[start[i] + t] != 255 and x[start[i] + t] != bit:
                    ok = False
                    break
                x[start[i] + t] = bit
            if not ok:
                break
        if not ok:
            continue
        count += 1
        c = oracle.cutval(g.u, g.v, None, x.astype(np.uint8))
        if c > best:
            best, best_x = c, x.astype(np.uint8)
    return best, best_x, count


@pytest.mark.parametrize("seed,M,K,n_sub", [(0, 2, 2, 4), (1, 3, 2, 5), (2, 4, 3, 4), (3, 5, 2, 4), (4, 3, 3, 6)])
def test_exhaustive_merge_equals_brute_force(seed, M, K, n_sub):
    nV, g, start, size, cand = _merge_instance(seed, M, K, n_sub)
    best, x, digits, leaves = oracle.merge(nV, start, size, g.u, g.v, None, cand, W=0)
    bb, bx, count = _brute_merge(nV, g, start, size, cand)
    assert best == bb and np.array_equal(x, bx)
    assert leaves == count == 2 * K ** M                     # pin 17: 2 K^M leaves
    assert oracle.cutval(g.u, g.v, None, x) == best


@pytest.mark.parametrize("seed,M,K,n_sub", [(5, 4, 3, 5), (6, 5, 2, 4), (7, 3, 4, 6)])
def test_beam_with_full_width_equals_exhaustive(seed, M, K, n_sub):
    nV, g, start, size, cand = _merge_instance(seed, M, K, n_sub, p=0.4)
    ex = oracle.merge(nV, start, size, g.u, g.v, None, cand, W=0)
    bm = oracle.merge(nV, start, size, g.u, g.v, None, cand, W=2 * K ** (M - 1))
    assert ex[0] == bm[0] and np.array_equal(ex[1], bm[1]) and np.array_equal(ex[2], bm[2])
    # a narrow beam can only do as well or worse, and its cut is consistent
    for narrow in (1, 2):
        nb = oracle.merge(nV, start, size, g.u, g.v, None, cand, W=narrow)
        assert nb[0] <= ex[0] and oracle.cutval(g.u, g.v, None, nb[1]) == nb[0]


def test_start_path_counts_from_paper():
    gold = json.load(open(GOLDEN))["start_paths"]
    K = gold["K"]
    nV, g, start, size, cand = _merge_instance(9, 3, K, 5)
    for L, cnt in zip(gold["L"], gold["count"]):
        # the first L levels alone enumerate the 2 K^L starting paths
        _, _, _, leaves = oracle.merge(start[L - 1] + size[L - 1], start[:L], size[:L],
                                       g.u[g.v < start[L - 1] + size[L - 1]],
                                       g.v[g.v < start[L - 1] + size[L - 1]], None, cand[:L], W=0)
        assert leaves == cnt


def test_concatenation_example_from_paper():
    gold = json.load(open(GOLDEN))["merge_concatenation_example"]
    enc = lambda s: sum(int(ch) << t for t, ch in enumerate(s))  # v1 is bit 0
    cand = np.array([[enc(gold["sub1"])], [enc(gold["sub2"])]], dtype=np.uint32)
    start = np.array([0, 2], dtype=np.int32)
    size = np.array([3, 3], dtype=np.int32)
    # no edges: every leaf ties, the first leaf in traversal order wins
    empty = np.zeros(0, np.int32)
    best, x, digits, leaves = oracle.merge(5, start, size, empty, empty, None, cand, W=0)
    assert "".join(str(b) for b in x) == gold["merged"] and leaves == 2


def test_cut_decomposition_invariant():
    # Sec. 3.4.1: Cut(B*) = sum_i Cut(b_i) + inter-partition term
    nV, g, start, size, cand = _merge_instance(12, 4, 3, 6, p=0.35)
    best, x, digits, _ = oracle.merge(nV, start, size, g.u, g.v, None, cand, W=7)
    intra = 0
    for s, n in zip(start, size):
        u, v, w = oracle.induced_edges(g.u, g.v, None, s, n)
        C = oracle.cut_table(n, u, v)
        z = sum(int(x[s + t]) << t for t in range(n))
        intra += int(C[z])
    inside = lambda a, b: any(s <= a < s + n and s <= b < s + n for s, n in zip(start, size))
    inter = sum(int(x[a] != x[b]) for a, b in zip(g.u, g.v) if not inside(a, b))
    assert intra + inter == best == oracle.cutval(g.u, g.v, None, x)


# ---------------------------------------------------------------- angle predictor
def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(3)
    in_dim, H, out = 5, 7, 3
    npar = oracle.mlp_num_params(in_dim, H, out)
    assert npar == H * in_dim + H + H * H + H + out * H + out
    P = rng.normal(0, 0.5, npar)
    X = rng.normal(0, 1, (6, in_dim))
    T = rng.normal(0, 1, (6, out))
    loss, G = oracle.mlp_loss_grad(P, X, T, H)
    Y = oracle.mlp_forward(P, X, H, out)
    assert loss == pytest.approx(np.mean((Y - T) ** 2), rel=1e-12)
    h = 1e-6
    for i in range(npar):
        e = np.zeros(npar)
        e[i] = h
        fd = (oracle.mlp_loss_grad(P + e, X, T, H)[0] - oracle.mlp_loss_grad(P - e, X, T, H)[0]) / (2 * h)
        assert abs(G[i] - fd) <= 1e-6 * max(1.0, abs(fd)), i


def test_mlp_forward_is_a_relu_network():
    # a single hidden unit path: with W1 = I-like, W2 = I, W3 = I the output
    # is relu(relu(x)) = relu(x)
    in_dim = H = out = 4
    W1 = np.eye(4)
    W2 = np.eye(4)
    W3 = np.eye(4)
    P = np.concatenate([W1.ravel(), np.zeros(4), W2.ravel(), np.zeros(4), W3.ravel(), np.zeros(4)])
    X = np.array([[1.0, -2.0, 0.5, -0.1]])
    assert np.allclose(oracle.mlp_forward(P, X, H, out), np.maximum(X, 0))
