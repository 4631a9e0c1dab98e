"""GPU parity at the sizes the 2000- and 16000-vertex workloads run.

* the adjoint gradient of one 24-qubit subgraph at depth 3 with the tuned
  group splits, against the FP64 oracle (the strided groups of 6-8 qubits
  and the 32-bit byte-offset path of the middle backward passes);
* the 2000-vertex ragged solve end to end, as the bench runs it (G(2000,
  0.01) seed 0, chain of 14..26-vertex subgraphs, edgeless ones skipped,
  p = 3, 50 Adam steps, top-16, beam 4096): the first gradient of sampled
  23..26-qubit subgraphs within 1e-4, the final states of two sampled
  subgraphs within 1e-5 with their <C> and top-16 lists, and the 104-level
  merge and CutVal bit-exact against the oracle's merge of the GPU's
  candidates;
* a 764-level merge shaped like the 16000-vertex workload (G(16000, 0.001)
  seed 0, chain of 20..24-vertex subgraphs, K = 16) at W = 256, bit-exact.

The FP64 oracle at 23..26 qubits takes seconds to a minute per subgraph; its
references are computed in a thread pool (the oracle's C calls release the
interpreter lock)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from paper_2603_26232_amd import autotune, synth
from paper_2603_26232_amd.batch import QaoaBatch
from paper_2603_26232_amd.partition import partition_chain
from paper_2603_26232_amd.solve import Solver, SolveConfig, cold_start, merge_beam

pytestmark = pytest.mark.gpu

G_TOL = 1e-4
AMP_TOL = 1e-5
E_TOL = 1e-5


def _grad_ref(args):
    n, edges, gamma, beta = args
    u, v, w = edges
    C = oracle.cut_table(n, u, v, w)
    return oracle.gradient(n, C, gamma, beta)


def _state_ref(args):
    n, edges, gamma, beta = args
    u, v, w = edges
    C = oracle.cut_table(n, u, v, w)
    psi = oracle.qaoa_state(n, C, gamma, beta)
    return psi, oracle.expectation(n, psi, C)


def _check_grad(E, dg, db, ref, what):
    e_ref, g_ref, b_ref = ref
    scale = max(1.0, float(np.abs(np.concatenate([g_ref, b_ref])).max()))
    assert abs(E - e_ref) <= E_TOL * max(1.0, abs(e_ref)), (what, E, e_ref)
    assert np.max(np.abs(dg - g_ref)) <= G_TOL * scale, (what, dg, g_ref)
    assert np.max(np.abs(db - b_ref)) <= G_TOL * scale, (what, db, b_ref)


@pytest.fixture
def tuned_splits():
    tuned = autotune.apply(autotune.DEFAULT_TABLE)
    yield tuned
    autotune.reset()


@pytest.mark.timeout(300)
@pytest.mark.parametrize("weighted", [False, True])
def test_gradient_24_qubits_tuned_split(tuned_splits, weighted):
    """Unit weights, and weights 20..60 whose sum brings C(z) near the 2047
    limit (the FP32 per-lane partial sums of the gradient terms then carry
    the largest values)."""
    n, p = 24, 3
    g = synth.erdos_renyi(n, 0.15, 2424)
    w = g.w
    if weighted:
        w = synth.random_weights(g.num_edges, 2426, 20, 60)
        while w.sum() > 2047:
            w = (w * 0.95).astype(np.int32)
    print(f"gradient parity: n={n}, p={p}, split {tuned_splits.get(n)}, weight sum {int(w.sum())}", flush=True)
    edges = [(g.u, g.v, w)]
    gamma, beta = synth.uniform_angles(2425, p, batch=1)
    if weighted:  # small gammas keep the landscape smooth at these weights
        gamma = gamma / 200.0
    bt = QaoaBatch([n], edges, max_p=p, max_k=4, gradient=True)
    E, dg, db = bt.expectation_grad(gamma, beta)
    torch.cuda.synchronize()
    ref = _grad_ref((n, edges[0], gamma[0], beta[0]))
    e_ref, g_ref, b_ref = ref
    rel = max(np.abs(dg.cpu().numpy()[0] - g_ref).max(), np.abs(db.cpu().numpy()[0] - b_ref).max()) / \
        max(1.0, float(np.abs(np.concatenate([g_ref, b_ref])).max()))
    print(f"  |E| {e_ref:.3f}, max |g| {np.abs(np.concatenate([g_ref, b_ref])).max():.3f}, "
          f"gradient error / max(1, max|g|) = {rel:.2e}", flush=True)
    _check_grad(float(E[0]), dg.cpu().numpy()[0], db.cpu().numpy()[0], ref, n)
    bt.close()


@pytest.mark.timeout(900)
def test_ragged2000_solve_end_to_end(tuned_splits):
    g = synth.erdos_renyi(2000, 0.01, 0)
    part = partition_chain(2000, synth.ragged_sizes(1, 14, 26, 2000))
    cfg = SolveConfig(p=3, iters=50, k=16, beam=4096)
    print(f"ragged2000: {part.M} subgraphs, sizes {part.size.min()}..{part.size.max()}", flush=True)
    S = Solver(g, part, cfg, skip_edgeless=True)
    nE = np.array([len(e[0]) for e in S.sub_edges])
    # sampled subgraphs with edges: the largest of 23, 24, 25 and 26 qubits
    sample = []
    for n in (23, 24, 25, 26):
        cands = [b for b in range(part.M) if part.size[b] == n and nE[b] > 0]
        sample.append(max(cands, key=lambda b: (nE[b], -b)))
    g0, b0 = cold_start(cfg.p, part.M)
    with ThreadPoolExecutor(max_workers=4) as pool:
        grad_refs = pool.map(_grad_ref, [(int(part.size[b]), S.sub_edges[b], g0[b], b0[b]) for b in sample])
        # the first gradient of the solve (cold-start angles)
        E, dg, db = S.batch.expectation_grad(g0, b0)
        E, dg, db = E.cpu().numpy(), dg.cpu().numpy(), db.cpu().numpy()
        S.run()
        r = S.result()
        # final states of two sampled subgraphs (26 and 23 qubits) at the GPU's final angles
        fin = [sample[3], sample[0]]
        state_refs = pool.map(_state_ref, [(int(part.size[b]), S.sub_edges[b], r.gamma[b], r.beta[b]) for b in fin])
        got = {b: S.batch.state(b).cpu().numpy() for b in fin}
        probs = S.prob.view(part.M, -1).cpu().numpy()
        for b, ref in zip(sample, grad_refs):
            print(f"  first gradient b={b} n={part.size[b]} edges={nE[b]}", flush=True)
            _check_grad(E[b], dg[b], db[b], ref, (b, int(part.size[b])))
        from test_gpu_sim import _accept_topk
        for b, (psi, e_ref) in zip(fin, state_refs):
            print(f"  final state b={b} n={part.size[b]}", flush=True)
            assert np.max(np.abs(got[b] - psi)) <= AMP_TOL
            assert abs(r.energies[b] - e_ref) <= E_TOL * max(1.0, e_ref)
            u, v, w = S.sub_edges[b]
            _accept_topk(r.cand[b], probs[b], psi, cfg.k, free=oracle.free_mask(int(part.size[b]), u, v, w))
    # 104-level merge of the GPU's candidates and CutVal, bit-exact
    ref_cut, ref_x, _, _ = oracle.merge(2000, part.start, part.size, g.u, g.v, g.w, r.cand, W=cfg.beam)
    print(f"  merge: {part.M} levels, cut {r.cut} (oracle {ref_cut})", flush=True)
    assert r.cut == ref_cut and np.array_equal(r.assignment, ref_x)
    assert oracle.cutval(g.u, g.v, g.w, r.assignment) == r.cut
    # edgeless subgraphs are closed-form: <C> = 0, top-16 = the first 16
    # strings of their single tie group in the oracle's rank order
    for b in np.nonzero(nE == 0)[0][:5]:
        n = int(part.size[b])
        uniform = np.full(1 << n, 2.0 ** (-n / 2), dtype=np.complex128)
        oi, _, _ = oracle.topk(n, uniform, cfg.k, True, (1 << n) - 1)
        assert r.energies[b] == 0.0 and np.array_equal(r.cand[b], oi)
    S.close()


@pytest.mark.timeout(600)
def test_merge_764_levels_w256():
    g = synth.erdos_renyi(16000, 0.001, 0)
    part = partition_chain(16000, synth.ragged_sizes(1, 20, 24, 16000))
    K, W = 16, 256
    rng = np.random.default_rng(16000)
    cand = np.full((part.M, K), 0xFFFFFFFF, dtype=np.uint32)
    for i in range(part.M):
        half = 1 << (int(part.size[i]) - 1)  # canonical candidates (bit 0 clear); the last subgraph may be short
        kk = min(K, half)
        cand[i, :kk] = 2 * rng.choice(half, kk, replace=False)
    print(f"merge: {part.M} levels, K={K}, W={W}", flush=True)
    best, cut, _ = merge_beam(g, part, torch.as_tensor(cand.view(np.int32), device="cuda"), K, W)
    ref_cut, ref_x, _, _ = oracle.merge(16000, part.start, part.size, g.u, g.v, g.w, cand, W=W)
    words = best.cpu().numpy().view(np.uint32)
    x = ((words[np.arange(16000) // 32] >> (np.arange(16000) % 32).astype(np.uint32)) & 1).astype(np.uint8)
    assert int(cut.cpu()[0]) == ref_cut
    assert np.array_equal(x, ref_x)
    assert oracle.cutval(g.u, g.v, g.w, x) == ref_cut
