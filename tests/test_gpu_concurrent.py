"""Concurrent qubit-group classes (QAOA_FLAG_CONCURRENT_CLASSES): the classes
of a ragged batch, and the small-subgraph kernel, run on the library's side
streams, forked from and joined back into the caller's stream. Every kernel
and every reduction is the same as in the serial order, so the results must be
bit-identical: eagerly, through the fused optimiser, and replayed from a
captured HIP graph."""
import numpy as np
import pytest
import torch

from paper_2603_26232_amd import synth
from paper_2603_26232_amd.batch import QaoaBatch
from paper_2603_26232_amd.partition import partition_chain
from paper_2603_26232_amd.solve import Solver, SolveConfig, cold_start

pytestmark = pytest.mark.gpu

# small-subgraph kernel (5, 9, 12), one-group classes of several shapes
# (14, 16, 17, 20) and two-group classes (21, 22, 23)
SIZES = [21, 9, 14, 16, 20, 22, 12, 17, 23, 5]


def _edges(sizes, seed):
    out = []
    for i, n in enumerate(sizes):
        g = synth.erdos_renyi(n, 0.3, seed + i)
        out.append((g.u, g.v, g.w))
    return out


def _run(bt, gamma, beta):
    bt.apply_layers(gamma, beta)
    E = bt.expectation().clone()
    idx, prob = bt.topk(8)
    states = [bt.reduced_state(b).clone() for b in range(len(SIZES))]
    Eg, dg, db = bt.expectation_grad(gamma, beta)
    torch.cuda.synchronize()
    return [E, idx.clone(), prob.clone(), Eg.clone(), dg.clone(), db.clone()] + states


@pytest.mark.parametrize("memory", ["checkpoints", "inplace"])
def test_batch_calls_bit_identical(memory):
    edges = _edges(SIZES, 40)
    gamma, beta = synth.uniform_angles(41, 3, batch=len(SIZES))
    ser = QaoaBatch(SIZES, edges, max_p=3, max_k=8, gradient=True, gradient_memory=memory)
    con = QaoaBatch(SIZES, edges, max_p=3, max_k=8, gradient=True, gradient_memory=memory,
                    concurrent_classes=True)
    ref = _run(ser, gamma, beta)
    for rep in range(2):
        got = _run(con, gamma, beta)
        for i, (a, b) in enumerate(zip(ref, got)):
            assert torch.equal(a, b), (rep, i)
    ser.close()
    con.close()


@pytest.mark.parametrize("mixer", ["mfma_f32", "mfma_bf16x4"])
def test_forward_matrix_core_modes_bit_identical(mixer):
    """Forward-only batches with a matrix-core mixer mode (their group-0
    passes are another kernel family) give the same states, <C> and top-k."""
    edges = _edges(SIZES, 60)
    gamma, beta = synth.uniform_angles(61, 2, batch=len(SIZES))
    out = []
    for conc in (False, True):
        bt = QaoaBatch(SIZES, edges, max_p=2, max_k=8, mixer=mixer, concurrent_classes=conc)
        bt.apply_layers(gamma, beta)
        E = bt.expectation().clone()
        idx, prob = bt.topk(8)
        st = [bt.reduced_state(b).clone() for b in range(len(SIZES))]
        torch.cuda.synchronize()
        out.append([E, idx.clone(), prob.clone()] + st)
        bt.close()
    for i, (a, b) in enumerate(zip(*out)):
        assert torch.equal(a, b), i


def _ragged():
    g = synth.erdos_renyi(240, 0.05, 11)
    part = partition_chain(240, synth.ragged_sizes(3, 10, 22, 240))
    return g, part


def test_solve_bit_identical_eager_and_graph():
    """Whole solves (Adam loop, finish, merge, CutVal) with and without the
    concurrent classes; then the Adam loop replayed from one captured graph
    (forks and joins inside the graph), checked on every replay with eager
    work in between."""
    g, part = _ragged()
    cfg = SolveConfig(p=3, iters=8, k=8, beam=128)
    ser = Solver(g, part, cfg, skip_edgeless=True)
    con = Solver(g, part, cfg, skip_edgeless=True, concurrent_classes=True)
    ser.run()
    con.run()
    torch.cuda.synchronize()
    for name in ("theta", "m", "v", "E"):
        assert torch.equal(getattr(ser, name), getattr(con, name)), name
    rs, rc = ser.result(), con.result()
    assert rs.cut == rc.cut
    assert np.array_equal(rs.assignment, rc.assignment)
    assert np.array_equal(rs.cand, rc.cand)
    ref_theta = ser.theta.clone()
    g0, b0 = cold_start(cfg.p, part.M)
    for rep in range(3):
        con.set_angles(g0, b0)
        con.optimise_graph(cfg.iters)
        torch.cuda.synchronize()
        assert torch.equal(con.theta, ref_theta), rep
        con.finish()
        torch.cuda.synchronize()
    ser.close()
    con.close()
