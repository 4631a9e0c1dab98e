"""C-ABI checks that need no GPU: the library loads, exports every function
the header declares, and rejects bad arguments before touching the device."""
import numpy as np
import pytest

from paper_2603_26232_amd import _abi
from paper_2603_26232_amd.partition import batch_arrays, bucket_edges, partition_chain, partition_equal
from paper_2603_26232_amd import synth
import oracle


def test_library_exports_every_declared_symbol():
    L = _abi.lib()
    names = _abi.header_functions()
    assert "qaoa_batch_create" in names and "maxcut_eval" in names
    for n in names:
        assert hasattr(L, n), f"{n} declared in include/paraqaoa.h but not exported"


def test_status_strings():
    assert _abi.qaoa_status_string(0) == "ok"
    assert _abi.qaoa_status_string(3) == "workspace too small"


def _ws(sizes, edges, **kw):
    nq, off, u, v, w = batch_arrays(sizes, edges)
    return _abi.qaoa_workspace_bytes(len(sizes), nq, off, kw.get("w", w), kw.get("max_p", 3),
                                     kw.get("max_k", 16), kw.get("flags", 0))


def test_workspace_size_grows_with_state_and_gradient():
    e = (np.array([0], np.int32), np.array([1], np.int32), np.array([1], np.int32))
    a = _ws([14], [e])
    b = _ws([15], [e])
    c = _ws([15], [e], flags=_abi.QAOA_FLAG_GRADIENT)
    assert 8 * (1 << 13) < a < b < c  # the stored half-state of 14 qubits
    assert c - b >= 8 * (1 << 14)  # the adjoint state


@pytest.mark.parametrize("n,status", [(0, 2), (31, 2)])
def test_qubit_range(n, status):
    e = (np.zeros(0, np.int32),) * 3
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([n], [e])
    assert ei.value.status == status


def test_empty_batch_is_rejected():
    with pytest.raises(_abi.QaoaError) as ei:
        _abi.qaoa_workspace_bytes(0, np.zeros(0, np.int32), np.zeros(1, np.int64), np.zeros(0, np.int32), 3, 16, 0)
    assert ei.value.status == 1
    assert "B = 0" in str(ei.value)


def test_argument_errors():
    e = (np.array([0], np.int32), np.array([1], np.int32), np.array([1], np.int32))
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([5], [e], max_p=0)
    assert ei.value.status == 2
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([5], [e], max_k=65)
    assert ei.value.status == 2
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([5], [e], flags=0x200)  # an unknown flag bit
    assert ei.value.status == 1
    # the concurrent-classes flag is known and changes no workspace size
    assert _ws([5, 20, 23], [e] * 3, flags=_abi.QAOA_FLAG_GRADIENT | _abi.QAOA_FLAG_CONCURRENT_CLASSES) == \
        _ws([5, 20, 23], [e] * 3, flags=_abi.QAOA_FLAG_GRADIENT)
    heavy = (np.array([0], np.int32), np.array([1], np.int32), np.array([5000], np.int32))
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([5], [heavy])
    assert ei.value.status == 6
    neg = (np.array([0], np.int32), np.array([1], np.int32), np.array([-1], np.int32))
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([5], [neg])
    assert ei.value.status == 1


def test_create_validates_edges_before_any_device_work():
    # bad local ids and self-loops are rejected on the host; no device pointer
    # is needed to see it (a NULL workspace would be the next error)
    for bad in [(0, 5), (2, 2), (-1, 1)]:
        nq, off, u, v, w = batch_arrays([5], [(np.array([bad[0]], np.int32), np.array([bad[1]], np.int32),
                                               np.array([1], np.int32))])
        with pytest.raises(_abi.QaoaError) as ei:
            _abi.qaoa_batch_create(1, nq, off, u, v, w, 2, 4, 0, 0, 1 << 20, 0)
        assert ei.value.status == 1 and "invalid" in ei.value.detail
    # well-formed edges, but no workspace
    nq, off, u, v, w = batch_arrays([5], [(np.array([0], np.int32), np.array([1], np.int32),
                                           np.array([1], np.int32))])
    with pytest.raises(_abi.QaoaError) as ei:
        _abi.qaoa_batch_create(1, nq, off, u, v, w, 2, 4, 0, 0, 1 << 20, 0)
    assert ei.value.status == 1 and "workspace" in ei.value.detail
    with pytest.raises(_abi.QaoaError) as ei:
        _abi.qaoa_batch_create(1, nq, off, u, v, w, 2, 4, 0, 256, 16, 0)
    assert ei.value.status == 3


def test_calls_on_null_handle_are_rejected():
    for fn, args in [(_abi.qaoa_apply_layers, (0, 1, 8, 8, 0)), (_abi.qaoa_expectation, (0, 8, 0)),
                     (_abi.qaoa_topk, (0, 4, 8, 8, 0)),
                     (_abi.qaoa_expectation_grad, (0, 1, 8, 8, 8, 8, 8, 0)),
                     (_abi.qaoa_optimize, (0, 1, 5, 8, 8, 8, 8, 0.05, 0.9, 0.999, 1e-8, 0, 0))]:
        with pytest.raises(_abi.QaoaError) as ei:
            fn(*args)
        assert ei.value.status == 1
    _abi.qaoa_batch_destroy(0)  # NULL is accepted


def test_adam_arguments_are_checked_on_the_host():
    # (count, theta, grad, m, v, step, lr, beta1, beta2, eps): status
    cases = [((0, 8, 8, 8, 8, 8, 0.05, 0.9, 0.999, 1e-8), 1),
             ((4, 0, 8, 8, 8, 8, 0.05, 0.9, 0.999, 1e-8), 1),
             ((4, 8, 8, 8, 8, 0, 0.05, 0.9, 0.999, 1e-8), 1),
             ((4, 8, 8, 8, 8, 8, 0.05, 1.0, 0.999, 1e-8), 2),
             ((4, 8, 8, 8, 8, 8, 0.05, 0.9, 0.999, 0.0), 2),
             ((4, 8, 8, 8, 8, 8, -1.0, 0.9, 0.999, 1e-8), 2)]
    for args, status in cases:
        with pytest.raises(_abi.QaoaError) as ei:
            _abi.qaoa_adam_step(*args, 1, 0)
        assert ei.value.status == status, args


def test_gradient_memory_choice():
    """Forward checkpoints unless the single-slot states fit the 256 MB cache
    and the checkpoints would not: the 400-vertex batch (21 x 20 qubits,
    ~200 MB in place, ~370 MB with checkpoints) stays in place, the
    2000-vertex ragged batch takes checkpoints; both flags are rejected."""
    G, IP, CK = 0x1, 0x40, 0x80

    def ws(sizes, edges, flags):
        nq, off, u, v, w = batch_arrays(sizes, edges)
        return _abi.qaoa_workspace_bytes(len(nq), nq, off, w, 3, 16, flags)

    g = synth.erdos_renyi(400, 0.05, 0)
    part = partition_equal(400, 20)
    se, _ = bucket_edges(part, g.u, g.v, g.w)
    assert ws(part.size, se, G) == ws(part.size, se, G | IP) < ws(part.size, se, G | CK)
    g = synth.erdos_renyi(2000, 0.01, 0)
    part = partition_chain(2000, synth.ragged_sizes(1, 14, 26, 2000))
    se, _ = bucket_edges(part, g.u, g.v, g.w)
    assert ws(part.size, se, G | 0x4) == ws(part.size, se, G | 0x4 | CK) > ws(part.size, se, G | 0x4 | IP)
    with pytest.raises(_abi.QaoaError) as ei:
        ws(part.size, se, G | IP | CK)
    assert ei.value.status == 1


def test_warm_start_arguments_are_checked_on_the_host():
    # fake non-NULL device pointers: every case fails its checks before any launch
    for fn in (_abi.qaoa_warm_angles, _abi.qaoa_keep_better):
        for (B, p, ptrs), status in [((0, 3, (8, 8, 8, 8)), 1), ((4, 0, (8, 8, 8, 8)), 2),
                                     ((4, 33, (8, 8, 8, 8)), 2), ((4, 3, (0, 8, 8, 8)), 1),
                                     ((4, 3, (8, 8, 8, 0)), 1)]:
            with pytest.raises(_abi.QaoaError) as ei:
                fn(B, p, *ptrs, 0)
            assert ei.value.status == status, (fn.__name__, B, p, ptrs)


def test_noalloc_backward_checks_its_scratch_limit_on_the_host():
    # 9000 samples at 18 -> 128 -> 128 -> 6 need ~9.5 MB of scratch (limit 8 MiB)
    with pytest.raises(_abi.QaoaError) as ei:
        _abi.qaoa_mlp_backward_noalloc(9000, 18, 128, 6, 8, 8, 8, 8, 8, 8, 8, 0)
    assert ei.value.status == 2 and "8388608" in str(ei.value)
    with pytest.raises(_abi.QaoaError) as ei:
        _abi.qaoa_mlp_backward_noalloc(10, 18, 128, 6, 8, 0, 8, 8, 8, 8, 8, 0)
    assert ei.value.status == 1


def test_predictor_file_shape():
    """The committed predictor holds plain arrays of an 18 -> 128 -> 128 -> 6
    network (loaded without pickle)."""
    from paper_2603_26232_amd.learned import DEFAULT_MODEL, N_FEATURES, _hidden_width
    with np.load(DEFAULT_MODEL, allow_pickle=False) as z:
        assert int(z["p"]) == 3
        assert z["x_mu"].shape == (N_FEATURES,) and z["y_sd"].shape == (6,)
        assert _hidden_width(N_FEATURES, 6, z["params"].shape[0]) == 128
        assert np.all(np.isfinite(z["params"])) and np.all(z["y_sd"] > 0)


# ---------------------------------------------------------------- host prep
@pytest.mark.parametrize("nV,N", [(400, 20), (401, 20), (57, 5), (20, 20), (1000, 26)])
def test_partition_matches_oracle(nV, N):
    p = partition_equal(nV, N)
    s, z = oracle.partition_equal(nV, N)
    assert np.array_equal(p.start, s) and np.array_equal(p.size, z)


def test_chain_partition_matches_oracle():
    sizes = synth.ragged_sizes(1, 14, 26, 300)
    p = partition_chain(2000, sizes)
    s, z = oracle.partition_chain(2000, sizes)
    assert np.array_equal(p.start, s) and np.array_equal(p.size, z)


def test_bucketing_matches_getsubgraph():
    g = synth.erdos_renyi(150, 0.08, 4)
    p = partition_equal(150, 12)
    subs, inter = bucket_edges(p, g.u, g.v, g.w)
    total = sum(len(s[0]) for s in subs) + len(inter[0])
    assert total == g.num_edges
    for k in range(p.M):
        ou, ov, ow = oracle.induced_edges(g.u, g.v, g.w, p.start[k], p.size[k])
        assert np.array_equal(ou, subs[k][0]) and np.array_equal(ov, subs[k][1])


def test_generators_shapes():
    g = synth.erdos_renyi(400, 0.05, 0)
    assert abs(g.num_edges - 0.05 * 400 * 399 / 2) < 4 * np.sqrt(3990)
    assert np.all(g.u < g.v)
    r = synth.random_regular3(26, 5)
    deg = np.bincount(np.concatenate([r.u, r.v]), minlength=26)
    assert np.all(deg == 3) and r.num_edges == 39
    assert len(set(zip(r.u.tolist(), r.v.tolist()))) == 39
    # counter-based stream: any window equals the same slice of a longer draw
    a = synth.splitmix64(9, 0, 100)
    assert np.array_equal(a[40:60], synth.splitmix64(9, 40, 20))


def test_mixer_precision_flags():
    e = (np.array([0], np.int32), np.array([1], np.int32), np.array([1], np.int32))
    base = _ws([16], [e])
    for f in (_abi.QAOA_FLAG_MIXER_MFMA_F32, _abi.QAOA_FLAG_MIXER_MFMA_BF16X3, _abi.QAOA_FLAG_MIXER_MFMA_BF16X4):
        assert _ws([16], [e], flags=f) == base  # same layout, no extra memory
        with pytest.raises(_abi.QaoaError) as ei:
            _ws([16], [e], flags=f | _abi.QAOA_FLAG_GRADIENT)
        assert ei.value.status == 6
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([16], [e], flags=_abi.QAOA_FLAG_MIXER_MFMA_F32 | _abi.QAOA_FLAG_MIXER_MFMA_BF16X3)
    assert ei.value.status == 1
    with pytest.raises(_abi.QaoaError) as ei:
        _ws([16], [e], flags=_abi.QAOA_FLAG_MIXER_MFMA_BF16X3 | _abi.QAOA_FLAG_MIXER_MFMA_BF16X4)
    assert ei.value.status == 1


def test_group_split_tuning_validation():
    _abi.qaoa_tune_group_split(26, [6, 8])
    _abi.qaoa_tune_group_split(26, [2, 4, 8])
    _abi.qaoa_tune_group_split(26, None)  # back to the default
    for n, sizes, status in [(26, [7, 8], 1), (13, [1], 2), (31, [8, 8, 3], 2), (26, [9, 5], 2),
                             (30, [6, 6, 6, 0], 2)]:
        with pytest.raises(_abi.QaoaError) as ei:
            _abi.qaoa_tune_group_split(n, sizes)
        assert ei.value.status == status, (n, sizes)
