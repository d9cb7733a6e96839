"""Batched replicas: each replica of the persistent batched launch equals a
single-lattice run with its seed and replica index, and against the oracle;
per-replica statistics; graph replay; the 64-replica workload's FDT check."""

import numpy as np
import pytest
import torch

import flb_workloads as W
from helpers import gpu_params, oracle_params, rel_err

pytestmark = pytest.mark.gpu

C2 = dict(lattice="D3Q19", rho0=1.0, kT=1e-5, rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0)
DIMS = [(16, 16, 16), (24, 8, 12), (9, 7, 5), (33, 3, 2), (1, 1, 1), (40, 20, 10)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lattice", ["D3Q19", "D2Q9"])
def test_batch_replicas_match_single_runs_and_oracle(precision, lattice):
    from oracle import flb
    from paper_1012_3632_amd import Batch, Simulation
    dims = DIMS if lattice == "D3Q19" else [(nx, ny, 1) for (nx, ny, _) in DIMS]
    seeds = [11 + 3 * r for r in range(len(dims))]
    kw = dict(C2, lattice=lattice, precision=precision)
    b = Batch(gpu_params(**kw), dims, seeds)
    for cfg in range(1):
        b.step(12, stats_stride=3)
    s_b, q_b, n_b = b.moments()
    assert n_b == 4
    for r, (nx, ny, nz) in enumerate(dims):
        single = Simulation(gpu_params(**kw, nx=nx, ny=ny, nz=nz, seed=seeds[r], replica=r))
        single.step(12, stats_stride=3)
        got = b.replica_state(r)
        ref = single.state()
        assert torch.equal(got, ref), r
        s1, q1, n1 = single.moments()
        # FP32 runs form wavefront sums in FP32 over differently shaped tiles
        np.testing.assert_allclose(q_b[r], q1, rtol=1e-12 if precision == "fp64" else 1e-6)
        if r < 3:
            po = oracle_params(**kw, nx=nx, ny=ny, nz=nz, seed=seeds[r], replica=r)
            S, _ = flb.run(flb.initial_state(po), po, 12)
            w = single.populations().numpy()
            assert rel_err(w, S.numpy()) < (1e-12 if precision == "fp64" else 1e-5)


def test_batch_graph_replay_matches_eager():
    from paper_1012_3632_amd import Batch
    kw = dict(C2, precision="fp32")
    a = Batch(gpu_params(**kw), DIMS)
    c = Batch(gpu_params(**kw), DIMS)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        c.graph_capture(8, stats_stride=1)
        for k in range(3):
            a.step(8, stats_stride=1)
            c.graph_launch()
            torch.cuda.synchronize()
            for r in range(len(DIMS)):
                assert torch.equal(a.replica_state(r), c.replica_state(r)), (k, r)
    _, qa, na = a.moments()
    _, qc, nc = c.moments()
    assert na == nc == 24
    np.testing.assert_array_equal(qa, qc)


@pytest.mark.parametrize("pair_bytes", [0, 1 << 20])
def test_batch_graph_replay_after_an_odd_step(pair_bytes):
    """Capture 4, step 1, replay = 5 eager steps, bit for bit (the replay
    starts from the other buffer than at capture)."""
    from paper_1012_3632_amd import Batch
    kw = dict(C2, precision="fp32")
    a = Batch(gpu_params(**kw), DIMS)
    c = Batch(gpu_params(**kw), DIMS)
    a.set_pairs(pair_bytes)
    c.set_pairs(pair_bytes)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        c.graph_capture(4, stats_stride=1)
        c.step(1, stats_stride=1)
        c.graph_launch()
        a.step(5, stats_stride=1)
        torch.cuda.synchronize()
    for r in range(len(DIMS)):
        assert torch.equal(a.replica_state(r), c.replica_state(r)), r
    _, qa, na = a.moments()
    _, qc, nc = c.moments()
    assert na == nc == 5
    # the per-chunk sums are folded once per call, so the two runs group the
    # same FP64 additions differently
    np.testing.assert_allclose(qa, qc, rtol=1e-13)


@pytest.mark.parametrize("pair_bytes", [1, 60000, 1 << 40])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lattice", ["D3Q19", "D2Q9"])
def test_batch_pairs_bit_identical(lattice, precision, pair_bytes):
    """Group-by-group in-place pairs (each replica its own group, several per
    group, one group) give the ordinary schedule's states and statistics bit
    for bit, over odd and even step counts."""
    from paper_1012_3632_amd import Batch
    dims = DIMS if lattice == "D3Q19" else [(nx, ny, 1) for (nx, ny, _) in DIMS]
    kw = dict(C2, lattice=lattice, precision=precision)
    a = Batch(gpu_params(**kw), dims)
    c = Batch(gpu_params(**kw), dims)
    c.set_pairs(pair_bytes)
    nb, ng = c.pairs()
    assert nb == pair_bytes and 1 <= ng <= len(dims)
    if pair_bytes == 1:
        assert ng == len(dims)
    if pair_bytes == 1 << 40:
        assert ng == 1
    for n, stride in ((7, 2), (6, 3), (1, 1), (4, 0)):
        a.step(n, stats_stride=stride)
        c.step(n, stats_stride=stride)
    torch.cuda.synchronize()
    for r in range(len(dims)):
        assert torch.equal(a.replica_state(r), c.replica_state(r)), r
    for x, y in zip(a.moments(), c.moments()):
        np.testing.assert_array_equal(x, y)


def test_batch_pairs_graph_replay():
    from paper_1012_3632_amd import Batch
    kw = dict(C2, precision="fp32")
    a = Batch(gpu_params(**kw), DIMS)
    c = Batch(gpu_params(**kw), DIMS)
    c.set_pairs(60000)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        c.graph_capture(8, stats_stride=1)
        for k in range(3):
            a.step(8, stats_stride=1)
            c.graph_launch()
            torch.cuda.synchronize()
            for r in range(len(DIMS)):
                assert torch.equal(a.replica_state(r), c.replica_state(r)), (k, r)
    for x, y in zip(a.moments(), c.moments()):
        np.testing.assert_array_equal(x, y)


def test_batch_autotune_keeps_state():
    from paper_1012_3632_amd import Batch
    b = Batch(gpu_params(**C2, precision="fp32"), DIMS)
    b.step(2, stats_stride=1)
    before = [b.replica_state(r).clone() for r in range(len(DIMS))]
    m_before = b.moments()
    best, ms = b.autotune(repeats=2)
    assert all(t > 0 for t in ms) and all(0 <= c < 4 for c in best)
    nb, ng = b.pairs()
    assert nb in [0] + [m << 20 for m in (64, 128, 160, 192, 224, 256, 320)] and (ng == 0) == (nb == 0)
    for r in range(len(DIMS)):
        assert torch.equal(before[r], b.replica_state(r))
    m_after = b.moments()
    for x, y in zip(m_before, m_after):
        np.testing.assert_array_equal(x, y)


def test_batch64_workload_fdt():
    """The 64-replica workload (edges drawn from {32,...,96}, seeds 0..63,
    FP32): per-replica mode variances equal rho0 kT N_a / cs2 after burn-in,
    advanced by captured graphs."""
    from paper_1012_3632_amd import Batch, lattice_tables
    wl = W.WORKLOADS["d3q19_batch64"]
    edges = W.batch_edges(wl["replicas"], wl["edges"], wl["size_seed"])
    dims = [(e, e, e) for e in edges]
    kw = dict(C2, precision="fp32", kT=wl["kT"])
    b = Batch(gpu_params(**kw), dims, seeds=list(range(wl["replicas"])))
    b.autotune(repeats=2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.graph_capture(100, stats_stride=0)
        for _ in range(3):
            b.graph_launch()
        b.graph_capture(100, stats_stride=1)
        b.graph_launch()
        b.graph_launch()
    torch.cuda.synchronize()
    s, q, n = b.moments()
    assert n == 200
    # the statistics were accumulated only during the last two replays
    N = lattice_tables("D3Q19")["N"]
    G = kw["kT"] * N * 3
    for r, e in enumerate(edges):
        V = e ** 3
        var = q[r] / (n * V) - (s[r] / (n * V)) ** 2
        tol = 0.02 if e >= 48 else 0.03
        np.testing.assert_allclose(var[4:] / G[4:], 1.0, atol=tol, err_msg=f"replica {r} edge {e}")
