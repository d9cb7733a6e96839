"""GPU parity of the HIP library against the FP64 oracle (through the C ABI).

Bars: Philox words bit-exact; populations within 1e-12 (FP64) / 1e-5 (FP32)
relative to max|f| on unshifted populations; statistics to FP64 rounding.
Sizes span several tiles with ragged edges in every direction.
"""

import numpy as np
import pytest
import torch

import flb_workloads as W
from helpers import gpu_params, oracle_params, rel_err, run_pair, tol

pytestmark = pytest.mark.gpu

C2 = dict(lattice="D3Q19", rho0=1.0, kT=1e-5, rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0, seed=7)
LANDAU = dict(force_model=1, a=-0.01, b=0.1, rho_c=1.0, kappa=0.05)


def test_noise_words_bit_exact():
    from oracle import philox
    from paper_1012_3632_amd import noise_words
    p = gpu_params(**C2, nx=128, ny=128, nz=128, precision="fp32")
    for step, block, site0, n in ((0, 0, 0, 4096), (123, 3, 2_000_000, 97_152), (2**31 + 5, 1, 16_000_000, 777)):
        got = noise_words(p, step, block, site0, n).numpy()
        ref = philox.block_words(np.arange(site0, site0 + n, dtype=np.uint64), step, block, 7)
        np.testing.assert_array_equal(got, ref.T.astype(np.int64))
    p2 = gpu_params(**C2, nx=8, ny=8, nz=8, precision="fp64").with_(seed=0xDEADBEEF12345678, replica=9)
    got = noise_words(p2, 77, 2, 0, 512, tag=1).numpy()
    ref = philox.block_words(np.arange(512, dtype=np.uint64), 77, 2, 0xDEADBEEF12345678, tag=1,
                             replica=9)
    np.testing.assert_array_equal(got, ref.T.astype(np.int64))


@pytest.mark.parametrize("lattice", ["D3Q19", "D2Q9"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noise_normals_match_oracle(lattice, precision):
    """Box-Muller normals of 2^20 sites (every 16-bit angle many times over)
    against the oracle's numpy log/cos/sin, pair by pair with R the pair's
    radius.  FP64 (series sin/cos and log on the device): within 1e-15
    max(1, R), a few ulp.  FP32: u = (r + 1) 2^-32 is rounded to 24 bits for
    r >= 2^24 (an error up to 2^-25 in u near 1, i.e. up to ~3e-8 / R in R)
    and v_log/v_sqrt/v_sin/v_cos are hardware approximations: within
    4e-6 max(1, R) + 1e-7 / R."""
    from oracle import philox
    from paper_1012_3632_amd import noise_normals
    p = gpu_params(**dict(C2, lattice=lattice), nx=8, ny=8, nz=8 if lattice == "D3Q19" else 1,
                   precision=precision).with_(replica=3)
    n = 1 << 20
    got = noise_normals(p, 1234, 0, n).numpy().astype(np.float64).T
    ref = philox.normals(n, 1234, got.shape[0], 7, replica=3)
    err = np.abs(got - ref)
    R = np.repeat(np.hypot(ref[0::2], ref[1::2]), 2, axis=0)[:ref.shape[0]]
    if precision == "fp64":
        bar = 1e-15 * np.maximum(1.0, R)
    else:
        bar = 4e-6 * np.maximum(1.0, R) + 1e-7 / R
    assert (err <= bar).all(), (err.max(), (err / bar).max())
    # the first pair of site 5 at another step and site offset
    got2 = noise_normals(p, 99, 5, 3).numpy().astype(np.float64)
    ref2 = philox.normals(8, 99, got.shape[0], 7, replica=3)[:, 5:8].T
    np.testing.assert_allclose(got2, ref2, rtol=0, atol=1e-14 if precision == "fp64" else 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_parity_d2q9_ideal_full_run(precision):
    kw = dict(W.params_of("d2q9_32_fp64"), precision=precision)
    sim, fg, fr, _ = run_pair(kw, W.WORKLOADS["d2q9_32_fp64"]["steps"])
    assert rel_err(fg, fr) < tol(kw)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(9, 70, 5), (20, 18, 16), (3, 5, 130)])
def test_parity_d3q19_ideal(precision, shape):
    nz, ny, nx = shape
    kw = dict(C2, precision=precision, nx=nx, ny=ny, nz=nz)
    for launch in range(n_launch(kw)):
        sim, fg, fr, _ = run_pair(kw, 30, drho_amp=0.01, launch=launch)
        assert rel_err(fg, fr) < tol(kw), launch


def n_launch(kw):
    from paper_1012_3632_amd import Simulation
    s = Simulation(gpu_params(**kw))
    n, _ = s.launch_configs()
    s.close()
    return n


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_statistics_every_launch_d3q19(precision):
    """The per-block statistics slots give the oracle's mode sums for every
    launch shape, over a box ragged in x and y."""
    kw = dict(C2, precision=precision, nx=130, ny=21, nz=12)
    n = n_launch(kw)
    assert n >= 10
    ref = None
    for launch in range(n):
        sim, fg, fr, st = run_pair(kw, 12, drho_amp=0.01, launch=launch, stats_stride=2)
        s, s2, ns = sim.moments()
        assert ns == st["nsamples"] == 6
        if precision == "fp64":
            np.testing.assert_allclose(s2, st["sumsq"], rtol=1e-11, err_msg=str(launch))
            np.testing.assert_allclose(s, st["sum"], rtol=1e-9, atol=1e-10, err_msg=str(launch))
        else:
            # FP32 moments are summed in FP32 per 16-lane row before the FP64
            # reduction.  Each of the N = sites x samples terms of a mode sum is
            # off by ~1e-7 of its own size (FP32 storage of the shifted state and
            # the row sums), so by Cauchy-Schwarz the sum is off by at most
            # ~1e-7 sqrt(N sum m^2); bound it at 5e-6 sqrt(N sum m^2) against the
            # oracle (the sums themselves are ~sqrt(N) times larger than that
            # bound's scale for these zero-mean modes)
            np.testing.assert_allclose(s2, st["sumsq"], rtol=5e-5, err_msg=str(launch))
            N = kw["nx"] * kw["ny"] * kw["nz"] * ns
            bound = 5e-6 * np.sqrt(N * st["sumsq"])
            assert np.all(np.abs(s - st["sum"]) <= bound), (launch, np.abs(s - st["sum"]) / bound)
            if ref is None:
                ref = (s, s2)
            # every launch shape sums the same FP32 values (bitwise equal states)
            np.testing.assert_allclose(s2, ref[1], rtol=1e-6, err_msg=str(launch))
        sim.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("eta", [0, 1])
def test_parity_d2q9_landau(precision, eta):
    kw = dict(W.params_of("d2q9_256_adjoint", nx=70, ny=37), precision=precision, eta=eta)
    nsteps = 200 if eta == 0 else 60
    for launch in range(3):
        sim, fg, fr, _ = run_pair(kw, nsteps, drho_amp=0.01, launch=launch)
        assert rel_err(fg, fr) < tol(kw), launch


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("eta", [0, 1])
@pytest.mark.parametrize("shape", [(11, 13, 35), (37, 9, 67)])
def test_parity_d3q19_landau(precision, eta, shape):
    """Every launch shape of the force step (3-D tiles and z-marching columns;
    nz = 37 gives z-marching runs of 16 and 32 planes with a ragged last run)."""
    nz, ny, nx = shape
    kw = dict(W.params_of("d3q19_256_landau", nx=nx, ny=ny, nz=nz), precision=precision, eta=eta)
    for launch in range(n_launch(kw)):
        sim, fg, fr, _ = run_pair(kw, 12, drho_amp=0.01, launch=launch)
        assert rel_err(fg, fr) < tol(kw), launch


def test_landau_statistics_every_launch_d3q19():
    kw = dict(W.params_of("d3q19_256_landau", nx=67, ny=9, nz=37), precision="fp64", kT=1e-5)
    for launch in range(n_launch(kw)):
        sim, fg, fr, st = run_pair(kw, 6, drho_amp=0.01, launch=launch, stats_stride=2)
        s, s2, ns = sim.moments()
        assert ns == st["nsamples"] == 3
        np.testing.assert_allclose(s2, st["sumsq"], rtol=1e-11, err_msg=str(launch))
        np.testing.assert_allclose(s, st["sum"], rtol=1e-9, atol=1e-10, err_msg=str(launch))
        sim.close()


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (1, 1, 1)), ("D2Q9", (1, 3, 1)),
                                           ("D3Q19", (1, 1, 1)), ("D3Q19", (2, 1, 3)),
                                           ("D3Q19", (1, 2, 65))])
@pytest.mark.parametrize("force", [0, 1])
def test_parity_tiny_boxes(lattice, shape, force):
    nz, ny, nx = shape
    kw = dict(lattice=lattice, precision="fp64", nx=nx, ny=ny, nz=nz, kT=1e-4, rate_bulk=1.3,
              rate_shear=0.7, rate_ghost=1.9, seed=5)
    if force:
        kw.update(LANDAU)
    sim, fg, fr, _ = run_pair(kw, 12, drho_amp=0.01 if force else 0.0)
    assert rel_err(fg, fr) < 1e-12


def test_statistics_match_oracle():
    kw = dict(W.params_of("d2q9_32_fp64"), nx=33, ny=17)
    sim, fg, fr, st = run_pair(kw, 60, stats_stride=3)
    s, s2, n = sim.moments()
    assert n == st["nsamples"] == 20
    np.testing.assert_allclose(s2, st["sumsq"], rtol=1e-11)
    # the oracle forms m_0 - rho0 from unshifted f: its own rounding is ~1e-16 per term
    np.testing.assert_allclose(s, st["sum"], rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("force", [0, 1])
def test_fields_match_oracle(force):
    from oracle import flb
    kw = dict(C2, precision="fp64", nx=21, ny=10, nz=9)
    if force:
        kw.update(LANDAU, kT=1e-6)
    sim, fg, fr, _ = run_pair(kw, 7, drho_amp=0.01)
    rho, j = flb.fields(torch.as_tensor(fr), oracle_params(**kw))
    out = sim.fields().cpu().numpy()
    np.testing.assert_allclose(out[0], rho.numpy(), rtol=1e-13)
    np.testing.assert_allclose(out[1:], j.numpy(), rtol=0, atol=1e-14)


def test_full_size_step_parity_d3q19_128():
    """d3q19_128 at full size in the launch shape the autotuner picks (the one
    the benchmark times): the GPU state after 40 steps is advanced two steps by
    the oracle and by the GPU; every site is compared (FP32 bar)."""
    from oracle import flb
    from paper_1012_3632_amd import Simulation
    kw = dict(W.params_of("d3q19_128"), precision="fp32")
    sim = Simulation(gpu_params(**kw))
    sim.autotune(repeats=2)
    sim.step(40, stats_stride=1)
    S40 = sim.populations()
    sim.step(2, stats_stride=1)   # one in-place pair if the autotuner chose pairs
    got = sim.populations().numpy()
    po = oracle_params(**kw)
    ref = flb.step(flb.step(S40, 40, po), 41, po).numpy()
    assert rel_err(got, ref) < 1e-5
    del S40


def test_graph_replay_matches_eager():
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, precision="fp32", nx=40, ny=24, nz=16)
    a = Simulation(gpu_params(**kw))
    b = Simulation(gpu_params(**kw))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.graph_capture(10, stats_stride=2)
        for r in range(4):
            a.step(10, stats_stride=2)
            b.graph_launch()
            torch.cuda.synchronize()
            assert torch.equal(a.state(), b.state()), r
            x = torch.randn(1000, device="cuda").sum()  # eager work between replays
    torch.cuda.synchronize()
    assert a.step_index == b.step_index == 40
    sa, qa, na = a.moments()
    sb, qb, nb = b.moments()
    assert na == nb == 20
    np.testing.assert_array_equal(qa, qb)


@pytest.mark.parametrize("pairs", [False, True])
def test_graph_replay_after_an_odd_step(pairs):
    """A graph captured with the state in one buffer and replayed after an
    odd number of ordinary steps (the state then in the other buffer)
    continues the state: capture 4, step 1, replay = 5 eager steps, bit for
    bit, states and statistics; with in-place pairs as well."""
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, precision="fp32", nx=64, ny=12, nz=10)
    a = Simulation(gpu_params(**kw))
    b = Simulation(gpu_params(**kw))
    if pairs:
        n, _ = a.launch_configs()
        ip = [c for c in range(n) if a.launch_shape(c)[6]][0]
        a.set_launch(ip)
        b.set_launch(ip)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.graph_capture(4, stats_stride=1)
        b.step(1, stats_stride=1)
        b.graph_launch()
        b.step(1, stats_stride=1)   # back to the first buffer
        b.graph_launch()
        a.step(5, stats_stride=1)
        a.step(5, stats_stride=1)
        torch.cuda.synchronize()
    assert a.step_index == b.step_index == 10
    assert torch.equal(a.state(), b.state())
    sa, qa, na = a.moments()
    sb, qb, nb = b.moments()
    assert na == nb == 10
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(qa, qb)


@pytest.mark.parametrize("kind", ["d3q19_ideal_pairs", "d3q19_landau_march", "d2q9_landau_fused"])
def test_nonfinite_population_is_reported(kind):
    """A NaN written into one population from the host: with checks on,
    flb_step returns FLB_ERR_NONFINITE within the chunk that pulls it; with
    checks off it stays asynchronous and returns FLB_OK; after the state is
    reloaded and the flag cleared, steps succeed again."""
    from paper_1012_3632_amd import Simulation
    from paper_1012_3632_amd._lib import FLBError
    if kind == "d3q19_ideal_pairs":
        kw = dict(C2, precision="fp32", nx=64, ny=10, nz=6)
    elif kind == "d3q19_landau_march":
        kw = dict(C2, **LANDAU, precision="fp32", nx=64, ny=12, nz=20, kT=1e-6)
    else:
        kw = dict(W.params_of("d2q9_256_adjoint", nx=40, ny=24), precision="fp64")
    sim = Simulation(gpu_params(**kw))
    n, _ = sim.launch_configs()
    if kind == "d3q19_ideal_pairs":
        sim.set_launch([c for c in range(n) if sim.launch_shape(c)[6]][0])
    elif kind == "d3q19_landau_march":
        sim.set_launch([c for c in range(n) if sim.launch_shape(c)[5]][0])
    sim.set_check(4)
    sim.step(8, stats_stride=1)
    good = sim.state().clone()
    torch.cuda.synchronize()
    bad = sim.state()
    bad.view(-1)[bad.numel() // 3] = float("nan")
    with pytest.raises(FLBError) as e:
        sim.step(10, stats_stride=1)
    assert e.value.status == -3
    assert sim.step_index == 12        # stopped after the first chunk of 4
    # reads off: asynchronous, no error
    sim.set_check(0)
    sim.step(3)
    torch.cuda.synchronize()
    sim.load_state(good)
    sim.set_check(1)                   # clears the flag
    sim.step(5)
    assert np.isfinite(sim.state().cpu().numpy()).all()


def test_resume_is_bit_exact():
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, precision="fp32", nx=30, ny=20, nz=10)
    a = Simulation(gpu_params(**kw))
    a.step(20)
    b = Simulation(gpu_params(**kw))
    b.step(10)
    c = Simulation(gpu_params(**kw).with_(step0=10))
    c.load_state(b.state().clone())
    c.step(10)
    torch.cuda.synchronize()
    assert torch.equal(a.state(), c.state())


def test_launch_configs_bitwise_identical_and_autotune_keeps_state():
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, precision="fp32", nx=64, ny=32, nz=16)
    ref = None
    n = n_launch(kw)
    for cfg in range(n):
        s = Simulation(gpu_params(**kw))
        s.set_launch(cfg)
        s.step(6)
        st = s.state().clone()
        if ref is None:
            ref = st
        assert torch.equal(st, ref), cfg
    s = Simulation(gpu_params(**kw))
    s.step(3)
    s.step(2, stats_stride=1)
    before = s.state().clone()
    m_before = s.moments()
    best, ms = s.autotune(repeats=2)
    assert torch.equal(s.state(), before)
    m_after = s.moments()
    for x, y in zip(m_before, m_after):
        np.testing.assert_array_equal(x, y)
    assert s.launch_configs() == (n, (best[0], best[1], best[3]))
    assert all(t > 0 for t in ms) and 0 <= best[0] < n and 0 <= best[1] < n
    assert best[2] >= 0 and best[3] in (-1, best[2])


@pytest.mark.parametrize("lattice,precision", [("D3Q19", "fp32"), ("D3Q19", "fp64"),
                                               ("D2Q9", "fp32"), ("D2Q9", "fp64")])
@pytest.mark.parametrize("shape", [(5, 7, 130), (3, 64, 64), (1, 1, 1), (2, 3, 65)])
def test_in_place_pairs_bit_identical(lattice, precision, shape):
    """In-place pairs (one buffer) against ordinary steps (two buffers): same
    populations and statistics bit for bit, for odd and even step counts and
    statistics strides, over boxes ragged in x and y and boxes of one site."""
    from paper_1012_3632_amd import Simulation
    nz, ny, nx = shape
    if lattice == "D2Q9":
        nz = 1
    kw = dict(C2, lattice=lattice, precision=precision, nx=nx, ny=ny, nz=nz)
    drho = W.initial_drho((nz, ny, nx), 5, 0.01)
    probe = Simulation(gpu_params(**kw))
    shapes = [probe.launch_shape(c) for c in range(probe.launch_configs()[0])]
    probe.close()
    for ip in [c for c, sh in enumerate(shapes) if sh[6]]:
        # the reference takes one step per call: every step is then a lone
        # step, run by the ordinary kernel of the same tile (same FP64
        # reduction order of the statistics)
        ref = Simulation(gpu_params(**kw), drho_init=drho)
        ref.set_launch(ip)
        got = Simulation(gpu_params(**kw), drho_init=drho)
        got.set_launch(ip)
        assert got.launch_configs()[1][2] == ip
        for nsteps, stride in ((1, 1), (4, 1), (5, 2), (6, 3), (3, 0)):
            for k in range(nsteps):
                ref.step(1, stats_stride=1 if stride and (k + 1) % stride == 0 else 0)
            got.step(nsteps, stats_stride=stride)
            torch.cuda.synchronize()
            assert torch.equal(ref.state(), got.state()), (ip, nsteps, stride)
            assert ref.step_index == got.step_index
        for a, b in zip(ref.moments(), got.moments()):
            np.testing.assert_array_equal(a, b)
        ref.close()
        got.close()


def test_in_place_pairs_graph_replay():
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, precision="fp32", nx=64, ny=24, nz=16)
    a = Simulation(gpu_params(**kw))
    b = Simulation(gpu_params(**kw))
    ip = next(c for c in range(b.launch_configs()[0]) if b.launch_shape(c)[6])
    a.set_launch(next(c for c in range(a.launch_configs()[0])
                      if a.launch_shape(c)[:6] == b.launch_shape(ip)[:6] and not a.launch_shape(c)[6]))
    b.set_launch(ip)   # the first in-place shape (128 x 2) has an ordinary twin
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.graph_capture(6, stats_stride=2)
        for r in range(3):
            a.step(6, stats_stride=2)
            b.graph_launch()
            torch.cuda.synchronize()
            assert torch.equal(a.state(), b.state()), r
    np.testing.assert_array_equal(a.moments()[1], b.moments()[1])


def test_conservation_gpu():
    from paper_1012_3632_amd import Simulation, lattice_tables
    kw = dict(C2, precision="fp64", nx=24, ny=20, nz=16)
    s = Simulation(gpu_params(**kw), drho_init=W.initial_drho((16, 20, 24), 1, 0.01))
    c = torch.as_tensor(lattice_tables("D3Q19")["c"], dtype=torch.float64)
    f0 = s.state().cpu().double()
    s.step(200)
    f1 = s.state().cpu().double()
    assert abs(f1.sum() - f0.sum()) < 1e-12
    j0 = torch.einsum("ia,i...->a", c, f0)
    j1 = torch.einsum("ia,i...->a", c, f1)
    assert (j1 - j0).abs().max() < 1e-13


def test_rest_state_stays_exactly_zero():
    from paper_1012_3632_amd import Simulation
    for lat in ("D2Q9", "D3Q19"):
        kw = dict(C2, lattice=lat, precision="fp32", nx=17, ny=9, nz=1 if lat == "D2Q9" else 5,
                  kT=0.0)
        s = Simulation(gpu_params(**kw))
        s.step(10)
        assert torch.count_nonzero(s.state()) == 0


def test_determinism():
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, precision="fp32", nx=64, ny=64, nz=64)
    out = []
    for _ in range(2):
        s = Simulation(gpu_params(**kw))
        s.step(20, stats_stride=1)
        out.append((s.state().clone(), s.moments()))
    assert torch.equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1][1], out[1][1][1])


def test_invalid_arguments_rejected():
    from paper_1012_3632_amd import Simulation
    from paper_1012_3632_amd._lib import FLBError
    bad = [dict(kT=0.4), dict(rate_shear=2.0), dict(rate_bulk=0.0), dict(nz=2), dict(nx=0),
           dict(rho0=-1.0)]
    for b in bad:
        kw = dict(lattice="D2Q9", precision="fp64", nx=8, ny=8, nz=1)
        kw.update(b)
        with pytest.raises(FLBError):
            Simulation(gpu_params(**kw))


def _window_ids(n, start, size):
    return (start + np.arange(size)) % n


def test_full_size_landau_256_windows():
    """d3q19_256_landau at full size (256^3, FP32) in the launch shape the
    autotuner picks (the one the benchmark times).  A site's update depends on
    the state within three sites (pull, density, chemical potential, force),
    so 20^3 windows of the GPU state S_n (periodic in the big box, some across
    its edges) are advanced two steps by the oracle with the noise of their
    global site indices, and the inner 8^3 sites are compared with the GPU's
    S_{n+2}, both steps run in one call: the second step's density is the one
    the march forms itself where the shape does so."""
    from oracle import flb, philox
    from paper_1012_3632_amd import Simulation, lattice_tables
    wl = W.WORKLOADS["d3q19_256_landau"]
    kw = dict(W.params_of("d3q19_256_landau"), precision="fp32")
    n = kw["nx"]
    sim = Simulation(gpu_params(**kw), drho_init=W.initial_drho((n, n, n), 7, wl["init_noise"]))
    sim.autotune(repeats=2)
    sim.step(30, stats_stride=1)
    w = torch.as_tensor(lattice_tables("D3Q19")["w"]).view(-1, 1, 1, 1)
    rng = np.random.default_rng(11)
    starts = [(0, 0, 0), (n - 7, n - 7, n - 7), (120, 3, 250)] + \
             [tuple(int(v) for v in rng.integers(0, n, 3)) for _ in range(3)]
    Wd, M, NS = 20, 6, 2
    wins = []
    for (z0, y0, x0) in starts:
        iz, iy, ix = (torch.as_tensor(_window_ids(n, s0, Wd), device="cuda") for s0 in (z0, y0, x0))
        wins.append((iz, iy, ix))
    before = [sim.state()[:, iz][:, :, iy][:, :, :, ix].to("cpu", torch.float64) + w * kw["rho0"]
              for iz, iy, ix in wins]
    step_n = sim.step_index
    sim.step(NS, stats_stride=1)
    after = [sim.state()[:, iz][:, :, iy][:, :, :, ix].to("cpu", torch.float64) + w * kw["rho0"]
             for iz, iy, ix in wins]
    pw = oracle_params(**dict(kw, nx=Wd, ny=Wd, nz=Wd))
    lat = flb.lattice_of(pw)
    K = len(lat.noncons())
    worst = 0.0
    for (iz, iy, ix), S0, S1 in zip(wins, before, after):
        gz, gy, gx = (t.cpu().numpy().astype(np.int64) for t in (iz, iy, ix))
        sites = ((gz[:, None, None] * n + gy[None, :, None]) * n + gx[None, None, :]).reshape(-1)
        ref = S0
        for k in range(NS):
            z = torch.as_tensor(philox.normals(None, step_n + k, K, kw["seed"], sites=sites)).reshape(K, Wd, Wd, Wd)
            f = flb.pull(ref, lat)
            F = flb.landau_force(flb.density(f), pw, lat)
            ref = flb.collide(f, F, step_n + k, pw, lat, z=z)
        inner = (slice(None), slice(M, Wd - M), slice(M, Wd - M), slice(M, Wd - M))
        worst = max(worst, rel_err(S1[inner].numpy(), ref[inner].numpy()))
    assert worst < 1e-5, worst
    sim.close()


@pytest.mark.parametrize("eta", [0, 1])
@pytest.mark.parametrize("shape", [(18, 7, 130), (5, 3, 64), (4, 5, 65), (1, 1, 1), (2, 1, 3),
                                   (1, 2, 65)])
def test_partial_density_march_d3q19(shape, eta):
    """D3Q19 force shapes whose march forms the next step's density itself
    (in-tile sources through LDS and wavefront shifts, the rest added by a
    completion pass from whole rows and the segments' edge records): over a
    box of several x tiles with a ragged last tile and segment, ragged y tiles
    and z runs, and over several calls (each starts with a density pass),
    FP32 states stay within the oracle's tolerance and equal the plain march
    of the same tile to FP32 rounding; statistics likewise.  Tiny boxes (one
    site, a last x segment of one site, one or two planes and rows) put a
    site at both edges of its segment, tile and plane run.  In FP64 the
    shapes run the plain march, bit for bit."""
    from oracle import flb
    from paper_1012_3632_amd import Simulation
    nz, ny, nx = shape
    kw = dict(W.params_of("d3q19_256_landau", nx=nx, ny=ny, nz=nz), precision="fp32", eta=eta)
    drho = W.initial_drho(shape, 3, 0.01)
    probe = Simulation(gpu_params(**kw))
    shapes = [probe.launch_shape(c) for c in range(probe.launch_configs()[0])]
    probe.close()
    pd = [c for c, sh in enumerate(shapes) if sh[7] == 2]
    assert len(pd) == 3
    calls = (2, 4, 4)   # even calls keep every call's samples on the oracle's steps
    po = oracle_params(**kw)
    S, st = flb.run(flb.initial_state(po, drho), po, sum(calls), stats_stride=2)
    ref = S.numpy()
    for c in pd:
        twin = next(u for u, sh in enumerate(shapes) if sh[:7] == shapes[c][:7] and sh[7] == 0)
        got = {}
        for cfg in (c, twin):
            sim = Simulation(gpu_params(**kw), drho_init=drho)
            sim.set_launch(cfg)
            for n in calls:
                sim.step(n, stats_stride=2)
            torch.cuda.synchronize()
            got[cfg] = (sim.populations().numpy(), sim.moments())
            sim.close()
        f_pd, (s_pd, s2_pd, ns_pd) = got[c]
        f_tw, (s_tw, s2_tw, _) = got[twin]
        assert rel_err(f_pd, ref) < tol(kw), c
        assert rel_err(f_pd, f_tw) < 1e-6, (c, twin)
        # modes that a box conserves exactly (momentum in a one-site box) have
        # sums of squares at FP32 rounding level, ~1e-18 against ~1e-33 in
        # FP64: an absolute floor at 1e-7 of the largest mode covers them
        floor = 1e-7 * float(np.max(st["sumsq"]))
        np.testing.assert_allclose(s2_pd, st["sumsq"], rtol=5e-5, atol=floor, err_msg=str(c))
        np.testing.assert_allclose(s2_pd, s2_tw, rtol=1e-6, atol=floor, err_msg=str(c))
    kw64 = dict(kw, precision="fp64")
    for c in pd:
        twin = next(u for u, sh in enumerate(shapes) if sh[:7] == shapes[c][:7] and sh[7] == 0)
        a = Simulation(gpu_params(**kw64), drho_init=drho)
        b = Simulation(gpu_params(**kw64), drho_init=drho)
        a.set_launch(c)
        b.set_launch(twin)
        a.step(6, stats_stride=1)
        b.step(6, stats_stride=1)
        torch.cuda.synchronize()
        assert torch.equal(a.state(), b.state()), c
        a.close()
        b.close()


def test_partial_density_march_call_splits():
    """Shapes that form the next density: the same calls give the same bits;
    the same steps split into other calls (each call's first step takes the
    density pass's density) agree to FP32 rounding."""
    from paper_1012_3632_amd import Simulation
    shape = (18, 7, 130)
    kw = dict(W.params_of("d3q19_256_landau", nx=shape[2], ny=shape[1], nz=shape[0]),
              precision="fp32")
    drho = W.initial_drho(shape, 3, 0.01)
    probe = Simulation(gpu_params(**kw))
    pd = next(c for c in range(probe.launch_configs()[0]) if probe.launch_shape(c)[7] == 2)
    probe.close()
    states = []
    for calls in ((8,), (8,), (3, 5)):
        sim = Simulation(gpu_params(**kw), drho_init=drho)
        sim.set_launch(pd)
        for n in calls:
            sim.step(n)
        torch.cuda.synchronize()
        states.append(sim.populations().numpy())
        sim.close()
    assert np.array_equal(states[0], states[1])
    assert rel_err(states[2], states[0]) < 1e-6


def test_partial_density_march_graph_replays():
    """A captured graph of the march that forms the next density (4 steps:
    the density pass, then march and completion pass per step) replayed
    three times, with eager work and synchronizations between the replays,
    gives the bits of eager calls of 4 steps after every replay: states and
    statistics."""
    from paper_1012_3632_amd import Simulation
    shape = (18, 7, 130)
    kw = dict(W.params_of("d3q19_256_landau", nx=shape[2], ny=shape[1], nz=shape[0]),
              precision="fp32")
    drho = W.initial_drho(shape, 3, 0.01)
    a = Simulation(gpu_params(**kw), drho_init=drho)
    b = Simulation(gpu_params(**kw), drho_init=drho)
    pd = next(c for c in range(a.launch_configs()[0]) if a.launch_shape(c)[7] == 2)
    a.set_launch(pd)
    b.set_launch(pd)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.graph_capture(4, stats_stride=2)
        for rep in range(3):
            b.graph_launch()
            a.step(4, stats_stride=2)
            torch.cuda.synchronize()
            assert torch.equal(a.state(), b.state()), rep
            sa, qa, na = a.moments()
            sb, qb, nb = b.moments()
            assert na == nb == 2 * (rep + 1)
            np.testing.assert_array_equal(sa, sb)
            np.testing.assert_array_equal(qa, qb)
            torch.cuda.synchronize()
    a.close()
    b.close()


@pytest.mark.parametrize("eta", [0, 1])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shape", [(13, 37), (64, 64), (1, 1), (3, 200)])
def test_fused_density_bit_identical(shape, precision, eta):
    """D2Q9 force steps that form the density tile from the populations
    themselves (no density pass) give the bits of the same tile after a
    density pass: states and statistics, over ragged, tiny and thin boxes."""
    from paper_1012_3632_amd import Simulation
    ny, nx = shape
    kw = dict(C2, lattice="D2Q9", precision=precision, nx=nx, ny=ny, nz=1, kT=1e-5,
              rho0=1.0, eta=eta, **LANDAU)
    drho = W.initial_drho((1, ny, nx), 4, 0.01)
    probe = Simulation(gpu_params(**kw))
    shapes = [probe.launch_shape(c) for c in range(probe.launch_configs()[0])]
    probe.close()
    fused = [c for c, sh in enumerate(shapes) if sh[7]]
    assert len(fused) == 3
    for c in fused:
        plain = next(u for u, sh in enumerate(shapes) if sh[:7] == shapes[c][:7] and not sh[7])
        a = Simulation(gpu_params(**kw), drho_init=drho)
        b = Simulation(gpu_params(**kw), drho_init=drho)
        a.set_launch(plain)
        b.set_launch(c)
        for n, stride in ((3, 1), (4, 2), (1, 0)):
            a.step(n, stats_stride=stride)
            b.step(n, stats_stride=stride)
        torch.cuda.synchronize()
        assert torch.equal(a.state(), b.state()), (c, plain)
        for x, y in zip(a.moments(), b.moments()):
            np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("precision,dims", [("fp32", (1024, 1024, 1023)),
                                            ("fp64", (1024, 1024, 511))])
def test_maximum_size_windows(precision, dims):
    """The largest lattice 32-bit offsets within a population plane allow (a
    plane just below 4 GiB; the two buffers take ~163 GB of the 288 GB): the
    last sites of every plane are addressed like the first.  In the 128 x 2
    in-place shape, a lone (ordinary) step and then an in-place pair are
    compared on 8^3 windows (at the origin, across the periodic wrap of the
    far corner, at the last sites, and at random places) advanced by the
    oracle with the noise of their global site indices: one step with the
    inner 6^3, two steps with the inner 4^3."""
    from oracle import flb, philox
    from paper_1012_3632_amd import Simulation, lattice_tables
    nx, ny, nz = dims
    rb = 4 if precision == "fp32" else 8
    assert nx * ny * nz * rb < 2 ** 32 <= nx * ny * (nz + 1) * rb
    kw = dict(lattice="D3Q19", precision=precision, nx=nx, ny=ny, nz=nz, rho0=1.0, kT=1e-5,
              rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0, seed=7)
    sim = Simulation(gpu_params(**kw))
    sim.set_launch(10)
    sim.step(3, stats_stride=1)          # a pair in place, then a lone ordinary step
    w = torch.as_tensor(lattice_tables("D3Q19")["w"]).view(-1, 1, 1, 1)
    rng = np.random.default_rng(5)
    Wd = 8
    starts = [(0, 0, 0), (nz - 4, ny - 4, nx - 4), (nz - Wd, ny - Wd, nx - Wd)] + \
             [(int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx)))
              for _ in range(2)]
    ids = [tuple(torch.as_tensor(_window_ids(n, s0, Wd), device="cuda")
                 for n, s0 in zip((nz, ny, nx), st)) for st in starts]

    def windows():
        S = sim.state()
        return [S[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]]
                .to("cpu", torch.float64) + w * kw["rho0"] for iz, iy, ix in ids]

    pw = oracle_params(**dict(kw, nx=Wd, ny=Wd, nz=Wd))
    lat = flb.lattice_of(pw)
    K = len(lat.noncons())

    def advance(S, n0, steps, win):
        iz, iy, ix = (t.cpu().numpy().astype(np.int64) for t in win)
        sites = ((iz[:, None, None] * ny + iy[None, :, None]) * nx + ix[None, None, :]).reshape(-1)
        for k in range(steps):
            z = torch.as_tensor(philox.normals(None, n0 + k, K, kw["seed"], sites=sites))
            S = flb.collide(flb.pull(S, lat), None, n0 + k, pw, lat, z=z.reshape(K, Wd, Wd, Wd))
        return S

    tol = 1e-5 if precision == "fp32" else 1e-12
    for steps in (1, 2):                 # a lone step, then a pair in place
        before = windows()
        n0 = sim.step_index
        sim.step(steps, stats_stride=1)
        after = windows()
        M = steps
        inner = (slice(None),) + (slice(M, Wd - M),) * 3
        for win, S0, S1 in zip(ids, before, after):
            ref = advance(S0, n0, steps, win)
            assert rel_err(S1[inner].numpy(), ref[inner].numpy()) < tol, (steps, win[0][0].item())
    s1, s2, ns = sim.moments()
    assert ns == 6 and np.all(np.isfinite(s1)) and np.all(np.isfinite(s2))
    sim.close()
    del sim
    torch.cuda.empty_cache()


def test_maximum_size_landau_march_windows():
    """The largest FP32 lattice the 32-bit plane offsets allow (1024 x 1024 x
    1023; the populations take 163 GB, the work area 35 GB) for the
    square-gradient fluid, in the z-marching shape that forms the next
    density (partial sums, edge records, ghost rows: the largest of their
    32-bit indices here).  The density fluctuations come from the noise
    (kT = 1e-4, four steps).  20^3 windows of the state (at the origin,
    across the periodic wrap of the far corner, at the last sites, at random
    places) are advanced two steps by the oracle with the noise of their
    global site indices and the inner 8^3 compared with the GPU's, both
    steps in one call (the second uses the density the march formed)."""
    from oracle import flb, philox
    from paper_1012_3632_amd import Simulation, lattice_tables
    nx, ny, nz = 1024, 1024, 1023
    assert nx * ny * nz * 4 < 2 ** 32 <= nx * ny * (nz + 1) * 4
    kw = dict(W.params_of("d3q19_256_landau", nx=nx, ny=ny, nz=nz), precision="fp32", kT=1e-4)
    sim = Simulation(gpu_params(**kw))
    pd = next(c for c in range(sim.launch_configs()[0]) if sim.launch_shape(c)[7] == 2)
    sim.set_launch(pd)
    sim.step(4, stats_stride=1)
    w = torch.as_tensor(lattice_tables("D3Q19")["w"]).view(-1, 1, 1, 1)
    rng = np.random.default_rng(9)
    Wd, M, NS = 20, 6, 2
    starts = [(0, 0, 0), (nz - 10, ny - 10, nx - 10), (nz - Wd, ny - Wd, nx - Wd)] + \
             [(int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx)))
              for _ in range(2)]
    ids = [tuple(torch.as_tensor(_window_ids(n, s0, Wd), device="cuda")
                 for n, s0 in zip((nz, ny, nx), st)) for st in starts]

    def windows():
        S = sim.state()
        return [S[:, iz[:, None, None], iy[None, :, None], ix[None, None, :]]
                .to("cpu", torch.float64) + w * kw["rho0"] for iz, iy, ix in ids]

    before = windows()
    n0 = sim.step_index
    sim.step(NS, stats_stride=1)
    after = windows()
    pw = oracle_params(**dict(kw, nx=Wd, ny=Wd, nz=Wd))
    lat = flb.lattice_of(pw)
    K = len(lat.noncons())
    inner = (slice(None),) + (slice(M, Wd - M),) * 3
    for win, S0, S1 in zip(ids, before, after):
        iz, iy, ix = (t.cpu().numpy().astype(np.int64) for t in win)
        sites = ((iz[:, None, None] * ny + iy[None, :, None]) * nx + ix[None, None, :]).reshape(-1)
        ref = S0
        for k in range(NS):
            z = torch.as_tensor(philox.normals(None, n0 + k, K, kw["seed"], sites=sites)).reshape(K, Wd, Wd, Wd)
            f = flb.pull(ref, lat)
            ref = flb.collide(f, flb.landau_force(flb.density(f), pw, lat), n0 + k, pw, lat, z=z)
        assert rel_err(S1[inner].numpy(), ref[inner].numpy()) < 1e-5, int(win[0][0])
    s1, s2, ns = sim.moments()
    assert ns == 6 and np.all(np.isfinite(s1)) and np.all(np.isfinite(s2))
    sim.close()
    del sim
    torch.cuda.empty_cache()


def test_full_size_batch64_replicas():
    """d3q19_batch64 at full size (64 replicas, 21.6 M sites) with the grid the
    autotuner picks, stepped through a captured graph as in the benchmark;
    the smallest, a middle and the largest replica are compared with the
    oracle run from the same initial state."""
    from oracle import flb
    from paper_1012_3632_amd import Batch
    wl = W.WORKLOADS["d3q19_batch64"]
    edges = W.batch_edges(wl["replicas"], wl["edges"], wl["size_seed"])
    kw = dict(lattice="D3Q19", precision="fp32", rho0=1.0, kT=wl["kT"], rate_bulk=wl["rate_bulk"],
              rate_shear=wl["rate_shear"], rate_ghost=wl["rate_ghost"])
    b = Batch(gpu_params(**kw), [(e, e, e) for e in edges], seeds=list(range(wl["replicas"])))
    b.autotune(repeats=2)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        b.graph_capture(4, stats_stride=1)
        b.graph_launch()
    torch.cuda.synchronize()
    order = np.argsort(edges, kind="stable")
    for r in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        e = int(edges[r])
        po = oracle_params(**dict(kw, nx=e, ny=e, nz=e, seed=r, replica=r))
        S, _ = flb.run(flb.initial_state(po), po, 4)
        w = torch.as_tensor(flb.lattice_of(po).w).view(-1, 1, 1, 1)
        got = b.replica_state(r).to("cpu", torch.float64) + w * 1.0
        assert rel_err(got.numpy(), S.numpy()) < 1e-5, (r, e)
    b.close()
