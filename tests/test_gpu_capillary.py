"""Interface heights and field spectra on the GPU (flb_interface_heights,
flb_field_spectrum) against the oracle, and the Sec. VI capillary run
against the capillary structure factor.

Heights: both sides start from the same mean-field stripe and advance the
same noisy steps; the GPU's fitted heights equal the oracle's fit of the
oracle's density within the error the population bar allows (the density
error times sum |m'| / sum m'^2 of the fit)."""

import numpy as np
import pytest
import torch

import flb_workloads as W
from helpers import F32_TOL, F64_TOL, gpu_params, oracle_params

pytestmark = pytest.mark.gpu

WELL = dict(force_model=1, a=-0.0125, b=0.1, rho_c=0.75, kappa=0.08, eta=1)
RL, RV = 1.0, 0.5

# (lattice, precision, (nz, ny, nx), (y1, y2), half_window)
CASES = [
    ("D2Q9", "fp64", (1, 48, 37), (12.3, 35.6), 7),
    ("D2Q9", "fp32", (1, 48, 37), (12.3, 35.6), 7),
    ("D2Q9", "fp64", (1, 40, 16), (1.4, 21.0), 6),      # window across the periodic wrap
    ("D3Q19", "fp64", (30, 5, 7), (7.6, 22.2), 5),
    ("D3Q19", "fp32", (30, 5, 7), (7.6, 22.2), 5),
]


def _width():
    from oracle import capillary as cap
    return cap.interface_width(RL, RV, WELL["kappa"], 0.1)


def _run_pair(kw, y12, nsteps):
    from oracle import flb
    from paper_1012_3632_amd import Simulation
    shape = (kw["nz"], kw["ny"], kw["nx"])
    drho = W.stripe_drho(shape, y12[0], y12[1], RL, RV, _width(), kw["rho0"])
    sim = Simulation(gpu_params(**kw), drho_init=drho)
    sim.step(nsteps)
    po = oracle_params(**kw)
    S, _ = flb.run(flb.initial_state(po, drho), po, nsteps)
    return sim, po, S


def _oracle_heights(S, po, y12, W_half):
    from oracle import capillary as cap
    from oracle import flb
    lat = flb.lattice_of(po)
    rho = flb.density(flb.pull(S, lat)).numpy()            # (nz, ny, nx)
    if lat.d == 2:
        cols = rho[0]                                       # (ny, nx): profile along y
    else:
        cols = rho.reshape(po.nz, po.ny * po.nx)            # profile along z
    hs = [cap.interface_heights(cols, y12[0], 1, W_half, RL, RV, _width()),
          cap.interface_heights(cols, y12[1], -1, W_half, RL, RV, _width())]
    return np.array(hs), cols


def _height_bound(cols, y12, W_half, drho_err):
    """max over columns of drho_err * sum |m'| / sum m'^2 for the window."""
    from oracle import capillary as cap
    n = cols.shape[0]
    w = _width()
    out = []
    for y_ref, sg in ((y12[0], 1), (y12[1], -1)):
        y0 = int(np.floor(y_ref + 0.5))
        ys = np.arange(y0 - W_half, y0 + W_half + 1)
        t = np.tanh(2 * (ys - y_ref) / w)
        mp = np.abs(0.5 * (RL - RV) * (1 - t * t) * 2 / w)
        out.append(drho_err * mp.sum() / (mp * mp).sum())
    return max(out)


@pytest.mark.parametrize("case", CASES, ids=lambda c: "-".join(map(str, c[:3])))
def test_heights_match_oracle(case):
    lat, prec, shape, y12, W_half = case
    nz, ny, nx = shape
    kw = dict(lattice=lat, precision=prec, nx=nx, ny=ny, nz=nz, rho0=0.75, kT=1e-5,
              rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0, seed=8, **WELL)
    sim, po, S = _run_pair(kw, y12, 4)
    ifs = [(y12[0], 1, W_half), (y12[1], -1, W_half)]
    h_gpu = sim.interface_heights(ifs, RL, RV, _width()).cpu().numpy().reshape(2, -1)
    h_ref, cols = _oracle_heights(S, po, y12, W_half)
    tol = F64_TOL if prec == "fp64" else F32_TOL
    drho_err = (9 if lat == "D2Q9" else 19) * tol * 0.5      # Q populations, max |f| < 0.5
    bound = _height_bound(cols, y12, W_half, drho_err) + 1e-9
    err = np.abs(h_gpu - h_ref).max()
    assert err <= bound, (err, bound)
    # the heights are near the stripe's interfaces
    assert np.all(np.abs(h_gpu[0] - y12[0]) < 2) and np.all(np.abs(h_gpu[1] - y12[1]) < 2)


def test_full_size_capillary_heights():
    """The 1024 x 400 stripe workload (FP32) after 3 steps: heights of both
    interfaces in every column against the oracle."""
    wl = W.WORKLOADS["d2q9_capillary"]
    kw = dict(W.params_of("d2q9_capillary"), precision="fp32", kT=1e-5, rho0=wl["rho0"])
    y12 = wl["stripe"]
    sim, po, S = _run_pair(kw, y12, 3)
    ifs = [(y12[0], 1, 25), (y12[1], -1, 25)]
    h_gpu = sim.interface_heights(ifs, RL, RV, _width()).cpu().numpy()
    h_ref, cols = _oracle_heights(S, po, y12, 25)
    bound = _height_bound(cols, y12, 25, 9 * F32_TOL * 0.5) + 1e-9
    assert np.abs(h_gpu - h_ref).max() <= bound


@pytest.mark.parametrize("shape", [(3, 1, 1, 7), (2, 1, 5, 9), (3, 4, 6, 10), (1, 1, 1, 1024),
                                   (1, 1, 1, 1)])
def test_field_spectrum_matches_fft(shape):
    from paper_1012_3632_amd import field_spectrum
    rng = np.random.default_rng(11)
    a = rng.standard_normal(shape)
    b = rng.standard_normal(shape)
    spec = field_spectrum(torch.as_tensor(a, device="cuda"))
    field_spectrum(torch.as_tensor(b, device="cuda"), spec)
    torch.cuda.synchronize()
    ref = (np.abs(np.fft.fftn(a, axes=(1, 2, 3))) ** 2 + np.abs(np.fft.fftn(b, axes=(1, 2, 3))) ** 2)
    np.testing.assert_allclose(spec.cpu().numpy(), ref, rtol=1e-10, atol=1e-10 * ref.max())


def test_heights_and_spectrum_reject_bad_arguments():
    from paper_1012_3632_amd import Simulation, field_spectrum
    from paper_1012_3632_amd._lib import FLBError
    ideal = Simulation(gpu_params(lattice="D2Q9", precision="fp32", nx=8, ny=20, kT=0.0))
    with pytest.raises(FLBError):
        ideal.interface_heights([(5.0, 1, 3)], RL, RV, 5.0)
    sim = Simulation(gpu_params(lattice="D2Q9", precision="fp32", nx=8, ny=20, rho0=0.75,
                                **WELL))
    for ifs in ([(5.0, 1, 10)], [(25.0, 1, 3)], [(5.0, 0, 3)], [(5.0, 1, 3)] * 9):
        with pytest.raises(FLBError):
            sim.interface_heights(ifs, RL, RV, 5.0)
    with pytest.raises(FLBError):
        sim.interface_heights([(5.0, 1, 3)], RL, RL, 5.0)
    with pytest.raises(FLBError):
        field_spectrum(torch.zeros((1, 1, 1, 1025), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()


def _bins(spec, nsnap, th, k, lo, hi):
    sel = (k >= lo) & (k < hi)
    return float(np.mean(spec[:, sel] / (nsnap * th[sel])))


def test_capillary_run_height_spectrum():
    """Sec. VI on the GPU: the 1024 x 400 stripe (the paper's parameters),
    2 x 10^5 steps, 300 snapshots.  The height spectrum of both interfaces has
    the capillary form A kT / (sigma_cw (2 - 2 cos k)) at small k: the ratio
    to it with sigma_cw fitted on 0.1 <= k < 0.4 is within 20 % of 1 for
    k < 0.1.  The scheme does not reach eq. capill-static with the paper's
    tension: sigma_cw is ~1.4-1.5 times eq. surf-tension's, and the scheme's
    own mechanical tension (the oracle's Laplace drops, tests/golden) is
    ~0.66 times it, so the spectrum is ~0.7 of the law with eq.
    surf-tension's sigma and under 0.6 of it with the mechanical one."""
    import json
    import os
    from paper_1012_3632_amd import capillary as C
    wl = W.WORKLOADS["d2q9_capillary"]
    p = C.paper_params(seed=wl["seed"])
    w = C.mean_field_width(wl["rho_L"], wl["rho_V"], wl["kappa"], wl["beta"])
    spec, nsnap, means, _ = C.run(p, wl["stripe"], wl["rho_L"], wl["rho_V"], w, 200000,
                                  50000, 500)
    assert nsnap == 300
    k = 2 * np.pi * np.arange(p.nx) / p.nx
    s_mf = C.surface_tension(wl["rho_L"], wl["rho_V"], wl["kappa"], wl["beta"])
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                       "laplace_tension.json")))
    s_mech = gold["sigma_inf"]
    th_mf = C.capillary_theory(p, p.kT, s_mf)
    r_mid = _bins(spec, nsnap, th_mf, k, 0.1, 0.4)
    s_cw = s_mf / r_mid                     # the tension the spectrum shows
    th_cw = C.capillary_theory(p, p.kT, s_cw)
    lo = _bins(spec, nsnap, th_cw, k, 0.01, 0.1)
    r_mech = _bins(spec, nsnap, C.capillary_theory(p, p.kT, s_mech), k, 0.01, 0.4)
    print("sigma_cw / sigma_eq %.3f; k<0.1 ratio to sigma_cw law %.3f; ratio to the "
          "mechanical-tension law %.3f" % (s_cw / s_mf, lo, r_mech))
    assert abs(lo - 1) < 0.2
    assert 1.25 < s_cw / s_mf < 1.7
    assert _bins(spec, nsnap, th_mf, k, 0.01, 0.4) < 0.8
    assert r_mech < 0.6
    # the interfaces stayed put (mass conservation) near the stripe's edges
    assert abs(means[0] - wl["stripe"][0]) < 6 and abs(means[1] - wl["stripe"][1]) < 6
