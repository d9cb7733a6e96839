"""Pins of the oracle's time step against what the paper and the mathematics fix.

* kT = 0, u = 0: the equilibrium is a fixed point.
* equal non-conserved rates: the MRT update reduces to lattice BGK with the
  second-order forcing (Sec. V eq. lbe-gen with Lambda = lam I), written out
  independently here in population space.
* shear-wave decay at the viscosity nu = cs2 (1/lam^LB - 1/2) (Sec. V lam^LB,
  App. B nu_s = cs2/lam_s).
* exact mass and momentum conservation with noise (Sec. IV.A, after eq.
  noise-ideal), momentum gain F per step under a body force (eq. lbe-mom).
* one-step noise variance rho kT N_a lam(2 - lam)/cs2 (Sec. V eq. noise-lbe).
* stationary mode variances G_aa = rho0 kT N_a / cs2 (Sec. IV.A eqs. G-ideal,
  mu-ideal) and a flat ideal-gas structure factor rho0 kT/cs2 (eq. S-ideal).
"""

import numpy as np
import pytest
import torch

import flb_workloads as W
from oracle import flb, lattice

F64 = torch.float64


def _params(**kw):
    return flb.Params(**kw)


def test_rest_state_is_fixed_point():
    for lat_name, shape in (("D2Q9", (1, 8, 8)), ("D3Q19", (4, 4, 4))):
        p = _params(lattice=lat_name, nz=shape[0], ny=shape[1], nx=shape[2], rho0=1.1,
                    rate_bulk=1.2, rate_shear=1.6, rate_ghost=0.7)
        S0 = flb.initial_state(p)
        S, _ = flb.run(S0, p, 5)
        np.testing.assert_allclose(S.numpy(), S0.numpy(), rtol=1e-14, atol=0)


def _bgk_step(S, F, lam, lat):
    """Lattice BGK with second-order forcing, in population space:
    f* = f - lam (f - f^eq) + (1 - lam/2) Phi, then pull-stream."""
    c = lat.c
    f = torch.stack([torch.roll(S[i], shifts=(int(c[i, 2]), int(c[i, 1]), int(c[i, 0])),
                                dims=(-3, -2, -1)) for i in range(lat.q)])
    rho = f.sum(0)
    cc = torch.as_tensor(c[:, : lat.d], dtype=F64)
    j = torch.einsum("ia,i...->a...", cc, f)
    u = (j + 0.5 * F) / rho
    w = torch.as_tensor(lat.w).view(-1, 1, 1, 1)
    uc = torch.einsum("ia,a...->i...", cc, u)
    Fc = torch.einsum("ia,a...->i...", cc, F)
    usq = (u * u).sum(0)
    feq = w * rho * (1 + 3 * uc + 4.5 * uc * uc - 1.5 * usq)
    Phi = w * (3 * Fc + 9 * uc * Fc - 3 * (u * F).sum(0))
    return f - lam * (f - feq) + (1 - lam / 2) * Phi


@pytest.mark.parametrize("lat_name,shape", [("D2Q9", (1, 12, 10)), ("D3Q19", (5, 6, 7))])
def test_equal_rates_reduce_to_bgk(lat_name, shape):
    lam = 1.37
    p = _params(lattice=lat_name, nz=shape[0], ny=shape[1], nx=shape[2], rate_bulk=lam,
                rate_shear=lam, rate_ghost=lam)
    lat = flb.lattice_of(p)
    S = flb.initial_state(p) + torch.as_tensor(W.random_populations(lat.q, shape, 5, 1e-3))
    F = torch.as_tensor(W.random_populations(lat.d, shape, 6, 1e-4))
    Sa = Sb = S
    for n in range(6):
        Sa = flb.collide(flb.pull(Sa, lat), F, n, p, lat)
        Sb = _bgk_step(Sb, F, lam, lat)
    np.testing.assert_allclose(Sa.numpy(), Sb.numpy(), rtol=0, atol=2e-15)


@pytest.mark.parametrize("lam", [0.8, 1.2, 1.7])
def test_shear_wave_viscosity(lam):
    nx = 128
    p = _params(lattice="D2Q9", nz=1, ny=1, nx=nx, rate_shear=lam, rate_bulk=1.0, rate_ghost=1.0)
    lat = flb.lattice_of(p)
    k = 2 * np.pi / nx
    x = np.arange(nx)
    uy = torch.as_tensor(1e-6 * np.sin(k * x)).view(1, 1, nx)
    u = torch.stack([torch.zeros_like(uy), uy])
    S = flb.equilibrium(torch.ones_like(uy), u, lat)
    amps = []
    for n in range(400):
        S = flb.step(S, n, p, lat)
        if n >= 100:
            rho, j = flb.fields(S, p, lat)
            amps.append(abs(np.fft.fft(j[1].numpy().ravel())[1]))
    rate = -np.polyfit(np.arange(len(amps)), np.log(amps), 1)[0]
    nu = lattice.CS2 * (1 / lam - 0.5)
    np.testing.assert_allclose(rate, nu * k * k, rtol=2e-3)


def test_conservation_with_noise():
    p = _params(lattice="D3Q19", nz=8, ny=10, nx=12, kT=1e-5, rate_bulk=1.2, rate_shear=1.6,
                rate_ghost=1.0, seed=9)
    lat = flb.lattice_of(p)
    S0 = flb.initial_state(p, W.initial_drho((8, 10, 12), 3, 0.01))
    S, _ = flb.run(S0, p, 20)
    c = torch.as_tensor(lat.c[:, :3], dtype=F64)
    m0 = S0.sum().item()
    m1 = S.sum().item()
    assert abs(m1 - m0) / m0 < 1e-13
    j0 = torch.einsum("ia,i...->a", c, S0)
    j1 = torch.einsum("ia,i...->a", c, S)
    assert (j1 - j0).abs().max().item() < 1e-13
    # noise is on: the state did move
    assert (S - S0).abs().max().item() > 1e-4


def test_constant_force_momentum_gain():
    p = _params(lattice="D2Q9", nz=1, ny=16, nx=16, kT=1e-4, seed=3, rate_shear=1.3)
    lat = flb.lattice_of(p)
    S = flb.initial_state(p, W.initial_drho((1, 16, 16), 4, 0.01))
    Fv = torch.tensor([2e-5, -3e-5], dtype=F64)
    F = Fv.view(2, 1, 1, 1).expand(2, 1, 16, 16).clone()
    c = torch.as_tensor(lat.c[:, :2], dtype=F64)
    j0 = torch.einsum("ia,i...->a", c, S)
    nsteps = 25
    for n in range(nsteps):
        S = flb.collide(flb.pull(S, lat), F, n, p, lat)
    j1 = torch.einsum("ia,i...->a", c, S)
    np.testing.assert_allclose((j1 - j0).numpy(), (nsteps * 256 * Fv).numpy(), rtol=1e-10, atol=1e-15)


@pytest.mark.parametrize("noise_rho_local", [1, 0])
def test_one_step_noise_variance(noise_rho_local):
    """From the rest state the post-collision moments are m^eq + xi; every
    non-conserved xi_a has variance rho0 kT N_a lam_a (2 - lam_a) / cs2, the
    conserved ones receive none."""
    n = 64
    p = _params(lattice="D3Q19", nz=n, ny=n, nx=n, kT=1e-5, rate_bulk=1.2, rate_shear=1.6,
                rate_ghost=1.0, seed=7, noise_rho_local=noise_rho_local)
    lat = flb.lattice_of(p)
    S1 = flb.step(flb.initial_state(p), 0, p, lat)
    m = flb.moments(S1, lat).reshape(lat.q, -1).numpy()
    m[0] -= p.rho0
    lam = flb.rates(lat, p).numpy()
    var = p.kT * lat.N * lam * (2 - lam) / lattice.CS2
    V = n ** 3
    for a in range(lat.q):
        if a <= lat.d:
            assert np.abs(m[a]).max() < 1e-15
        else:
            assert abs(m[a].mean()) < 5 * np.sqrt(var[a] / V)
            assert abs((m[a] ** 2).mean() / var[a] - 1) < 5 * np.sqrt(2 / V)


def _run_fdt(p, nsteps, burn):
    lat = flb.lattice_of(p)
    S = flb.initial_state(p)
    S, _ = flb.run(S, p, burn)
    snaps = []
    ssum = np.zeros(lat.q)
    ssq = np.zeros(lat.q)
    for k in range(nsteps - burn):
        f = flb.pull(S, lat)
        a, b = flb.mode_sums(f, p, lat)
        ssum += a
        ssq += b
        snaps.append(f.sum(0).numpy() - p.rho0)
        S = flb.step(S, burn + k, p, lat)
    V = p.nx * p.ny * p.nz
    ns = nsteps - burn
    return lat, ssq / (ns * V), np.array(snaps)


def test_fdt_stationary_variances_d2q9():
    w = W.WORKLOADS["d2q9_32_fp64"]
    p = _params(**W.params_of("d2q9_32_fp64"))
    lat, var, snaps = _run_fdt(p, w["steps"], 500)
    G = p.rho0 * p.kT * lat.N / lattice.CS2
    V = p.nx * p.ny
    ratio = var / G
    nc = lat.noncons()
    np.testing.assert_allclose(ratio[nc], 1.0, atol=0.01)
    # conserved modes: the k = 0 part is frozen, so the site variance is G (1 - 1/V)
    np.testing.assert_allclose(ratio[: lat.d + 1], 1 - 1 / V, atol=0.03)
    # flat ideal-gas structure factor S(k) = <|drho_k|^2>/V = rho0 kT/cs2 (eq. S-ideal)
    rk = np.fft.fftn(snaps.reshape(len(snaps), p.ny, p.nx), axes=(1, 2))
    Sk = (np.abs(rk) ** 2).mean(0) / V
    Sk[0, 0] = np.nan
    target = p.rho0 * p.kT / lattice.CS2
    kx = np.fft.fftfreq(p.nx) * 2 * np.pi
    kmag = np.sqrt(kx[None, :] ** 2 + kx[:, None] ** 2)
    for lo, hi in ((0.1, 1.0), (1.0, 2.0), (2.0, 3.0), (3.0, 4.5)):
        sel = (kmag >= lo) & (kmag < hi)
        np.testing.assert_allclose(np.nanmean(Sk[sel]) / target, 1.0, atol=0.06)


def test_fdt_stationary_variances_d3q19():
    p = _params(**W.params_of("d3q19_128", nx=16, ny=16, nz=16))
    lat, var, _ = _run_fdt(p, 600, 300)
    G = p.rho0 * p.kT * lat.N / lattice.CS2
    ratio = var / G
    nc = lat.noncons()
    np.testing.assert_allclose(ratio[nc], 1.0, atol=0.01)
    np.testing.assert_allclose(ratio[: lat.d + 1], 1.0, atol=0.03)
