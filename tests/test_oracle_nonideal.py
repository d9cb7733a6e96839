"""Pins of the oracle's non-ideal (force-based) fluid.

* stencils: on a plane wave the isotropic gradient and Laplacian have the
  closed-form symbols of central differences.
* the force conserves mass exactly (Guo forcing has no mass moment).
* eta = 1 (App. A eq. he-force) at kT = 0: a flat liquid slab relaxes to the
  mean-field tanh profile of Sec. VI eq. denprof with the coexistence densities
  of the double well (eq. f0-bulk) and the width of eq. interf-width.
* eta = 0 at kT > 0: small-k structure factor of Ornstein-Zernike form
  S(k) = rho0 kT / c_s^2(k) (App. A eqs. he-cs2 and the OZ form after
  eq. freeE-funct), with c_s^2(k) = cs2 + rho0 psi''(rho0) + kappa rho0 k^2
  (the LB ideal pressure cs2 adds to psi when the force omits it).
  At all k the oracle's S(k) is pinned through the exact linearized step
  (``test_oracle_spectra.py``).
"""

import numpy as np
import pytest
import torch
from scipy.optimize import curve_fit

import flb_workloads as W
from oracle import flb, lattice

F64 = torch.float64


@pytest.mark.parametrize("lat_name", ["D2Q9", "D3Q19"])
def test_stencil_symbols(lat_name):
    lat = lattice.get(lat_name)
    n = 16
    shape = (1, n, n) if lat.d == 2 else (n, n, n)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    k = 2 * np.pi * 3 / n
    phi = torch.as_tensor(np.cos(k * x))
    g = flb.grad_h(phi, lat).numpy()
    np.testing.assert_allclose(g[0], -np.sin(k * x) * np.sin(k), atol=1e-14)
    np.testing.assert_allclose(g[1:], 0, atol=1e-14)
    lap = flb.lap_h(phi, lat).numpy()
    np.testing.assert_allclose(lap, -(2 - 2 * np.cos(k)) * np.cos(k * x), atol=1e-14)
    # diagonal wave: symbol of the isotropic stencil along (1,1)
    phi = torch.as_tensor(np.cos(k * (x + y)))
    lap = flb.lap_h(phi, lat).numpy()
    c = lat.c[:, :3].astype(float)
    sym = 2 / lattice.CS2 * sum(lat.w[i] * (np.cos(k * (c[i, 0] + c[i, 1])) - 1) for i in range(lat.q))
    np.testing.assert_allclose(lap, sym * np.cos(k * (x + y)), atol=1e-14)
    # small-k limit of that symbol is -|k|^2 = -2 k^2
    ks = 1e-3
    sym_s = 2 / lattice.CS2 * sum(lat.w[i] * (np.cos(ks * (c[i, 0] + c[i, 1])) - 1) for i in range(lat.q))
    np.testing.assert_allclose(sym_s, -2 * ks * ks, rtol=1e-5)


def test_landau_mass_conservation():
    p = flb.Params(**W.params_of("d2q9_256_adjoint", nx=24, ny=20))
    S0 = flb.initial_state(p, W.initial_drho((1, 20, 24), 1, 0.01))
    S, _ = flb.run(S0, p, 30)
    assert abs(S.sum().item() - S0.sum().item()) / S0.sum().item() < 1e-13


def test_flat_interface_tanh_profile():
    """eta = 1, kT = 0: a flat slab relaxes to a tanh profile (Sec. VI eq.
    denprof) between the coexistence densities rho_c +- sqrt(-a/2b) of the
    double well (eq. f0-bulk).  Its width follows eq. interf-width,
    w^2 = 4 kappa_eff / (-a), with kappa_eff = kappa + 1/12: at rest the Guo
    forcing's second-order streaming term F''/4 (1-D, all rates 1) turns the
    large cs2 grad rho part of the eta = 1 force into an extra square-gradient
    coefficient cs2/4 (a lattice correction derived for this test, not printed
    in the paper)."""
    ny = 64
    p = flb.Params(lattice="D2Q9", nx=1, ny=ny, nz=1, kT=0.0, force_model=1, a=-0.01, b=0.1,
                   rho_c=1.0, kappa=0.05, eta=1)
    dr = np.sqrt(-p.a / (2 * p.b))                      # rho_L,V = rho_c +- dr
    idx = np.arange(ny)
    y1, y2 = ny / 4, 3 * ny / 4
    start = dr * np.tanh(2 * (idx - y1) / 4.0) * np.tanh(2 * (y2 - idx) / 4.0)
    S = flb.initial_state(p, start.reshape(1, ny, 1))
    S, _ = flb.run(S, p, 6000)
    rho, j = flb.fields(S, p)
    prof = rho.numpy()[0, :, 0]
    assert np.abs(j.numpy()).max() < 1e-6           # (nearly) at rest
    np.testing.assert_allclose(prof[ny // 2], p.rho_c + dr, rtol=1e-2)
    np.testing.assert_allclose(prof[0], p.rho_c - dr, rtol=1e-2)

    def tanh(x, rl, rv, x0, w):
        return 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(2 * (x - x0) / w)

    sel = slice(2, ny // 2 - 2)
    popt, _ = curve_fit(tanh, idx[sel], prof[sel], p0=[1.2, 0.8, y1, 5.0])
    resid = np.abs(tanh(idx[sel], *popt) - prof[sel]).max()
    assert resid < 0.01 * 2 * dr
    w_eff = 2 * np.sqrt((p.kappa + 1 / 12) / (-p.a))
    np.testing.assert_allclose(popt[3], w_eff, rtol=0.03)


def test_ornstein_zernike_structure_factor():
    n = 32
    p = flb.Params(lattice="D2Q9", nx=n, ny=n, nz=1, kT=1e-5, force_model=1, a=0.05, b=0.0,
                   rho_c=1.0, kappa=0.05, eta=0, seed=21)
    lat = flb.lattice_of(p)
    S = flb.initial_state(p)
    S, _ = flb.run(S, p, 300)
    acc = np.zeros((n, n))
    ns = 0
    for k in range(4000):
        S = flb.step(S, 300 + k, p, lat)
        if k % 4 == 0:
            rho = flb.density(flb.pull(S, lat)).numpy()[0] - p.rho0
            acc += np.abs(np.fft.fft2(rho)) ** 2
            ns += 1
    Sk = acc / ns / (n * n)
    kk = np.fft.fftfreq(n) * 2 * np.pi
    KX, KY = np.meshgrid(kk, kk, indexing="xy")
    c = lat.c[:, :2].astype(float)
    lap_sym = -2 / lattice.CS2 * sum(lat.w[i] * (np.cos(KX * c[i, 0] + KY * c[i, 1]) - 1)
                                     for i in range(lat.q))
    oz = p.rho0 * p.kT / (lattice.CS2 + p.rho0 * 2 * p.a + p.kappa * p.rho0 * lap_sym)
    ideal = p.rho0 * p.kT / lattice.CS2
    kmag = np.sqrt(KX ** 2 + KY ** 2)
    sel = (kmag > 0) & (kmag < 0.7)
    r = (Sk[sel] / oz[sel]).mean()
    assert abs(r - 1) < 0.05, r
    # the non-ideal terms are resolved: ideal-gas S(k) is far off
    assert abs((Sk[sel] / ideal).mean() - 1) > 0.15
