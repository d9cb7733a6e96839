"""Pins of the oracle's capillary analysis (``oracle.capillary``, Sec. VI).

* the height fit returns the exact shift of a mean-field profile (eq.
  denprof) placed anywhere in the window, for both orientations, across the
  periodic wrap, and the centre of a symmetric profile of another width;
* eq. surf-tension equals the square-gradient integrals int kappa rho'^2 dy
  over the profile of eqs. denprof / interf-width and
  int sqrt(2 kappa W) drho over the double well of eq. f0-bulk;
* the lattice capillary theory's k^2 -> 2 - 2 cos k is the symbol of the
  nearest-neighbour line tension: sum_x (h(x+1) - h(x))^2 =
  (1/L) sum_k (2 - 2 cos k) |h(k)|^2, with height_spectrum's normalisation;
* the effective square-gradient coefficient kappa_eff equals the one the
  exact linearized step gives at small k (fitted), for random wells, rates,
  densities and both force forms;
* mechanics: p0 = rho psi' - psi is the scheme's bulk pressure (a flat
  interface relaxes to equal p0 in the two phases), and drops obey the 2-D
  Young-Laplace law p_in - p_out = sigma / R with one tension sigma, below
  eq. surf-tension's.
"""

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import capillary as cap
from oracle import flb, spectra

RL, RV, BETA, KAPPA = 1.0, 0.5, 0.1, 0.08


@pytest.mark.parametrize("sign", [1, -1])
@pytest.mark.parametrize("h0,yref", [(100.0, 100.0), (100.37, 100.0), (97.81, 99.6), (1.25, 0.7)])
def test_fit_recovers_the_shift(sign, h0, yref):
    n, ncol = 400, 5
    w = cap.interface_width(RL, RV, KAPPA, BETA)
    y = np.arange(n)
    # periodic image nearest the window
    yy = np.where(y - h0 > n / 2, y - n, y)
    rho = np.repeat(cap.mean_field_profile(yy, h0, RL, RV, w, sign)[:, None], ncol, axis=1)
    h = cap.interface_heights(rho, yref, sign, 20, RL, RV, w)
    np.testing.assert_allclose(h, h0, atol=1e-9)
    # a symmetric profile of another width: the fitted centre is still h0
    rho2 = cap.mean_field_profile(yy, h0, RL, RV, 1.6 * w, sign)[:, None]
    np.testing.assert_allclose(cap.interface_heights(rho2, yref, sign, 20, RL, RV, w), h0,
                               atol=1e-9)


def test_surface_tension_is_the_square_gradient_integral():
    sig = cap.surface_tension(RL, RV, KAPPA, BETA)
    w = cap.interface_width(RL, RV, KAPPA, BETA)
    d = lambda y: 0.5 * (RL - RV) * (2 / w) / np.cosh(2 * y / w) ** 2   # rho_MF'
    np.testing.assert_allclose(quad(lambda y: KAPPA * d(y) ** 2, -80, 80, epsabs=1e-15)[0], sig,
                               rtol=1e-10)
    W = lambda r: BETA * (r - RV) ** 2 * (r - RL) ** 2
    np.testing.assert_allclose(quad(lambda r: np.sqrt(2 * KAPPA * W(r)), RV, RL)[0], sig,
                               rtol=1e-12)


def test_line_tension_symbol():
    rng = np.random.default_rng(2)
    for shape in ((64,), (12, 20)):
        h = rng.standard_normal(shape)
        L = h.size
        ks = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
        lap = sum(2 - 2 * np.cos(k) for k in ks)
        grad2 = sum(((np.roll(h, -1, axis=ax) - h) ** 2).sum() for ax in range(h.ndim))
        np.testing.assert_allclose((lap * cap.height_spectrum(h)).sum() / L, grad2, rtol=1e-12)
        th = cap.capillary_theory(ks, 1e-7, 2e-3, L)
        assert np.isnan(th.flat[0]) and np.all(th.flat[1:] > 0)


def test_effective_kappa_is_the_linearized_steps():
    rng = np.random.default_rng(5)
    checked = 0
    while checked < 6:
        lat = "D2Q9" if checked % 2 == 0 else "D3Q19"
        eta = checked % 3 != 0
        rho0 = rng.uniform(0.5, 1.5)
        p = flb.Params(lattice=lat, nx=1, ny=1, nz=1, kT=1e-7, force_model=1,
                       a=rng.uniform(-0.03, 0.05), b=rng.uniform(0, 0.2),
                       rho_c=rng.uniform(0.5, 1.2), kappa=rng.uniform(0.01, 0.2), eta=int(eta),
                       rho0=rho0, rate_bulk=rng.uniform(0.5, 1.9),
                       rate_shear=rng.uniform(0.5, 1.9), rate_ghost=rng.uniform(0.5, 1.9))
        cs2_0 = (1 - p.eta) / 3 + rho0 * spectra.psi2(p, rho0)
        if cs2_0 <= 0.01:
            continue
        ks = np.linspace(0.004, 0.06, 25)
        th = rng.uniform(0, 1.5)
        st = spectra.stationary_spectrum(p, K=(ks * np.cos(th), ks * np.sin(th), 0 * ks))
        y = (rho0 * p.kT / st[0] - cs2_0) / (rho0 * ks ** 2)
        A = np.stack([np.ones_like(ks), ks ** 2, ks ** 4, ks ** 6], 1)
        kap0 = np.linalg.lstsq(A, y, rcond=None)[0][0]
        np.testing.assert_allclose(kap0 * rho0, cap.effective_kappa(p, rho0) * rho0, atol=2e-5)
        checked += 1


def _capillary_params():
    return flb.Params(lattice="D2Q9", rho0=0.75, kT=0.0, force_model=1,
                      a=-0.5 * BETA * (RL - RV) ** 2, b=BETA, rho_c=0.5 * (RL + RV),
                      kappa=KAPPA, eta=1)


def test_flat_interface_balances_the_bulk_pressure():
    """A flat stripe of the capillary workload relaxed at kT = 0: the two
    phases end at equal bulk pressure p0 (zero curvature, zero Laplace
    pressure), which makes p0 the pressure the drop test compares.  Their
    psi' differ by ~2.4e-4, three times the largest Laplace jump measured
    below: the steady state is mechanical, not that of a free energy with
    bulk density psi."""
    p = _capillary_params().with_(nx=1, ny=96)
    w = cap.interface_width(RL, RV, KAPPA, BETA)
    y = np.arange(96) + 0.5
    rho = RV + 0.5 * (RL - RV) * (np.tanh(2 * (y - 24) / w) - np.tanh(2 * (y - 72) / w))
    S = flb.initial_state(p, (rho - p.rho0).reshape(1, 96, 1))
    S, _ = flb.run(S, p, 6000)
    d = flb.fields(S, p)[0].numpy()[0, :, 0]
    rin, rout = d[48], d[0]
    assert abs(cap.bulk_pressure(p, rin) - cap.bulk_pressure(p, rout)) < 2e-6
    dpsi = lambda r: 2 * p.a * (r - p.rho_c) + 4 * p.b * (r - p.rho_c) ** 3
    assert dpsi(rin) - dpsi(rout) > 1e-4


@pytest.mark.slow
def test_laplace_drops_fix_the_mechanical_tension():
    """Two drops (R 20 in 80^2, R 28 in 112^2) relaxed at kT = 0: the bulk
    pressure jump falls as 1/R (Young-Laplace in 2-D), sigma = R dp agreeing
    within 10 % (the smaller drop's curvature correction); the tension is
    0.55-0.8 of eq. surf-tension's."""
    p = _capillary_params()
    w = cap.interface_width(RL, RV, KAPPA, BETA)
    d1 = cap.laplace_drop(p, 80, 20.0, 3000, RL, RV, w)
    d2 = cap.laplace_drop(p, 112, 28.0, 4000, RL, RV, w)
    assert d1["dp"] > d2["dp"] > 0
    assert abs(d1["sigma"] / d2["sigma"] - 1) < 0.1
    s_eq = cap.surface_tension(RL, RV, KAPPA, BETA)
    for d in (d1, d2):
        assert 0.55 < d["sigma"] / s_eq < 0.8
