"""Capillary fluctuations of a planar interface (Sec. VI, capillary fluctuations).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper's second test: a liquid stripe in a periodic box; the local height
h of each interface (eq. height-def: rho(r) = rho_int(y - h(x))) is obtained
by fitting the mean-field profile of eq. denprof to the density of every
column, and the equal-time spectrum of h is compared with the capillary
structure factor kT / (sigma k^2) (eq. capill-static), k^2 read on the lattice
as 2 - 2 cos k, sigma from eq. surf-tension.

* ``mean_field_profile`` eq. denprof, rising (sign +1) or falling (sign -1).
* ``interface_heights``  per column, the h minimizing the squared misfit of
                         the profile over the 2 W + 1 sites nearest y_ref (a
                         bounded scalar minimization, then the zero of the
                         misfit's derivative to full precision).
* ``height_spectrum``    |h(k)|^2, h(k) = sum_x h(x) exp(-i k.x) over the
                         interface plane (1-D for D2Q9, 2-D for D3Q19).
* ``surface_tension``    eq. surf-tension; ``capillary_theory`` the expected
                         |h(k)|^2 = A kT / (sigma sum_a (2 - 2 cos k_a)), A the
                         interface area in sites.
* ``bulk_pressure``      p0 = rho psi'(rho) - psi(rho), the bulk pressure of
                         the eta = 1 force (the LB ideal pressure is replaced),
                         App. A eq. he-force.
* ``laplace_drop``       the interface tension of this scheme by mechanics: a
                         2-D drop relaxed at kT = 0, its equimolar radius R and
                         the bulk pressures inside and outside; Young-Laplace
                         in 2-D gives sigma = R (p_in - p_out).
* ``effective_kappa``    kappa_eff(rho0) = kappa + (eta cs2 - rho0 psi''(rho0))
                         / (4 rho0): the coefficient of k^2 in this lattice
                         scheme's small-k density fluctuations (Ornstein-
                         Zernike form), pinned against the exact linearized
                         step (``spectra.stationary_spectrum``).

Pins: ``tests/test_oracle_capillary.py``.
"""

import numpy as np
from scipy.optimize import brentq, minimize_scalar

from . import lattice as _lattice

CS2 = _lattice.CS2


def mean_field_profile(y, h, rho_L, rho_V, width, sign):
    """(rho_L + rho_V)/2 + sign (rho_L - rho_V)/2 tanh(2 (y - h) / width)."""
    return 0.5 * (rho_L + rho_V) + sign * 0.5 * (rho_L - rho_V) * np.tanh(2.0 * (y - h) / width)


def interface_heights(rho, y_ref, sign, half_window, rho_L, rho_V, width):
    """Height of one interface in every column.

    rho: array (n, ncol), the density along the profile axis (periodic, n
    sites) for each column.  The window is y = y0 + j, j = -W..W, with
    y0 = floor(y_ref + 1/2), read at y mod n; h is returned in the same
    (unwrapped) coordinate, searched in [y0 - W, y0 + W]."""
    rho = np.asarray(rho, dtype=np.float64)
    n, ncol = rho.shape
    y0 = int(np.floor(y_ref + 0.5))
    ys = np.arange(y0 - half_window, y0 + half_window + 1)
    win = rho[ys % n]
    out = np.empty(ncol)
    lo, hi = y0 - half_window, y0 + half_window
    for c in range(ncol):
        r = win[:, c]

        def misfit(h):
            return np.sum((r - mean_field_profile(ys, h, rho_L, rho_V, width, sign)) ** 2)

        def slope(h):
            # -dE/dh / 2 = sum (rho - m) dm/dy at y - h: zero at the minimizer
            t = np.tanh(2.0 * (ys - h) / width)
            m = 0.5 * (rho_L + rho_V) + sign * 0.5 * (rho_L - rho_V) * t
            return np.sum((r - m) * sign * 0.5 * (rho_L - rho_V) * (1 - t * t) * 2.0 / width)

        # the bounded minimizer stops at a relative tolerance of sqrt(eps) |h|;
        # the stationarity condition is then solved to full precision
        h = minimize_scalar(misfit, bounds=(lo, hi), method="bounded",
                            options={"xatol": 1e-12, "maxiter": 500}).x
        a, b = max(lo, h - 1e-4), min(hi, h + 1e-4)
        if slope(a) * slope(b) < 0:
            h = brentq(slope, a, b, xtol=1e-14, rtol=4 * np.finfo(float).eps)
        out[c] = h
    return out


def height_spectrum(h):
    """|h(k)|^2 of heights over the interface plane (shape (nx,) or (ny, nx))."""
    return np.abs(np.fft.fftn(np.asarray(h, dtype=np.float64))) ** 2


def surface_tension(rho_L, rho_V, kappa, beta):
    """sigma = (rho_L - rho_V)^3 sqrt(2 kappa beta) / 6 (eq. surf-tension)."""
    return (rho_L - rho_V) ** 3 / 6.0 * np.sqrt(2.0 * kappa * beta)


def interface_width(rho_L, rho_V, kappa, beta):
    """w = sqrt(8 kappa / beta) / (rho_L - rho_V) (eq. interf-width)."""
    return np.sqrt(8.0 * kappa / beta) / (rho_L - rho_V)


def capillary_theory(k_axes, kT, sigma, area):
    """Expected |h(k)|^2 of one snapshot: area kT / (sigma sum_a (2 - 2 cos k_a))
    (eq. capill-static with the lattice Laplacian's symbol for k^2); NaN at 0."""
    lap = sum(2.0 - 2.0 * np.cos(k) for k in k_axes)
    with np.errstate(divide="ignore"):
        return np.where(lap > 0, area * kT / (sigma * np.where(lap > 0, lap, 1.0)), np.nan)


def _psi(p, r):
    d = r - p.rho_c
    return p.a * d * d + p.b * d ** 4


def _psi2(p, r):
    return 2 * p.a + 12 * p.b * (r - p.rho_c) ** 2


def effective_kappa(p, rho):
    """kappa + (eta cs2 - rho psi''(rho)) / (4 rho): the square-gradient
    coefficient of this lattice scheme's small-k density fluctuations."""
    return p.kappa + (p.eta * CS2 - rho * _psi2(p, rho)) / (4.0 * rho)


def bulk_pressure(p, rho):
    """p0 = rho psi'(rho) - psi(rho): the pressure of a uniform phase under the
    eta = 1 force (F = -rho grad mu + cs2 grad rho cancels the LB pressure
    rho cs2, and -rho grad psi' = -grad p0)."""
    d = rho - p.rho_c
    return rho * (2 * p.a * d + 4 * p.b * d ** 3) - _psi(p, rho)


def laplace_drop(p, L, R0, nsteps, rho_L, rho_V, width):
    """A liquid drop of radius R0 (mean-field profile of eq. denprof, width
    ``width``) centred in an L x L periodic D2Q9 box of vapour, relaxed with
    the oracle step at kT = 0 for ``nsteps`` steps.

    Returns dict(R, rho_in, rho_out, dp, sigma): the bulk densities (the mean
    density at distance below R0 - 3 width from the centre, and above
    R0 + 3 width), the equimolar radius R = sqrt(sum (rho - rho_out) /
    (pi (rho_in - rho_out))), the bulk pressure difference
    dp = p0(rho_in) - p0(rho_out), and sigma = R dp, the tension by the 2-D
    Young-Laplace law dp = sigma / R."""
    from . import flb
    if p.lattice != "D2Q9" or p.force_model != 1 or p.eta != 1:
        raise ValueError("the drop is a D2Q9 run with the eta = 1 force")
    q = p.with_(nx=L, ny=L, nz=1, kT=0.0)
    y, x = np.mgrid[0:L, 0:L] + 0.5 - L / 2
    r = np.hypot(x, y)
    rho = 0.5 * (rho_L + rho_V) - 0.5 * (rho_L - rho_V) * np.tanh(2 * (r - R0) / width)
    lat = flb.lattice_of(q)
    S = flb.initial_state(q, (rho - q.rho0)[None])
    for k in range(nsteps):
        S = flb.step(S, k, q, lat)
    d = flb.fields(S, q, lat)[0][0].numpy()
    rin = float(d[r < R0 - 3 * width].mean())
    rout = float(d[r > R0 + 3 * width].mean())
    R = float(np.sqrt((d - rout).sum() / (np.pi * (rin - rout))))
    dp = float(bulk_pressure(q, rin) - bulk_pressure(q, rout))
    return dict(R=R, rho_in=rin, rho_out=rout, dp=dp, sigma=R * dp)
