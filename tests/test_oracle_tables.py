"""Pins of the oracle's lattice tables against what the paper prints or fixes.

Paper passages: Sec. III eqs. feq, forcing-term, moments, moments-inv, T-orthog,
T-complete, adv-fourier; Sec. IV eqs. G-ideal, noise-ideal, force-mom and the
identity A G = -G A^dagger stated after eq. noise-ideal; Sec. V lam^LB and
eq. noise-lbe; App. B table tab:modes-d2q9 and eq. TD2Q9; App. C eq. adv-op.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
import torch

from oracle import flb, lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_blocks(name):
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            if line.isalpha():
                cur = line
                blocks[cur] = []
                continue
            blocks[cur].append([float(Fraction(t)) for t in line.split()])
    return {k: np.array(v) for k, v in blocks.items()}


LATS = [lattice.d2q9(), lattice.d3q19()]


def test_d2q9_basis_equals_printed_matrix():
    g = _read_blocks("d2q9_basis.txt")
    lat = lattice.d2q9()
    np.testing.assert_array_equal(lat.T, g["T"])
    np.testing.assert_allclose(lat.N, g["N"][0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(lat.w.sum(), 1.0, atol=1e-15)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_orthogonality_and_completeness(lat):
    # eq. T-orthog: sum_i w_i T_ai T_bi = N_a delta_ab
    G = (lat.T * lat.w) @ lat.T.T
    np.testing.assert_allclose(G, np.diag(lat.N), atol=1e-15)
    # eq. T-complete: w_i sum_a T_ai T_aj / N_a = delta_ij
    C = lat.w[:, None] * (lat.T.T / lat.N) @ lat.T
    np.testing.assert_allclose(C, np.eye(lat.q), atol=1e-14)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_lattice_isotropy(lat):
    """Weights make the moments isotropic through fourth order with cs2 = 1/3
    (needed for eq. feq to give the stated moments)."""
    c = lat.c[:, : lat.d].astype(float)
    w = lat.w
    d = lat.d
    cs2 = lattice.CS2
    np.testing.assert_allclose(w.sum(), 1.0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), cs2 * np.eye(d), atol=1e-15)
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic->abc", w, c, c, c), 0, atol=1e-15)
    dd = np.eye(d)
    iso4 = cs2 ** 2 * (np.einsum("ab,cd->abcd", dd, dd) + np.einsum("ac,bd->abcd", dd, dd)
                       + np.einsum("ad,bc->abcd", dd, dd))
    np.testing.assert_allclose(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c), iso4, atol=1e-15)


def test_d2q9_equilibrium_moments_printed():
    """m^eq column of table tab:modes-d2q9: rho, rho u, 3 rho u^2,
    rho(ux^2 - uy^2), rho ux uy and zero on the ghosts."""
    lat = lattice.d2q9()
    rng = np.random.default_rng(0)
    rho = torch.tensor(1 + 0.1 * rng.standard_normal(50))
    u = torch.tensor(0.05 * rng.standard_normal((2, 50)))
    m = flb.moments(flb.equilibrium(rho, u, lat), lat).numpy()
    r, ux, uy = rho.numpy(), u[0].numpy(), u[1].numpy()
    expect = np.stack([r, r * ux, r * uy, 3 * r * (ux ** 2 + uy ** 2), r * (ux ** 2 - uy ** 2),
                       r * ux * uy, 0 * r, 0 * r, 0 * r])
    np.testing.assert_allclose(m, expect, atol=1e-15)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_equilibrium_has_no_ghost_projection(lat):
    """Sec. III: with the w-weighted basis, T_ai f^eq_i = 0 on ghost modes,
    and the stress moments are those of rho u u (eq. f-moments)."""
    rng = np.random.default_rng(1)
    rho = torch.tensor(1 + 0.1 * rng.standard_normal(40))
    u = torch.tensor(0.05 * rng.standard_normal((lat.d, 40)))
    feq = flb.equilibrium(rho, u, lat)
    m = flb.moments(feq, lat).numpy()
    ghosts = [a for a, k in enumerate(lat.classes) if k == lattice.GHOST]
    np.testing.assert_allclose(m[ghosts], 0, atol=1e-15)
    c = lat.c[:, : lat.d].astype(float)
    # second moment: sum_i f^eq c c = rho cs2 I + rho u u
    P = np.einsum("ix,iy,in->xyn", c, c, feq.numpy())
    expect = (np.einsum("n,xy->xyn", rho.numpy(), lattice.CS2 * np.eye(lat.d))
              + np.einsum("n,xn,yn->xyn", rho.numpy(), u.numpy(), u.numpy()))
    np.testing.assert_allclose(P, expect, atol=1e-15)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_forcing_moments(lat):
    """Sec. IV eq. force-mom and Sec. V eq. lbe-moments: the forcing term has no
    mass, momentum moment F, second moment uF + Fu, no ghost projection."""
    rng = np.random.default_rng(2)
    u = torch.tensor(0.05 * rng.standard_normal((lat.d, 30)))
    F = torch.tensor(1e-3 * rng.standard_normal((lat.d, 30)))
    Phi = flb.forcing(u, F, lat).numpy()
    c = lat.c[:, : lat.d].astype(float)
    np.testing.assert_allclose(Phi.sum(0), 0, atol=1e-18)
    np.testing.assert_allclose(np.einsum("ix,in->xn", c, Phi), F.numpy(), atol=1e-17)
    P = np.einsum("ix,iy,in->xyn", c, c, Phi)
    uF = np.einsum("xn,yn->xyn", u.numpy(), F.numpy())
    np.testing.assert_allclose(P, uF + uF.transpose(1, 0, 2), atol=1e-17)
    m = flb.moments(torch.tensor(Phi), lat).numpy()
    ghosts = [a for a, k in enumerate(lat.classes) if k == lattice.GHOST]
    np.testing.assert_allclose(m[ghosts], 0, atol=1e-17)


def _advection(lat, k):
    """T diag(k.c) T^-1, the operator of eq. adv-fourier without the -i."""
    kc = lat.c[:, : lat.d] @ k
    return lat.T @ np.diag(kc) @ lat.Tinv


def test_d2q9_advection_equals_printed_matrix():
    """App. C eq. adv-op.  (The printed general formula divides by N_a; the
    printed matrix, and T c T^-1 with (T^-1)_ib = w_i T_bi / N_b, divide by N_b.)"""
    g = _read_blocks("d2q9_advection.txt")
    lat = lattice.d2q9()
    np.testing.assert_allclose(_advection(lat, np.array([1.0, 0.0])), g["AX"], atol=1e-15)
    np.testing.assert_allclose(_advection(lat, np.array([0.0, 1.0])), g["AY"], atol=1e-15)


@pytest.mark.parametrize("lat", LATS, ids=lambda l: l.name)
def test_ideal_gas_fdt(lat):
    """Sec. IV.A: with G = mu rho0 diag(N_a), mu = kT/cs2 (eqs. G-ideal, mu-ideal),
    A G = -G A^dagger, hence L G + G L^dagger = diag(2 lam_a G_aa) (eq. noise-ideal),
    and the momentum variance is rho0 kT (eq. momtm-correl-l)."""
    rng = np.random.default_rng(3)
    kT, rho0 = 1e-5, 1.3
    G = kT / lattice.CS2 * rho0 * np.diag(lat.N)
    mom = [a for a, k in enumerate(lat.classes) if k == lattice.MOM]
    np.testing.assert_allclose(np.diag(G)[mom], rho0 * kT, rtol=1e-14)
    lam = np.array([0.0 if k in (lattice.RHO, lattice.MOM) else rng.uniform(0.2, 1.8)
                    for k in lat.classes])
    for _ in range(5):
        k = rng.uniform(-np.pi, np.pi, lat.d)
        A = -1j * _advection(lat, k)
        np.testing.assert_allclose(A @ G, -G @ A.conj().T, atol=1e-18)
        L = A + np.diag(lam)
        Xi = L @ G + G @ L.conj().T
        np.testing.assert_allclose(Xi, np.diag(2 * lam * np.diag(G)), atol=1e-18)


def test_lb_noise_factor():
    """Sec. V: with lam^LB = 2 lam/(2 + lam), (1 - lam^LB/2)^2 * 2 lam equals
    lam^LB (2 - lam^LB) -- the LB variance of eq. noise-lbe follows from the
    DBE variance of eq. noise-ideal with the factor (1 - lam^LB/2) of
    eq. lbe-mom (the printed (1 + lam^LB/2) would not give it)."""
    lam = np.linspace(0.01, 50, 200)
    lb = 2 * lam / (2 + lam)
    np.testing.assert_allclose((1 - lb / 2) ** 2 * 2 * lam, lb * (2 - lb), rtol=1e-14)
    assert not np.allclose((1 + lb / 2) ** 2 * 2 * lam, lb * (2 - lb))
