"""Pins of oracle.modeq (the linearized modified-equilibrium model, Sec. IV.B)
against what the paper prints and against independent routes:

* the DBE noise of eq. noise-yeo (diagonal as printed; the (e, eps) entry at
  half the printed value, the reading stated in the module, with the
  positive-semidefiniteness argument for it),
* eq. s-nonideal (density correlation) and eq. momtm-correl-l (momentum
  correlation rho0 kT) from G,
* A G = -G A^dagger for this model (stated after eq. noise-yeo),
* the ideal-gas limit (c_s^2 = cs2, kappa = 0): the noise of Sec. V
  eq. noise-lbe, rho0 kT N_a lam (2 - lam) / cs2 on the diagonal,
* mass and momentum conservation of the noise,
* G is the stationary covariance of the LB step (Lyapunov solve),
* the real-space step equals the k-space matrix S(k) C(k) (no noise),
* the generated noise has the covariance Xi(k) (sample average).
"""

import numpy as np
import pytest

from oracle import lattice as L
from oracle import modeq as M

CS2 = 1.0 / 3.0
PAPER = dict(cs2_0=0.265 ** 2, kappa=0.08, rho0=1.0, kT=1e-7)


def _grid(p):
    return M.wavevectors(p)


def _printed_dbe(c2, le, lq, leps, ls, rho0, kT):
    """eq. noise-yeo, entries as printed (D2Q9 norms of App. B)."""
    N = L.get("D2Q9").N
    pre = 2 * rho0 * kT / CS2
    X = np.zeros(np.shape(c2) + (9, 9))
    X[..., 3, 3] = pre * N[3] * (2 - 3 * c2) * le
    X[..., 4, 4] = pre * N[4] * ls
    X[..., 5, 5] = pre * N[5] * ls
    X[..., 6, 6] = pre * N[6] * lq
    X[..., 7, 7] = pre * N[7] * lq
    X[..., 8, 8] = pre * N[8] * (1.25 - 0.75 * c2) * leps
    X[..., 3, 8] = X[..., 8, 3] = pre * 12 * (c2 - CS2) * (le + leps)
    return X


def test_dbe_noise_matches_printed_matrix():
    p = M.ModEqParams(nx=16, ny=12, rate_bulk=0.7, rate_shear=1.3, rate_ghost=0.9, **PAPER)
    K = _grid(p)
    leps = 1.7                                      # distinct from lam_q
    Xi = M.noise_covariance_dbe(p, K, rate_eps=leps)
    c2 = M.sound_speed2(p, K)
    P = _printed_dbe(c2, p.rate_bulk, p.rate_ghost, leps, p.rate_shear, p.rho0, p.kT)
    scale = np.abs(P).max()
    diag = np.eye(9, dtype=bool)
    np.testing.assert_allclose(Xi[..., diag], P[..., diag], atol=1e-13 * scale)
    # (e, eps): half the printed value (reading), every other off-diagonal zero
    np.testing.assert_allclose(Xi[..., 3, 8], 0.5 * P[..., 3, 8], atol=1e-13 * scale)
    np.testing.assert_allclose(Xi[..., 8, 3], 0.5 * P[..., 8, 3], atol=1e-13 * scale)
    off = ~diag
    off[3, 8] = off[8, 3] = False
    assert np.abs(Xi[..., off]).max() < 1e-13 * scale


@pytest.mark.parametrize("c2", [0.07, 0.3, 0.45, 0.55, 0.59])
def test_dbe_noise_reading_is_the_positive_one(c2):
    """With G a covariance (fbar >= 0 up to c_s^2 = 0.6) the computed (e, eps)
    block is positive semidefinite; the printed one is not above ~0.53."""
    p = M.ModEqParams(nx=1, ny=1, cs2_0=c2, kappa=0.0, kT=1.0, rate_bulk=1.0,
                      rate_ghost=1.0)
    K = (np.zeros(1), np.zeros(1))
    assert M.fbar(p, K).min() >= 0
    Xi = M.noise_covariance_dbe(p, K)[0]
    blk = Xi[np.ix_([3, 8], [3, 8])]
    assert np.linalg.eigvalsh(blk).min() >= -1e-12
    P = _printed_dbe(np.array(c2), 1.0, 1.0, 1.0, 1.0, 1.0, 1.0)
    pblk = P[np.ix_([3, 8], [3, 8])]
    if c2 > 0.54:
        assert np.linalg.eigvalsh(pblk).min() < 0


def test_correlations_follow_structure_factor_and_temperature():
    p = M.ModEqParams(nx=20, ny=14, **PAPER)
    K = _grid(p)
    G = M.correlation(p, K)
    c2 = M.sound_speed2(p, K)
    np.testing.assert_allclose(G[..., 0, 0], p.rho0 * p.kT / c2, rtol=1e-13)      # eq. s-nonideal
    for a in (1, 2):
        np.testing.assert_allclose(G[..., a, a], p.rho0 * p.kT, rtol=1e-13)       # eq. momtm-correl-l
    assert np.abs(G[..., 1, 2]).max() < 1e-13 * p.kT
    # the equilibrium moments of fbar are eq. meq-yeo's
    m = M.fbar(p, K) @ L.get("D2Q9").T.T
    d = 6 * (c2 - CS2)
    np.testing.assert_allclose(m[..., 0], p.rho0, rtol=1e-13)
    np.testing.assert_allclose(m[..., 3], p.rho0 * d, atol=1e-13)
    np.testing.assert_allclose(m[..., 8], -p.rho0 * d, atol=1e-13)
    assert np.abs(m[..., [1, 2, 4, 5, 6, 7]]).max() < 1e-13


def test_advection_contribution_vanishes():
    p = M.ModEqParams(nx=9, ny=16, **PAPER)
    K = _grid(p)
    G = M.correlation(p, K)
    A = M.advection_matrix(K)
    R = A @ G + G @ np.conj(np.swapaxes(A, -1, -2))
    assert np.abs(R).max() < 1e-13 * np.abs(G).max()
    assert np.abs(A @ G).max() > 1e-3 * np.abs(G).max()   # not trivially zero


def test_ideal_gas_limit_is_the_lbe_noise():
    p = M.ModEqParams(nx=8, ny=8, cs2_0=CS2, kappa=0.0, kT=2e-5, rho0=1.3, rate_bulk=1.2,
                      rate_shear=1.6, rate_ghost=0.8)
    K = _grid(p)
    Xi = M.noise_covariance(p, K)
    N = L.get("D2Q9").N
    lam = np.array([0, 0, 0, 1.2, 1.6, 1.6, 0.8, 0.8, 0.8])
    want = np.diag(p.rho0 * p.kT * N * lam * (2 - lam) / CS2)       # Sec. V eq. noise-lbe
    np.testing.assert_allclose(Xi, np.broadcast_to(want, Xi.shape), atol=1e-13 * want.max())


def test_noise_conserves_mass_and_momentum_and_is_white_off_the_block():
    p = M.ModEqParams(nx=12, ny=10, rate_bulk=1.1, rate_shear=1.7, rate_ghost=1.3, **PAPER)
    K = _grid(p)
    Xi = M.noise_covariance(p, K)
    s = np.abs(Xi).max()
    assert np.abs(Xi[..., :3, :]).max() < 1e-13 * s
    assert np.abs(Xi[..., :, :3]).max() < 1e-13 * s
    for a in (4, 5, 6, 7):
        np.testing.assert_allclose(Xi[..., a, a], Xi[0, 0, a, a], rtol=1e-12)
    # positive semidefinite at every k
    assert np.linalg.eigvalsh(Xi).min() >= -1e-13 * s


@pytest.mark.parametrize("rates", [(1.0, 1.0, 1.0), (1.2, 1.6, 0.7), (0.4, 1.9, 1.5)])
def test_G_is_the_stationary_covariance(rates):
    rb, rs, rg = rates
    p = M.ModEqParams(nx=12, ny=10, rate_bulk=rb, rate_shear=rs, rate_ghost=rg, **PAPER)
    K = _grid(p)
    P = M.stationary_covariance(p, K).reshape(p.ny, p.nx, 9, 9)
    G = M.correlation(p, K)
    ok = np.isfinite(P[..., 0, 0].real)
    assert ok.sum() >= p.nx * p.ny - 4
    assert np.abs(P - G)[ok].max() < 1e-11 * np.abs(G).max()


def test_real_space_step_is_the_k_space_matrix():
    p = M.ModEqParams(nx=11, ny=7, rate_bulk=1.2, rate_shear=1.6, rate_ghost=0.9,
                      **dict(PAPER, kT=0.0))
    rng = np.random.default_rng(5)
    S = rng.standard_normal((9, p.ny, p.nx))
    S1 = M.step(S, 0, p)
    K = _grid(p)
    T, Ti = L.get("D2Q9").T, L.get("D2Q9").Tinv
    # state in k: pulled moments m(k) = Sm(k) T S(k); post-collision C m
    Sk = np.fft.fft2(S, axes=(1, 2))
    phase = np.exp(-1j * (K[0][None] * L.get("D2Q9").c[:, 0, None, None]
                          + K[1][None] * L.get("D2Q9").c[:, 1, None, None]))
    mk = np.einsum("ai,iyx->ayx", T, phase * Sk)
    C = M.collision_matrix(p, K)
    mk1 = np.einsum("yxab,byx->ayx", C, mk)
    S1k = np.einsum("ia,ayx->iyx", Ti, mk1)
    np.testing.assert_allclose(S1, np.fft.ifft2(S1k, axes=(1, 2)).real, atol=1e-12)


def test_generated_noise_has_the_covariance_Xi():
    """Sample covariance of xi_hat(k) over 400 draws against V Xi(k): the
    average ratio over k to 1.5 %, the ratio at each k to 6 sigma."""
    p = M.ModEqParams(nx=16, ny=12, rate_bulk=1.2, rate_shear=1.6, rate_ghost=0.9, seed=77,
                      **dict(PAPER, kT=1e-5))
    K = _grid(p)
    V = p.nx * p.ny
    Xi = M.noise_covariance(p, K)
    nd = 400
    acc = np.zeros((p.ny, p.nx, 6, 6), dtype=complex)
    for n in range(nd):
        xk = np.fft.fft2(M.noise(n, p), axes=(1, 2))
        acc += np.einsum("ayx,byx->yxab", xk, np.conj(xk))
    acc /= nd * V
    want = Xi[..., M.NONCONS, :][..., M.NONCONS]
    for a, b in ((0, 0), (5, 5), (1, 1), (3, 3)):
        r = acc[..., a, b].real / want[..., a, b]
        assert abs(r.mean() - 1) < 0.015, (a, b, r.mean())
        assert np.abs(r - 1).max() < 6 / np.sqrt(nd)
    # cross term: compare Re <xi_e xi_eps*> against Xi_e,eps on the scale of the block
    sc = np.sqrt(want[..., 0, 0] * want[..., 5, 5])
    dev = (acc[..., 0, 5].real - want[..., 0, 5]) / sc
    assert abs(dev.mean()) < 0.015 and np.abs(dev).max() < 6 / np.sqrt(nd)
    # distinct white modes are uncorrelated
    assert np.abs(acc[..., 1, 2]).mean() / np.sqrt(want[..., 1, 1] * want[..., 2, 2]).mean() < 0.1


def test_run_reaches_G():
    """A 16 x 16 run: the time-averaged |m_a(k)|^2 / (V G_aa(k)) is 1 within
    sampling error (the paper's equilibration measure, for this model)."""
    p = M.ModEqParams(nx=16, ny=16, rate_bulk=1.0, rate_shear=1.0, rate_ghost=1.0, seed=4,
                      **dict(PAPER, kT=1e-5))
    K = _grid(p)
    V = p.nx * p.ny
    G = M.correlation(p, K)
    T = L.get("D2Q9").T
    S = M.run(M.initial_state(p), p, 200)
    acc = np.zeros((9, p.ny, p.nx))
    ns = 0
    for n in range(200, 1400):
        S = M.step(S, n, p)
        if n % 4 == 0:
            mk = np.fft.fft2(np.tensordot(T, M.pull(S), axes=([1], [0])), axes=(1, 2))
            acc += np.abs(mk) ** 2
            ns += 1
    Gd = np.stack([G[..., a, a] for a in range(9)])
    r = acc / (ns * V * Gd)
    r[:, 0, 0] = np.nan
    for a in range(9):
        assert abs(np.nanmean(r[a]) - 1) < 0.06, (a, np.nanmean(r[a]))
