"""The equilibration test of Sec. VI on the HIP library.

A homogeneous fluid at rest is driven by the fluctuating step; after a
burn-in, the equal-time spectra of all LB modes are summed over snapshots on
the GPU (``Simulation.accumulate_spectrum``, i.e. flb_mode_spectrum) and
divided by the variance the theory assigns to each mode and wavevector
(Sec. IV eq. g-mat-forcing): the equilibration ratio, 1 where a mode is
equilibrated.  The paper's run is D2Q9 128^2 at rho0 = 1, kappa 0.08,
c_s 0.265, T 1e-7, tau 1, averaged over 400 snapshots.

The GPU does the stepping and the spectra.  This module adds the host-side
closed forms: G_aa(k), the Landau double well of Sec. VI eq. f0-bulk in the
library's (a, b, rho_c) form, and the averages over |k| shells.
"""

import numpy as np
import torch

from .sim import Params, Simulation, lattice_tables

CS2 = 1.0 / 3.0


def double_well(rho_L, rho_V, cs, rho0=1.0):
    """(a, b, rho_c) with a (r - rho_c)^2 + b (r - rho_c)^4 = beta (r - rho_V)^2
    (r - rho_L)^2 + const (Sec. VI eq. f0-bulk) and beta = cs^2 / (2 rho0
    (rho_L - rho_V)^2), the speed of sound of that well at rho0 = rho_L."""
    beta = cs * cs / (2.0 * rho0 * (rho_L - rho_V) ** 2)
    return -0.5 * beta * (rho_L - rho_V) ** 2, beta, 0.5 * (rho_L + rho_V)


def paper_params(nx=128, ny=128, kT=1e-7, kappa=0.08, cs=0.265, rho_L=1.0, rho_V=0.5, rho0=1.0,
                 rate=1.0, seed=2010, precision="fp32"):
    """Params of the Sec. VI equilibration run: the paper's force (eta = 1),
    the double well set by cs, all rates 1/tau."""
    a, b, rc = double_well(rho_L, rho_V, cs, rho0)
    return Params(lattice="D2Q9", precision=precision, nx=nx, ny=ny, nz=1, rho0=rho0, kT=kT,
                  rate_bulk=rate, rate_shear=rate, rate_ghost=rate, force_model=1, a=a, b=b,
                  rho_c=rc, kappa=kappa, eta=1, seed=seed)


def wavevectors(p):
    """(kx, ky, kz) of every spectrum entry, arrays (nz, ny, nx), folded into
    (-pi, pi]."""
    def axis(n):
        k = 2.0 * np.pi * np.arange(n) / n
        return np.where(k > np.pi, k - 2.0 * np.pi, k)
    kz, ky, kx = np.meshgrid(axis(p.nz), axis(p.ny), axis(p.nx), indexing="ij")
    return kx, ky, kz


def paper_variance(p):
    """G_aa(k) (Sec. IV eq. g-mat-forcing), (q, nz, ny, nx): the density row is
    the structure factor rho0 kT / c_s^2(k) (eq. s-nonideal) with
    c_s^2(k) = (1 - eta) cs2 + rho0 psi''(rho0) + kappa rho0 Lambda(k)
    (App. A eq. he-cs2; Lambda(k) = (2/cs2) sum_i w_i (1 - cos k.c_i) is the
    lattice Laplacian's symbol, k^2 at small k), every other mode
    rho0 kT N_a / cs2.  Ideal gas: cs2 in place of c_s^2(k)."""
    t = lattice_tables(p.lattice)
    kx, ky, kz = wavevectors(p)
    lam = np.zeros_like(kx)
    for i in range(t["q"]):
        cx, cy, cz = t["c"][i]
        lam += t["w"][i] * (1.0 - np.cos(kx * cx + ky * cy + kz * cz))
    lam *= 2.0 / CS2
    if p.force_model == 1:
        d = p.rho0 - p.rho_c
        psi2 = 2.0 * p.a + 12.0 * p.b * d * d
        cs2k = (1 - p.eta) * CS2 + p.rho0 * psi2 + p.kappa * p.rho0 * lam
    else:
        cs2k = np.full_like(kx, CS2)
    G = np.empty((t["q"],) + kx.shape)
    G[0] = p.rho0 * p.kT / cs2k
    for a in range(1, t["q"]):
        G[a] = p.rho0 * p.kT * t["N"][a] / CS2
    return G


def run(p, snapshots=400, interval=250, burn_in=20000, sim=None):
    """Burn in, then add the mode spectra of ``snapshots`` states taken every
    ``interval`` steps.  The steps between snapshots are replayed from one
    captured HIP graph.  Returns (spectrum sum as float64 numpy
    (q + npairs, nz, ny, nx), the Simulation)."""
    sim = sim or Simulation(p)
    stream = torch.cuda.Stream()
    spec = sim.spectrum_buffer()
    with torch.cuda.stream(stream):
        sim.graph_capture(interval, stats_stride=0, stream=stream)
        for _ in range(burn_in // interval):
            sim.graph_launch(stream)
        if burn_in % interval:
            sim.step(burn_in % interval, stream=stream)
        for _ in range(snapshots):
            sim.graph_launch(stream)
            sim.accumulate_spectrum(spec, stream=stream)
    stream.synchronize()
    return spec.cpu().numpy(), sim


def equilibration_ratio(spec_sum, nsnap, p):
    """<|m_a(k)|^2> / (V G_aa(k)) for the q modes, (q, nz, ny, nx); NaN at k = 0."""
    G = paper_variance(p)
    V = p.nx * p.ny * p.nz
    r = np.asarray(spec_sum[: G.shape[0]], dtype=np.float64) / (nsnap * V * G)
    r[:, 0, 0, 0] = np.nan
    return r


def momentum_split(spec_sum, p):
    """Spectra of the momentum component along k (longitudinal) and of one
    component across k (transverse, the mean of the d - 1 of them):
    (2, nz, ny, nx), NaN at k = 0."""
    q, d = p.q, p.d
    K = wavevectors(p)[:d]
    k2 = sum(k * k for k in K)
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = np.where(k2 > 0, 1.0 / k2, np.nan)
    pairs = [(0, 1)] if d == 2 else [(0, 1), (1, 2), (2, 0)]
    par = sum(K[a] * K[a] * spec_sum[1 + a] for a in range(d))
    for n, (al, be) in enumerate(pairs):
        par = par + 2.0 * K[al] * K[be] * spec_sum[q + n]
    par = par * inv
    total = sum(spec_sum[1 + a] for a in range(d))
    return np.stack([par, (total - par) / (d - 1)])


def shell_average(r, p, nbins=16):
    """Mean of r (nz, ny, nx) over the wavevectors of each |k| shell of width
    pi / nbins in (0, pi] (the paper's average over directions at each |k|).
    Returns (shell centres, means, counts)."""
    kx, ky, kz = wavevectors(p)
    km = np.sqrt(kx * kx + ky * ky + kz * kz)
    b = np.minimum((km / (np.pi / nbins)).astype(np.int64), nbins - 1)
    ok = (km > 0) & (km <= np.pi) & np.isfinite(r)
    counts = np.bincount(b[ok], minlength=nbins)
    sums = np.bincount(b[ok], weights=r[ok], minlength=nbins)
    with np.errstate(invalid="ignore", divide="ignore"):
        means = np.where(counts > 0, sums / np.maximum(counts, 1), np.nan)
    return (np.arange(nbins) + 0.5) * np.pi / nbins, means, counts
