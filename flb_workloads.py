"""Seeded synthetic workloads shared by the tests, the bench and the smoke run.

This module holds parameters and seeded random inputs only -- none of the
method's arithmetic.  Both the HIP library's callers and the oracle's callers
take their inputs from here; neither side imports the other.

Workloads (all periodic, rho0 = 1, fluid initially at rest, lattice units):

* ``d2q9_32_fp64``     D2Q9 ideal gas 32x32, FP64, all rates 1.0, kT 1e-4,
                        seed 1234, 1000 steps (FDT and conservation case).
* ``d3q19_128``         D3Q19 ideal gas 128^3, FP32 shifted storage (and the
                        FP64 step beside it), rates bulk/shear/ghost
                        1.2/1.6/1.0, kT 1e-5, seed 7, 2000 steps.
* ``d3q19_256_landau``  D3Q19 non-ideal 256^3, FP32, psi = a(r-rc)^2 + b(r-rc)^4
                        with a -0.01, b 0.1, rc 1, kappa 0.05, all rates 1.0,
                        rho = rc + 0.01 N(0,1), kT 1e-6, seed 7, 5000 steps.
* ``d3q19_batch64``     64 ideal-gas D3Q19 replicas of edge drawn uniformly
                        from {32, 48, 64, 80, 96}, seeds 0..63, rates as
                        d3q19_128, kT 1e-5, FP32, 1000 steps.
* ``d2q9_256_adjoint``  D2Q9 non-ideal 256x256 (Landau as above), FP32, all
                        rates 1.0 at the evaluation point, target density from
                        the same run at shear rate 1.5, kT 1e-6, seed 1234,
                        400 steps, checkpoint every 20.

* ``d2q9_128_equilibration``  the equilibration test of Sec. VI: D2Q9 128^2,
                        homogeneous fluid at rho0 = 1 with the paper's force
                        (eta = 1), Landau double well with rho_L 1, rho_V 0.5 and
                        beta set by c_s 0.265 (a, b, rho_c below are that well
                        written about rho_c: a = -beta (rho_L - rho_V)^2 / 2,
                        b = beta, rho_c = (rho_L + rho_V) / 2, beta = c_s^2 /
                        (2 rho0 (rho_L - rho_V)^2) = 0.14045), kappa 0.08,
                        kT 1e-7, all rates 1.0 (tau = 1), FP32, seed 2010;
                        400 snapshots every 250 steps after 20000 steps of
                        burn-in (the paper states neither of the last two).

* ``d2q9_capillary``   the capillary-fluctuation test of Sec. VI: D2Q9
                        1024 x 400, a liquid stripe (rho_L 1) between y = 100
                        and y = 300 in vapour (rho_V 0.5), the paper's force
                        (eta = 1) and double well with beta 0.1 (a, b, rho_c as
                        above: a = -beta (rho_L - rho_V)^2 / 2, b = beta,
                        rho_c = 0.75), kappa 0.08, kT 1e-7, all rates 1.0,
                        FP32 with rho0 0.75, seed 1995; started from the
                        mean-field profile of width sqrt(8 kappa / beta) /
                        (rho_L - rho_V) (``stripe_drho``); 10^6 steps, 2000
                        snapshots (every 474 steps after 52000; the paper gives
                        neither the burn-in nor the spacing).

The paper's own runs use no public dataset; its 2-D demonstrations (128^2
homogeneous fluid, 1024x400 liquid stripe) are parameter sets, not data.
"""

import numpy as np

LANDAU = dict(force_model=1, a=-0.01, b=0.1, rho_c=1.0, kappa=0.05, eta=0)

WORKLOADS = {
    "d2q9_32_fp64": dict(lattice="D2Q9", precision="fp64", nx=32, ny=32, nz=1, rho0=1.0,
                         kT=1e-4, rate_bulk=1.0, rate_shear=1.0, rate_ghost=1.0,
                         seed=1234, steps=1000),
    "d3q19_128": dict(lattice="D3Q19", precision="fp32", nx=128, ny=128, nz=128, rho0=1.0,
                      kT=1e-5, rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0,
                      seed=7, steps=2000),
    "d3q19_256_landau": dict(lattice="D3Q19", precision="fp32", nx=256, ny=256, nz=256,
                             rho0=1.0, kT=1e-6, rate_bulk=1.0, rate_shear=1.0,
                             rate_ghost=1.0, seed=7, steps=5000, init_noise=0.01, **LANDAU),
    "d3q19_batch64": dict(lattice="D3Q19", precision="fp32", replicas=64,
                          edges=(32, 48, 64, 80, 96), size_seed=2024, rho0=1.0, kT=1e-5,
                          rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0, steps=1000),
    "d2q9_256_adjoint": dict(lattice="D2Q9", precision="fp32", nx=256, ny=256, nz=1,
                             rho0=1.0, kT=1e-6, rate_bulk=1.0, rate_shear=1.0,
                             rate_ghost=1.0, target_rate_shear=1.5, seed=1234, steps=400,
                             checkpoint_every=20, init_noise=0.01, **LANDAU),
    "d2q9_128_equilibration": dict(lattice="D2Q9", precision="fp32", nx=128, ny=128, nz=1,
                                   rho0=1.0, kT=1e-7, rate_bulk=1.0, rate_shear=1.0,
                                   rate_ghost=1.0, seed=2010, force_model=1,
                                   a=-0.01755625, b=0.14045, rho_c=0.75, kappa=0.08, eta=1,
                                   rho_L=1.0, rho_V=0.5, cs=0.265, snapshots=400,
                                   interval=250, burn_in=20000),
    "d2q9_capillary": dict(lattice="D2Q9", precision="fp32", nx=1024, ny=400, nz=1,
                           rho0=0.75, kT=1e-7, rate_bulk=1.0, rate_shear=1.0, rate_ghost=1.0,
                           seed=1995, force_model=1, a=-0.0125, b=0.1, rho_c=0.75,
                           kappa=0.08, eta=1, rho_L=1.0, rho_V=0.5, beta=0.1,
                           stripe=(100.0, 300.0), steps=1000000, burn_in=52000,
                           snapshots=2000, interval=474),
}

PARAM_KEYS = ("lattice", "nx", "ny", "nz", "rho0", "kT", "rate_bulk", "rate_shear",
              "rate_ghost", "force_model", "a", "b", "rho_c", "kappa", "eta", "seed")


# The modified-equilibrium model (Sec. IV.B) at the equilibration parameters
# of Sec. VI: D2Q9 128^2, rho0 1, c_s(0) 0.265, kappa 0.08, kT 1e-7, all
# rates 1 (tau = 1), FP32 deviations from rest, seed 1012; the run starts
# at rest, and after a burn-in of 20000 steps takes 400 snapshots 250 steps apart.
MODEQ_WORKLOADS = {
    "d2q9_128_modeq": dict(nx=128, ny=128, precision="fp32", rho0=1.0, kT=1e-7,
                           cs2_0=0.265 ** 2, kappa=0.08, rate_bulk=1.0, rate_shear=1.0,
                           rate_ghost=1.0, seed=1012, burn_in=20000, snapshots=400,
                           interval=250),
}
MODEQ_PARAM_KEYS = ("nx", "ny", "precision", "rho0", "kT", "cs2_0", "kappa", "rate_bulk",
                    "rate_shear", "rate_ghost", "seed")


def modeq_params_of(name, **override):
    d = {k: v for k, v in MODEQ_WORKLOADS[name].items() if k in MODEQ_PARAM_KEYS}
    d.update(override)
    return d


def params_of(name, **override):
    """The FLB parameters of a workload as a plain dict (keys of PARAM_KEYS)."""
    w = dict(WORKLOADS[name])
    w.update(override)
    return {k: w[k] for k in PARAM_KEYS if k in w}


def initial_drho(shape, seed, amplitude=0.01, offset=0.0):
    """rho(x) - rho0 for an initial state: offset + amplitude * N(0,1) per site,
    float64 array of ``shape`` (nz, ny, nx), from numpy's PCG64 with ``seed``."""
    rng = np.random.default_rng(seed)
    return offset + amplitude * rng.standard_normal(shape)


def stripe_drho(shape, y1, y2, rho_L, rho_V, width, rho0):
    """rho(y) - rho0 of a liquid stripe between y1 and y2 (periodic in y, the
    profile axis, which is y in 2-D and z in 3-D): the mean-field tanh
    interfaces of width ``width``, float64 array of ``shape`` (nz, ny, nx)."""
    nz, ny, nx = shape
    n = ny if nz == 1 else nz
    y = np.arange(n, dtype=np.float64)
    half = 0.5 * (rho_L - rho_V)
    prof = rho_V + half * (np.tanh(2 * (y - y1) / width) - np.tanh(2 * (y - y2) / width)) - rho0
    if nz == 1:
        return np.broadcast_to(prof[None, :, None], shape).copy()
    return np.broadcast_to(prof[:, None, None], shape).copy()


def batch_edges(replicas=64, edges=(32, 48, 64, 80, 96), seed=2024):
    """Cubic edge length of every replica, drawn uniformly from ``edges``."""
    rng = np.random.default_rng(seed)
    return [int(edges[k]) for k in rng.integers(0, len(edges), size=replicas)]


def random_populations(q, shape, seed, amplitude):
    """A seeded non-equilibrium perturbation of the populations, shape (q, *shape)."""
    rng = np.random.default_rng(seed)
    return amplitude * rng.standard_normal((q,) + tuple(shape))


def unit_direction(shape, seed):
    """A seeded unit-norm direction (float64) for directional derivatives."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(shape)
    return v / np.linalg.norm(v)
