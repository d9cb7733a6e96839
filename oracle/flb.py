"""The fluctuating lattice Boltzmann step, FP64, written as the paper states it.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Everything works on whole fields held as float64 torch tensors on the CPU
(torch only so that ``oracle.grad`` can differentiate it); populations are
kept unshifted, shape (q, nz, ny, nx) with x fastest (site = x + nx*(y + ny*z)).

One time step with index n takes the post-collision state S_n to S_{n+1}
(Sec. V, eq. lbe-mom, with Delta t = 1):

1. pull-stream        f_i(x) = S_{n,i}(x - c_i), periodic  (left side of eq. lbe-mom)
2. non-ideal only     rho(x) = sum_i f_i(x); mu = psi'(rho) - kappa lap rho;
                      F = -rho grad mu + eta * cs2 * grad rho    (App. A eq. he-force)
3. moments            m_a = sum_i T_ai f_i                       (Sec. III eq. moments)
                      rho = m_0, rho u = j + F/2                 (Sec. V eq. lbe-moments)
4. equilibrium and forcing moments by projection:
                      m^eq_a = sum_i T_ai f^eq_i(rho, u)         (Sec. III eq. feq)
                      m^F_a  = sum_i T_ai Phi_i(u, F)            (eq. forcing-term, Guo reading)
5. update             m*_a = m_a - lam_a (m_a - m^eq_a) + (1 - lam_a/2) m^F_a + xi_a
                      with lam_a = 0 on conserved modes and
                      <xi_a xi_b> = rho kT N_a lam_a (2 - lam_a) / cs2 delta_ab
                      (Sec. V eq. noise-lbe, Delta V = 1, sign of the printed
                      "(1 + lam/2)" read as "(1 - lam/2)", consistent with eq.
                      lbe-mom and the variance it states)
6. back to populations S_{n+1,i}(x) = w_i sum_a T_ai m*_a / N_a  (Sec. III eq. moments-inv)

Readings where the paper is silent or garbled are listed in the docstrings of
the functions that take them.
"""

from dataclasses import dataclass, replace

import numpy as np
import torch

from . import lattice as _lattice
from . import philox

CS2 = _lattice.CS2
F64 = torch.float64


@dataclass
class Params:
    """Parameters of one FLB run (oracle copy; plain floats, or 0-d float64
    tensors for the ones ``oracle.grad`` differentiates)."""

    lattice: str = "D2Q9"
    nx: int = 32
    ny: int = 32
    nz: int = 1
    rho0: float = 1.0
    kT: object = 0.0
    rate_bulk: object = 1.0
    rate_shear: object = 1.0
    rate_ghost: object = 1.0
    force_model: int = 0      # 0 ideal gas, 1 Landau square-gradient force
    a: float = 0.0            # psi = a (rho - rho_c)^2 + b (rho - rho_c)^4
    b: float = 0.0
    rho_c: float = 1.0
    kappa: float = 0.0
    eta: int = 0              # 1 adds cs2 grad rho to the force (App. A eq. he-force)
    noise_rho_local: int = 1  # 1: noise variance uses the local rho(x); 0: rho0
    seed: int = 0
    replica: int = 0

    def with_(self, **kw):
        return replace(self, **kw)


def lattice_of(p):
    return _lattice.get(p.lattice)


# ---------------------------------------------------------------- helpers

def _shape(p):
    return (p.nz, p.ny, p.nx)


def _tab(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64), dtype=F64)


def _shift(phi, s):
    """roll so that result[x] = phi[x - s] for an integer 3-vector s."""
    return torch.roll(phi, shifts=(int(s[2]), int(s[1]), int(s[0])), dims=(-3, -2, -1))


def rates(lat, p):
    """lam_a^LB for every mode (Sec. V, lam^LB = 2 lam / (2 + lam) in (0, 2)):
    0 on the conserved density and momentum (Sec. III eq. relax-eigenv), and one
    rate per class for bulk, shear and ghost modes (the classes of App. B)."""
    out = []
    for k in lat.classes:
        if k in (_lattice.RHO, _lattice.MOM):
            out.append(torch.zeros((), dtype=F64))
        elif k == _lattice.BULK:
            out.append(torch.as_tensor(p.rate_bulk, dtype=F64))
        elif k == _lattice.SHEAR:
            out.append(torch.as_tensor(p.rate_shear, dtype=F64))
        else:
            out.append(torch.as_tensor(p.rate_ghost, dtype=F64))
    return torch.stack(out)


def moments(f, lat):
    """m_a = sum_i T_ai f_i (Sec. III eq. moments)."""
    return torch.tensordot(_tab(lat.T), f, dims=([1], [0]))


def populations(m, lat):
    """f_i = w_i sum_a T_ai m_a / N_a (Sec. III eq. moments-inv)."""
    return torch.tensordot(_tab(lat.Tinv), m, dims=([1], [0]))


def _dot_c(v, lat):
    """(c_i . v)(x) for every i: shape (q, ...); v has d components."""
    c = _tab(lat.c[:, : lat.d])
    return torch.tensordot(c, v, dims=([1], [0]))


def equilibrium(rho, u, lat):
    """f^eq_i = w_i rho (1 + u.c_i/cs2 + u_a u_b Q_iab / (2 cs2^2)),
    Q_iab = c_ia c_ib - cs2 delta_ab (Sec. III eq. feq)."""
    w = _tab(lat.w).view(-1, *([1] * rho.dim()))
    uc = _dot_c(u, lat)
    uu = (u * u).sum(0)
    return w * rho * (1 + uc / CS2 + (uc * uc - CS2 * uu) / (2 * CS2 * CS2))


def forcing(u, F, lat):
    """Phi_i = w_i (F.c_i / cs2 + (uF + Fu):Q_i / (2 cs2^2)).

    Reading: the printed prefactors of Sec. III eq. forcing-term (an extra rho
    and cs2 instead of cs2^2 in the second term) contradict the moments the
    paper itself states (Sec. IV eq. force-mom: momentum moment F; Sec. V
    eq. lbe-moments: rho u = sum f c + F/2 and the second moment uF + Fu).
    This is the form whose moments are {0, F, uF + Fu, 0 on ghosts}, with F a
    force density."""
    w = _tab(lat.w).view(-1, *([1] * (F.dim() - 1)))
    uc = _dot_c(u, lat)
    Fc = _dot_c(F, lat)
    uF = (u * F).sum(0)
    return w * (Fc / CS2 + (2 * uc * Fc - 2 * CS2 * uF) / (2 * CS2 * CS2))


def pull(S, lat):
    """f_i(x) = S_i(x - c_i) with periodic wrap (streaming of eq. lbe-mom)."""
    return torch.stack([_shift(S[i], lat.c[i]) for i in range(lat.q)])


def grad_h(phi, lat):
    """Isotropic central gradient (1/cs2) sum_i w_i c_i phi(x + c_i): shape (d, ...).

    Reading: the paper's own runs use the Lee-Fischer differences (Sec. VI);
    this build uses the lattice's isotropic stencil (9 or 19 points)."""
    acc = torch.zeros((lat.d,) + tuple(phi.shape), dtype=F64)
    for i in range(1, lat.q):
        ph = _shift(phi, -lat.c[i])  # phi(x + c_i)
        for al in range(lat.d):
            if lat.c[i, al] != 0:
                acc[al] = acc[al] + lat.w[i] * lat.c[i, al] * ph
    return acc / CS2


def lap_h(phi, lat):
    """Isotropic Laplacian (2/cs2) sum_i w_i (phi(x + c_i) - phi(x))."""
    acc = torch.zeros_like(phi)
    for i in range(1, lat.q):
        acc = acc + lat.w[i] * (_shift(phi, -lat.c[i]) - phi)
    return 2.0 * acc / CS2


def chemical_potential(rho, p, lat):
    """mu = psi'(rho) - kappa lap rho, psi = a (rho - rho_c)^2 + b (rho - rho_c)^4
    (square-gradient functional, App. A eq. freeE-funct; Landau double well of
    Sec. VI eq. f0-bulk written about rho_c)."""
    d = rho - p.rho_c
    return 2 * p.a * d + 4 * p.b * d ** 3 - p.kappa * lap_h(rho, lat)


def landau_force(rho, p, lat):
    """F = -rho grad mu + eta cs2 grad rho.

    App. A eq. he-force is F = kappa rho grad lap rho - grad(p0 - rho cs2)
    = -rho grad mu + cs2 grad rho; eta = 1 is that form, eta = 0 keeps the LB
    ideal pressure and uses F = -rho grad mu alone."""
    F = -rho * grad_h(chemical_potential(rho, p, lat), lat)
    if p.eta:
        F = F + p.eta * CS2 * grad_h(rho, lat)
    return F


def noise(n, p, lat):
    """Standard normals z_k for the non-conserved modes at step n: (K, nz, ny, nx).

    Reading (Sec. VI asks only for independent per-site Gaussians): Philox
    counter (site, n, block, replica), key from the seed; see ``oracle.philox``."""
    K = len(lat.noncons())
    V = p.nx * p.ny * p.nz
    z = philox.normals(V, n, K, p.seed, tag=0, replica=p.replica)
    return torch.as_tensor(z, dtype=F64).reshape(K, *_shape(p))


def collide(f, F, n, p, lat, z=None):
    """Moment-space relaxation + forcing + noise at every site (steps 3-6 above).

    ``f`` are the pulled populations, ``F`` the force density (d, ...) or None.
    Returns the post-collision populations."""
    m = moments(f, lat)
    rho = m[0]
    j = m[1 : 1 + lat.d]
    if F is None:
        F = torch.zeros_like(j)
    u = (j + 0.5 * F) / rho
    meq = moments(equilibrium(rho, u, lat), lat)
    mF = moments(forcing(u, F, lat), lat)
    lam = rates(lat, p).view(-1, *([1] * rho.dim()))
    ms = m - lam * (m - meq) + (1 - 0.5 * lam) * mF
    kT = p.kT
    if isinstance(kT, torch.Tensor) or kT != 0.0:
        if z is None:
            z = noise(n, p, lat)
        nc = lat.noncons()
        lam_nc = rates(lat, p)[nc].view(-1, *([1] * rho.dim()))
        Nn = _tab(lat.N[nc]).view(-1, *([1] * rho.dim()))
        rho_n = rho if p.noise_rho_local else torch.full_like(rho, p.rho0)
        # sqrt(kT) is factored out so that d/dkT stays finite for kT > 0
        sig = torch.sqrt(torch.as_tensor(kT, dtype=F64)) * torch.sqrt(
            rho_n * Nn * lam_nc * (2 - lam_nc) / CS2)
        xi = torch.zeros_like(ms)
        xi[nc] = sig * z
        ms = ms + xi
    return populations(ms, lat)


def density(f):
    return f.sum(0)


def step(S, n, p, lat=None):
    """One FLB time step with index n: S_n -> S_{n+1} (eq. lbe-mom)."""
    lat = lat or lattice_of(p)
    f = pull(S, lat)
    F = None
    if p.force_model == 1:
        F = landau_force(density(f), p, lat)
    return collide(f, F, n, p, lat)


def initial_state(p, drho=None):
    """S_0,i = w_i rho(x): the u = 0 equilibrium (Sec. III eq. feq) at
    rho = rho0 + drho (drho a float64 array of shape (nz, ny, nx) or None)."""
    lat = lattice_of(p)
    rho = torch.full(_shape(p), p.rho0, dtype=F64)
    if drho is not None:
        rho = rho + torch.as_tensor(np.asarray(drho, dtype=np.float64).reshape(_shape(p)))
    w = _tab(lat.w).view(-1, 1, 1, 1)
    return w * rho


def mode_sums(f, p, lat):
    """Per-mode site sums (sum m_a, sum m_a^2) of the pulled populations f,
    with m_0 taken relative to rho0 (delta rho), FP64: two arrays of length q.
    These are the moments whose variances the FDT fixes (Sec. IV eq. G-ideal)."""
    m = moments(f, lat).reshape(lat.q, -1)
    m = m.clone()
    m[0] = m[0] - p.rho0
    return m.sum(1).numpy(), (m * m).sum(1).numpy()


def run(S, p, nsteps, n0=0, stats_stride=0):
    """Advance ``nsteps`` steps starting at step index n0.

    If stats_stride > 0, the pre-collision moments of every step k (0-based
    within this call) with (k + 1) % stats_stride == 0 are accumulated.
    Returns (S, stats) with stats = dict(sum, sumsq, nsamples)."""
    lat = lattice_of(p)
    ssum = np.zeros(lat.q)
    ssq = np.zeros(lat.q)
    ns = 0
    for k in range(nsteps):
        if stats_stride > 0 and (k + 1) % stats_stride == 0:
            a, b = mode_sums(pull(S, lat), p, lat)
            ssum += a
            ssq += b
            ns += 1
        S = step(S, n0 + k, p, lat)
    return S, dict(sum=ssum, sumsq=ssq, nsamples=ns)


def fields(S, p, lat=None):
    """Hydrodynamic fields of state S: rho(x) and rho u(x) = sum_i c_i f_i + F/2
    of the pulled populations (Sec. V eq. lbe-moments)."""
    lat = lat or lattice_of(p)
    f = pull(S, lat)
    m = moments(f, lat)
    rho = m[0]
    j = m[1 : 1 + lat.d]
    if p.force_model == 1:
        j = j + 0.5 * landau_force(rho, p, lat)
    return rho, j
