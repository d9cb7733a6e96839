"""Modified-equilibrium (Swift) fluctuating LB, linearized about rest, D2Q9.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. IV.B, subsection "Modified-equilibrium model": the non-ideal fluid enters
through the equilibrium moments instead of a force.  Linearized about a fluid
at rest with density rho0, in the D2Q9 basis of App. B (mode order rho, j_x,
j_y, e, p_xx, p_xy, q_x, q_y, eps), the equilibrium moments are (eq. meq-yeo)

    delta m^eq(k) = {drho, dj_x, dj_y, d(k) drho, 0, 0, 0, 0, -d(k) drho},
    d(k) = 6 (c_s^2(k) - cs2),

with c_s(k) the generalized sound speed, S(k) = rho0 kT / c_s^2(k)
(eq. s-nonideal).  The equal-time correlations are (eq. f-correl-yeo)

    <df_i(k) df_j(-k)> = S(k) / rho0 fbar_i(k) delta_ij,

fbar(k) the populations whose moments are rho0 {1, 0, 0, d, 0, 0, 0, 0, -d};
projected on the basis as in eq. g-correl this is G(k) = (S / rho0) T
diag(fbar) T^T.

Readings (the paper gives the DBE, continuous in time):

* c_s^2(k) = cs2_0 + kappa rho0 Lambda(k), Lambda(k) = (2 / cs2) sum_i w_i
  (1 - cos k.c_i) the symbol of the isotropic 9-point Laplacian, i.e. the
  linearized square-gradient pressure on the lattice; then d(k) drho is the
  local stencil 6 (cs2_0 - cs2) drho - 6 kappa rho0 lap_h drho.
* The time step is the LB form of eq. FDBE-yeo: pull streaming, then
  m* = m - lam (m - m^eq) + xi with the lattice rates lam^LB of Sec. V.
* The noise covariance is fixed by the lattice FDT: G must be the stationary
  covariance of the step.  Streaming leaves G invariant (it is diagonal in
  the populations), so Xi = G - C G C^T with C = 1 - Lam (1 - E) the collision
  matrix.  Its small-rate limit is the DBE result Lam' G + G Lam'^T of
  eq. dbe-fdt.  That limit reproduces the diagonal of the printed eq. noise-yeo;
  its (e, eps) entry is 12 (c_s^2 - cs2)(lam_e + lam_eps) rho0 kT / cs2,
  half the printed value.  The printed value would make Xi indefinite for
  0.53 < c_s^2 <= 0.6, where G is still a covariance (fbar >= 0); the
  computed one is positive semidefinite exactly where fbar >= 0.
* Only the (e, eps) block of Xi depends on k; the other non-conserved modes
  get white noise.  The (e, eps) noise is drawn as white normals z_e, z_eps,
  filtered in Fourier space by the lower Cholesky factor L(k) of that block:
  xi_hat(k) = L(k) z_hat(k), xi = inverse DFT.  The normals are those of the
  force-based step (``oracle.philox.normals`` with 6 per site, z_k for mode
  3 + k).

Pins: ``tests/test_oracle_modeq.py``.
"""

from dataclasses import dataclass, replace

import numpy as np

from . import lattice as _lattice
from . import philox

CS2 = _lattice.CS2
LAT = _lattice.get("D2Q9")
Q = 9
E_MODE, EPS_MODE = 3, 8        # bulk e and ghost eps in the App. B order
NONCONS = [3, 4, 5, 6, 7, 8]   # z_k drives mode 3 + k


@dataclass
class ModEqParams:
    nx: int = 16
    ny: int = 16
    rho0: float = 1.0
    kT: float = 0.0
    cs2_0: float = CS2         # c_s^2 at k = 0
    kappa: float = 0.0         # c_s^2(k) = cs2_0 + kappa rho0 Lambda(k)
    rate_bulk: float = 1.0     # lam_e
    rate_shear: float = 1.0    # lam_s (p_xx, p_xy)
    rate_ghost: float = 1.0    # lam_q = lam_eps
    seed: int = 0

    def with_(self, **kw):
        return replace(self, **kw)


def rates(p, rate_eps=None):
    """lam_a for every mode (0 on rho, j); ``rate_eps`` overrides lam_eps."""
    g = p.rate_ghost
    return np.array([0, 0, 0, p.rate_bulk, p.rate_shear, p.rate_shear, g, g,
                     g if rate_eps is None else rate_eps], dtype=np.float64)


def wavevectors(p):
    """(kx, ky) on the DFT grid, each (ny, nx), folded to (-pi, pi]."""
    ks = []
    for n in (p.nx, p.ny):
        k = 2 * np.pi * np.arange(n) / n
        ks.append(np.where(k > np.pi, k - 2 * np.pi, k))
    KY, KX = np.meshgrid(ks[1], ks[0], indexing="ij")
    return KX, KY


def _kc(K):
    KX, KY = K
    return KX[..., None] * LAT.c[:, 0] + KY[..., None] * LAT.c[:, 1]   # (..., q)


def laplacian_symbol(K):
    """Lambda(k) = (2 / cs2) sum_i w_i (1 - cos k.c_i) = k^2 + O(k^4)."""
    return 2.0 / CS2 * (LAT.w * (1.0 - np.cos(_kc(K)))).sum(-1)


def sound_speed2(p, K):
    """c_s^2(k) = cs2_0 + kappa rho0 Lambda(k) (a reading, see module doc)."""
    return p.cs2_0 + p.kappa * p.rho0 * laplacian_symbol(K)


def structure_factor(p, K):
    """S(k) = rho0 kT / c_s^2(k) (eq. s-nonideal)."""
    return p.rho0 * p.kT / sound_speed2(p, K)


def d_of(c2):
    """d(k) = 6 (c_s^2(k) - cs2) (eq. meq-yeo)."""
    return 6.0 * (c2 - CS2)


def fbar(p, K):
    """Populations with moments rho0 {1, 0, 0, d, 0, 0, 0, 0, -d}: (..., q)."""
    d = d_of(sound_speed2(p, K))
    mb = np.zeros(np.shape(d) + (Q,))
    mb[..., 0] = p.rho0
    mb[..., E_MODE] = p.rho0 * d
    mb[..., EPS_MODE] = -p.rho0 * d
    return mb @ LAT.Tinv.T                      # f_i = sum_a (T^-1)_ia m_a


def correlation(p, K):
    """G(k) = (S(k) / rho0) T diag(fbar(k)) T^T (eqs. f-correl-yeo, g-correl):
    (..., q, q)."""
    fb = fbar(p, K)
    S = structure_factor(p, K)
    return (S / p.rho0)[..., None, None] * np.einsum("ai,...i,bi->...ab", LAT.T, fb, LAT.T)


def equilibrium_matrix(p, K):
    """E(k) with m^eq = E m: identity on rho, j; e = d rho, eps = -d rho."""
    d = d_of(sound_speed2(p, K))
    E = np.zeros(np.shape(d) + (Q, Q))
    for a in range(3):
        E[..., a, a] = 1.0
    E[..., E_MODE, 0] = d
    E[..., EPS_MODE, 0] = -d
    return E


def collision_matrix(p, K, rate_eps=None):
    """C(k) = 1 - Lam (1 - E(k)): m* = C m + xi."""
    E = equilibrium_matrix(p, K)
    lam = rates(p, rate_eps)
    return np.eye(Q) - lam[:, None] * (np.eye(Q) - E)


def advection_matrix(K):
    """The DBE's advection in mode space, A = T diag(i k.c_i) T^-1 (eq. FDBE-yeo)."""
    return np.einsum("ai,...i,ib->...ab", LAT.T, 1j * _kc(K), LAT.Tinv)


def streaming_matrix(K):
    """One LB streaming step in mode space: T diag(exp(-i k.c_i)) T^-1."""
    return np.einsum("ai,...i,ib->...ab", LAT.T, np.exp(-1j * _kc(K)), LAT.Tinv)


def noise_covariance_dbe(p, K, rate_eps=None):
    """Xi = L G + G L^dagger (eq. dbe-fdt) with the relaxation part of L,
    Lam (1 - E); the advective part A G + G A^dagger vanishes for this model."""
    G = correlation(p, K)
    E = equilibrium_matrix(p, K)
    lam = rates(p, rate_eps)
    Lr = lam[:, None] * (np.eye(Q) - E)
    return Lr @ G + G @ np.swapaxes(Lr, -1, -2)


def noise_covariance(p, K, rate_eps=None):
    """Xi = G - C G C^T: the per-site covariance that keeps G stationary
    under the LB step (a reading, see module doc)."""
    G = correlation(p, K)
    C = collision_matrix(p, K, rate_eps)
    return G - C @ G @ np.swapaxes(C, -1, -2)


def stationary_covariance(p, K):
    """Covariance of the pulled moments in the stationary state of the step,
    by a direct solve of P = A P A^H + S Xi S^H (A = S C, S streaming) in its
    Kronecker form; (n, q, q) for the n wavevectors of K (flattened)."""
    kx, ky = (np.ravel(K[0]), np.ravel(K[1]))
    Kf = (kx, ky)
    Sm = streaming_matrix(Kf)
    A = Sm @ collision_matrix(p, Kf)
    Xi = noise_covariance(p, Kf)
    Qm = Sm @ Xi @ np.conj(np.swapaxes(Sm, -1, -2))
    n = len(kx)
    out = np.full((n, Q, Q), np.nan, dtype=complex)
    # where two eigenvalues of A satisfy l_i conj(l_j) = 1 (k = 0: the
    # conserved modes) the solution depends on the initial state: NaN there
    ev = np.linalg.eigvals(A)
    gap = np.abs(1 - ev[:, :, None] * np.conj(ev[:, None, :])).min(axis=(1, 2))
    good = np.flatnonzero(gap > 1e-9)
    a = A[good]
    M = np.eye(Q * Q)[None] - np.einsum("nik,njl->nijkl", a, np.conj(a)).reshape(
        len(good), Q * Q, Q * Q)
    out[good] = np.linalg.solve(M, Qm[good].reshape(len(good), Q * Q, 1)).reshape(len(good), Q, Q)
    return out


def white_amplitudes(p):
    """sqrt(Xi_aa) of the k-independent modes p_xx, p_xy, q_x, q_y (index
    into NONCONS 1..4); from the k = 0 covariance."""
    Xi = noise_covariance(p, (np.zeros(1), np.zeros(1)))[0]
    return np.sqrt(np.maximum([Xi[a, a] for a in NONCONS[1:5]], 0.0))


def noise_filter(p, K):
    """Lower Cholesky factor of the (e, eps) block of Xi(k): (L11, L21, L22),
    each of the shape of K[0]."""
    Xi = noise_covariance(p, K)
    see, sep, spp = Xi[..., E_MODE, E_MODE], Xi[..., E_MODE, EPS_MODE], Xi[..., EPS_MODE, EPS_MODE]
    l11 = np.sqrt(np.maximum(see, 0.0))
    l21 = np.where(l11 > 0, sep / np.where(l11 > 0, l11, 1.0), 0.0)
    l22 = np.sqrt(np.maximum(spp - l21 * l21, 0.0))
    return l11, l21, l22


def noise(n, p, z=None):
    """xi_a(x) of step n for the 6 non-conserved modes: (6, ny, nx)."""
    V = p.nx * p.ny
    if z is None:
        z = philox.normals(V, n, 6, p.seed).reshape(6, p.ny, p.nx)
    K = wavevectors(p)
    xi = np.empty_like(z)
    amp = white_amplitudes(p)
    for k in range(1, 5):
        xi[k] = amp[k - 1] * z[k]
    l11, l21, l22 = noise_filter(p, K)
    ze, zp = np.fft.fft2(z[0]), np.fft.fft2(z[5])
    xi[0] = np.fft.ifft2(l11 * ze).real
    xi[5] = np.fft.ifft2(l21 * ze + l22 * zp).real
    return xi


def pull(S):
    """f_i(x) = S_i(x - c_i), periodic: S of shape (q, ny, nx)."""
    return np.stack([np.roll(S[i], (LAT.c[i, 1], LAT.c[i, 0]), axis=(0, 1)) for i in range(Q)])


def lap_h(phi):
    """(2 / cs2) sum_i w_i (phi(x + c_i) - phi(x))."""
    acc = np.zeros_like(phi)
    for i in range(1, Q):
        acc += LAT.w[i] * (np.roll(phi, (-LAT.c[i, 1], -LAT.c[i, 0]), axis=(0, 1)) - phi)
    return 2.0 / CS2 * acc


def step(S, n, p, z=None):
    """One step with index n of the linearized model: S_n -> S_{n+1}, S the
    deviations delta f_i (q, ny, nx) from the uniform rest state."""
    f = pull(S)
    m = np.tensordot(LAT.T, f, axes=([1], [0]))
    drho = m[0]
    D = 6.0 * (p.cs2_0 - CS2) * drho - 6.0 * p.kappa * p.rho0 * lap_h(drho)  # d(k) drho
    meq = np.zeros_like(m)
    meq[0:3] = m[0:3]
    meq[E_MODE] = D
    meq[EPS_MODE] = -D
    lam = rates(p)[:, None, None]
    ms = m - lam * (m - meq)
    if p.kT != 0.0:
        ms[NONCONS] += noise(n, p, z)
    return np.tensordot(LAT.Tinv, ms, axes=([1], [0]))


def initial_state(p, drho=None):
    """delta f_i = w_i drho (drho (ny, nx) or None for the rest state)."""
    d = np.zeros((p.ny, p.nx)) if drho is None else np.asarray(drho, np.float64).reshape(p.ny, p.nx)
    return LAT.w[:, None, None] * d[None]


def run(S, p, nsteps, n0=0):
    for k in range(nsteps):
        S = step(S, n0 + k, p)
    return S
