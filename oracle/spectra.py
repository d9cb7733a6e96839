"""Equal-time mode spectra and their theoretical values (Sec. VI, equilibration tests).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. VI checks a fluctuating non-ideal fluid by the equilibration ratio: the
equal-time correlation <|delta m_a(k)|^2> of every LB mode, averaged over
snapshots, divided by the variance the theory gives for it.  This module is
the plain version of that analysis:

* ``mode_fields``   the mode densities of a state after streaming
                    (Sec. III eq. moments), with the density taken relative to
                    rho0 and the momentum rows replaced by rho u = j + F/2
                    (Sec. V eq. lbe-moments), so that the conserved rows are the
                    hydrodynamic fields.
* ``mode_spectrum`` |m_a(k)|^2 of every mode and Re(j_a(k) conj j_b(k)) of every
                    momentum pair, with m(k) = sum_x m(x) exp(-i k.x) (numpy's
                    FFT as the library step).
* ``theory_variance`` G_aa(k) of the force-based model (Sec. IV eq.
                    g-mat-forcing): the structure factor S(k) = rho0 kT / c_s^2(k)
                    (eq. s-nonideal, OZ form of App. A) for the density and
                    rho0 kT N_a / cs2 for every other mode.
* ``stationary_spectrum`` the exact stationary spectra of the step linearized
                    about rest (``linear_step``: pull streaming, the moment
                    collision with the stencil force and Guo forcing, the noise
                    of Sec. V eq. noise-lbe), from the discrete Lyapunov equation
                    at every wavevector: what a run of this lattice scheme must
                    reproduce at small kT, at all k.
* ``double_well``   the Landau double well of Sec. VI eq. f0-bulk written as
                    psi = a (rho - rho_c)^2 + b (rho - rho_c)^4, with beta from
                    the speed of sound (the relation after eq. f0-bulk).

Pins: ``tests/test_oracle_spectra.py`` -- brute-force DFT, Parseval against
``flb.mode_sums``, closed forms of a streamed plane wave (with and without the
force), the linear force against ``flb.landau_force``, the ideal-gas
stationary spectra equal to G exactly (the FDT of the lattice noise), the
small-k Ornstein-Zernike limit, the paper's beta-c_s relation, and an oracle
run at the paper's equilibration parameters against ``stationary_spectrum``
in every |k| shell.  ``theory_variance`` at large k is the paper's G(k) with
the lattice Laplacian symbol in place of k^2 (a reading); this lattice scheme
does not reach it there for the density, which the runs resolve.
"""

import numpy as np

from . import flb
from . import lattice as _lattice

CS2 = _lattice.CS2


def momentum_pairs(d):
    """(alpha, beta) momentum component pairs of the cross spectra: (x, y) in
    2-D; (x, y), (y, z), (z, x) in 3-D."""
    return [(0, 1)] if d == 2 else [(0, 1), (1, 2), (2, 0)]


def mode_fields(S, p, lat=None):
    """All q mode densities of state S after streaming, float64 numpy
    (q, nz, ny, nx): m_0 - rho0, rho u_a = j_a + F_a / 2 for the momentum rows,
    m_a = sum_i T_ai f_i for the others (Sec. III eq. moments, Sec. V eq.
    lbe-moments)."""
    lat = lat or flb.lattice_of(p)
    f = flb.pull(S, lat)
    m = flb.moments(f, lat).clone()
    if p.force_model == 1:
        F = flb.landau_force(m[0], p, lat)
        m[1 : 1 + lat.d] = m[1 : 1 + lat.d] + 0.5 * F
    m[0] = m[0] - p.rho0
    return m.numpy()


def mode_spectrum(S, p, lat=None):
    """Equal-time spectra of state S: array (q + npairs, nz, ny, nx) holding
    |m_a(k)|^2 for a < q and Re(j_alpha(k) conj j_beta(k)) for the momentum
    pairs, k = 2 pi (kx / nx, ky / ny, kz / nz), DFT sign exp(-i k.x)."""
    lat = lat or flb.lattice_of(p)
    m = mode_fields(S, p, lat)
    mk = np.fft.fftn(m, axes=(1, 2, 3))
    out = [np.abs(mk[a]) ** 2 for a in range(lat.q)]
    for al, be in momentum_pairs(lat.d):
        out.append((mk[1 + al] * np.conj(mk[1 + be])).real)
    return np.stack(out)


def wavevectors(p):
    """k_x, k_y, k_z on the FFT grid, each (nz, ny, nx), folded to (-pi, pi]."""
    ks = []
    for n in (p.nx, p.ny, p.nz):
        k = 2 * np.pi * np.arange(n) / n
        ks.append(np.where(k > np.pi, k - 2 * np.pi, k))
    KZ, KY, KX = np.meshgrid(ks[2], ks[1], ks[0], indexing="ij")
    return KX, KY, KZ


def laplacian_symbol(p, lat=None, K=None):
    """-(symbol of flb.lap_h): (2 / cs2) sum_i w_i (1 - cos(k.c_i)), which is
    k^2 + O(k^4); on the grid (nz, ny, nx), or at the wavevectors K = (kx, ky,
    kz) (arrays of one shape)."""
    lat = lat or flb.lattice_of(p)
    KX, KY, KZ = wavevectors(p) if K is None else K
    acc = np.zeros_like(KX)
    for i in range(lat.q):
        kc = KX * lat.c[i, 0] + KY * lat.c[i, 1] + KZ * lat.c[i, 2]
        acc += lat.w[i] * (1 - np.cos(kc))
    return 2 / CS2 * acc


def psi2(p, rho):
    """psi''(rho) of psi = a (rho - rho_c)^2 + b (rho - rho_c)^4."""
    return 2 * p.a + 12 * p.b * (rho - p.rho_c) ** 2


def sound_speed2(p, lat=None, K=None):
    """c_s^2(k) of the linearized force (App. A eqs. he-force, he-cs2):
    rho0 psi''(rho0) + kappa rho0 Lambda(k), plus the LB ideal part cs2 when the
    force keeps it (eta = 0; eta = 1 cancels it).  Ideal gas: cs2."""
    lat = lat or flb.lattice_of(p)
    lap = laplacian_symbol(p, lat, K)
    if p.force_model != 1:
        return np.full(lap.shape, CS2)
    return ((1 - p.eta) * CS2 + p.rho0 * psi2(p, p.rho0) + p.kappa * p.rho0 * lap)


def theory_variance(p, lat=None, K=None):
    """G_aa(k) of Sec. IV eq. g-mat-forcing, array (q, nz, ny, nx) (or
    (q, *K[0].shape)): S(k) = rho0 kT / c_s^2(k) for the density (eq.
    s-nonideal) and rho0 kT N_a / cs2 for every other mode (mass parameter
    kT / cs2)."""
    lat = lat or flb.lattice_of(p)
    cs2k = sound_speed2(p, lat, K)
    G = np.empty((lat.q,) + cs2k.shape)
    G[0] = p.rho0 * p.kT / cs2k
    for a in range(1, lat.q):
        G[a] = p.rho0 * p.kT * lat.N[a] / CS2
    return G


def equilibration_ratio(spec_sum, nsnap, p, lat=None):
    """<|delta m_a(k)|^2> / (V G_aa(k)) for every mode, from spectra summed
    over nsnap snapshots; (q, nz, ny, nx), k = 0 set to NaN (the conserved
    totals do not fluctuate)."""
    lat = lat or flb.lattice_of(p)
    V = p.nx * p.ny * p.nz
    r = np.asarray(spec_sum[: lat.q], dtype=np.float64) / (nsnap * V * theory_variance(p, lat))
    r[:, 0, 0, 0] = np.nan
    return r


def momentum_split(spec_sum, p, lat=None):
    """Longitudinal and transverse momentum spectra (per transverse
    component), from the |j_a|^2 and cross spectra: (2, nz, ny, nx).
    |j_par|^2 = sum_ab khat_a khat_b Re(j_a conj j_b); the transverse total is
    sum_a |j_a|^2 - |j_par|^2, divided by d - 1."""
    lat = lat or flb.lattice_of(p)
    d = lat.d
    K = wavevectors(p)[:d]
    k2 = sum(k * k for k in K)
    k2 = np.where(k2 == 0, np.nan, k2)
    C = [[None] * d for _ in range(d)]
    for a in range(d):
        C[a][a] = spec_sum[1 + a]
    for n, (al, be) in enumerate(momentum_pairs(d)):
        C[al][be] = C[be][al] = spec_sum[lat.q + n]
    par = sum(K[a] * K[b] * C[a][b] for a in range(d) for b in range(d)) / k2
    tot = sum(C[a][a] for a in range(d))
    return np.stack([par, (tot - par) / (d - 1)])


def shell_average(r, p, nbins):
    """Average of r (nz, ny, nx) over wavevectors in |k| shells of width
    pi / nbins on (0, pi]; returns (k_centres, means, counts)."""
    KX, KY, KZ = wavevectors(p)
    km = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    edges = np.linspace(0, np.pi, nbins + 1)
    idx = np.digitize(km, edges[1:-1])
    ok = (km > 0) & (km <= np.pi) & np.isfinite(r)
    means = np.full(nbins, np.nan)
    counts = np.zeros(nbins, dtype=np.int64)
    for b in range(nbins):
        sel = ok & (idx == b)
        counts[b] = sel.sum()
        if counts[b]:
            means[b] = r[sel].mean()
    return 0.5 * (edges[1:] + edges[:-1]), means, counts


def force_symbol(p, lat=None, K=None):
    """Linear force per unit density fluctuation, F(k) = Fk(k) drho(k), of the
    stencil force of ``flb.landau_force`` about rest at rho0: (d, nz, ny, nx)
    complex.  With i g(k) the symbol of flb.grad_h, g_a = (1/cs2) sum_i w_i c_ia
    sin(k.c_i), and -Lambda(k) that of flb.lap_h:
    Fk = i g(k) (eta cs2 - rho0 (psi''(rho0) + kappa Lambda(k)))."""
    lat = lat or flb.lattice_of(p)
    KX, KY, KZ = wavevectors(p) if K is None else K
    if p.force_model != 1:
        return np.zeros((lat.d,) + KX.shape, dtype=complex)
    g = np.zeros((lat.d,) + KX.shape)
    for i in range(lat.q):
        sk = np.sin(KX * lat.c[i, 0] + KY * lat.c[i, 1] + KZ * lat.c[i, 2])
        for al in range(lat.d):
            g[al] += lat.w[i] * lat.c[i, al] * sk / CS2
    amp = p.eta * CS2 - p.rho0 * (psi2(p, p.rho0) + p.kappa * laplacian_symbol(p, lat, K))
    return 1j * g * amp


def linear_step(p, lat=None, K=None):
    """The step linearized about rest at rho0, per wavevector (flattened k):
    returns (A, B, O, Xi) with m(k) of the pulled populations advancing as
    m' = A m + B xi, the observed fields (momentum rows j + F/2) o = O m, and
    Xi the per-site noise covariance of xi (Sec. V eq. noise-lbe at rho0).

    Collision (steps 3-5 of ``oracle.flb``): m*_0 = m_0, m*_j = j + F, and for
    every other mode m*_a = (1 - lam_a) m_a + xi_a (the equilibrium and forcing
    moments of those modes are quadratic in u, F).  Streaming: f_i(x) moves to
    x + c_i, a phase exp(-i k.c_i) on population i, i.e. T diag(phase) T^-1 in
    mode space."""
    lat = lat or flb.lattice_of(p)
    q, d = lat.q, lat.d
    KX, KY, KZ = wavevectors(p) if K is None else K
    n = KX.size
    kc = (np.outer(KX.ravel(), lat.c[:, 0]) + np.outer(KY.ravel(), lat.c[:, 1])
          + np.outer(KZ.ravel(), lat.c[:, 2]))
    phase = np.exp(-1j * kc)                                    # (n, q)
    Sm = np.einsum("ai,ni,ib->nab", lat.T, phase, lat.Tinv)     # streaming in mode space
    lam = flb.rates(lat, p).numpy()
    Fk = force_symbol(p, lat, K).reshape(d, n)
    C = np.zeros((n, q, q), dtype=complex)
    C[:, np.arange(q), np.arange(q)] = 1 - lam
    O = np.zeros((n, q, q), dtype=complex)
    O[:, np.arange(q), np.arange(q)] = 1
    for al in range(d):
        C[:, 1 + al, 0] += Fk[al]
        O[:, 1 + al, 0] += 0.5 * Fk[al]
    A = Sm @ C
    Xi = np.diag(p.rho0 * p.kT * lat.N * lam * (2 - lam) / CS2)
    return A, Sm, O, Xi


def stationary_spectrum(p, lat=None, K=None, chunk=2048):
    """Expected mode_spectrum of one snapshot in the stationary state of the
    linearized step (``linear_step``): V (O P O^H) with P the per-site
    covariance solving P = A P A^H + B Xi B^H (a direct solve of the
    Kronecker form).  Same layout as ``mode_spectrum`` (or (q + npairs,
    *K[0].shape) at given wavevectors K).  Where A has two
    eigenvalues with lam_i conj(lam_j) = 1 (k = 0, and a few Nyquist
    wavevectors at which a conserved combination is not reached by the noise)
    the stationary variance depends on the initial state: those k are NaN."""
    lat = lat or flb.lattice_of(p)
    q, d = lat.q, lat.d
    A, B, O, Xi = linear_step(p, lat, K)
    n = A.shape[0]
    shape = (p.nz, p.ny, p.nx) if K is None else np.shape(K[0])
    V = p.nx * p.ny * p.nz
    pairs = momentum_pairs(d)
    out = np.full((q + len(pairs), n), np.nan)
    eye = np.eye(q * q)
    ev = np.linalg.eigvals(A)
    gap = np.abs(1 - ev[:, :, None] * np.conj(ev[:, None, :])).min(axis=(1, 2))
    good = np.flatnonzero(gap > 1e-9)
    for s in range(0, len(good), chunk):
        idx = good[s : s + chunk]
        a, b, o = A[idx], B[idx], O[idx]
        K = eye[None] - np.einsum("nik,njl->nijkl", a, np.conj(a)).reshape(len(idx), q * q, q * q)
        Qm = b @ Xi @ np.conj(np.transpose(b, (0, 2, 1)))
        P = np.linalg.solve(K, Qm.reshape(len(idx), q * q, 1)).reshape(len(idx), q, q)
        Oo = o @ P @ np.conj(np.transpose(o, (0, 2, 1)))
        out[:q, idx] = V * np.real(np.einsum("naa->na", Oo)).T
        for m, (al, be) in enumerate(pairs):
            out[q + m, idx] = V * np.real(Oo[:, 1 + al, 1 + be])
    return out.reshape((q + len(pairs),) + tuple(shape))


def double_well(rho_L, rho_V, cs, rho0):
    """(a, b, rho_c) of psi = a (rho - rho_c)^2 + b (rho - rho_c)^4 equal (up
    to a constant) to beta (rho - rho_V)^2 (rho - rho_L)^2 (Sec. VI eq.
    f0-bulk), with beta = c_s^2 / (2 rho0 (rho_L - rho_V)^2) (the relation
    after eq. f0-bulk)."""
    beta = cs * cs / (2 * rho0 * (rho_L - rho_V) ** 2)
    half = 0.5 * (rho_L - rho_V)
    return -2 * beta * half * half, beta, 0.5 * (rho_L + rho_V)


def run_snapshots(p, burn_in, nsnap, interval, S=None):
    """Advance the oracle burn_in steps from S (default: rest at rho0), then sum
    mode_spectrum over nsnap snapshots taken every ``interval`` steps.
    Returns (spec_sum, S, next step index)."""
    lat = flb.lattice_of(p)
    S = flb.initial_state(p) if S is None else S
    n = 0
    for _ in range(burn_in):
        S = flb.step(S, n, p, lat)
        n += 1
    acc = None
    for _ in range(nsnap):
        for _ in range(interval):
            S = flb.step(S, n, p, lat)
            n += 1
        sp = mode_spectrum(S, p, lat)
        acc = sp if acc is None else acc + sp
    return acc, S, n
