"""The linearized modified-equilibrium (Swift) model on the HIP library.

Sec. IV.B, subsection on the modified-equilibrium model: the non-ideal fluid
enters through the equilibrium moments (eq. meq-yeo) and the noise is
k-dependent, so that the equal-time correlations are those of
eq. f-correl-yeo.  The step and its Fourier-filtered noise run in
``csrc/modeq.hip`` behind ``flb_modeq_*`` of include/flb.h; this module only
marshals arguments.
"""

import ctypes as C
from dataclasses import dataclass, replace

import torch

from ._lib import call, flb_modeq_params
from .sim import _ptr, _stream

CS2 = 1.0 / 3.0


@dataclass
class ModEqParams:
    nx: int = 128
    ny: int = 128
    precision: str = "fp32"
    rho0: float = 1.0
    kT: float = 0.0
    cs2_0: float = CS2          # c_s^2 at k = 0
    kappa: float = 0.0          # c_s^2(k) = cs2_0 + kappa rho0 Lambda(k)
    rate_bulk: float = 1.0
    rate_shear: float = 1.0
    rate_ghost: float = 1.0
    seed: int = 0

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def dtype(self):
        return torch.float32 if self.precision == "fp32" else torch.float64

    def to_c(self):
        p = flb_modeq_params()
        p.nx, p.ny = int(self.nx), int(self.ny)
        p.precision = 0 if self.precision == "fp32" else 1
        p.reserved = 0
        p.rho0, p.kT = float(self.rho0), float(self.kT)
        p.cs2_0, p.kappa = float(self.cs2_0), float(self.kappa)
        p.rate_bulk, p.rate_shear = float(self.rate_bulk), float(self.rate_shear)
        p.rate_ghost = float(self.rate_ghost)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        return p


def paper_params(nx=128, ny=128, seed=0, precision="fp32"):
    """The equilibration parameters of Sec. VI (rho0 1, kappa 0.08,
    c_s 0.265, kT 1e-7, tau 1) for this model: c_s^2(0) = 0.265^2."""
    return ModEqParams(nx=nx, ny=ny, precision=precision, rho0=1.0, kT=1e-7, cs2_0=0.265 ** 2,
                       kappa=0.08, rate_bulk=1.0, rate_shear=1.0, rate_ghost=1.0, seed=seed)


def work_bytes(p):
    b = C.c_size_t()
    call("flb_modeq_work_bytes", C.byref(p.to_c()), C.byref(b))
    return b.value


class ModEq:
    """Two population buffers (9, ny, nx) of the deviations from rest, and
    the noise work space, on the current device."""

    def __init__(self, p, f0=None, device="cuda", batch=16):
        """``batch``: steps whose noise ``step`` draws and filters together
        (the work buffer holds that many; results do not depend on it)."""
        self.p = p
        self.c = p.to_c()
        self.f = torch.zeros((9, p.ny, p.nx), dtype=p.dtype, device=device)
        if f0 is not None:
            self.f.copy_(torch.as_tensor(f0).reshape(9, p.ny, p.nx))
        self.tmp = torch.empty_like(self.f)
        self.nbytes = work_bytes(p) * max(1, int(batch))
        self.work = torch.empty(max(self.nbytes, 1), dtype=torch.uint8, device=device)
        self.n = 0

    def step(self, nsteps=1, stream=None):
        call("flb_modeq_run", C.byref(self.c), _ptr(self.f), _ptr(self.tmp), int(self.n),
             int(nsteps), _ptr(self.work), int(self.nbytes), _stream(stream))
        self.n += nsteps

    def step_into(self, fin, fout, n, stream=None):
        """One step with index n from fin to fout (distinct tensors)."""
        call("flb_modeq_step", C.byref(self.c), _ptr(fin), _ptr(fout), int(n), _ptr(self.work),
             int(self.nbytes), _stream(stream))

    def step_into_noalloc(self, fin, fout, n, stream=None):
        """The step of ``step_into`` with the library's fixed device work
        array (no work buffer; lattices of at most 699050 sites in FP32,
        349525 in FP64)."""
        call("flb_modeq_step_noalloc", C.byref(self.c), _ptr(fin), _ptr(fout), int(n),
             _stream(stream))

    def moments(self, out=None, stream=None):
        """Moment fields of the pulled populations: (9, ny, nx) float64."""
        if out is None:
            out = torch.empty((9, self.p.ny, self.p.nx), dtype=torch.float64, device=self.f.device)
        call("flb_modeq_moments", C.byref(self.c), _ptr(self.f), _ptr(out), _stream(stream))
        return out

    def noise(self, n, stream=None):
        """The filtered (e, eps) noise of step n: (2, ny, nx) in the state's
        precision."""
        out = torch.empty((2, self.p.ny, self.p.nx), dtype=self.p.dtype, device=self.f.device)
        call("flb_modeq_noise", C.byref(self.c), int(n), _ptr(out), _ptr(self.work),
             int(self.nbytes), _stream(stream))
        return out


def equal_time_variances(p):
    """G_aa(k) of eq. f-correl-yeo projected as in eq. g-correl, in closed
    form for the D2Q9 basis: (9, ny, nx) float64 numpy.  With c2 = c_s^2(k):
    rho kT / c2, rho kT (j_x, j_y), 4 rho kT / c2 (e), 4/3, 1/3 rho kT (p_xx,
    p_xy), 2 rho kT (q_x, q_y), 4 rho kT (9 c2 + 1) / c2 (eps)."""
    import numpy as np
    kx = 2 * np.pi * np.arange(p.nx) / p.nx
    ky = 2 * np.pi * np.arange(p.ny) / p.ny
    cx, cy = np.cos(kx)[None, :], np.cos(ky)[:, None]
    lap = (4.0 / 3.0) * (2.0 - cx - cy) + (2.0 / 3.0) * (1.0 - cx * cy)
    c2 = p.cs2_0 + p.kappa * p.rho0 * lap
    g = p.rho0 * p.kT
    one = np.ones_like(c2)
    return np.stack([g / c2, g * one, g * one, 4 * g / c2, 4 / 3 * g * one, g / 3 * one,
                     2 * g * one, 2 * g * one, 4 * g * (9 * c2 + 1) / c2])


def run_spectra(p, burn_in, snapshots, interval, stream=None):
    """From rest: burn_in steps, then ``snapshots`` snapshots ``interval``
    steps apart, each adding |m_a(k)|^2 of the pulled moments (the
    equilibration measure of Sec. VI) to a (9, ny, nx) FP64 sum: the moment
    fields (flb_modeq_moments) and their spectra (flb_field_spectrum).
    Returns (spectrum sum, the ModEq)."""
    from .sim import field_spectrum
    sim = ModEq(p)
    spec = torch.zeros((9, 1, p.ny, p.nx), dtype=torch.float64, device="cuda")
    m = torch.empty((9, 1, p.ny, p.nx), dtype=torch.float64, device="cuda")
    work = torch.empty(16 * spec.numel(), dtype=torch.uint8, device="cuda")
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        sim.step(burn_in, stream=s)
        for _ in range(snapshots):
            sim.step(interval, stream=s)
            sim.moments(out=m, stream=s)
            field_spectrum(m, spec, work=work, stream=s)
    s.synchronize()
    return spec.reshape(9, p.ny, p.nx), sim
