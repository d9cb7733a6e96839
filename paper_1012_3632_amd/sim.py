"""Python front end of the HIP library: torch provides device memory and the
stream, every step of the method runs in libflb.so.

    sim = Simulation(Params(lattice="D3Q19", precision="fp32", nx=128, ny=128, nz=128,
                            kT=1e-5, rate_bulk=1.2, rate_shear=1.6, seed=7))
    sim.step(1000, stats_stride=1)
    msum, msq, n = sim.moments()
"""

import ctypes as C
from dataclasses import asdict, dataclass, fields, replace

import numpy as np
import torch

from . import _lib
from ._lib import call, lib

LATTICES = {"D2Q9": (_lib.FLB_D2Q9, 9, 2), "D3Q19": (_lib.FLB_D3Q19, 19, 3)}
PRECISIONS = {"fp32": (_lib.FLB_FP32, torch.float32), "fp64": (_lib.FLB_FP64, torch.float64)}


@dataclass
class Params:
    """Run parameters (see include/flb.h, struct flb_params)."""

    lattice: str = "D2Q9"
    precision: str = "fp64"
    nx: int = 32
    ny: int = 32
    nz: int = 1
    rho0: float = 1.0
    kT: float = 0.0
    rate_bulk: float = 1.0
    rate_shear: float = 1.0
    rate_ghost: float = 1.0
    force_model: int = 0
    a: float = 0.0
    b: float = 0.0
    rho_c: float = 1.0
    kappa: float = 0.0
    eta: int = 0
    noise_rho_local: int = 1
    seed: int = 0
    step0: int = 0
    replica: int = 0

    @classmethod
    def from_dict(cls, d):
        names = {f.name for f in fields(cls)}
        return cls(**{k: v for k, v in d.items() if k in names})

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def q(self):
        return LATTICES[self.lattice][1]

    @property
    def d(self):
        return LATTICES[self.lattice][2]

    @property
    def dtype(self):
        return PRECISIONS[self.precision][1]

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def to_c(self):
        p = _lib.flb_params()
        p.lattice = LATTICES[self.lattice][0]
        p.precision = PRECISIONS[self.precision][0]
        p.nx, p.ny, p.nz = int(self.nx), int(self.ny), int(self.nz)
        p.force_model = int(self.force_model)
        p.eta = int(self.eta)
        p.noise_rho_local = int(self.noise_rho_local)
        p.rho0, p.kT = float(self.rho0), float(self.kT)
        p.rate_bulk, p.rate_shear, p.rate_ghost = (float(self.rate_bulk), float(self.rate_shear),
                                                    float(self.rate_ghost))
        p.a, p.b, p.rho_c, p.kappa = float(self.a), float(self.b), float(self.rho_c), float(self.kappa)
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        p.step0 = int(self.step0)
        p.replica = int(self.replica)
        return p


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def query_sizes(params):
    pop, scr, sta = C.c_size_t(), C.c_size_t(), C.c_size_t()
    call("flb_query_sizes", C.byref(params.to_c()), C.byref(pop), C.byref(scr), C.byref(sta))
    return pop.value, scr.value, sta.value


def lattice_tables(lattice):
    """The library's constant tables (host call, no GPU needed)."""
    code, q, d = LATTICES[lattice]
    qq = C.c_int32()
    c = (C.c_int32 * (3 * q))()
    w = (C.c_double * q)()
    T = (C.c_double * (q * q))()
    N = (C.c_double * q)()
    cls = (C.c_int32 * q)()
    call("flb_lattice_tables", code, C.byref(qq), c, w, T, N, cls)
    return dict(q=qq.value, c=np.array(c[:]).reshape(q, 3), w=np.array(w[:]),
                T=np.array(T[:]).reshape(q, q), N=np.array(N[:]), cls=np.array(cls[:]))


def field_spectrum(fields, spec=None, work=None, stream=None):
    """Add |DFT|^2 of each real field to spec: fields float64 CUDA (nf, nz, ny, nx)
    (or (nf, ny, nx), (nf, nx)); spec of the same shape, zero-filled if None.
    Returns spec."""
    f = fields.contiguous()
    assert f.dtype == torch.float64 and f.is_cuda and f.dim() >= 2
    dims = list(f.shape[1:])
    while len(dims) < 3:
        dims.insert(0, 1)
    nz, ny, nx = dims
    if spec is None:
        spec = torch.zeros_like(f)
    assert spec.shape == f.shape and spec.dtype == torch.float64 and spec.is_contiguous()
    need = 16 * f.numel()
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 256), dtype=torch.uint8, device=f.device)
    call("flb_field_spectrum", _ptr(f), int(f.shape[0]), int(nx), int(ny), int(nz), _ptr(work),
         _ptr(spec), _stream(stream))
    return spec


def noise_words(params, step, block, site0, nsites, tag=0, device="cuda", stream=None):
    """Raw Philox words of noise block ``block`` at ``step`` for a range of sites:
    uint32 values as an int64 CPU tensor of shape (nsites, 4)."""
    out = torch.empty((nsites, 4), dtype=torch.int32, device=device)
    call("flb_noise_words", C.byref(params.to_c()), int(step), int(block), int(tag), int(site0),
         int(nsites), _ptr(out), _stream(stream))
    return out.cpu().to(torch.int64) & 0xFFFFFFFF


def noise_normals(params, step, site0, nsites, device="cuda", stream=None):
    """The Box-Muller normals the collision of ``step`` draws at a range of
    sites: CPU tensor of shape (nsites, 2P) in the parameters' precision,
    P = 8 pairs (D3Q19) or 3 (D2Q9)."""
    npair = 8 if params.q == 19 else 3
    out = torch.empty((nsites, 2 * npair), dtype=params.dtype, device=device)
    call("flb_noise_normals", C.byref(params.to_c()), int(step), int(site0), int(nsites),
         _ptr(out), _stream(stream))
    return out.cpu()


class Simulation:
    """One lattice advanced by the HIP library; buffers are torch tensors."""

    def __init__(self, params, drho_init=None, device="cuda", stream=None):
        self.params = params
        self.device = torch.device(device)
        pop, scr, sta = query_sizes(params)
        self._pop_bytes = pop
        mk = lambda n: torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
        self.fa, self.fb = mk(pop), mk(pop)
        self.scratch, self.stats = mk(scr), mk(sta)
        drho = None
        if drho_init is not None:
            drho = torch.as_tensor(np.asarray(drho_init, dtype=np.float64).reshape(-1),
                                   device=self.device).contiguous()
            assert drho.numel() == params.nx * params.ny * params.nz
        h = C.c_void_p()
        call("flb_init", C.byref(params.to_c()), _ptr(self.fa), _ptr(self.fb), _ptr(self.scratch),
             _ptr(self.stats), _ptr(drho), _stream(stream), C.byref(h))
        self._h = h
        self._bufs = {self.fa.data_ptr(): self.fa, self.fb.data_ptr(): self.fb}

    # -- helpers
    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("simulation is closed")
        return self._h

    def _view(self, buf):
        p = self.params
        n = p.q * p.nx * p.ny * p.nz
        return buf.view(p.dtype)[:n].view(p.q, *p.shape)

    # -- API
    def step(self, nsteps, stats_stride=0, stream=None):
        call("flb_step", self.handle, int(nsteps), int(stats_stride), _stream(stream))

    def set_check(self, every, stream=None):
        """every > 0: step() reads the library's non-finite flag every
        ``every`` steps and raises FLBError (FLB_ERR_NONFINITE) once a NaN or
        Inf population has been pulled; 0 turns the reads off.  Clears the flag."""
        call("flb_set_check", self.handle, int(every), _stream(stream))

    def seek(self, step, stream=None):
        """Set the index of the next step (noise counter) without touching the state."""
        call("flb_seek", self.handle, int(step), _stream(stream))

    @property
    def step_index(self):
        s = C.c_uint64()
        call("flb_state", self.handle, None, None, C.byref(s))
        return s.value

    def state(self):
        """View of the current shifted populations delta f, shape (q, nz, ny, nx)."""
        cur = C.c_void_p()
        call("flb_state", self.handle, C.byref(cur), None, None)
        return self._view(self._bufs[cur.value])

    def other(self):
        oth = C.c_void_p()
        call("flb_state", self.handle, None, C.byref(oth), None)
        return self._view(self._bufs[oth.value])

    def populations(self):
        """Unshifted populations f = delta f + w rho0 as float64 on the CPU."""
        w = torch.as_tensor(lattice_tables(self.params.lattice)["w"])
        f = self.state().detach().to("cpu", torch.float64)
        return f + w.view(-1, 1, 1, 1) * self.params.rho0

    def load_state(self, delta_f):
        """Overwrite the current state with shifted populations (q, nz, ny, nx)."""
        self.state().copy_(torch.as_tensor(delta_f).to(self.device, self.params.dtype))

    def moments(self, stream=None):
        q = self.params.q
        s = (C.c_double * q)()
        s2 = (C.c_double * q)()
        n = C.c_int64()
        call("flb_moments", self.handle, s, s2, C.byref(n), _stream(stream))
        return np.array(s[:]), np.array(s2[:]), n.value

    def reset_stats(self, stream=None):
        call("flb_reset_stats", self.handle, _stream(stream))

    def fields(self, stream=None):
        """rho and rho u after streaming (rho u = sum c f + F/2): (1 + d, nz, ny, nx)."""
        p = self.params
        out = torch.empty((1 + p.d,) + p.shape, dtype=p.dtype, device=self.device)
        call("flb_fields", self.handle, _ptr(out), _stream(stream))
        return out

    def mode_fields(self, stream=None):
        """All q mode densities after streaming, float64 (q, nz, ny, nx): row 0
        is rho - rho0, the momentum rows are rho u = j + F/2."""
        p = self.params
        out = torch.empty((p.q,) + p.shape, dtype=torch.float64, device=self.device)
        call("flb_mode_fields", self.handle, _ptr(out), _stream(stream))
        return out

    def spectrum_buffer(self):
        """A zeroed float64 buffer (q + npairs, nz, ny, nx) for accumulate_spectrum:
        |m_a(k)|^2 for the q modes, then Re(j_al conj j_be) for the momentum
        pairs (x, y) [2-D] or (x, y), (y, z), (z, x) [3-D]."""
        p = self.params
        npairs = 1 if p.d == 2 else 3
        return torch.zeros((p.q + npairs,) + p.shape, dtype=torch.float64, device=self.device)

    def accumulate_spectrum(self, spec, stream=None):
        """Add the equal-time mode spectra of the current state to spec (see
        spectrum_buffer); k = (kx, ky, kz) is at spec[:, kz, ky, kx]."""
        if getattr(self, "_spec_work", None) is None:
            n = C.c_size_t()
            call("flb_spectrum_work_bytes", self.handle, C.byref(n))
            self._spec_work = torch.empty(max(n.value, 256), dtype=torch.uint8,
                                          device=self.device)
        assert spec.dtype == torch.float64 and spec.is_contiguous()
        p = self.params
        assert spec.numel() == (p.q + (1 if p.d == 2 else 3)) * p.nx * p.ny * p.nz
        call("flb_mode_spectrum", self.handle, _ptr(self._spec_work), _ptr(spec),
             _stream(stream))
        return spec

    def interface_heights(self, interfaces, rho_L, rho_V, width, stream=None):
        """Heights of planar interfaces across the profile axis (y in 2-D, z in
        3-D) by fitting the mean-field profile to every column: interfaces is a
        list of (y_ref, sign, half_window); returns float64 (n_if, nx) in 2-D,
        (n_if, ny, nx) in 3-D."""
        p = self.params
        arr = (_lib.flb_interface * len(interfaces))()
        for j, (y, sg, w) in enumerate(interfaces):
            arr[j].y_ref, arr[j].sign, arr[j].half_window = float(y), int(sg), int(w)
        plane = (p.nx,) if p.d == 2 else (p.ny, p.nx)
        out = torch.empty((len(interfaces),) + plane, dtype=torch.float64, device=self.device)
        call("flb_interface_heights", self.handle, arr, len(interfaces), float(rho_L),
             float(rho_V), float(width), _ptr(out), _stream(stream))
        return out

    def density(self, s, stream=None):
        """rho - rho0 after streaming of state s (q, nz, ny, nx)."""
        p = self.params
        out = torch.empty(p.shape, dtype=p.dtype, device=self.device)
        call("flb_density", self.handle, _ptr(s.contiguous()), _ptr(out), _stream(stream))
        return out

    def graph_capture(self, nsteps, stats_stride=0, stream=None):
        call("flb_graph_capture", self.handle, int(nsteps), int(stats_stride), _stream(stream))

    def graph_launch(self, stream=None):
        call("flb_graph_launch", self.handle, _stream(stream))

    def autotune(self, repeats=5, stream=None):
        """Time every launch shape; returns
        ((shape_plain, shape_stats, best_in_place or -1, in_place_in_use or -1),
         (ms_plain, ms_stats, ms_in_place))."""
        best, ms = (C.c_int32 * 4)(), (C.c_double * 3)()
        call("flb_autotune", self.handle, int(repeats), best, ms, _stream(stream))
        return tuple(best[:]), tuple(ms[:])

    def set_launch(self, config):
        call("flb_set_launch", self.handle, int(config))

    def launch_configs(self):
        """(number of launch shapes, (shape of plain steps, shape of steps with
        statistics, in-place shape or -1))."""
        n, cur = C.c_int32(), (C.c_int32 * 3)()
        call("flb_launch_configs", self.handle, C.byref(n), cur)
        return n.value, tuple(cur[:])

    def launch_shape(self, config):
        """(tx, ty, tz, sites_per_thread, nontemporal, z_planes_per_block,
        in_place, fused_density) of a launch configuration."""
        sh = (C.c_int32 * 8)()
        call("flb_launch_shape", self.handle, int(config), sh)
        return tuple(sh[:])

    def adjoint_seed(self, rhobar, stream=None):
        p = self.params
        out = torch.empty((p.q,) + p.shape, dtype=p.dtype, device=self.device)
        call("flb_adjoint_density_seed", self.handle, _ptr(rhobar.contiguous()), _ptr(out),
             _stream(stream))
        return out

    def adjoint_step(self, s_n, abar_np1, n, out=None, grad=None, stream=None):
        """abar_n = dL/dS_n from abar_{n+1}; if ``grad`` (a length-4 float64
        numpy array) is given, this step's parameter derivatives are added to it
        (order: rate_shear, kT, rate_bulk, rate_ghost)."""
        p = self.params
        if out is None:
            out = torch.empty((p.q,) + p.shape, dtype=p.dtype, device=self.device)
        g = (C.c_double * 4)(*(grad if grad is not None else [0.0] * 4)) if grad is not None else None
        call("flb_adjoint_step", self.handle, _ptr(s_n.contiguous()), _ptr(abar_np1.contiguous()),
             _ptr(out), g, int(n), _stream(stream))
        if grad is not None:
            grad[:] = np.array(g[:])
        return out

    def adjoint_segment(self, s_k0, abar, k0, k1, work=None, grad=None, stream=None):
        """In place: abar = dL/dS_{k1} -> dL/dS_{k0}, recomputing the segment's
        states from s_k0 on the GPU.  ``work`` may be a preallocated uint8
        device tensor of at least adjoint_segment_bytes(k1 - k0) bytes."""
        need = self.adjoint_segment_bytes(k1 - k0)
        if work is None or work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=self.device)
        g = (C.c_double * 4)(*grad) if grad is not None else None
        call("flb_adjoint_segment", self.handle, _ptr(s_k0.contiguous()), _ptr(abar), _ptr(work),
             int(k0), int(k1), g, _stream(stream))
        if grad is not None:
            grad[:] = np.array(g[:])
        return work

    def adjoint_segment_bytes(self, nsteps):
        n = C.c_size_t()
        call("flb_adjoint_segment_bytes", self.handle, int(nsteps), C.byref(n))
        return n.value

    def adjoint_run(self, ckpts, abar, seg_len, nsteps, work=None, grad=None, stream=None):
        """In place: abar = dL/dS_N -> dL/dS_0 over a run checkpointed every
        ``seg_len`` steps (``ckpts[s]`` = state at step s * seg_len); the
        recompute of each earlier segment overlaps the reverse sweep of the
        later one on a second stream.  Returns the work tensor for reuse."""
        n = C.c_size_t()
        call("flb_adjoint_run_bytes", self.handle, int(seg_len), C.byref(n))
        if work is None or work.numel() < n.value:
            work = torch.empty(n.value, dtype=torch.uint8, device=self.device)
        cks = [c.contiguous() for c in ckpts]
        arr = (C.c_void_p * len(cks))(*[c.data_ptr() for c in cks])
        g = (C.c_double * 4)(*grad) if grad is not None else None
        call("flb_adjoint_run", self.handle, arr, len(cks), int(seg_len), int(nsteps), _ptr(abar),
             _ptr(work), g, _stream(stream))
        if grad is not None:
            grad[:] = np.array(g[:])
        return work

    def close(self):
        if self._h is not None:
            lib.flb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent ideal-gas replicas of uneven size advanced together
    (one persistent launch per step over a flat tile table)."""

    def __init__(self, params, dims, seeds=None, device="cuda", stream=None):
        self.params = params
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.nrep = len(self.dims)
        self.device = torch.device(device)
        d = (C.c_int32 * (3 * self.nrep))(*[v for dd in self.dims for v in dd])
        self._dims_c = d
        pop, scr, sta = C.c_size_t(), C.c_size_t(), C.c_size_t()
        call("flb_batch_query_sizes", C.byref(params.to_c()), self.nrep, d, C.byref(pop),
             C.byref(scr), C.byref(sta))
        mk = lambda n: torch.empty(max(n, 256), dtype=torch.uint8, device=self.device)
        self.fa, self.fb = mk(pop.value), mk(pop.value)
        self.scratch, self.stats = mk(scr.value), mk(sta.value)
        seeds = list(range(self.nrep)) if seeds is None else [int(s) for s in seeds]
        sd = (C.c_uint64 * self.nrep)(*seeds)
        h = C.c_void_p()
        call("flb_batch_init", C.byref(params.to_c()), self.nrep, d, sd, _ptr(self.fa),
             _ptr(self.fb), _ptr(self.scratch), _ptr(self.stats), _stream(stream), C.byref(h))
        self._h = h
        self._bufs = {self.fa.data_ptr(): self.fa, self.fb.data_ptr(): self.fb}
        self.sites = [a * b * c for (a, b, c) in self.dims]

    def step(self, nsteps, stats_stride=0, stream=None):
        call("flb_batch_step", self._h, int(nsteps), int(stats_stride), _stream(stream))

    def graph_capture(self, nsteps, stats_stride=0, stream=None):
        call("flb_batch_graph_capture", self._h, int(nsteps), int(stats_stride), _stream(stream))

    def graph_launch(self, stream=None):
        call("flb_batch_graph_launch", self._h, _stream(stream))

    def autotune(self, repeats=3, stream=None):
        """((grid plain, grid with statistics), (ms plain, ms with statistics))."""
        best, ms = (C.c_int32 * 2)(), (C.c_double * 2)()
        call("flb_batch_autotune", self._h, int(repeats), best, ms, _stream(stream))
        return tuple(best[:]), tuple(ms[:])

    def set_pairs(self, pair_bytes):
        """0: all replicas every step (alternating buffers); > 0: groups of
        replicas up to pair_bytes, each taken through all steps of a call in
        place, pairs of steps in one buffer (the same bits either way)."""
        call("flb_batch_set_pairs", self._h, int(pair_bytes))

    def pairs(self):
        """(pair_bytes, number of groups) of the current schedule."""
        nb, ng = C.c_uint64(), C.c_int32()
        call("flb_batch_pairs", self._h, C.byref(nb), C.byref(ng))
        return nb.value, ng.value

    def moments(self, stream=None):
        q = self.params.q
        s = (C.c_double * (q * self.nrep))()
        s2 = (C.c_double * (q * self.nrep))()
        n = C.c_int64()
        call("flb_batch_moments", self._h, s, s2, C.byref(n), _stream(stream))
        return (np.array(s[:]).reshape(self.nrep, q), np.array(s2[:]).reshape(self.nrep, q), n.value)

    def reset_stats(self, stream=None):
        call("flb_batch_reset_stats", self._h, _stream(stream))

    def replica_state(self, r):
        """View of replica r's shifted populations, shape (q, nz, ny, nx)."""
        cur = C.c_void_p()
        call("flb_batch_state", self._h, C.byref(cur), None, None)
        buf = self._bufs[cur.value].view(self.params.dtype)
        q = self.params.q
        off = q * sum(self.sites[:r])
        nx, ny, nz = self.dims[r]
        return buf[off: off + q * self.sites[r]].view(q, nz, ny, nx)

    def close(self):
        if self._h is not None:
            lib.flb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
