"""The allocation-free modified-equilibrium step (flb_modeq_step_noalloc)
against flb_modeq_step with a caller work buffer: bit-identical states on two
calls in a row, the second on a smaller lattice (the fixed device work array
keeps the first call's contents), in FP32 and FP64, through the C ABI."""

import ctypes as C

import numpy as np
import pytest
import torch

import flb_workloads as W

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _one(lib_call, p, f0, n):
    from paper_1012_3632_amd.modeq import work_bytes
    c = p.to_c()
    fin = torch.as_tensor(f0).to("cuda", p.dtype).contiguous()
    ref = torch.empty_like(fin)
    got = torch.full_like(fin, float("nan"))
    work = torch.empty(work_bytes(p), dtype=torch.uint8, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib_call("flb_modeq_step", C.byref(c), _ptr(fin), _ptr(ref), int(n), _ptr(work),
             int(work.numel()), s)
    lib_call("flb_modeq_step_noalloc", C.byref(c), _ptr(fin), _ptr(got), int(n), s)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_step_equals_the_work_buffer_step(precision):
    from paper_1012_3632_amd._lib import call
    from paper_1012_3632_amd.modeq import ModEqParams
    base = W.modeq_params_of("d2q9_128_modeq", precision=precision)
    # the first call on the full workload (128 x 128), the second on a smaller,
    # ragged lattice: the fixed array still holds the first call's spectra
    for (nx, ny), n, seed in (((128, 128), 7, 1), ((48, 20), 3, 2)):
        p = ModEqParams(**dict(base, nx=nx, ny=ny, kT=1e-5))
        f0 = W.random_populations(9, (ny, nx), seed, 1e-3)
        print(f"noalloc {precision} {nx}x{ny} step {n}", flush=True)
        ref, got = _one(call, p, f0, n)
        assert np.isfinite(ref).all()
        np.testing.assert_array_equal(got, ref)


def test_noalloc_rejects_lattices_beyond_the_array():
    """The fixed array holds 16 MiB: 1024 x 512 in FP64 (48 V bytes) and
    1024 x 1024 in FP32 (24 V bytes) are rejected before anything is queued."""
    from paper_1012_3632_amd._lib import FLBError, call
    from paper_1012_3632_amd.modeq import ModEqParams
    nbytes = C.c_size_t()
    call("flb_modeq_static_work_bytes", C.byref(nbytes))
    for prec, ny, per in (("fp64", 512, 48), ("fp32", 1024, 24)):
        p = ModEqParams(**dict(W.modeq_params_of("d2q9_128_modeq", precision=prec), nx=1024,
                               ny=ny, kT=1e-5))
        assert per * 1024 * ny > nbytes.value
        a = torch.zeros((9, ny, 1024), dtype=p.dtype, device="cuda")
        b = torch.zeros_like(a)
        with pytest.raises(FLBError) as e:
            call("flb_modeq_step_noalloc", C.byref(p.to_c()), _ptr(a), _ptr(b), 0, None)
        assert e.value.status == -1
