"""FP32 shifted storage against the FP64 GPU step over the full lengths of the
two 3-D workloads (the precision extension: the error against FP64 stated per
result).  The FP64 GPU step is the reference: it matches the FP64 oracle to
1e-12 in the parity tests, and the oracle cannot run these lengths.

* d3q19_128: 128^3 ideal gas, 2000 steps (FP32 in the launch shape the
  autotuner picks, as the benchmark times it).
* d3q19_256_landau: 256^3 square-gradient fluid, eta = 0, 5000 steps.

Error measures on the final states, unshifted populations f = delta f + w rho0:
max |f32 - f64| / max |f64| (the 1e-5 bar) and the RMS of the shifted
difference over the RMS of delta f64 (stricter, informational); the total
mass of both runs is compared as well."""

import numpy as np
import pytest
import torch

import flb_workloads as W
from helpers import gpu_params

pytestmark = pytest.mark.gpu


def _errors(s32, s64, w, rho0):
    d = s32.double() - s64
    f64max = (s64 + w * rho0).abs().max()
    return (float(d.abs().max() / f64max),
            float(torch.sqrt((d * d).mean()) / torch.sqrt((s64 * s64).mean())))


def run_fp32_fp64(name, nsteps, drho=None, fp64_launch=None):
    from paper_1012_3632_amd import Simulation, lattice_tables
    kw = W.params_of(name)
    out = {}
    for prec in ("fp64", "fp32"):
        sim = Simulation(gpu_params(**dict(kw, precision=prec)), drho_init=drho)
        if prec == "fp32":
            sim.autotune(repeats=2)
        elif fp64_launch is not None:
            sim.set_launch(fp64_launch)
        sim.step(nsteps)
        torch.cuda.synchronize()
        out[prec] = sim.state().clone()
        assert sim.step_index == nsteps
        sim.close()
        del sim
        torch.cuda.empty_cache()
    q = 19
    w = torch.as_tensor(lattice_tables("D3Q19")["w"], device="cuda").view(q, 1, 1, 1)
    e_max, e_rms = _errors(out["fp32"], out["fp64"], w, kw["rho0"])
    m32, m64 = float(out["fp32"].double().sum()), float(out["fp64"].sum())
    return e_max, e_rms, m32, m64


def test_d3q19_128_full_length_fp32_vs_fp64():
    e_max, e_rms, m32, m64 = run_fp32_fp64("d3q19_128", 2000)
    print(f"d3q19_128 2000 steps: max rel {e_max:.3e}, rms rel (shifted) {e_rms:.3e}", flush=True)
    assert e_max < 1e-5
    assert abs(m32 - m64) < 1e-6 * 128 ** 3


def test_d3q19_256_landau_full_length_fp32_vs_fp64():
    drho = W.initial_drho((256, 256, 256), 7, W.WORKLOADS["d3q19_256_landau"]["init_noise"])
    # the z-marching force step (128 x 2 columns, 16 planes) for the FP64 run
    e_max, e_rms, m32, m64 = run_fp32_fp64("d3q19_256_landau", 5000, drho, fp64_launch=7)
    print(f"d3q19_256_landau 5000 steps: max rel {e_max:.3e}, rms rel (shifted) {e_rms:.3e}",
          flush=True)
    assert e_max < 1e-5
    assert abs(m32 - m64) < 1e-6 * 256 ** 3
