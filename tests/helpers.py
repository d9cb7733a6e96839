"""Shared helpers of the GPU parity tests: run the HIP library and the oracle
on the same seeded inputs and compare populations."""

import numpy as np
import torch

import flb_workloads as W

F32_TOL = 1e-5    # relative population error, FP32 shifted storage vs the FP64 oracle
F64_TOL = 1e-12   # relative population error, FP64 GPU step vs the FP64 oracle


def gpu_params(**kw):
    from paper_1012_3632_amd import Params
    return Params.from_dict(kw)


def oracle_params(**kw):
    from oracle import flb
    names = set(flb.Params.__dataclass_fields__)
    return flb.Params(**{k: v for k, v in kw.items() if k in names})


def rel_err(f_gpu, f_ref):
    f_gpu = np.asarray(f_gpu, dtype=np.float64)
    f_ref = np.asarray(f_ref, dtype=np.float64)
    return float(np.abs(f_gpu - f_ref).max() / np.abs(f_ref).max())


def run_pair(kw, nsteps, drho_amp=0.0, drho_seed=3, stats_stride=0, launch=None):
    """Run the GPU library and the oracle for nsteps from the same initial state.
    Returns (sim, f_gpu (unshifted, float64 numpy), f_ref, oracle stats)."""
    from oracle import flb
    from paper_1012_3632_amd import Simulation

    shape = (kw.get("nz", 1), kw["ny"], kw["nx"])
    drho = W.initial_drho(shape, drho_seed, drho_amp) if drho_amp else None
    sim = Simulation(gpu_params(**kw), drho_init=drho)
    if launch is not None:
        sim.set_launch(launch)
    sim.step(nsteps, stats_stride=stats_stride)
    torch.cuda.synchronize()
    f_gpu = sim.populations().numpy()
    po = oracle_params(**kw)
    S0 = flb.initial_state(po, drho)
    S, st = flb.run(S0, po, nsteps, stats_stride=stats_stride)
    return sim, f_gpu, S.numpy(), st


def tol(kw):
    return F64_TOL if kw.get("precision", "fp64") == "fp64" else F32_TOL
