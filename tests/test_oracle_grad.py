"""Pin of the oracle's reference gradient: FP64 central differences.

The loss is mean((rho_N - rho_target)^2) of the density after N steps at a
fixed noise seed; the target is the final density of the same run at another
shear rate.  Scalars use a relative step theta(1 +- 1e-6); the initial
populations are probed along seeded unit directions with an absolute step.
"""

import numpy as np
import pytest
import torch

import flb_workloads as W
from oracle import flb, grad


def _setup(lattice_name, force):
    if lattice_name == "D2Q9":
        kw = W.params_of("d2q9_256_adjoint", nx=12, ny=10) if force else \
            W.params_of("d2q9_32_fp64", nx=12, ny=10, kT=1e-5)
        shape = (1, 10, 12)
    else:
        kw = W.params_of("d3q19_128", nx=6, ny=5, nz=4)
        shape = (4, 5, 6)
    p = flb.Params(**kw)
    S0 = flb.initial_state(p, W.initial_drho(shape, 5, 0.01))
    target = grad.final_density(S0, p.with_(rate_shear=1.5), 8)
    return p, S0, target


@pytest.mark.parametrize("lattice_name,force", [("D2Q9", True), ("D2Q9", False), ("D3Q19", False)])
def test_reference_gradient_matches_central_differences(lattice_name, force):
    p, S0, target = _setup(lattice_name, force)
    nsteps = 8
    L, gS, gth = grad.loss_and_grads(S0, p, nsteps, target, checkpoint_every=3)
    assert L > 0
    for name in ("rate_shear", "rate_bulk", "rate_ghost", "kT"):
        th = float(getattr(p, name))
        h = 1e-6 * abs(th)
        lp = grad.loss_only(S0, p.with_(**{name: th + h}), nsteps, target)
        lm = grad.loss_only(S0, p.with_(**{name: th - h}), nsteps, target)
        fd = (lp - lm) / (2 * h)
        np.testing.assert_allclose(gth[name], fd, rtol=1e-5, atol=1e-9 * abs(L) / abs(th))
    for seed in (1, 2, 3):
        v = torch.as_tensor(W.unit_direction(S0.shape, seed))
        h = 1e-6
        lp = grad.loss_only(S0 + h * v, p, nsteps, target)
        lm = grad.loss_only(S0 - h * v, p, nsteps, target)
        fd = (lp - lm) / (2 * h)
        np.testing.assert_allclose(float((gS * v).sum()), fd, rtol=1e-5)
