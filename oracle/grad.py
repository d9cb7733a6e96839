"""Reference gradients of the FLB run (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The loss is a function of the density after the last step,
    rho_N(x) = sum_i S_{N,i}(x - c_i),
i.e. the density of the populations after the final streaming.  The gradient
is the plain derivative of ``oracle.flb.run`` w.r.t. the initial populations
S_0, the relaxation rates and kT at a fixed noise seed, obtained by reverse-mode
automatic differentiation of the FP64 forward (torch autograd; segments of
``checkpoint_every`` steps are recomputed to bound memory, which does not change
the arithmetic).  It is pinned in the tests by FP64 central differences of the
same forward.
"""

import torch
from torch.utils.checkpoint import checkpoint

from . import flb

F64 = torch.float64


def final_density(S0, p, nsteps, n0=0, checkpoint_every=20):
    lat = flb.lattice_of(p)

    def segment(S, k0, k1):
        for n in range(k0, k1):
            S = flb.step(S, n0 + n, p, lat)
        return S

    S = S0
    for k0 in range(0, nsteps, checkpoint_every):
        k1 = min(k0 + checkpoint_every, nsteps)
        if S.requires_grad:
            S = checkpoint(segment, S, k0, k1, use_reentrant=False)
        else:
            S = segment(S, k0, k1)
    return flb.density(flb.pull(S, lat))


def mse_loss(rho, rho_target):
    """L = mean over sites of (rho - rho_target)^2."""
    return ((rho - rho_target) ** 2).mean()


def loss_only(S0, p, nsteps, rho_target, n0=0):
    with torch.no_grad():
        return float(mse_loss(final_density(S0, p, nsteps, n0), rho_target))


def loss_and_grads(S0, p, nsteps, rho_target, n0=0, checkpoint_every=20):
    """Returns (L, dL/dS0, dict(rate_shear, rate_bulk, rate_ghost, kT))."""
    S0 = S0.detach().clone().requires_grad_(True)
    th = {k: torch.tensor(float(getattr(p, k)), dtype=F64, requires_grad=True)
          for k in ("rate_shear", "rate_bulk", "rate_ghost", "kT")}
    q = p.with_(**th)
    rho = final_density(S0, q, nsteps, n0, checkpoint_every)
    L = mse_loss(rho, torch.as_tensor(rho_target, dtype=F64))
    L.backward()
    return float(L.detach()), S0.grad.detach(), {k: float(v.grad) for k, v in th.items()}
