"""GPU adjoint against the oracle: one-step vector-Jacobian products against
reverse-mode differentiation of the FP64 oracle step, and whole-run gradients
(through FLBRun with checkpointing) against the oracle's reference gradient and
FP64 central differences."""

import numpy as np
import pytest
import torch

import flb_workloads as W
from helpers import gpu_params, oracle_params, rel_err

pytestmark = pytest.mark.gpu

F64 = torch.float64
C2 = dict(lattice="D3Q19", rho0=1.0, kT=1e-5, rate_bulk=1.2, rate_shear=1.6, rate_ghost=1.0, seed=7)
LANDAU = dict(force_model=1, a=-0.01, b=0.1, rho_c=1.0, kappa=0.05)
GRAD_KEYS = ("rate_shear", "kT", "rate_bulk", "rate_ghost")


def oracle_vjp(kw, S_unshifted, abar, n):
    """(dL/dS_n, dL/dtheta) for L = <abar, step_n(S_n)> by autograd of the oracle."""
    from oracle import flb
    S = torch.as_tensor(S_unshifted, dtype=F64).clone().requires_grad_(True)
    th = {k: torch.tensor(float(kw[k]), dtype=F64, requires_grad=True) for k in GRAD_KEYS}
    po = oracle_params(**kw).with_(**th)
    out = flb.step(S, n, po)
    L = (out * torch.as_tensor(abar, dtype=F64)).sum()
    L.backward()
    return S.grad.numpy(), np.array([float(th[k].grad) for k in GRAD_KEYS])


CASES = [
    ("D2Q9", False, (1, 13, 70)),
    ("D2Q9", True, (1, 37, 70)),
    ("D3Q19", False, (9, 10, 70)),
    ("D3Q19", True, (11, 13, 35)),
]


@pytest.mark.parametrize("lattice,force,shape", CASES)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("eta", [0, 1])
def test_adjoint_step_matches_oracle_vjp(lattice, force, shape, precision, eta):
    from paper_1012_3632_amd import Simulation, lattice_tables
    if eta and not force:
        pytest.skip("eta only affects the force model")
    nz, ny, nx = shape
    kw = dict(C2, lattice=lattice, precision=precision, nx=nx, ny=ny, nz=nz, rate_bulk=1.3,
              rate_shear=0.8, rate_ghost=1.7)
    if force:
        kw.update(LANDAU, kT=1e-6, eta=eta)
    q = 9 if lattice == "D2Q9" else 19
    w = lattice_tables(lattice)["w"].reshape(-1, 1, 1, 1)
    dS = W.random_populations(q, shape, 11, 1e-3) * w * 10
    dS[:] += w * W.initial_drho(shape, 12, 0.01)[None]
    abar = W.random_populations(q, shape, 13, 1.0)
    n = 17
    sim = Simulation(gpu_params(**kw))
    dt = sim.params.dtype
    g = np.zeros(4)
    out = sim.adjoint_step(torch.as_tensor(dS, dtype=dt, device="cuda"),
                           torch.as_tensor(abar, dtype=dt, device="cuda"), n, grad=g)
    got = out.cpu().double().numpy()
    # the oracle sees exactly the populations the GPU stored
    dS_used = torch.as_tensor(dS, dtype=dt).double().numpy()
    ref, gref = oracle_vjp(kw, dS_used + w * kw["rho0"], abar, n)
    tol_pop = 1e-12 if precision == "fp64" else 2e-5
    assert rel_err(got, ref) < tol_pop
    scale = np.abs(gref).max()
    tol_g = 1e-9 if precision == "fp64" else 1e-4
    np.testing.assert_allclose(g, gref, rtol=tol_g, atol=tol_g * scale)


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (1, 20, 33)), ("D3Q19", (6, 7, 9))])
def test_adjoint_density_seed(lattice, shape):
    from oracle import flb
    from paper_1012_3632_amd import Simulation
    kw = dict(C2, lattice=lattice, precision="fp64", nx=shape[2], ny=shape[1], nz=shape[0])
    sim = Simulation(gpu_params(**kw))
    rb = W.initial_drho(shape, 4, 1.0)
    got = sim.adjoint_seed(torch.as_tensor(rb, device="cuda")).cpu().numpy()
    po = oracle_params(**kw)
    lat = flb.lattice_of(po)
    S = torch.zeros((lat.q,) + shape, dtype=F64, requires_grad=True)
    (flb.density(flb.pull(S, lat)) * torch.as_tensor(rb)).sum().backward()
    np.testing.assert_allclose(got, S.grad.numpy(), rtol=0, atol=1e-15)


def _run_grad_case(kw, shape, nsteps, ck, drho_amp=0.01):
    """GPU FLBRun gradient and the oracle reference gradient of
    L = mean((rho_N - rho_target)^2)."""
    from oracle import flb, grad
    from paper_1012_3632_amd import lattice_tables
    from paper_1012_3632_amd.autograd import FLBRun
    po = oracle_params(**kw)
    drho = W.initial_drho(shape, 5, drho_amp)
    S0 = flb.initial_state(po, drho)
    target = grad.final_density(S0, po.with_(rate_shear=1.5), nsteps)
    p = gpu_params(**kw)
    w = torch.as_tensor(lattice_tables(kw["lattice"])["w"]).view(-1, 1, 1, 1)
    df0 = (S0 - w * kw["rho0"]).to("cuda", p.dtype).requires_grad_(True)
    rs = torch.tensor(kw["rate_shear"], dtype=F64, requires_grad=True)
    kT = torch.tensor(kw["kT"], dtype=F64, requires_grad=True)
    rho = FLBRun.apply(df0, rs, kT, p, nsteps, ck)
    L = ((rho.double() - target.to("cuda")) ** 2).mean()
    L.backward()
    Lr, gS, gth = grad.loss_and_grads(S0, po, nsteps, target, checkpoint_every=ck)
    return dict(L=float(L), gS=df0.grad.double().cpu().numpy(), rs=float(rs.grad), kT=float(kT.grad),
                extra=FLBRun.last_grads), dict(L=Lr, gS=gS.numpy(), **gth), (po, S0, target)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("lattice,force", [("D2Q9", True), ("D3Q19", False), ("D3Q19", True)])
def test_run_gradient_matches_oracle(precision, lattice, force):
    if lattice == "D2Q9":
        kw = dict(W.params_of("d2q9_256_adjoint", nx=40, ny=34), precision=precision)
        shape = (1, 34, 40)
    else:
        kw = dict(C2, precision=precision, nx=12, ny=10, nz=9)
        if force:
            kw.update(LANDAU, kT=1e-6)
        shape = (9, 10, 12)
    got, ref, _ = _run_grad_case(kw, shape, 30, 7)
    tol = 1e-9 if precision == "fp64" else 1e-4
    np.testing.assert_allclose(got["L"], ref["L"], rtol=1e-9 if precision == "fp64" else 1e-3)
    assert rel_err(got["gS"], ref["gS"]) < tol
    np.testing.assert_allclose(got["rs"], ref["rate_shear"], rtol=tol)
    np.testing.assert_allclose(got["kT"], ref["kT"], rtol=tol)
    np.testing.assert_allclose(got["extra"]["rate_bulk"], ref["rate_bulk"], rtol=tol)
    np.testing.assert_allclose(got["extra"]["rate_ghost"], ref["rate_ghost"], rtol=tol)


def test_run_gradient_with_float_parameters():
    """Rate and kT passed as plain floats: backward returns dL/d(delta f0)
    (equal to the run with tensor parameters) and no parameter gradients."""
    from paper_1012_3632_amd.autograd import final_density
    kw = dict(W.params_of("d2q9_256_adjoint", nx=40, ny=34), precision="fp32")
    p = gpu_params(**kw)
    df0 = torch.as_tensor(W.random_populations(9, (1, 34, 40), 3, 1e-3)).to("cuda", p.dtype)
    grads = []
    for as_tensor in (False, True):
        x = df0.clone().requires_grad_(True)
        rs, kT = kw["rate_shear"], kw["kT"]
        if as_tensor:
            rs = torch.tensor(rs, dtype=F64, requires_grad=True)
            kT = torch.tensor(kT, dtype=F64, requires_grad=True)
        rho = final_density(x, rs, kT, p, 30, 10)
        (rho ** 2).mean().backward()
        grads.append(x.grad.clone())
        if as_tensor:
            assert rs.grad is not None and kT.grad is not None
    assert torch.equal(grads[0], grads[1])


def test_d2q9_256_adjoint_full_size_vs_fd():
    """The differentiable workload at full size (D2Q9 256^2, FP32, 400 steps,
    checkpoint every 20): GPU gradients w.r.t. the shear rate, kT and the
    initial populations (two seeded directions) against FP64 central
    differences of the oracle (relative step 1e-6 for scalars)."""
    from oracle import grad
    wl = W.WORKLOADS["d2q9_256_adjoint"]
    kw = dict(W.params_of("d2q9_256_adjoint"), precision="fp32")
    shape = (1, 256, 256)
    nsteps, ck = wl["steps"], wl["checkpoint_every"]
    from oracle import flb
    from paper_1012_3632_amd import lattice_tables
    from paper_1012_3632_amd.autograd import FLBRun
    po = oracle_params(**kw)
    drho = W.initial_drho(shape, 1234, wl["init_noise"])
    S0 = flb.initial_state(po, drho)
    target = grad.final_density(S0, po.with_(rate_shear=wl["target_rate_shear"]), nsteps)
    p = gpu_params(**kw)
    w = torch.as_tensor(lattice_tables("D2Q9")["w"]).view(-1, 1, 1, 1)
    df0 = (S0 - w).to("cuda", torch.float32).requires_grad_(True)
    rs = torch.tensor(kw["rate_shear"], dtype=F64, requires_grad=True)
    kT = torch.tensor(kw["kT"], dtype=F64, requires_grad=True)
    rho = FLBRun.apply(df0, rs, kT, p, nsteps, ck)
    L = ((rho.double() - target.to("cuda")) ** 2).mean()
    L.backward()
    for name, gpu_val in (("rate_shear", float(rs.grad)), ("kT", float(kT.grad))):
        th = float(kw[name])
        h = 1e-6 * th
        lp = grad.loss_only(S0, po.with_(**{name: th + h}), nsteps, target)
        lm = grad.loss_only(S0, po.with_(**{name: th - h}), nsteps, target)
        fd = (lp - lm) / (2 * h)
        np.testing.assert_allclose(gpu_val, fd, rtol=1e-4)
    gS = df0.grad.double().cpu()
    for seed in (1, 2):
        v = torch.as_tensor(W.unit_direction(S0.shape, seed))
        h = 1e-6
        lp = grad.loss_only(S0 + h * v, po, nsteps, target)
        lm = grad.loss_only(S0 - h * v, po, nsteps, target)
        fd = (lp - lm) / (2 * h)
        np.testing.assert_allclose(float((gS * v).sum()), fd, rtol=1e-4)


@pytest.mark.parametrize("lattice,force,precision,nsteps,ck", [
    ("D2Q9", True, "fp32", 47, 10), ("D2Q9", True, "fp64", 20, 20), ("D3Q19", False, "fp32", 9, 2),
    ("D3Q19", True, "fp64", 13, 4), ("D2Q9", False, "fp64", 5, 5)])
def test_adjoint_run_equals_segment_loop(lattice, force, precision, nsteps, ck):
    """flb_adjoint_run (recompute of segment s - 1 on a helper stream beside
    the reverse sweep of segment s) gives dL/dS_0 and the parameter
    derivatives bit for bit equal to flb_adjoint_segment called per segment
    from last to first, for ragged last segments and single segments."""
    from paper_1012_3632_amd import Simulation
    shape = (1, 37, 70) if lattice == "D2Q9" else (9, 10, 21)
    kw = dict(C2, lattice=lattice, precision=precision, nz=shape[0], ny=shape[1], nx=shape[2])
    if force:
        kw.update(LANDAU, kT=1e-6)
    sim = Simulation(gpu_params(**kw), drho_init=W.initial_drho(shape, 3, 0.01))
    ckpts = []
    for k0 in range(0, nsteps, ck):
        ckpts.append(sim.state().clone())
        sim.step(min(ck, nsteps - k0))
    rhobar = torch.as_tensor(W.initial_drho(shape, 4, 1.0), dtype=sim.params.dtype, device="cuda")
    seed = sim.adjoint_seed(rhobar)
    a1, g1 = seed.clone(), np.zeros(4)
    for s in range(len(ckpts) - 1, -1, -1):
        k0 = s * ck
        sim.adjoint_segment(ckpts[s], a1, k0, min(k0 + ck, nsteps), grad=g1 if s == 0 else None)
    a2, g2 = seed.clone(), np.zeros(4)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sim.adjoint_run(ckpts, a2, ck, nsteps, grad=g2, stream=stream)
    torch.cuda.synchronize()
    assert torch.equal(a1, a2)
    np.testing.assert_array_equal(g1, g2)
    sim.close()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_one_launch_recompute_equals_density_pass_recompute(precision):
    """The D2Q9 force recompute in a shape that forms its own density tile
    writes each recomputed state's density from the step itself; the
    gradients equal, bit for bit, those of a shape whose recompute runs the
    density pass after every step (the two forward paths are bit-identical)."""
    from paper_1012_3632_amd import Simulation
    shape = (1, 37, 70)
    nsteps, ck = 23, 8
    kw = dict(C2, lattice="D2Q9", precision=precision, nz=1, ny=37, nx=70, **LANDAU)
    kw["kT"] = 1e-6
    out = []
    for cfg in (3, 0):   # 64 x 4 forming its density tile; 64 x 4 reading a density pass
        sim = Simulation(gpu_params(**kw), drho_init=W.initial_drho(shape, 3, 0.01))
        sim.set_launch(cfg)
        ckpts = []
        for k0 in range(0, nsteps, ck):
            ckpts.append(sim.state().clone())
            sim.step(min(ck, nsteps - k0))
        rhobar = torch.as_tensor(W.initial_drho(shape, 4, 1.0), dtype=sim.params.dtype,
                                 device="cuda")
        a, g = sim.adjoint_seed(rhobar), np.zeros(4)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            sim.adjoint_run(ckpts, a, ck, nsteps, grad=g, stream=stream)
        torch.cuda.synchronize()
        out.append((sim.state().clone(), a.clone(), g.copy()))
        sim.close()
    assert torch.equal(out[0][0], out[1][0])
    assert torch.equal(out[0][1], out[1][1])
    np.testing.assert_array_equal(out[0][2], out[1][2])
