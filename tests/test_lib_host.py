"""Host-side checks of the HIP library (no GPU needed): the shared library
loads, exports every symbol include/flb.h declares, its constant tables equal
the oracle's independently built ones, and invalid parameters are rejected."""

import numpy as np
import pytest

from oracle import lattice


def test_library_exports_every_declared_symbol():
    from paper_1012_3632_amd import _lib
    names = _lib.declared_symbols()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(_lib.lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_library_tables_equal_oracle(name):
    from paper_1012_3632_amd import lattice_tables
    t = lattice_tables(name)
    lat = lattice.get(name)
    assert t["q"] == lat.q
    np.testing.assert_array_equal(t["c"], lat.c)
    np.testing.assert_allclose(t["w"], lat.w, rtol=1e-15)
    np.testing.assert_array_equal(t["T"], lat.T)
    np.testing.assert_allclose(t["N"], lat.N, rtol=1e-15)
    names = ["rho", "j", "bulk", "shear", "ghost"]
    assert [names[k] for k in t["cls"]] == lat.classes


def test_sizes_and_validation():
    from paper_1012_3632_amd import Params, query_sizes
    from paper_1012_3632_amd._lib import FLBError
    pop, scr, sta = query_sizes(Params(lattice="D3Q19", precision="fp32", nx=128, ny=128, nz=128))
    assert pop == 19 * 128 ** 3 * 4
    pop64, _, _ = query_sizes(Params(lattice="D3Q19", precision="fp64", nx=128, ny=128, nz=128))
    assert pop64 == 2 * pop
    assert sta >= 2 * 19 * 8
    # the D3Q19 force step in FP32 also holds a second density field (the
    # march forms the next step's density there) and one 64 B edge record
    # per 64-wide x segment of every row; FP64 does not
    landau = dict(lattice="D3Q19", nx=130, ny=7, nz=5, force_model=1, a=-0.01, b=0.1,
                  rho_c=1.0, kappa=0.05)
    _, scr32, _ = query_sizes(Params(precision="fp32", **landau))
    _, scr64, _ = query_sizes(Params(precision="fp64", **landau))
    V = 130 * 7 * 5
    assert scr32 >= 2 * V * 4 + 3 * 7 * 5 * 64
    # the rest of the work area (density, adjoint fields) scales with the
    # precision, so FP32 exceeds half of FP64 by at least the second field
    assert scr32 - scr64 // 2 >= V * 4
    bad = [dict(kT=1 / 3), dict(kT=-1e-9), dict(rate_shear=2.0), dict(rate_ghost=0.0),
           dict(nz=2), dict(nx=0), dict(rho0=0.0), dict(lattice="D3Q19", nx=2048, ny=2048, nz=1024),
           dict(force_model=1, kappa=-1.0), dict(force_model=1, eta=2), dict(force_model=3)]
    for b in bad:
        kw = dict(lattice="D2Q9", precision="fp64", nx=8, ny=8, nz=1)
        kw.update(b)
        with pytest.raises(FLBError):
            query_sizes(Params(**kw))


def test_product_path_does_not_use_oracle():
    """The package never imports the oracle (and vice versa)."""
    import ast
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    for pkg, forbidden in (("paper_1012_3632_amd", "oracle"), ("oracle", "paper_1012_3632_amd")):
        for dirpath, _, files in os.walk(os.path.join(root, pkg)):
            for fn in files:
                if not fn.endswith(".py"):
                    continue
                tree = ast.parse(open(os.path.join(dirpath, fn)).read())
                for node in ast.walk(tree):
                    if isinstance(node, ast.Import):
                        assert all(not a.name.startswith(forbidden) for a in node.names), fn
                    elif isinstance(node, ast.ImportFrom) and node.module:
                        assert not node.module.startswith(forbidden), fn


@pytest.mark.parametrize("eta", [0, 1])
def test_equilibration_theory_equals_oracle(eta):
    """The library's host-side Sec. VI closed forms (G_aa(k), the double well,
    the longitudinal/transverse momentum split) equal the oracle's,
    written independently."""
    import flb_workloads as W
    from oracle import flb, spectra
    from paper_1012_3632_amd import equilibration as E
    wl = W.WORKLOADS["d2q9_128_equilibration"]
    np.testing.assert_allclose(E.double_well(wl["rho_L"], wl["rho_V"], wl["cs"], wl["rho0"]),
                               spectra.double_well(wl["rho_L"], wl["rho_V"], wl["cs"],
                                                   wl["rho0"]), rtol=1e-15)
    for lat, shape in (("D2Q9", (1, 12, 20)), ("D3Q19", (6, 5, 8))):
        p = E.paper_params(nx=shape[2], ny=shape[1]).with_(lattice=lat, nz=shape[0], eta=eta)
        po = flb.Params(lattice=lat, nx=p.nx, ny=p.ny, nz=p.nz, rho0=p.rho0, kT=p.kT,
                        force_model=1, a=p.a, b=p.b, rho_c=p.rho_c, kappa=p.kappa, eta=eta)
        np.testing.assert_allclose(E.paper_variance(p), spectra.theory_variance(po), rtol=1e-13)
        np.testing.assert_allclose(E.paper_variance(p.with_(force_model=0)),
                                   spectra.theory_variance(po.with_(force_model=0)), rtol=1e-13)
        rng = np.random.default_rng(4)
        spec = rng.random((p.q + (1 if p.d == 2 else 3),) + shape)
        a, b = E.momentum_split(spec, p), spectra.momentum_split(spec, po)
        np.testing.assert_allclose(a, b, rtol=1e-12, equal_nan=True)


def test_capillary_theory_equals_oracle():
    """The library's host-side capillary closed forms (eq. surf-tension, the
    lattice capillary structure factor, the stripe's mean-field profile) equal the oracle's and the shared input generator's."""
    import flb_workloads as W
    from oracle import capillary as cap
    from oracle import flb
    from paper_1012_3632_amd import capillary as C
    wl = W.WORKLOADS["d2q9_capillary"]
    p = C.paper_params(nx=64, ny=40)
    assert (p.a, p.b, p.rho_c) == (wl["a"], wl["b"], wl["rho_c"])
    np.testing.assert_allclose(C.surface_tension(1.0, 0.5, 0.08, 0.1),
                               cap.surface_tension(1.0, 0.5, 0.08, 0.1), rtol=1e-15)
    k = [2 * np.pi * np.arange(64) / 64]
    np.testing.assert_allclose(C.capillary_theory(p, 1e-7, 3e-3),
                               cap.capillary_theory(k, 1e-7, 3e-3, 64), rtol=1e-14,
                               equal_nan=True)
    w = C.mean_field_width(1.0, 0.5, 0.08, 0.1)
    np.testing.assert_allclose(w, cap.interface_width(1.0, 0.5, 0.08, 0.1), rtol=1e-15)
    np.testing.assert_allclose(C.stripe(p, 10.0, 30.0, 1.0, 0.5, w),
                               W.stripe_drho(p.shape, 10.0, 30.0, 1.0, 0.5, w, p.rho0),
                               atol=1e-15)


def test_modeq_validation_and_sizes():
    """flb_modeq_work_bytes: 24 V bytes in FP32, 48 V in FP64; invalid extents, rates, kT, c_s^2(k)
    above 0.6 and rates that leave the (e, eps) covariance indefinite are
    rejected on the host."""
    from paper_1012_3632_amd._lib import FLBError
    from paper_1012_3632_amd.modeq import ModEqParams, paper_params, work_bytes
    ok = ModEqParams(nx=8, ny=8, kT=1e-5, cs2_0=0.07, kappa=0.08, rate_bulk=1.2, rate_shear=1.6,
                     rate_ghost=0.9)
    assert work_bytes(ok) == 24 * 64
    assert work_bytes(ok.with_(precision="fp64")) == 48 * 64
    assert work_bytes(paper_params()) == 24 * 128 * 128
    bad = [ok.with_(nx=1025), ok.with_(ny=0), ok.with_(rate_shear=2.0), ok.with_(kT=-1.0),
           ok.with_(cs2_0=0.0), ok.with_(kappa=0.2),
           ok.with_(cs2_0=0.55, kappa=0.0, rate_bulk=1.0, rate_ghost=1.9)]
    for p in bad:
        with pytest.raises(FLBError):
            work_bytes(p)


def test_modeq_entry_points_reject_bad_pointers():
    """flb_modeq_step / _run / _noise / _moments check their pointers on the
    host before any device work: NULL, aliased or unaligned buffers and a
    too-small work buffer are errors (no device memory is touched)."""
    import ctypes as C

    from paper_1012_3632_amd._lib import FLBError, call
    from paper_1012_3632_amd.modeq import ModEqParams
    p = ModEqParams(nx=8, ny=8, kT=1e-5, cs2_0=0.07, kappa=0.08, precision="fp32").to_c()
    A, B, Wk = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p(3 << 20)
    odd = C.c_void_p((1 << 20) + 8)
    need = 24 * 64   # FP32 work bytes of 8 x 8 sites
    bad_calls = [
        ("flb_modeq_step", C.byref(p), None, B, 0, Wk, need, None),
        ("flb_modeq_step", C.byref(p), A, A, 0, Wk, need, None),
        ("flb_modeq_step", C.byref(p), odd, B, 0, Wk, need, None),
        ("flb_modeq_step", C.byref(p), A, B, 0, Wk, need - 1, None),
        ("flb_modeq_step", C.byref(p), A, B, 0, None, need, None),
        ("flb_modeq_run", C.byref(p), A, A, 0, 4, Wk, need, None),
        ("flb_modeq_run", C.byref(p), A, B, 0, -1, Wk, need, None),
        ("flb_modeq_noise", C.byref(p), 0, None, Wk, need, None),
        ("flb_modeq_noise", C.byref(p), 0, A, Wk, need - 1, None),
        ("flb_modeq_moments", C.byref(p), None, A, None),
        ("flb_modeq_moments", C.byref(p), odd, A, None),
    ]
    for name, *args in bad_calls:
        with pytest.raises(FLBError) as e:
            call(name, *args)
        assert e.value.status == -1, (name, e.value)   # FLB_ERR_INVALID_ARG: rejected on the host


def test_modeq_noalloc_step_rejects_on_the_host():
    """flb_modeq_step_noalloc checks its parameters, pointers and the size of
    its fixed 16 MiB work array on the host, before any device call."""
    import ctypes as C

    from paper_1012_3632_amd._lib import FLBError, call
    from paper_1012_3632_amd.modeq import ModEqParams
    nbytes = C.c_size_t()
    call("flb_modeq_static_work_bytes", C.byref(nbytes))
    assert nbytes.value == 16 << 20
    ok = ModEqParams(nx=8, ny=8, kT=1e-5, cs2_0=0.07, kappa=0.08)
    A, B, odd = C.c_void_p(1 << 20), C.c_void_p(2 << 20), C.c_void_p((1 << 20) + 8)
    big64 = ok.with_(nx=1024, ny=342, precision="fp64")   # 48 V = 16.03 MiB
    big32 = ok.with_(nx=1024, ny=683, precision="fp32")   # 24 V = 16.01 MiB
    assert 48 * 1024 * 342 > nbytes.value and 24 * 1024 * 683 > nbytes.value
    bad_calls = [
        (ok.to_c(), None, B), (ok.to_c(), A, A), (ok.to_c(), odd, B),
        (ok.with_(rate_bulk=2.5).to_c(), A, B), (big64.to_c(), A, B), (big32.to_c(), A, B),
    ]
    for p, fin, fout in bad_calls:
        with pytest.raises(FLBError) as e:
            call("flb_modeq_step_noalloc", C.byref(p), fin, fout, 0, None)
        assert e.value.status == -1, e.value


def test_batch64_edge_file_is_the_draw():
    """tests/golden/d3q19_batch64_edges.json holds the replica edges the
    batched workload draws (the realised list of the 64-replica run)."""
    import json
    import os

    import flb_workloads as W
    wl = W.WORKLOADS["d3q19_batch64"]
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                    "d3q19_batch64_edges.json")))
    edges = W.batch_edges(wl["replicas"], wl["edges"], wl["size_seed"])
    assert d["edges"] == edges and len(edges) == 64
    assert d["sites"] == sum(e ** 3 for e in edges)
