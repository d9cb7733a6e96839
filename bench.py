"""Benchmark of the fused fluctuating-LB step on one MI355X.

Workload (metric's configuration): D3Q19 ideal gas 128^3, FP32 shifted
populations, rates bulk/shear/ghost 1.2/1.6/1.0, kT 1e-5, seed 7, with the FP64
moment statistics accumulated every step.  A "step" is one full time step of
the hot path (pull, moments, relaxation + Philox/Box-Muller noise, inverse,
store, statistics).  Inputs are resident in HBM before the timed region.

Prints one JSON line: MLUPS (whole job), the roofline of the dominant kernel
(algorithmic bytes 2 Q s per site over the kernel's average launch time, HIP
events on the launch stream), the FP64 step beside it, the other workloads
(non-ideal 256^3, 64-replica batch, adjoint/forward ratio) and the CPU oracle
timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-extras]
"""

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def src_hash():
    h = hashlib.sha256()
    # the step kernel's device sources: kernels.hip and the headers it
    # includes, with comments left out and white space collapsed (an edit of
    # comments or layout leaves the counters valid)
    csrc = os.path.join(ROOT, "paper_1012_3632_amd", "csrc")
    for p in [os.path.join(csrc, "kernels.hip")] + sorted(glob.glob(os.path.join(csrc, "*.h"))):
        text = re.sub(r"/\*.*?\*/", " ", open(p).read(), flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel_keys):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy)
    from the committed rocprofv3 counter summary, averaged over the given
    kernels (the two phases of an in-place pair), or None if the counters were
    taken on other kernel sources than the ones built now."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if d.get("src_hash") != src_hash():
            return None
        vals = [d["bytes_per_launch"].get(k) for k in kernel_keys]
        if any(v is None for v in vals):
            return None
        return round(sum(vals) / len(vals))
    except Exception:
        return None


def time_steps(sim, steps, stride, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps, stats_stride=stride, stream=stream)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / steps   # ms per step


def fdt_check(sim):
    """Measured variance of each non-conserved mode over the sampled sites and
    steps against the fluctuation-dissipation value rho0 kT N_a / cs2."""
    import numpy as np

    from paper_1012_3632_amd import lattice_tables
    p = sim.params
    s, s2, n = sim.moments()
    cnt = float(n) * p.nx * p.ny * p.nz
    var = s2 / cnt - (s / cnt) ** 2
    N = lattice_tables("D3Q19" if p.q == 19 else "D2Q9")["N"]
    d = 3 if p.q == 19 else 2
    ratio = var[d + 1:] / (p.rho0 * p.kT * N[d + 1:] * 3.0)
    return {"samples": int(n), "max_rel_dev": round(float(np.abs(ratio - 1).max()), 5),
            "mean_ratio": round(float(ratio.mean()), 5)}


def profile_key(shape):
    """Name(s) of a stats-on D3Q19 FP32 step launch in the committed counter
    table (an in-place shape has one entry per phase of a pair)."""
    tx, ty, tz, spt, nt, _, ip, _ = shape
    if ip:
        sp = "x%d" % spt if spt > 1 else ""
        return ["k_step_ip_d3q19_fp32_stats_%dx%d%s_ph%d" % (tx, ty, sp, ph) for ph in (0, 1)]
    return ["k_step_d3q19_fp32_stats_%dx%dx%dx%d%s" % (tx, ty, tz, spt, "_nt" if nt else "")]


def bench_main(args):
    import numpy as np
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation

    stream = torch.cuda.Stream()   # non-null stream: graph capture needs one
    torch.cuda.set_stream(stream)
    kw = W.params_of("d3q19_128")
    p = Params.from_dict(dict(kw, precision="fp32"))
    V = p.nx * p.ny * p.nz
    sim = Simulation(p)
    tuned = sim.autotune(repeats=5)
    (plain_cfg, best_cfg, _, pair_cfg), _ = tuned
    run_cfg = pair_cfg if pair_cfg >= 0 else best_cfg
    sim.step(args.warmup, stats_stride=1)
    sim.reset_stats()   # the statistics of the timed steps alone (after the burn-in)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = time_steps(sim, args.steps, 1, stream)
    wall = time.perf_counter() - t0
    fdt = fdt_check(sim)
    mlups = V / (ms * 1e-3) / 1e6
    bytes_site = 2 * 19 * 4
    achieved = bytes_site * V / (ms * 1e-3) / 1e9
    out = {
        "metric": "D3Q19 FLB MLUPS + % HBM roofline, FP32 vs FP64; adjoint/forward time ratio",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "d3q19_128 ideal-gas FLB, 128^3 periodic, FP32 shifted storage, "
                               "rates 1.2/1.6/1.0, kT 1e-5, seed 7, FP64 statistics every step",
                   "lattice": "D3Q19", "sites": V, "launch_config": run_cfg,
                   "launch_shape": list(sim.launch_shape(run_cfg)),
                   "in_place_pairs": pair_cfg >= 0},
        # in-place pairs keep one 159 MB population buffer, which stays largely
        # resident in the 256 MB last-level (Infinity) cache: the rate is that
        # of HBM and that cache together ("hbm+llc"); d3q19_256_ideal below is
        # the same step on a state 8 times larger, bound by HBM alone
        "roofline": {"bound": "hbm+llc" if pair_cfg >= 0 else "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profiles(profile_key(sim.launch_shape(run_cfg))),
                     "kernel": ("k_step_ip<D3Q19,float,stats> (in-place pair, phases 0 and 1)"
                                if pair_cfg >= 0 else "k_step<D3Q19,float,ideal,stats>"),
                     "bytes_per_site": bytes_site,
                     "working_set_bytes": (1 if pair_cfg >= 0 else 2) * 19 * 4 * V},
        "wall_timed_s": round(wall, 3),
        "fdt": fdt,
        "autotune": {"shapes": list(tuned[0]), "ms_per_step": [round(x, 5) for x in tuned[1]]},
    }
    # the same step without statistics
    ms_ns = time_steps(sim, args.steps, 0, stream)
    out["fp32_nostats"] = {"ms_per_step": round(ms_ns, 5),
                           "MLUPS": round(V / (ms_ns * 1e-3) / 1e6, 1),
                           "hbm_frac": round(bytes_site * V / (ms_ns * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "launch_config": pair_cfg if pair_cfg >= 0 else plain_cfg}
    sim.close()
    del sim
    # context: what a plain device copy reaches on this GPU (read + write bytes)
    a = torch.empty(1 << 27, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(20):
        b.copy_(a)
    e1.record(stream)
    e1.synchronize()
    copy_gbs = 2 * a.numel() * 4 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    out["roofline"]["measured_copy_GBps"] = round(copy_gbs, 1)
    out["roofline"]["frac_of_measured_copy"] = round(achieved / copy_gbs, 4)
    del a, b
    torch.cuda.empty_cache()
    out["d3q19_256_ideal"] = ideal_256(stream, copy_gbs)
    # FP64 step beside it
    p64 = p.with_(precision="fp64")
    s64 = Simulation(p64)
    (_, cfg64, _, ip64), _ = s64.autotune(repeats=3)
    s64.step(args.warmup, stats_stride=1)
    ms64 = time_steps(s64, max(args.steps // 2, 10), 1, stream)
    out["fp64"] = {"ms_per_step": round(ms64, 5), "MLUPS": round(V / (ms64 * 1e-3) / 1e6, 1),
                   "hbm_frac": round(2 * 19 * 8 * V / (ms64 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                   "frac_of_measured_copy": round(2 * 19 * 8 * V / (ms64 * 1e-3) / 1e9 / copy_gbs, 4),
                   # the 318 MB state exceeds the last-level cache: the autotuner
                   # may prefer two buffers to the in-place pairs
                   "launch_config": ip64 if ip64 >= 0 else cfg64,
                   "launch_shape": list(s64.launch_shape(ip64 if ip64 >= 0 else cfg64)),
                   "in_place_pairs": ip64 >= 0}
    s64.close()
    del s64
    torch.cuda.empty_cache()

    if not args.no_extras:
        out.update(extras(args, stream))
        # a correctness field, run after every timing: its 5000 FP64 steps
        # at 256^3 are the longest GPU work of the benchmark
        out["fp32_vs_fp64"] = long_parity(stream)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


def ideal_256(stream, copy_gbs):
    """The headline step on a 256^3 lattice (1.27 GB per FP32 population
    buffer, five times the last-level cache): in-place pairs and two buffers,
    statistics every step, against 8 TB/s, the measured copy rate and the
    measured rate of a plain in-place pass over a buffer of the same size."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation
    p = Params.from_dict(dict(W.params_of("d3q19_128", nx=256, ny=256, nz=256), precision="fp32"))
    V = p.nx * p.ny * p.nz
    sim = Simulation(p)
    (_, best_stats, best_ip, _), tms = sim.autotune(repeats=3)
    res = {"workload": "d3q19_128's parameters on 256^3 (16.8 M sites), FP32, FP64 statistics "
                       "every step", "sites": V}
    for name, cfg in (("in_place_pairs", best_ip), ("two_buffers", best_stats)):
        if cfg < 0:
            continue
        sim.set_launch(cfg)
        sim.step(40, stats_stride=1)
        ms = time_steps(sim, 200, 1, stream)
        gbs = 152 * V / (ms * 1e-3) / 1e9
        res[name] = {"launch_config": cfg, "launch_shape": list(sim.launch_shape(cfg)),
                     "ms_per_step": round(ms, 5), "MLUPS": round(V / (ms * 1e-3) / 1e6, 1),
                     "achieved_GBps_152B": round(gbs, 1), "frac_of_8TBps": round(gbs / HBM_PEAK_GBS, 4),
                     "frac_of_measured_copy": round(gbs / copy_gbs, 4)}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    # measured ceilings: a flat in-place pass (x *= 1, torch) over one buffer
    # of the state's size, and the step's own access pattern without its
    # arithmetic (19 planes read and written per site, in place and between
    # two buffers: flb_plane_stream_probe)
    import ctypes as C

    from paper_1012_3632_amd._lib import call
    n = 19 * V
    a = torch.ones(n, device="cuda")
    bb = torch.ones(n, device="cuda")

    def rate(fn):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(20):
            fn()
        e1.record(stream)
        e1.synchronize()
        return 2 * n * 4 * 20 / (e0.elapsed_time(e1) * 1e-3) / 1e9

    sp = C.c_void_p(stream.cuda_stream)
    pa, pb = C.c_void_p(a.data_ptr()), C.c_void_p(bb.data_ptr())
    ip_gbs = rate(lambda: a.mul_(1.0))
    pat_ip = rate(lambda: call("flb_plane_stream_probe", pa, pa, 19, V, 1, sp))
    pat_two = rate(lambda: call("flb_plane_stream_probe", pa, pb, 19, V, 1, sp))
    del a, bb
    torch.cuda.empty_cache()
    res["measured_inplace_pass_GBps"] = round(ip_gbs, 1)
    res["measured_copy_GBps"] = round(copy_gbs, 1)
    res["measured_19plane_pattern_GBps"] = {"in_place": round(pat_ip, 1), "two_buffers": round(pat_two, 1)}
    if "in_place_pairs" in res:
        g = res["in_place_pairs"]["achieved_GBps_152B"]
        res["in_place_pairs"]["frac_of_measured_inplace_pass"] = round(g / ip_gbs, 4)
        res["in_place_pairs"]["frac_of_19plane_pattern"] = round(g / pat_ip, 4)
    if "two_buffers" in res:
        res["two_buffers"]["frac_of_19plane_pattern"] = round(
            res["two_buffers"]["achieved_GBps_152B"] / pat_two, 4)
    res["roofline"] = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "kernel": "k_step_ip<D3Q19,float,stats> (in-place pair)"}
    best = min((v for k, v in res.items() if k in ("in_place_pairs", "two_buffers")),
               key=lambda v: v["ms_per_step"])
    res["roofline"].update(achieved=best["achieved_GBps_152B"], frac=best["frac_of_8TBps"])
    return res


def long_parity(stream):
    """FP32 against the FP64 GPU step over the full lengths of the two 3-D
    workloads (d3q19_128: 2000 steps; d3q19_256_landau, eta = 0: 5000 steps),
    from the same initial state: max |f32 - f64| / max |f64| on unshifted
    populations and the RMS of the shifted difference over the RMS of delta f64."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation, lattice_tables
    w = torch.as_tensor(lattice_tables("D3Q19")["w"], device="cuda").view(19, 1, 1, 1)
    res = {}
    for name, nsteps in (("d3q19_128", 2000), ("d3q19_256_landau", 5000)):
        kw = W.params_of(name)
        drho = (W.initial_drho((kw["nz"], kw["ny"], kw["nx"]), 7, W.WORKLOADS[name]["init_noise"])
                if kw.get("force_model") else None)
        st, t = {}, {}
        for prec in ("fp64", "fp32"):
            sim = Simulation(Params.from_dict(dict(kw, precision=prec)), drho_init=drho)
            if prec == "fp32":
                sim.autotune(repeats=2)
            elif kw.get("force_model"):
                sim.set_launch(7)    # z-marching force step, 128 x 2 columns
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            sim.step(nsteps, stream=stream)
            e1.record(stream)
            e1.synchronize()
            t[prec] = e0.elapsed_time(e1) / nsteps
            st[prec] = sim.state().clone()
            sim.close()
            del sim
            torch.cuda.empty_cache()
        d = st["fp32"].double() - st["fp64"]
        fmax = (st["fp64"] + w * kw["rho0"]).abs().max()
        res[name] = {"steps": nsteps,
                     "max_rel_err_unshifted": float("%.3e" % float(d.abs().max() / fmax)),
                     "rms_rel_err_shifted": float("%.3e" % float(
                         torch.sqrt((d * d).mean()) / torch.sqrt((st["fp64"] ** 2).mean()))),
                     "mass_fp32_minus_fp64": float("%.3e" % float(st["fp32"].double().sum() - st["fp64"].sum())),
                     "ms_per_step_fp32": round(t["fp32"], 4), "ms_per_step_fp64": round(t["fp64"], 4)}
        del st, d
        torch.cuda.empty_cache()
    return res


def extras(args, stream):
    import numpy as np
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation

    res = {}
    # non-ideal fluid 256^3
    kw = W.params_of("d3q19_256_landau")
    p = Params.from_dict(dict(kw, precision="fp32"))
    V = p.nx * p.ny * p.nz
    drho = W.initial_drho(p.shape, 7, W.WORKLOADS["d3q19_256_landau"]["init_noise"])
    s = Simulation(p, drho_init=drho)
    del drho
    (cfg_plain, cfg_stats, _, _), _ = s.autotune(repeats=3)
    s.step(5, stats_stride=1)
    n = max(args.steps // 4, 100)
    ms = time_steps(s, n, 1, stream)
    shape = list(s.launch_shape(cfg_stats))
    if shape[7] == 2:
        # the march forms the next step's density itself: it moves 152 B of
        # populations, reads the density (4 B), writes the partial density
        # (4 B), the x-segment edge records (40 B per 64 sites) and the ghost
        # rows of the neighbouring tiles' edge rows (4 B per edge row: 8 / TY
        # B); the completion pass reads the partial density and writes the
        # density (8 B), reads the ghost rows (8 / TY B), the populations that
        # cross the plane run's z edges (40 / 16 B) and the edge records; the
        # first step of a call adds a density pass (80 B)
        ty = shape[1]
        bytes_site = 152 + 8 + 40 / 64 + 8 / ty + 8 + 8 / ty + 40 / 16 + 40 / 64
        pattern = "march forming the next density + completion pass (a call's first step: density pass)"
    else:
        # the density pass (19 reads + 1 write) and the force step (19 reads +
        # 19 writes + the density): 80 + 156 = 236 B per site
        bytes_site = 236
        pattern = "density pass + march"
    # the same steps without statistics (the autotuner's plain shape)
    ms_plain = time_steps(s, n, 0, stream)
    res["d3q19_256_landau"] = {"ms_per_step": round(ms, 4), "MLUPS": round(V / (ms * 1e-3) / 1e6, 1),
                               "steps_timed": n, "pattern": pattern,
                               "ms_per_step_without_statistics": round(ms_plain, 4),
                               "hbm_frac_algorithmic_160B_without_statistics":
                                   round(160 * V / (ms_plain * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "bytes_per_site": round(bytes_site, 2),
                               "hbm_frac_algorithmic": round(bytes_site * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               # the method's minimum: populations in and out plus
                               # one density write and read (152 + 8 B)
                               "hbm_frac_algorithmic_160B": round(160 * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "launch_config": cfg_stats, "launch_shape": shape,
                               "launch_config_without_statistics": cfg_plain,
                               "statistics": "every step"}
    s.close()
    del s
    torch.cuda.empty_cache()
    # the paper's own force (eta = 1: the ideal-gas pressure replaced), same cost
    s = Simulation(p.with_(eta=1), drho_init=W.initial_drho(p.shape, 7, W.WORKLOADS["d3q19_256_landau"]["init_noise"]))
    (_, cfg_stats, _, _), _ = s.autotune(repeats=3)
    s.step(5, stats_stride=1)
    ms = time_steps(s, n, 1, stream)
    res["d3q19_256_landau_eta1"] = {"ms_per_step": round(ms, 4), "MLUPS": round(V / (ms * 1e-3) / 1e6, 1),
                                    "launch_config": cfg_stats, "statistics": "every step"}
    s.close()
    del s
    torch.cuda.empty_cache()

    # 64 replicas of uneven size (the realised draw is tests/golden/
    # d3q19_batch64_edges.json), one persistent launch per step, the
    # workload's 1000 steps captured in one graph
    from paper_1012_3632_amd import Batch, lattice_tables
    wl = W.WORKLOADS["d3q19_batch64"]
    edges = W.batch_edges(wl["replicas"], wl["edges"], wl["size_seed"])
    pb = Params.from_dict(dict(lattice="D3Q19", precision="fp32", rho0=1.0, kT=wl["kT"],
                               rate_bulk=wl["rate_bulk"], rate_shear=wl["rate_shear"],
                               rate_ghost=wl["rate_ghost"]))
    b = Batch(pb, [(e, e, e) for e in edges], seeds=list(range(wl["replicas"])))
    (_, best), _ = b.autotune(repeats=3)
    pair_bytes, ngroups = b.pairs()
    gsteps = wl["steps"]

    def batch_graph_ms(fdt=False):
        b.graph_capture(gsteps, stats_stride=1, stream=stream)
        b.graph_launch(stream=stream)          # warm-up and burn-in: 1000 steps
        b.reset_stats(stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        b.graph_launch(stream=stream)
        e1.record(stream)
        e1.synchronize()
        return e0.elapsed_time(e1) / gsteps

    ms = batch_graph_ms()
    # per-replica fluctuation-dissipation check on the timed steps
    s1, s2, nsamp = b.moments()
    Nn = lattice_tables("D3Q19")["N"]
    vol = np.array([e ** 3 for e in edges], dtype=np.float64)[:, None]
    cnt = vol * nsamp
    ratio = (s2 / cnt - (s1 / cnt) ** 2)[:, 4:] / (pb.rho0 * pb.kT * Nn[4:] * 3.0)
    fdt_b = {"samples": int(nsamp), "max_rel_dev_all_replicas_modes": round(float(np.abs(ratio - 1).max()), 5),
             "max_rel_dev_replica_mean": round(float(np.abs(ratio.mean(1) - 1).max()), 5)}
    # the other schedule, for the record
    b.set_pairs(0 if pair_bytes else 128 << 20)
    ms_other = batch_graph_ms()
    b.set_pairs(pair_bytes)
    Vt = sum(e ** 3 for e in edges)
    res["d3q19_batch64"] = {"ms_per_step": round(ms, 4), "MLUPS": round(Vt / (ms * 1e-3) / 1e6, 1),
                            "sites": Vt, "grid_config": best,
                            "hbm_frac": round(152 * Vt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            # groups taken through all steps in place stay
                            # near the last-level cache size
                            "bound": "hbm+llc" if pair_bytes else "hbm",
                            "in_place_pair_groups": ngroups, "pair_group_bytes": pair_bytes,
                            ("ms_per_step_replica_interleaved" if pair_bytes else
                             "ms_per_step_pairs_128MiB_groups"): round(ms_other, 4),
                            "graph_steps": gsteps, "statistics": "every step", "fdt": fdt_b,
                            "edges_file": "tests/golden/d3q19_batch64_edges.json",
                            "count_by_edge": {str(e): edges.count(e) for e in wl["edges"]}}
    b.close()
    del b
    torch.cuda.empty_cache()

    # the equilibration test of Sec. VI: D2Q9 128^2, the paper's parameters
    from paper_1012_3632_amd import equilibration as E
    wl = W.WORKLOADS["d2q9_128_equilibration"]
    pe = E.paper_params(nx=wl["nx"], ny=wl["ny"], kT=wl["kT"], kappa=wl["kappa"], cs=wl["cs"],
                        rho_L=wl["rho_L"], rho_V=wl["rho_V"], seed=wl["seed"])
    se = Simulation(pe)
    spec = se.spectrum_buffer()
    se.graph_capture(wl["interval"], stats_stride=0, stream=stream)
    se.graph_launch(stream=stream)
    se.accumulate_spectrum(spec, stream=stream)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    torch.cuda.synchronize()
    e0.record(stream)
    se.graph_launch(stream=stream)
    e1.record(stream)
    nspec = 20
    for _ in range(nspec):
        se.accumulate_spectrum(spec, stream=stream)
    e2.record(stream)
    e2.synchronize()
    ms_step = e0.elapsed_time(e1) / wl["interval"]
    us_spec = e1.elapsed_time(e2) / nspec * 1e3
    Ve = pe.nx * pe.ny
    # direct DFT along x then y: 8 FP64 flops per complex multiply-add
    dft_flops = 8 * pe.q * Ve * (pe.nx + pe.ny)
    se.close()
    del se, spec
    t0 = time.perf_counter()
    spec_sum, se = E.run(pe, wl["snapshots"], wl["interval"], wl["burn_in"])
    run_s = time.perf_counter() - t0
    se.close()
    r = E.equilibration_ratio(spec_sum, wl["snapshots"], pe)
    kc, dens, _ = E.shell_average(r[0], pe, 16)
    dev = lambda rows: float(max(np.nanmax(np.abs(E.shell_average(r[a], pe, 16)[1][kc < 2.5] - 1))
                                 for a in rows))
    res["d2q9_128_equilibration"] = {
        "ms_per_step": round(ms_step, 5), "MLUPS": round(Ve / (ms_step * 1e-3) / 1e6, 1),
        "spectrum_us": round(us_spec, 2),
        "spectrum_fp64_tflops": round(dft_flops / (us_spec * 1e-6) / 1e12, 3),
        "run_s": round(run_s, 3), "steps": wl["burn_in"] + wl["snapshots"] * wl["interval"],
        "snapshots": wl["snapshots"],
        "density_ratio_by_shell": [round(float(x), 3) for x in dens],
        "momentum_max_dev_k_lt_2.5": round(dev(range(1, 3)), 4),
        "nonconserved_max_dev_k_lt_2.5": round(dev(range(3, 9)), 4)}

    # the modified-equilibrium (Swift) model at the same parameters (Sec. IV.B)
    from paper_1012_3632_amd import modeq as MQ
    wl = W.MODEQ_WORKLOADS["d2q9_128_modeq"]
    pm = MQ.ModEqParams(**W.modeq_params_of("d2q9_128_modeq"))
    sm = MQ.ModEq(pm)
    with torch.cuda.stream(stream):
        sm.step(200, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        nms = 2000
        e0.record(stream)
        sm.step(nms, stream=stream)
        e1.record(stream)
        e1.synchronize()
    ms_step = e0.elapsed_time(e1) / nms
    del sm
    t0 = time.perf_counter()
    spec_m, sm = MQ.run_spectra(pm, wl["burn_in"], wl["snapshots"], wl["interval"], stream=stream)
    run_s = time.perf_counter() - t0
    Vm = pm.nx * pm.ny
    rm = spec_m.cpu().numpy() / (wl["snapshots"] * Vm * MQ.equal_time_variances(pm))
    rm[:, 0, 0] = np.nan
    res["d2q9_128_modeq"] = {
        "ms_per_step": round(ms_step, 5), "MLUPS": round(Vm / (ms_step * 1e-3) / 1e6, 1),
        "run_s": round(run_s, 3), "steps": wl["burn_in"] + wl["snapshots"] * wl["interval"],
        "snapshots": wl["snapshots"],
        "ratio_to_G_by_mode": [round(float(x), 4) for x in np.nanmean(rm.reshape(9, -1), 1)]}
    del sm, spec_m
    # the same workload with FP64 state and step arithmetic
    sm64 = MQ.ModEq(pm.with_(precision="fp64"))
    with torch.cuda.stream(stream):
        sm64.step(200, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        sm64.step(2000, stream=stream)
        e1.record(stream)
        e1.synchronize()
    res["d2q9_128_modeq"]["fp64_ms_per_step"] = round(e0.elapsed_time(e1) / 2000, 5)
    del sm64
    # the same model at 1024^2, the largest extent of its transforms: one
    # step moves 232 B per site (noise: 32 B written by the row transforms,
    # 64 B read and written by the column pass, 48 B by the inverse rows;
    # step: 36 B of populations in, 36 B out, 16 B of filtered noise)
    pm2 = pm.with_(nx=1024, ny=1024)
    sm2 = MQ.ModEq(pm2)
    with torch.cuda.stream(stream):
        sm2.step(32, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        nms = 160
        e0.record(stream)
        sm2.step(nms, stream=stream)
        e1.record(stream)
        e1.synchronize()
    ms2 = e0.elapsed_time(e1) / nms
    V2 = pm2.nx * pm2.ny
    res["d2q9_1024_modeq"] = {"ms_per_step": round(ms2, 5), "MLUPS": round(V2 / (ms2 * 1e-3) / 1e6, 1),
                              "GBps_232B_per_site": round(232 * V2 / (ms2 * 1e-3) / 1e9, 1),
                              "hbm_frac": round(232 * V2 / (ms2 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    del sm2
    torch.cuda.empty_cache()

    # the capillary-fluctuation test of Sec. VI: 1024 x 400 stripe, 10^6 steps
    from paper_1012_3632_amd import capillary as CAP
    from paper_1012_3632_amd import field_spectrum
    wl = W.WORKLOADS["d2q9_capillary"]
    pc = CAP.paper_params(seed=wl["seed"])
    wc = CAP.mean_field_width(wl["rho_L"], wl["rho_V"], wl["kappa"], wl["beta"])
    sc = Simulation(pc, drho_init=CAP.stripe(pc, *wl["stripe"], wl["rho_L"], wl["rho_V"], wc))
    ifs = [(wl["stripe"][0], 1, 25), (wl["stripe"][1], -1, 25)]
    sc.graph_capture(wl["interval"], stats_stride=0, stream=stream)
    sc.graph_launch(stream=stream)
    hh = sc.interface_heights(ifs, wl["rho_L"], wl["rho_V"], wc, stream=stream)
    hspec = torch.zeros_like(hh)
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    torch.cuda.synchronize()
    e0.record(stream)
    sc.graph_launch(stream=stream)
    e1.record(stream)
    for _ in range(20):
        hh = sc.interface_heights(ifs, wl["rho_L"], wl["rho_V"], wc, stream=stream)
    e2.record(stream)
    for _ in range(20):
        field_spectrum(hh, hspec, stream=stream)
    e3.record(stream)
    e3.synchronize()
    ms_step = e0.elapsed_time(e1) / wl["interval"]
    us_h, us_s = e1.elapsed_time(e2) / 20 * 1e3, e2.elapsed_time(e3) / 20 * 1e3
    sc.close()
    del sc, hh, hspec
    t0 = time.perf_counter()
    spec_c, nsnap, means, sc = CAP.run(pc, wl["stripe"], wl["rho_L"], wl["rho_V"], wc,
                                        wl["steps"], wl["burn_in"], wl["interval"])
    run_s = time.perf_counter() - t0
    sc.close()
    kc = 2 * np.pi * np.arange(pc.nx) / pc.nx
    s_mf = CAP.surface_tension(wl["rho_L"], wl["rho_V"], wl["kappa"], wl["beta"])
    # the scheme's own tension by mechanics (Laplace drops on the oracle,
    # written by tests/golden/make_laplace_tension.py)
    s_mech = json.load(open(os.path.join(ROOT, "tests", "golden", "laplace_tension.json")))["sigma_inf"]
    ratio = lambda sig, lo, hi: round(float(np.mean(
        spec_c[:, (kc >= lo) & (kc < hi)] / (nsnap * CAP.capillary_theory(pc, pc.kT, sig)[(kc >= lo) & (kc < hi)]))), 3)
    s_cw = s_mf / ratio(s_mf, 0.1, 0.4)
    Vc = pc.nx * pc.ny
    res["d2q9_capillary"] = {
        "ms_per_step": round(ms_step, 5), "MLUPS": round(Vc / (ms_step * 1e-3) / 1e6, 1),
        "heights_us": round(us_h, 2), "height_spectrum_us": round(us_s, 2),
        "run_s": round(run_s, 3), "steps": wl["steps"], "snapshots": nsnap,
        "capillary_law_reached": False,
        "sigma_eq_surf_tension": round(float(s_mf), 6),
        "sigma_mechanical_laplace": round(float(s_mech), 6),
        "sigma_from_spectrum_0.1-0.4": round(float(s_cw), 6),
        "spectrum_over_theory_sigma": {"k<0.1": ratio(s_mf, 0.005, 0.1),
                                       "0.1-0.4": ratio(s_mf, 0.1, 0.4),
                                       "0.4-1": ratio(s_mf, 0.4, 1.0)},
        "spectrum_over_theory_sigma_mechanical": {"k<0.1": ratio(s_mech, 0.005, 0.1),
                                                  "0.1-0.4": ratio(s_mech, 0.1, 0.4)},
        "mean_heights": [round(float(x), 3) for x in means]}

    # differentiable run: adjoint / forward time
    from paper_1012_3632_amd.autograd import FLBRun
    wl = W.WORKLOADS["d2q9_256_adjoint"]
    pa = Params.from_dict(dict(W.params_of("d2q9_256_adjoint"), precision="fp32"))
    drho = W.initial_drho(pa.shape, 1234, wl["init_noise"])
    w = torch.tensor([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, dtype=torch.float64).view(-1, 1, 1, 1)
    df0 = (w * torch.as_tensor(drho)).to("cuda", torch.float32)
    target = torch.ones(pa.shape, dtype=torch.float64, device="cuda")
    # HIP events on the launch stream around the forward (FLBRun.forward:
    # the steps and the checkpoints) and the backward (seed, recompute,
    # reverse sweep): median and range over 7 repeats after one warm-up
    fwd, bwd = [], []
    for rep in range(8):
        x = df0.clone().requires_grad_(True)
        rs = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
        kT = torch.tensor(pa.kT, dtype=torch.float64, requires_grad=True)
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        torch.cuda.synchronize()
        e0.record(stream)
        rho = FLBRun.apply(x, rs, kT, pa, wl["steps"], wl["checkpoint_every"])
        L = ((rho - target) ** 2).mean()
        e1.record(stream)
        L.backward()
        e2.record(stream)
        e2.synchronize()
        if rep:
            fwd.append(e0.elapsed_time(e1))
            bwd.append(e1.elapsed_time(e2))
    ratios = sorted(b_ / f_ for f_, b_ in zip(fwd, bwd))
    res["d2q9_256_adjoint"] = {"forward_ms_median": round(float(np.median(fwd)), 3),
                               "backward_ms_median": round(float(np.median(bwd)), 3),
                               "adjoint_forward_ratio": round(float(np.median(ratios)), 3),
                               "ratio_range": [round(ratios[0], 3), round(ratios[-1], 3)],
                               "repeats": len(ratios), "steps": wl["steps"],
                               "checkpoint_every": wl["checkpoint_every"]}
    return res


def cpu_baseline():
    """The FP64 oracle on the host cores, on bounded samples of the workloads,
    with all the threads torch uses and with one: d3q19_128 (the headline
    workload; full-size steps until about 8 s of wall time, at least one),
    d2q9_32_fp64 (200 steps) and d2q9_256_adjoint (the forward step, 10 steps).
    ``value`` is the d3q19_128 figure with all threads."""
    import os as _os

    import torch

    import flb_workloads as W
    from oracle import flb

    def mlups(name, min_steps, seconds):
        kw = W.params_of(name)
        po = flb.Params(**{k: v for k, v in kw.items() if k in flb.Params.__dataclass_fields__})
        drho = (W.initial_drho((po.nz, po.ny, po.nx), 7, W.WORKLOADS[name]["init_noise"])
                if po.force_model else None)
        S = flb.initial_state(po, drho)
        S = flb.step(S, 0, po)   # untimed first step (allocator warm-up)
        n = 0
        t0 = time.perf_counter()
        while n < min_steps or time.perf_counter() - t0 < seconds:
            n += 1
            S = flb.step(S, n, po)
        dt = time.perf_counter() - t0
        return V_of(po) * n / dt / 1e6, n, dt

    V_of = lambda po: po.nx * po.ny * po.nz
    all_threads = torch.get_num_threads()
    res = {}
    for threads in (all_threads, 1):
        torch.set_num_threads(threads)
        for name, mn, sec in (("d3q19_128", 1, 8.0 if threads > 1 else 0.0),
                              ("d2q9_32_fp64", 200, 0.0), ("d2q9_256_adjoint", 10, 0.0)):
            v, n, dt = mlups(name, mn, sec)
            res[f"{name}_{threads}thr"] = {"MLUPS": round(v, 4), "steps": n, "s": round(dt, 2)}
    torch.set_num_threads(all_threads)
    return {"value": res[f"d3q19_128_{all_threads}thr"]["MLUPS"], "unit": "MLUPS",
            "cores": all_threads, "kind": "oracle",
            "sample": "full-size d3q19_128 steps of the FP64 torch/numpy oracle, "
                      f"{res[f'd3q19_128_{all_threads}thr']['steps']} steps on {all_threads} threads "
                      f"(host has {_os.cpu_count()} CPUs); per-workload figures at all threads and at "
                      "one thread in 'workloads'",
            "workloads": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--profile-modeq", type=int, metavar="N",
                    help="only run the modified-equilibrium model on an N x N lattice (FP32, "
                         "the equilibration parameters), 64 steps after 32 warm-up steps")
    ap.add_argument("--inplace-probe", action="store_true",
                    help="only time a plain in-place elementwise pass over buffers of 32 MB to 1 GiB")
    ap.add_argument("--profile-step", choices=["fp32", "fp64"],
                    help="only run the d3q19_128 step (fixed launch shape, statistics on)")
    ap.add_argument("--profile-landau", action="store_true",
                    help="only run the d3q19_256_landau step (FP32, statistics every step) in "
                         "launch configuration 9 (z-marching 128 x 2 columns, 16 planes, forming "
                         "the next density), 6 steps")
    ap.add_argument("--profile-batch", action="store_true",
                    help="only run the d3q19_batch64 replicas (FP32, statistics every step), "
                         "in-place groups of up to 256 MiB, 4 steps")
    ap.add_argument("--profile-256", action="store_true",
                    help="only run the d3q19_128 step on 256^3 (FP32, statistics every step): "
                         "in-place pairs (128 x 2) and two buffers (128 x 2), 20 steps each")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(domain decomposition is design only).", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
    elif args.inplace_probe:
        inplace_probe()
    elif args.profile_modeq:
        profile_modeq(args.profile_modeq)
    elif args.profile_step:
        profile_step(args)
    elif args.profile_256:
        profile_256()
    elif args.profile_landau:
        profile_landau()
    elif args.profile_batch:
        profile_batch()
    else:
        bench_main(args)


def copy_probe():
    """A plain copy of 2^28 floats (1 GiB read, 1 GiB written), 5 times."""
    import torch
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": a.numel() * 4, "copy_probe_bytes_written": b.numel() * 4}))


def profile_modeq(n):
    """The modified-equilibrium model at n x n for per-kernel profiles."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import modeq as MQ
    pm = MQ.ModEqParams(**W.modeq_params_of("d2q9_128_modeq", nx=n, ny=n))
    sm = MQ.ModEq(pm)
    sm.step(32)
    torch.cuda.synchronize()
    sm.step(64)
    torch.cuda.synchronize()
    print(json.dumps({"profile_modeq": n, "steps": 96}))


def inplace_probe():
    """Read-and-write rate of a plain in-place pass (x *= 1) over one buffer,
    by buffer size: the ceiling a one-buffer in-place step can reach when its
    working set does or does not fit the last-level cache."""
    import torch
    out = {}
    for mb in (32, 64, 128, 159, 200, 256, 320, 512, 1024):
        n = mb * 2 ** 20 // 4
        a = torch.ones(n, device="cuda")
        for _ in range(30):
            a.mul_(1.0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(200):
            a.mul_(1.0)
        e1.record()
        e1.synchronize()
        out[f"{mb}MB"] = round(2 * n * 4 / (e0.elapsed_time(e1) / 200 * 1e-3) / 1e12, 3)
        del a
    print(json.dumps({"inplace_probe_TBps": out}))


def profile_step(args):
    """Every launch shape of the d3q19_128 step, with and without statistics,
    a few steps each (for per-kernel hardware counters)."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation
    p = Params.from_dict(dict(W.params_of("d3q19_128"), precision=args.profile_step))
    sim = Simulation(p)
    n, _ = sim.launch_configs()
    for cfg in range(n):
        sim.set_launch(cfg)
        sim.step(args.steps, stats_stride=1)
        sim.step(args.steps, stats_stride=0)
    torch.cuda.synchronize()
    print(json.dumps({"profile_step": args.profile_step, "configs": n, "steps_each": args.steps}))


def profile_landau():
    """The 256^3 square-gradient step for kernel counters: the z-marching force
    step that forms the next density (128 x 2 columns, non-temporal stores,
    launch configuration 9, the shape the benchmark's autotuner picks) with
    its completion pass; the first step of the call has a density pass."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation
    p = Params.from_dict(dict(W.params_of("d3q19_256_landau"), precision="fp32"))
    drho = W.initial_drho(p.shape, 7, W.WORKLOADS["d3q19_256_landau"]["init_noise"])
    sim = Simulation(p, drho_init=drho)
    sim.set_launch(9)
    sim.step(6, stats_stride=1)
    torch.cuda.synchronize()
    print(json.dumps({"profile_landau": 9, "steps": 6}))


def profile_batch():
    """The 64 uneven replicas in the grouped in-place schedule (groups of up
    to 256 MiB, default grid), for kernel counters."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Batch, Params
    wl = W.WORKLOADS["d3q19_batch64"]
    edges = W.batch_edges(wl["replicas"], wl["edges"], wl["size_seed"])
    pb = Params.from_dict(dict(lattice="D3Q19", precision="fp32", rho0=1.0, kT=wl["kT"],
                               rate_bulk=wl["rate_bulk"], rate_shear=wl["rate_shear"],
                               rate_ghost=wl["rate_ghost"]))
    b = Batch(pb, [(e, e, e) for e in edges], seeds=list(range(wl["replicas"])))
    b.set_pairs(256 << 20)
    b.step(4, stats_stride=1)
    torch.cuda.synchronize()
    print(json.dumps({"profile_batch": list(b.pairs()), "steps": 4}))


def profile_256():
    """The 256^3 ideal-gas step in its in-place pair and two-buffer shapes
    (launch configurations 10 and 1: 128 x 2 tiles), for kernel traces."""
    import torch

    import flb_workloads as W
    from paper_1012_3632_amd import Params, Simulation
    p = Params.from_dict(dict(W.params_of("d3q19_128", nx=256, ny=256, nz=256), precision="fp32"))
    sim = Simulation(p)
    for cfg in (10, 1):
        sim.set_launch(cfg)
        sim.step(20, stats_stride=1)
    torch.cuda.synchronize()
    print(json.dumps({"profile_256": [10, 1], "steps_each": 20}))


if __name__ == "__main__":
    main()
