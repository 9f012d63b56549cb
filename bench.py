#!/usr/bin/env python3
"""Benchmark of the coupled IB-LB droplet timestep on one MI355X.

Headline workload (single droplet, FP32 populations): 256^3 box with moving
walls, tau = 0.8, droplet of rest radius 32 on a level-6 icosphere (40962
vertices, 81920 triangles), and a seeded traceless Ornstein-Uhlenbeck velocity
gradient A(t) (correlation time 2000 steps, rms capillary number 0.15 at
R/eta = 0.472). Its two population copies (2.55 GB) are far beyond the 256 MB
last-level cache. One step is the whole coupled update: forces, spreading,
fused collide-stream with the moving walls, interpolation + Euler, HC
smoothing.

Prints one JSON line: throughput in MLUPS (lattice node updates per second,
whole job; the median of five timed runs of --steps steps), the fused lattice
kernel's HBM roofline fraction (algorithmic 2 x 19 x s bytes per node update
over its HIP-event-timed average duration), the same box with FP64, FP16 and
BF16 population storage, the 128^3 single droplet, the 64-droplet ensemble
against the same droplets one at a time, the adjoint, and the FP64 CPU oracle
timed on bounded samples.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def workload(storage="f32"):
    from paper_2403_01161_amd.inputs import box_center, icosphere
    L = (128, 128, 128)
    R, level, tau = 16.0, 5, 0.8
    nu = (tau - 0.5) / 3.0
    G = (0.472 ** 2) * nu / R ** 2          # 1/tau_eta at R/eta = 0.472
    Ca = 0.1
    sigma = nu * R * G / Ca                 # mu = rho0 nu
    V, T = icosphere(level, R, box_center(L))
    return dict(L=L, R=R, tau=tau, G=G, Ca=Ca, sigma=sigma, V=V, T=T, storage=storage,
                corr=2000.0, seed=2)


def ensemble_workload(n=64, seed=3, level=4):
    """64 independent droplets: box sides drawn from {48, 64, 96}, R = L/8,
    level-4 icospheres (2562 vertices), tau = 1, rms Ca uniform in
    [0.05, 0.2] at R/eta = 0.472, own OU gradient table (seed 1000 + d)."""
    import numpy as np
    from paper_2403_01161_amd.inputs import box_center, icosphere
    rng = np.random.default_rng(seed)
    sides = rng.choice([48, 64, 96], size=n)
    cas = rng.uniform(0.05, 0.2, size=n)
    members, rms = [], []
    for d in range(n):
        L = int(sides[d])
        R, tau = L / 8.0, 1.0
        nu = (tau - 0.5) / 3.0
        G = (0.472 ** 2) * nu / R ** 2
        V, T = icosphere(level, R, box_center((L, L, L)))
        members.append(dict(L=(L, L, L), tau=tau, sigma=nu * R * G / cas[d], radius=R, vertices=V,
                            triangles=T))
        rms.append(G)
    return members, rms


def ensemble_bench(steps, warmup=20):
    import numpy as np
    import torch
    from paper_2403_01161_amd import ibmlb
    from paper_2403_01161_amd.inputs import ou_gradient_table
    members, rms = ensemble_workload()
    n = len(members)
    tabs = np.stack([ou_gradient_table(warmup + steps, 2000.0, rms[d], seed=1000 + d) for d in range(n)])
    for d in range(n):
        members[d]["A0"] = tabs[d, 0]
    nodes = sum(int(np.prod(m["L"])) for m in members)
    ens = ibmlb.Ensemble(members, storage="f32")
    variant = ens.autotune(5)
    ens.step(tabs[:, :warmup])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ens.step(tabs[:, warmup:])
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    obs = ens.observables()
    ens.close()
    del ens
    # the same droplets one at a time: each a one-member ensemble, so the solo
    # runs use the same batched kernels and the same captured graph replays
    solos = []
    for d in range(n):
        e = ibmlb.Ensemble([members[d]], storage="f32")
        e.autotune(3)
        e.step(tabs[d:d + 1, :warmup])
        solos.append(e)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in range(n):
        solos[d].step(tabs[d:d + 1, warmup:])
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    for e in solos:
        e.close()
    return {"workload": "64 droplets, boxes drawn from {48,64,96}^3, R = L/8, 2562-vertex icospheres, "
                        "tau 1, OU A(t) per droplet, rms Ca U(0.05, 0.2), f32",
            "droplets": n, "nodes": nodes, "vertices": sum(len(m["vertices"]) for m in members),
            "steps": steps, "batched_mlups": round(nodes * steps / t_batch / 1e6, 1),
            "solo_mlups": round(nodes * steps / t_solo / 1e6, 1),
            "solo": "each droplet as a one-member ensemble, one after another (same kernels, same graphs)",
            "batched_over_solo": round(t_solo / t_batch, 3),
            "batched_ms_per_step": round(t_batch / steps * 1e3, 4),
            "batched_hbm_frac": round(152 * nodes * steps / t_batch / 1e9 / HBM_PEAK_GBS, 4),
            "lattice_variant": variant,
            "max_D": round(max(o["D"] for o in obs), 5)}


def describe_variant(v):
    """Step-variant bits as named fields (see ibm_lb_set_variant)."""
    rows = bool(v & 16)
    d = {"layout": "rows" if rows else "linear", "nontemporal_loads": bool(v & 1),
         "block": (128, 256, 512, 64)[(v >> 1) & 3]}
    if rows:
        d["nontemporal_stores"] = bool(v & 8)
    else:
        d["xcd_grouped_order"] = bool(v & 8)
    d["smoothing_finish_in_force_kernel"] = bool(v & 32)
    d["in_place_streaming"] = bool(v & 64)
    return d


def lattice_kernel_name(v, chi=1.0, collision="bgk"):
    if collision == "mrt":
        return "k_lattice_rows<..., MRT>" if v & 16 else "k_lattice_mrt"
    if chi != 1.0:
        return "k_lattice_rows<..., CHI>" if v & 16 else "k_lattice_chi"
    if v & 64:
        return "k_lattice_aa"
    return "k_lattice_rows" if v & 16 else "k_lattice"


STORAGE_BYTES = {"f64": 8, "f32": 4, "f16dev": 2, "bf16dev": 2}
DTYPE = {"f64": "f64", "f32": "f32", "f16dev": "f16", "bf16dev": "bf16"}


def droplet_leg(dev, w, storage, K, W, reps=5, variant=None, chi=1.0, collision="bgk", walls="link",
                deterministic=False, box="256cubed"):
    """One droplet workload `w` with `storage` populations: W warm-up steps,
    then `reps` timed runs of K whole steps (hipStream synchronised around
    each; the median is reported), then K more steps with HIP events stamped
    by every lattice dispatch for the lattice kernel's average duration."""
    import numpy as np
    import torch
    from paper_2403_01161_amd import ibmlb
    from paper_2403_01161_amd.inputs import ou_gradient_table
    table = ou_gradient_table(W + (reps + 1) * K + 1, w["corr"], w["G"], seed=w["seed"])
    sim = ibmlb.Simulation(w["L"], w["tau"], w["sigma"], w["R"], w["V"], w["T"], storage=storage,
                           A0=table[0], device=dev, chi=chi, collision=collision, walls=walls,
                           deterministic=deterministic)
    dtab = torch.from_numpy(table).to(dev)
    nodes = int(np.prod(w["L"]))
    nv = len(w["V"])
    if variant is None:
        variant = sim.autotune(5)
    else:
        sim.set_variant(variant)
    sim.step_table(dtab[:W])
    obs0 = sim.observables()  # synchronises
    times = []
    for r in range(reps):
        t0 = time.perf_counter()
        sim.step_table(dtab[W + r * K:W + (r + 1) * K])
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[reps // 2]
    sim.timing(True)
    t1 = time.perf_counter()
    sim.step_table(dtab[W + reps * K:W + (reps + 1) * K])
    torch.cuda.synchronize()
    dt_ev = time.perf_counter() - t1
    lat_ms, launches = sim.timing_read()
    sim.timing(False)
    obs = sim.observables()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    alg = 2 * 19 * STORAGE_BYTES[storage] * nodes
    avg_s = lat_ms / 1e3 / max(launches, 1)
    ach = alg / avg_s / 1e9
    plain = chi == 1.0 and collision == "bgk" and walls == "link"
    return {"mlups": round(nodes * K / dt / 1e6, 2), "ms_per_step": round(dt / K * 1e3, 5),
            "rep_ms_per_step": [round(t / K * 1e3, 5) for t in times],
            "ms_per_step_with_kernel_events": round(dt_ev / K * 1e3, 5),
            "vertex_updates_per_s": round(nv * K / dt, 1),
            "hbm_frac_whole_step": round(alg * K / dt / 1e9 / HBM_PEAK_GBS, 4),
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4),
                         "traffic": counter_traffic(storage, box, variant) if plain else None,
                         "kernel": lattice_kernel_name(variant, chi, collision), "alg_bytes_per_launch": alg,
                         "avg_launch_us": round(avg_s * 1e6, 3), "launches": launches,
                         "variant": describe_variant(variant)},
            "observables": {"step": obs["step"], "D": obs["D"], "theta_deg": obs["theta_deg"],
                            "beta": obs["beta"], "reg_iters": obs["reg_iters"],
                            "mass_drift_rel": (obs["mass"] - obs0["mass"]) / obs0["mass"]}}


def workload_name(w, storage, chi=1.0, collision="bgk", walls="link", deterministic=False):
    L = w["L"][0]
    return (f"single droplet, {L}^3 moving-wall box, tau {w['tau']:g}, R {w['R']:g}, {len(w['V'])}-vertex "
            f"icosphere, OU traceless A(t) rms Ca {w['Ca']:g}, {storage} populations"
            + (f", viscosity ratio {chi:g}" if chi != 1.0 else "")
            + (", MRT collision" if collision == "mrt" else "")
            + (", wet-node walls" if walls == "wet" else "")
            + (", deterministic spreading" if deterministic else ""))


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("kernels.hip", "lattice_kernels.h", "lattice_common.h", "device_common.h"):
        with open(os.path.join(ROOT, "paper_2403_01161_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def counter_traffic(storage, box="128cubed", variant=None):
    """HBM bytes per lattice launch from a committed rocprofv3 counter summary
    (profiles/lattice_{storage}_{box}[_v{variant}]_counters.md), valid only
    while the kernel source is the one profiled and the lattice kernel variant
    (bits 0-4 and 6 of the step variant) is the profiled one."""
    prof = os.path.join(ROOT, "profiles")
    if not os.path.isdir(prof):
        return None
    for fn in sorted(os.listdir(prof)):
        if not (fn.startswith(f"lattice_{storage}_{box}") and fn.endswith("_counters.md")) or "diagnostic" in fn:
            continue
        txt = open(os.path.join(prof, fn)).read()
        m = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]{16})", txt)
        t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
        v = re.search(r"lattice_variant:\s*([0-9]+)", txt)
        if not m or not t or not v or m.group(1) != kernel_source_hash():
            continue
        if variant is not None and int(v.group(1)) != (variant & 95):
            continue
        return float(t.group(1))
    return None


def _oracle_rate(w, steps, warm=2, seed=None, threads=None):
    """FP64 oracle MLUPS on workload w: `warm` untimed steps, then `steps`
    timed steps (its own OU table, or w["A"] when given)."""
    import numpy as np
    import oracle
    from paper_2403_01161_amd.inputs import ou_gradient_table
    if "A" in w:
        table = np.asarray(w["A"])[:1 + warm + steps]
    else:
        table = ou_gradient_table(1 + warm + steps, w["corr"], w["G"], seed=w["seed"] if seed is None else seed)
    ref = oracle.Oracle(w["L"], w["tau"], sigma=w["sigma"], radius=w["R"], vertices=w["V"], triangles=w["T"],
                        A0=table[0])
    ref.step_table(table[1:1 + warm])
    t0 = time.perf_counter()
    ref.step_table(table[1 + warm:1 + warm + steps])
    dt = time.perf_counter() - t0
    ref.close()
    return int(np.prod(w["L"])) * steps / dt / 1e6, dt


def cpu_baseline(w, steps=20, single_steps=3, per_config=True):
    """The FP64 oracle on this host's cores (its lattice sweeps use OpenMP over
    z-planes, the IB part is serial) on a bounded sample of the headline
    workload, then on one thread for a shorter sample; then the other
    configurations: the plain-method run in full (32^3, 1000 steps) and
    20 timed steps of the others, whose full-run times are extrapolated."""
    import ctypes
    import numpy as np
    from paper_2403_01161_amd.inputs import box_center, icosphere, ou_gradient_table, simple_shear
    gomp = ctypes.CDLL("libgomp.so.1")  # the OpenMP runtime the oracle library uses
    cores = int(gomp.omp_get_max_threads())
    value, dt = _oracle_rate(w, steps)
    gomp.omp_set_num_threads(1)
    try:
        single, dt1 = _oracle_rate(w, single_steps, warm=0, seed=w["seed"] + 1)
    finally:
        gomp.omp_set_num_threads(cores)
    nodes = int(np.prod(w["L"]))
    out = {"value": round(value, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
           "sample": f"FP64 oracle, the headline {w['L'][0]}^3 workload: {steps} steps after 2 warm-up steps "
                     f"({dt:.1f} s) on {cores} threads (OpenMP over z-planes for the lattice, serial IB); "
                     f"then {single_steps} steps from a fresh start on 1 thread ({dt1:.1f} s)",
           "single_thread_value": round(single, 3)}
    if not per_config:
        return out
    pc = {}
    # plain method: 32^3, tau 1, R 5 (642 vertices), simple shear Ca 0.05, 1000 steps, in full
    from oracle import Oracle
    g = 1e-3
    V, T = icosphere(3, 5.0, box_center((32, 32, 32)))
    ref = Oracle((32, 32, 32), 1.0, sigma=(1 / 6) * g * 5.0 / 0.05, radius=5.0, vertices=V, triangles=T,
                 A0=simple_shear(g))
    t0 = time.perf_counter()
    ref.step(simple_shear(g), 1000)
    t1k = time.perf_counter() - t0
    D = ref.observables()["D"]
    ref.close()
    pc["plain_32cubed_1000_steps"] = {"mlups": round(32 ** 3 * 1000 / t1k / 1e6, 3), "seconds": round(t1k, 2),
                                      "D": D, "measured": "full run"}
    w2 = workload("f32")
    m2, _ = _oracle_rate(w2, 20)
    pc["single_128cubed_20000_steps"] = {"mlups": round(m2, 3), "measured": "20 steps after 2 warm-up",
                                        "full_run_seconds_extrapolated": round(128 ** 3 * 20000 / m2 / 1e6, 0)}
    pc["precision_256cubed_5000_steps"] = {"mlups": round(value, 3), "measured": f"{steps} steps (above)",
                                          "full_run_seconds_extrapolated": round(nodes * 5000 / value / 1e6, 0)}
    members, rms = ensemble_workload()
    t_ens, n_ens = 0.0, 0
    for d, m in enumerate(members):
        wd = dict(L=m["L"], tau=m["tau"], sigma=m["sigma"], R=m["radius"], V=m["vertices"], T=m["triangles"],
                  corr=2000.0, G=rms[d], seed=1000 + d)
        _, dtd = _oracle_rate(wd, 20)
        t_ens += dtd
        n_ens += int(np.prod(m["L"])) * 20
    pc["ensemble_64_droplets_10000_steps"] = {
        "mlups": round(n_ens / t_ens / 1e6, 3), "measured": "20 steps of each droplet after 2 warm-up",
        "full_run_seconds_extrapolated": round(n_ens / 20 * 10000 / (n_ens / t_ens), 0)}
    wa = adjoint_workload()
    ma, _ = _oracle_rate(dict(wa, corr=0, G=0, seed=0), 20)
    pc["adjoint_64cubed_500_steps_forward"] = {"mlups": round(ma, 3), "measured": "20 steps after 2 warm-up",
                                               "full_run_seconds_extrapolated": round(64 ** 3 * 500 / ma / 1e6, 1)}
    out["per_config"] = pc
    return out


def adjoint_workload():
    """64^3 box, tau 1, R 8 on a level-4 icosphere (2562 vertices); simple shear
    at Ca 0.1 (gamma 5.8e-4, sigma = mu R gamma / Ca) plus a seeded OU
    perturbation of rms 0.1 gamma and correlation time 100 steps (seed 5);
    500 steps, checkpoints every 50."""
    from paper_2403_01161_amd.inputs import box_center, icosphere, ou_gradient_table
    L = (64, 64, 64)
    R, tau, gamma, Ca = 8.0, 1.0, 5.80e-4, 0.1
    nu = (tau - 0.5) / 3.0
    V, T = icosphere(4, R, box_center(L))
    A = ou_gradient_table(500, 100.0, 0.1 * gamma, seed=5)
    A[:, 1] += gamma
    return dict(L=L, R=R, tau=tau, sigma=nu * R * gamma / Ca, V=V, T=T, A=A, K=50)


def adjoint_bench(dev):
    """Forward (with a checkpoint every K steps) and backward (recompute + adjoint
    sweep of every segment) of J = D(r^T), timed separately after one untimed
    pass; FP32 populations. The FP64-forward gradient is reported beside it."""
    import numpy as np
    import torch
    from paper_2403_01161_amd import ibmlb
    w = adjoint_workload()
    A = torch.from_numpy(w["A"]).to(dev)
    n, K = A.shape[0], w["K"]

    def run(storage, timed):
        sim = ibmlb.Simulation(w["L"], w["tau"], w["sigma"], w["R"], w["V"], w["T"], storage=storage,
                               A0=w["A"][0], device=dev)
        sim.autotune(5)
        ck = [torch.empty(sim.state_bytes(), dtype=torch.uint8, device=dev) for _ in range(0, n, K)]
        fbuf = torch.empty(19 * sim.N, dtype=torch.float64, device=dev)
        rnext = torch.empty((sim.nv, 3), dtype=torch.float64, device=dev)
        dA = torch.empty((n, 9), dtype=torch.float64, device=dev)
        dsig = torch.zeros(1, dtype=torch.float64, device=dev)
        times = []
        for rep in range(2 if timed else 1):
            st0 = sim.save()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i, s0 in enumerate(range(0, n, K)):
                sim.save(ck[i])
                sim.step_table(A[s0:s0 + K])
            D, rbar = sim.objective_grad()
            t1 = time.perf_counter()
            dsig.zero_()
            fbar = None
            for i in reversed(range(len(ck))):
                s0 = i * K
                sim.adjoint_segment(ck[i], A[s0:s0 + K], fbar, rbar, fbuf, rnext, dA[s0:s0 + K], dsig)
                fbar = fbuf
                rbar, rnext = rnext, rbar
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times.append((t1 - t0, t2 - t1))
            sim.load(st0)
        out = (D, float(dsig[0]), dA.cpu().numpy(), times[-1])
        sim.close()
        return out

    D32, s32, a32, (tf, tb) = run("f32", True)
    D64, s64, a64, _ = run("f64", False)
    return {"workload": "64^3 box, tau 1, R 8, 2562-vertex icosphere, shear Ca 0.1 + OU perturbation, "
                        "500 steps, checkpoints every 50, f32 populations, FP64 adjoint",
            "objective": "D(r^T)", "D": round(D32, 8), "forward_ms": round(tf * 1e3, 2),
            "backward_ms": round(tb * 1e3, 2), "backward_over_forward": round(tb / tf, 3),
            "dD_dsigma": s32, "f32_vs_f64_forward": {
                "dD_dsigma_rel": abs(s32 - s64) / abs(s64),
                "dD_dA_rel": float(np.linalg.norm(a32 - a64) / np.linalg.norm(a64))}}


def precision_workload():
    """256^3 box, tau 0.8, R 32 on a level-6 icosphere (40962 vertices), OU
    traceless A(t) with rms Ca 0.15 at R/eta = 0.472, correlation 2000 steps,
    seed 4."""
    from paper_2403_01161_amd.inputs import box_center, icosphere
    L = (256, 256, 256)
    R, tau, Ca = 32.0, 0.8, 0.15
    nu = (tau - 0.5) / 3.0
    G = (0.472 ** 2) * nu / R ** 2
    V, T = icosphere(6, R, box_center(L))
    return dict(L=L, R=R, tau=tau, G=G, Ca=Ca, sigma=nu * R * G / Ca, V=V, T=T, corr=2000.0, seed=4)


def precision_bench(dev, steps, every=500):
    """Every population storage format on the same 256^3 run: throughput, the
    lattice kernel's roofline fraction, D and theta along the run and the
    final velocity field, each against the FP64-storage run."""
    import numpy as np
    import torch
    from paper_2403_01161_amd import ibmlb
    from paper_2403_01161_amd.inputs import ou_gradient_table
    w = precision_workload()
    table = ou_gradient_table(steps, w["corr"], w["G"], seed=w["seed"])
    dtab = torch.from_numpy(table).to(dev)
    nodes = int(np.prod(w["L"]))
    res, ref = {}, None
    for storage, sb in (("f64", 8), ("f32", 4), ("f16dev", 2), ("bf16dev", 2)):
        sim = ibmlb.Simulation(w["L"], w["tau"], w["sigma"], w["R"], w["V"], w["T"], storage=storage,
                               A0=table[0], device=dev)
        variant = sim.autotune(10)
        sim.timing(True)
        Ds, th = [], []
        mass0 = sim.observables()["mass"]
        torch.cuda.synchronize()
        t_run = 0.0
        for s0 in range(0, steps, every):
            t0 = time.perf_counter()
            sim.step_table(dtab[s0:s0 + every])
            torch.cuda.synchronize()
            t_run += time.perf_counter() - t0
            o = sim.observables()
            Ds.append(o["D"])
            th.append(o["theta_deg"])
        mass_drift = (o["mass"] - mass0) / mass0
        lat_ms, launches = sim.timing_read()
        _, u = sim.fields()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        r = {"mlups": round(nodes * steps / t_run / 1e6, 1),
             "lattice_frac": round(2 * 19 * sb * nodes / (lat_ms / 1e3 / launches) / 1e9 / HBM_PEAK_GBS, 4),
             "lattice_variant": variant, "D_final": Ds[-1], "theta_final_deg": th[-1],
             "mass_rel_drift": mass_drift}
        if ref is None:
            ref = (np.array(Ds), np.array(th), u)
        else:
            Dr, thr, ur = ref
            r["D_rel_err_max"] = float(np.max(np.abs(np.array(Ds) - Dr) / np.abs(Dr)))
            r["theta_err_max_deg"] = float(np.max(np.abs(np.array(th) - thr)))
            r["u_err_rel"] = float(np.abs(u - ur).max() / np.abs(ur).max())
        res[storage] = r
        print(json.dumps({"precision_format_done": storage, **r}), flush=True)
    return {"workload": "256^3 moving-wall box, tau 0.8, R 32, 40962-vertex icosphere, OU A(t) rms Ca 0.15",
            "steps": steps, "sample_every": every, "formats": res}


def counters_sequence(dev, storage, box="128", fixed_variant=None):
    """Kernels whose HBM counters are read: a plain 256 MiB copy whose source
    was first pushed out of the 256 MB last-level cache by a 1 GiB fill (three
    times; the known 256 MiB read + 256 MiB write calibrate the counters), and
    20 steps of the single-droplet workload (128^3, or the 256^3 droplet) after
    5 warm-up steps."""
    import torch
    from paper_2403_01161_amd import ibmlb
    from paper_2403_01161_amd.inputs import ou_gradient_table
    src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    flush = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device=dev)
    for _ in range(3):
        flush.fill_(1.0)
        dst.copy_(src)
    torch.cuda.synchronize()
    del flush
    w = workload(storage) if box == "128" else dict(precision_workload(), storage=storage)
    table = ou_gradient_table(26, w["corr"], w["G"], seed=w["seed"])
    sim = ibmlb.Simulation(w["L"], w["tau"], w["sigma"], w["R"], w["V"], w["T"], storage=w["storage"],
                           A0=table[0], device=dev)
    variant = sim.autotune(5) if fixed_variant is None else fixed_variant
    sim.set_variant(variant)
    sim.step_table(table[:5])
    sim.step_table(table[5:25])
    torch.cuda.synchronize()
    print(json.dumps({"counters_sequence": "done", "storage": storage, "box": box, "variant": variant,
                      "kernel": lattice_kernel_name(variant)}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000, help="steps per timed run (five runs; median)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--box", default="256", choices=["256", "128"],
                    help="single-droplet workload of the headline leg: 256^3 (R 32) or 128^3 (R 16)")
    ap.add_argument("--storage", default="f32", choices=["f32", "f64", "f16dev", "bf16dev"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-formats", action="store_true", help="skip the other storage formats of the box")
    ap.add_argument("--no-extras", action="store_true",
                    help="headline leg only (no other formats, 128^3 leg, ensemble, adjoint or CPU baseline)")
    ap.add_argument("--ensemble-steps", type=int, default=300)
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--precision", type=int, default=0, metavar="STEPS",
                    help="run only the storage-precision study (256^3, every format) for STEPS steps")
    ap.add_argument("--variant", type=int, default=None,
                    help="run this step variant instead of the autotuner's choice (the headline leg "
                         "and --counters)")
    ap.add_argument("--chi", type=float, default=1.0,
                    help="viscosity ratio of the droplet for the headline leg (1: one fluid)")
    ap.add_argument("--collision", default="bgk", choices=["bgk", "mrt"],
                    help="collision of the headline leg (MRT: default rates)")
    ap.add_argument("--walls", default="link", choices=["link", "wet"],
                    help="wall rule of the headline leg (wet: the wet-node velocity walls)")
    ap.add_argument("--deterministic", action="store_true",
                    help="headline leg with the deterministic (fixed-order gather) spreading")
    ap.add_argument("--counters", nargs="?", const="128", choices=["128", "256"], default=None,
                    help="short fixed sequence for hardware-counter runs: 3 device copies of "
                         "256 MiB (calibration) and 20 steps of the single-droplet workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the ensemble and a "
                                   "z-slab split are the multi-GPU designs (not run here)"}))
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    if args.counters:
        counters_sequence(dev, args.storage, args.counters, args.variant)
        return
    if args.precision:
        print(json.dumps({"precision": precision_bench(dev, args.precision)}), flush=True)
        return
    K, W = args.steps, args.warmup
    variant_kw = dict(chi=args.chi, collision=args.collision, walls=args.walls, deterministic=args.deterministic)
    w = precision_workload() if args.box == "256" else workload(args.storage)
    box = f"{args.box}cubed"
    head = droplet_leg(dev, w, args.storage, K, W, variant=args.variant, box=box, **variant_kw)
    print(json.dumps({"leg_done": "headline", "mlups": head["mlups"], "frac": head["roofline"]["frac"]}),
          file=sys.stderr, flush=True)
    line = {
        "metric": "IB-LB MLUPS",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.storage],
        "data": "synthetic",
        "config": {"workload": workload_name(w, args.storage, **variant_kw), "box": list(w["L"]),
                   "vertices": len(w["V"]), "storage": args.storage, "chi": args.chi,
                   "collision": args.collision, "walls": args.walls, "deterministic": args.deterministic,
                   "timing": "median of 5 timed runs of `steps` steps"},
        "roofline": head["roofline"],
    }
    for k in ("rep_ms_per_step", "ms_per_step_with_kernel_events", "vertex_updates_per_s",
              "hbm_frac_whole_step", "observables"):
        line[k] = head[k]
    extras = not args.no_extras
    plain = args.chi == 1.0 and args.collision == "bgk" and args.walls == "link" and not args.deterministic
    if extras and not args.no_formats and plain:
        fm = {}
        for st in ("f64", "f32", "f16dev", "bf16dev"):
            if st == args.storage:
                continue
            leg = droplet_leg(dev, w, st, K, W, box=box)
            fm[st] = {"workload": workload_name(w, st), **{k: leg[k] for k in (
                "mlups", "ms_per_step", "rep_ms_per_step", "hbm_frac_whole_step", "roofline", "observables")}}
            print(json.dumps({"leg_done": st, "mlups": leg["mlups"], "frac": leg["roofline"]["frac"]}),
                  file=sys.stderr, flush=True)
        line["storage_formats"] = fm
    if extras and args.box == "256" and plain:
        w2 = workload("f32")
        leg = droplet_leg(dev, w2, "f32", K, W, box="128cubed")
        line["single_droplet_128cubed"] = {"workload": workload_name(w2, "f32"), **leg}
        print(json.dumps({"leg_done": "128cubed", "mlups": leg["mlups"]}), file=sys.stderr, flush=True)
    if extras and args.ensemble_steps > 0:
        line["ensemble"] = ensemble_bench(args.ensemble_steps)
        print(json.dumps({"leg_done": "ensemble"}), file=sys.stderr, flush=True)
    if extras and not args.no_adjoint:
        line["adjoint"] = adjoint_bench(dev)
        print(json.dumps({"leg_done": "adjoint"}), file=sys.stderr, flush=True)
    if extras and not args.no_cpu and args.chi == 1.0 and args.box == "256":
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
