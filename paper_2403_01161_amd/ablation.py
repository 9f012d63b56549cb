"""Regularisation ablation: the same droplet run with and without the mesh
smoothing of Sec. 3.3, tracking lambda_max / R^2 (Fig. 3(a)) and the mesh
quality that the smoothing exists to protect (the loosening and clustering
of elements shown in Fig. 3(b, c)): the smallest triangle angle and the
longest-to-shortest edge ratio. A run that ends in a domain or non-finite
error records the step at which it was detected.

Host code driving `ibmlb.Simulation`; the observables are computed on the
GPU (FP64 reductions)."""
from __future__ import annotations

import numpy as np

from . import ibmlb


def track(sim, A, nsteps: int, every: int, radius: float):
    """Advance `sim` by nsteps with the gradient A (row-major 9), reading the
    observables every `every` steps. Returns per-reading arrays (step,
    lmax_over_R2, D, volume, min_angle_deg, edge_ratio) and blowup_step (the
    first reading that failed, or None)."""
    rec = {k: [] for k in ("step", "lmax_over_R2", "D", "volume", "min_angle_deg", "edge_ratio")}
    blowup = None
    done = 0
    while done < nsteps:
        k = min(every, nsteps - done)
        try:
            sim.step(A, k)
            ob = sim.observables()
        except ibmlb.IbmLbError as e:
            if e.code not in (ibmlb.EDOMAIN, ibmlb.ENONFINITE):
                raise
            blowup = done + k
            break
        done += k
        rec["step"].append(done)
        rec["lmax_over_R2"].append(ob["eigval"][0] / (radius * radius))
        rec["D"].append(ob["D"])
        rec["volume"].append(ob["volume"])
        rec["min_angle_deg"].append(ob["min_angle_deg"])
        rec["edge_ratio"].append(ob["edge_max"] / ob["edge_min"])
    out = {k: np.asarray(v) for k, v in rec.items()}
    out["blowup_step"] = blowup
    return out


def regularisation_ablation(L, radius, vertices, triangles, tau, sigma, A, nsteps, every, storage="f32",
                            reg_iters=(50, 0), **kw):
    """The droplet under the constant gradient A, once per smoothing cap in
    `reg_iters` (0 switches the smoothing off). Returns {cap: track}."""
    out = {}
    for cap in reg_iters:
        sim = ibmlb.Simulation(L, tau, sigma=sigma, radius=radius, vertices=vertices, triangles=triangles,
                               A0=A, storage=storage, reg_max_iter=cap, **kw)
        try:
            out[cap] = track(sim, A, nsteps, every, radius)
        finally:
            sim.close()
    return out
