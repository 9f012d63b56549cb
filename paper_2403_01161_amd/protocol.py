"""The paper's protocol for sub-Kolmogorov droplets driven by turbulent
velocity gradients, and the linear theory it is validated against.

Unit matching (Sec. "Outer Flow and matching between DNSU and LBU"):
lengths scale by C_x = R / R_lbu (Eq. eq:cl), times by
C_t = C_x^2 nu_lbu / nu (Eq. eq:ct). A gradient frame of the DNS becomes
C_t grad(u) in lattice units (Eq. eq:strain_conversion) and is held for
N = dt / C_t lattice steps, which scales as (eta / R)^2 (Eq. eq:N_Reta). The
capillary time tau_sigma = Ca tau_eta (Eq. capillary) becomes tau_sigma / C_t
steps, and the surface tension sigma_lbu = mu_lbu R_lbu / tau_sigma_lbu
(Eq. surfacetensionconversion).

Linear theory (Eq. eq:LT): for a viscosity ratio chi,
    dS/dt = -(1 / tau_sigma) k(chi) (S - R^2 I) + 2 R^2 d(chi) E(t),
    k(chi) = 40 (chi + 1) / ((2 chi + 3)(19 chi + 16)),  d(chi) = 5 / (2 chi + 3),
with E the symmetric part of the gradient. The gradient is held constant for
N steps per frame, so each frame has the closed-form propagator used here.

Everything in this module runs on the host: the matching is arithmetic on a
few scalars, and the linear theory is a 3x3 ODE; the droplet itself runs in
the HIP library through `ibmlb.Simulation` / `ibmlb.Ensemble`.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class DnsScales:
    """Scales of the turbulent flow in DNS units (the values of the paper's
    database: Kolmogorov length and time, viscosity, frame spacing)."""
    eta: float = 4.2e-3
    tau_eta: float = 2.3e-2
    nu: float = 8e-4
    dt: float = 2.25e-3


@dataclasses.dataclass(frozen=True)
class Matching:
    """DNS-to-lattice matching of one (R / eta, Ca) point."""
    R_over_eta: float
    Ca: float
    R_lbu: float
    tau_f: float
    rho0: float
    C_x: float            # DNS length per lattice length
    C_t: float            # DNS time per lattice step
    steps_per_frame: float  # dt / C_t before rounding
    N: int                # lattice steps each frame is held for (>= 1)
    nu_lbu: float
    tau_sigma_lbu: float  # capillary time in lattice steps
    sigma_lbu: float

    def gradient_lbu(self, grad_dnsu):
        """Eq. eq:strain_conversion: C_t grad(u), row-major [..., 9]."""
        return self.C_t * np.asarray(grad_dnsu, dtype=np.float64)


def match_units(R_over_eta: float, Ca: float, R_lbu: float, tau_f: float, rho0: float = 1.0,
                scales: DnsScales = DnsScales()) -> Matching:
    """Lattice parameters of a droplet of radius R = (R / eta) eta and
    capillary number Ca, resolved with radius R_lbu at relaxation time tau_f."""
    if not (R_over_eta > 0 and Ca > 0 and R_lbu > 0 and tau_f > 0.5):
        raise ValueError("need R/eta > 0, Ca > 0, R_lbu > 0 and tau_f > 1/2")
    nu_lbu = (tau_f - 0.5) / 3.0
    C_x = R_over_eta * scales.eta / R_lbu
    C_t = C_x * C_x * nu_lbu / scales.nu
    spf = scales.dt / C_t
    tau_sigma_lbu = Ca * scales.tau_eta / C_t
    sigma_lbu = rho0 * nu_lbu * R_lbu / tau_sigma_lbu
    return Matching(R_over_eta, Ca, R_lbu, tau_f, rho0, C_x, C_t, spf, max(1, int(round(spf))), nu_lbu,
                    tau_sigma_lbu, sigma_lbu)


def lt_coefficients(chi: float = 1.0):
    """(k, d) of Eq. eq:LT: relaxation and strain coefficients."""
    return 40.0 * (chi + 1.0) / ((2.0 * chi + 3.0) * (19.0 * chi + 16.0)), 5.0 / (2.0 * chi + 3.0)


def lt_propagate(S, A, h, R, tau_sigma, chi=1.0):
    """S after h time units of Eq. eq:LT with the gradient A (row-major 9,
    held constant): S(h) = R^2 I + e^{-a h}(S - R^2 I) + (1 - e^{-a h}) 2 R^2 d E / a,
    a = k / tau_sigma."""
    k, d = lt_coefficients(chi)
    a = k / tau_sigma
    G = np.asarray(A, dtype=np.float64).reshape(3, 3)
    E = 0.5 * (G + G.T)
    I = np.eye(3)
    e = math.exp(-a * h)
    return R * R * I + e * (np.asarray(S) - R * R * I) + (1.0 - e) * (2.0 * R * R * d / a) * E


def lt_integrate(A_frames, N, R, tau_sigma, chi=1.0, S0=None):
    """S at the end of every frame: frame f holds the gradient A_frames[f]
    (lattice units, row-major) for N steps. S0 defaults to the sphere R^2 I.
    Returns [F, 3, 3]."""
    A_frames = np.asarray(A_frames, dtype=np.float64).reshape(-1, 9)
    S = R * R * np.eye(3) if S0 is None else np.array(S0, dtype=np.float64).reshape(3, 3)
    out = np.empty((len(A_frames), 3, 3))
    for f, A in enumerate(A_frames):
        S = lt_propagate(S, A, float(N), R, tau_sigma, chi)
        out[f] = S
    return out


def descriptors(S, A):
    """Deformation D = (sqrt(l1) - sqrt(l3)) / (sqrt(l1) + sqrt(l3)), the
    orientation beta = v1.E.v1 / |E|_F (Eq. beta) and theta = atan2(v1_y, v1_x)
    folded into (-90, 90] degrees, for morphological tensors S [..., 3, 3] and
    gradients A [..., 9] (beta is 0 where E vanishes)."""
    S = np.asarray(S, dtype=np.float64).reshape(-1, 3, 3)
    G = np.asarray(A, dtype=np.float64).reshape(-1, 3, 3)
    lam, vec = np.linalg.eigh(0.5 * (S + np.swapaxes(S, 1, 2)))
    l1, l3 = lam[:, 2], lam[:, 0]
    v = vec[:, :, 2]
    with np.errstate(invalid="ignore"):  # NaN where S is not positive (the theory beyond its range)
        D = (np.sqrt(l1) - np.sqrt(l3)) / (np.sqrt(l1) + np.sqrt(l3))
    E = 0.5 * (G + np.swapaxes(G, 1, 2))
    nE = np.sqrt((E * E).sum(axis=(1, 2)))
    vEv = np.einsum("ni,nij,nj->n", v, E, v)
    beta = np.where(nE > 0, vEv / np.where(nE > 0, nE, 1.0), 0.0)
    th = np.degrees(np.arctan2(v[:, 1], v[:, 0]))
    th = np.where(th > 90.0, th - 180.0, np.where(th <= -90.0, th + 180.0, th))
    return D, beta, th


def run(sim, frames_dnsu, m: Matching):
    """Drive a droplet through DNS gradient frames (DNS units, [F, 9]): each
    frame converted and held for m.N steps (the protocol's steps 1-4), with
    the droplet's observables read after every frame. Returns a dict of
    per-frame arrays (D, beta, theta, S [F, 3, 3], A_lbu [F, 9])."""
    A = m.gradient_lbu(np.asarray(frames_dnsu, dtype=np.float64).reshape(-1, 9))
    F = len(A)
    out = {k: np.empty(F) for k in ("D", "beta", "theta")}
    out["S"] = np.empty((F, 3, 3))
    for f in range(F):
        sim.step(A[f], m.N)
        ob = sim.observables()
        out["D"][f], out["beta"][f], out["theta"][f] = ob["D"], ob["beta"], ob["theta_deg"]
        out["S"][f] = np.asarray(ob["S"]).reshape(3, 3)
    out["A_lbu"] = A
    return out


def run_ensemble(ens, frames_dnsu, m: Matching, stop_on_error: bool = False):
    """As `run` for an ensemble whose members share the matching, member i
    following trajectory frames_dnsu[i] ([n, F, 9]). Returns per-frame arrays
    [n, F] (D, beta, theta). With stop_on_error, a domain or non-finite error
    (a droplet reaching a wall, an unstable lattice) ends the run instead of
    raising: the arrays then hold the frames before it and "failed_at" the
    frame whose read failed."""
    from . import ibmlb
    A = m.gradient_lbu(np.asarray(frames_dnsu, dtype=np.float64))
    n, F = A.shape[0], A.shape[1]
    out = {k: np.empty((n, F)) for k in ("D", "beta", "theta")}
    out["failed_at"] = None
    for f in range(F):
        try:
            ens.step(np.repeat(A[:, f:f + 1, :], m.N, axis=1))
            obs = ens.observables()
        except ibmlb.IbmLbError as e:
            if not stop_on_error or e.code not in (ibmlb.EDOMAIN, ibmlb.ENONFINITE):
                raise
            out["failed_at"] = f
            for k in ("D", "beta", "theta"):
                out[k] = out[k][:, :f]
            A = A[:, :f]
            break
        for i, ob in enumerate(obs):
            out["D"][i, f], out["beta"][i, f], out["theta"][i, f] = ob["D"], ob["beta"], ob["theta_deg"]
    out["A_lbu"] = A
    return out


def compare_with_theory(m: Matching, res, skip: int = 5, chi: float = 1.0):
    """Frame-by-frame agreement of driven droplets with the linear theory
    for the viscosity ratio chi.
    res holds per-frame D, beta, theta and A_lbu, either [F] (one droplet) or
    [n, F] (an ensemble). Returns the mean of D / D_LT, the correlation of D
    with D_LT and of beta with beta_LT, and the mean |theta - theta_LT|
    (degrees, folded to [0, 90]) over every droplet's frames after `skip`
    where the theory's S stays positive (at large Ca the linear theory drives
    an eigenvalue of S negative); lt_valid_frac is the share of such frames."""
    D, beta, theta = (np.atleast_2d(res[k]) for k in ("D", "beta", "theta"))
    A = np.asarray(res["A_lbu"]).reshape(D.shape[0], D.shape[1], 9)
    out = {"D_over_D_lt": [], "corr_D": [], "corr_beta": [], "theta_err_deg": [], "lt_valid_frac": []}
    for i in range(D.shape[0]):
        S = lt_integrate(A[i], m.N, m.R_lbu, m.tau_sigma_lbu, chi=chi)
        Dl, bl, tl = descriptors(S, A[i])
        ok = np.isfinite(Dl)
        ok[:skip] = False
        out["lt_valid_frac"].append(ok[skip:].mean())
        if ok.sum() < 3:
            continue
        out["D_over_D_lt"].append(D[i, ok].mean() / Dl[ok].mean())
        out["corr_D"].append(np.corrcoef(D[i, ok], Dl[ok])[0, 1])
        out["corr_beta"].append(np.corrcoef(beta[i, ok], bl[ok])[0, 1])
        dt = np.abs(theta[i, ok] - tl[ok]) % 180.0
        out["theta_err_deg"].append(np.minimum(dt, 180.0 - dt).mean())
    return {k: (float(np.mean(v)) if v else None) for k, v in out.items()}


def sweep(R_over_eta=(0.5,), Ca=(0.05, 0.1, 0.2, 0.4), members=8, frames=200, R_lbu=8.0, L=64, tau_f=1.0,
          level=4, storage="f32", seed=100):
    """The protocol over a grid of (R / eta, Ca): for each point an ensemble
    of `members` droplets (R_lbu, level-`level` icospheres in L^3 boxes) on
    independent synthetic trajectories, run batched on the GPU, compared with
    the linear theory frame by frame. Returns one record per point; a point
    whose run stops with a domain or non-finite error records the error.

    The lattice gradient is C_t / tau_eta ~ nu_lbu / R_lbu^2 and the wall
    speed grows with L / R_lbu, so small droplets need a small tau_f to keep
    the walls' Mach number near the paper's (R_lbu 19, L 200, tau_f 1.5)."""
    from . import ibmlb
    from .inputs import box_center, dns_gradient_frames, icosphere
    V, T = icosphere(level, R_lbu, box_center((L, L, L)))
    fr = np.stack([dns_gradient_frames(frames, seed=seed + i) for i in range(members)])
    out = []
    for r in R_over_eta:
        for ca in Ca:
            m = match_units(r, ca, R_lbu, tau_f)
            mem = [dict(L=(L, L, L), tau=tau_f, sigma=m.sigma_lbu, radius=R_lbu, vertices=V, triangles=T,
                        A0=m.gradient_lbu(fr[i, 0])) for i in range(members)]
            rec = {"R_over_eta": r, "Ca": ca, "steps_per_frame": m.N, "frames": frames, "members": members,
                   "tau_f": tau_f, "R_lbu": R_lbu, "L": L}
            ens = ibmlb.Ensemble(mem, storage=storage)
            try:
                res = run_ensemble(ens, fr, m, stop_on_error=True)
            finally:
                ens.close()
            rec["frames_completed"] = res["D"].shape[1]
            if res["failed_at"] is not None:
                rec["stopped"] = "a droplet stencil reached a wall or the state turned non-finite"
            if res["D"].shape[1] > 10:
                rec.update(compare_with_theory(m, res))
                rec["mean_D"] = float(np.mean(res["D"][:, 5:]))
                rec["max_D"] = float(np.max(res["D"]))
            out.append(rec)
    return out


if __name__ == "__main__":
    import argparse
    import json
    ap = argparse.ArgumentParser(description="the paper's protocol against the linear theory (GPU ensembles)")
    ap.add_argument("--r-over-eta", type=float, nargs="+", default=[0.5])
    ap.add_argument("--ca", type=float, nargs="+", default=[0.05, 0.1, 0.2, 0.4])
    ap.add_argument("--members", type=int, default=8)
    ap.add_argument("--frames", type=int, default=200)
    ap.add_argument("--tau", type=float, default=1.0)
    ap.add_argument("--R", type=float, default=8.0, help="droplet radius in lattice units")
    ap.add_argument("--L", type=int, default=64, help="box side")
    ap.add_argument("--level", type=int, default=4, help="icosphere subdivision level")
    a = ap.parse_args()
    for rec in sweep(tuple(a.r_over_eta), tuple(a.ca), a.members, a.frames, R_lbu=a.R, L=a.L, tau_f=a.tau,
                     level=a.level):
        print(json.dumps(rec), flush=True)
