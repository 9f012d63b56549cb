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


def run_ensemble(ens, frames_dnsu, m: Matching):
    """As `run` for an ensemble whose members share the matching, member i
    following trajectory frames_dnsu[i] ([n, F, 9]). Returns per-frame arrays
    [n, F] (D, beta, theta)."""
    A = m.gradient_lbu(np.asarray(frames_dnsu, dtype=np.float64))
    n, F = A.shape[0], A.shape[1]
    out = {k: np.empty((n, F)) for k in ("D", "beta", "theta")}
    for f in range(F):
        ens.step(np.repeat(A[:, f:f + 1, :], m.N, axis=1))
        for i, ob in enumerate(ens.observables()):
            out["D"][i, f], out["beta"][i, f], out["theta"][i, f] = ob["D"], ob["beta"], ob["theta_deg"]
    out["A_lbu"] = A
    return out
