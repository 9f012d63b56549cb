"""GPU: the paper's protocol (DNS frames converted to lattice units and held
for N steps each) through the HIP library.

* One droplet, FP64 storage: the deformation and orientation after every
  frame equal the FP64 oracle's (same protocol), and follow the linear
  theory at small Ca.
* An ensemble of four droplets on independent synthetic trajectories
  (FP32 storage, batched launches): each follows the linear theory.
"""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd import protocol as P
from paper_2403_01161_amd.inputs import dns_gradient_frames

from .test_protocol import _against_linear_theory, _protocol_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01161_amd import ibmlb
    ibmlb.lib()
    return ibmlb


def test_protocol_single_droplet_matches_oracle(ib):
    m, L, kw, fr = _protocol_case(40)
    print(f"case protocol L={L} N={m.N} frames={len(fr)}", flush=True)
    sim = ib.Simulation(L, storage="f64", **kw)
    res = P.run(sim, fr, m)
    sim.close()
    o = oracle.Oracle(L, **kw)
    ref = P.run(o, fr, m)
    o.close()
    assert np.abs(res["D"] - ref["D"]).max() <= 1e-9 * ref["D"].max()
    assert np.abs(res["beta"] - ref["beta"]).max() <= 1e-8
    assert np.abs(res["S"] - ref["S"]).max() <= 1e-9 * np.abs(ref["S"]).max()
    cD, ratio, cb = _against_linear_theory(m, res)
    assert cD > 0.8 and 1.0 < ratio < 1.5 and cb > 0.95


def test_protocol_ensemble_follows_linear_theory(ib):
    m, L, kw, _ = _protocol_case(1)
    n, F = 4, 40
    frames = np.stack([dns_gradient_frames(F, seed=100 + i) for i in range(n)])
    members = []
    for i in range(n):
        d = dict(kw)
        d["A0"] = m.gradient_lbu(frames[i, 0])
        members.append(dict(L=L, **d))
    print(f"case protocol ensemble n={n} N={m.N} frames={F}", flush=True)
    ens = ib.Ensemble(members, storage="f32")
    res = P.run_ensemble(ens, frames, m)
    ens.close()
    for i in range(n):
        one = {"D": res["D"][i], "beta": res["beta"][i], "theta": res["theta"][i], "A_lbu": res["A_lbu"][i]}
        cD, ratio, cb = _against_linear_theory(m, one)
        print(f"  member {i}: corr D {cD:.3f}  D/D_LT {ratio:.3f}  corr beta {cb:.3f}", flush=True)
        assert cD > 0.8 and 1.0 < ratio < 1.5 and cb > 0.95
