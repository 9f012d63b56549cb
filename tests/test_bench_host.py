"""bench.py's host side (CPU): the one-GPU contract, the workloads' shapes,
the variant naming and the counter-traffic lookup that feeds
roofline.traffic."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_workloads_have_the_stated_shapes():
    w = bench.workload("f32")
    assert w["L"] == (128, 128, 128) and w["R"] == 16.0 and len(w["V"]) == 10242 and len(w["T"]) == 20480
    # sigma from Ca = mu R G / sigma with mu = rho0 nu
    nu = (w["tau"] - 0.5) / 3
    assert abs(nu * w["R"] * w["G"] / w["sigma"] - w["Ca"]) < 1e-15
    p = bench.precision_workload()
    assert p["L"] == (256, 256, 256) and len(p["V"]) == 40962 and len(p["T"]) == 81920 and p["Ca"] == 0.15
    a = bench.adjoint_workload()
    assert a["L"] == (64, 64, 64) and len(a["V"]) == 2562 and a["A"].shape == (500, 9) and a["K"] == 50
    members, rms = bench.ensemble_workload()
    sides = [m["L"][0] for m in members]
    assert len(members) == 64 and set(sides) <= {48, 64, 96} and len(set(sides)) == 3
    assert all(m["radius"] == m["L"][0] / 8 and len(m["vertices"]) == 2562 for m in members)


def test_describe_variant_bits():
    d = bench.describe_variant(57)
    assert d == {"layout": "rows", "nontemporal_loads": True, "block": 128, "nontemporal_stores": True,
                 "smoothing_finish_in_force_kernel": True, "in_place_streaming": False}
    d = bench.describe_variant(2 | 8 | 64)
    assert d["layout"] == "linear" and d["block"] == 256 and d["xcd_grouped_order"] and d["in_place_streaming"]


def _summary(tmp_path, storage, box, variant, sha, nbytes):
    prof = tmp_path / "profiles"
    prof.mkdir(exist_ok=True)
    (prof / f"lattice_{storage}_{box}_counters.md").write_text(
        f"# test\n\nhbm_bytes_per_launch: {nbytes}\nlattice_variant: {variant}\nkernel_source_sha256_16: {sha}\n")


def test_counter_traffic_only_for_the_profiled_kernel(tmp_path, monkeypatch):
    sha = bench.kernel_source_hash()
    _summary(tmp_path, "f32", "256cubed", 57 & 95, sha, 2582617607)
    _summary(tmp_path, "f16dev", "256cubed", 2, "0" * 16, 1294139420)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha)
    assert bench.counter_traffic("f32", "256cubed", 57) == 2582617607.0
    assert bench.counter_traffic("f32", "256cubed", 57 | 64) is None  # another lattice variant
    assert bench.counter_traffic("f32", "256cubed", 57 & ~32) == 2582617607.0  # bit 5 is not a lattice bit
    assert bench.counter_traffic("f16dev", "256cubed", 34) is None  # profiled from another kernel source
    assert bench.counter_traffic("bf16dev", "256cubed", 34) is None  # no summary
    # a second summary of the same box, for another variant
    (tmp_path / "profiles" / "lattice_f32_256cubed_v36_counters.md").write_text(
        f"# test\n\nhbm_bytes_per_launch: 2582000000\nlattice_variant: 4\nkernel_source_sha256_16: {sha}\n")
    assert bench.counter_traffic("f32", "256cubed", 36) == 2582000000.0
    assert bench.counter_traffic("f32", "256cubed", 57) == 2582617607.0


def test_committed_counter_summaries_are_consistent():
    """Every committed summary names its variant and the kernel source it was
    taken from, and its bytes lie within 2 % above the algorithmic bytes."""
    prof = os.path.join(ROOT, "profiles")
    nodes = {"256cubed": 256 ** 3, "128cubed": 128 ** 3}
    found = 0
    for fn in sorted(os.listdir(prof)):
        if not (fn.startswith("lattice_") and fn.endswith("_counters.md")) or "diagnostic" in fn:
            continue
        storage, box = fn[len("lattice_"):-len("_counters.md")].split("_")[:2]
        txt = open(os.path.join(prof, fn)).read()
        nbytes = float(txt.split("hbm_bytes_per_launch:")[1].split()[0])
        alg = 2 * 19 * bench.STORAGE_BYTES[storage] * nodes[box]
        assert 1.0 <= nbytes / alg <= 1.02, (fn, nbytes / alg)
        assert "lattice_variant:" in txt and "kernel_source_sha256_16:" in txt
        found += 1
    assert found >= 5


def test_ou_table_rms_matches_the_gradient_scale():
    from paper_2403_01161_amd.inputs import ou_gradient_table
    w = bench.workload("f32")
    table = ou_gradient_table(20001, w["corr"], w["G"], seed=w["seed"])
    rms = np.sqrt(np.mean(np.sum(table ** 2, axis=1)))
    assert abs(rms / w["G"] - 1) < 0.3  # one correlation time is 2000 steps: ten samples' worth
    assert np.abs(table[:, 0] + table[:, 4] + table[:, 8]).max() < 1e-15 * w["G"] * 10
