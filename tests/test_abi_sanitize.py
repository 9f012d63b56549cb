"""The library's host-side validation and set-up under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU).

api.hip is compiled again with the sanitizers on its host code only (the
device code is unchanged), linked with the library's other objects into the
driver `abi_sanitize_check.cpp`, and run on an icosphere: every valid
configuration the set-up distinguishes, every rejected parameter and mesh
defect, and an ensemble that refuses a member. The run must be clean and
every call must return the expected code. Needs the objects of a prior
build (`__graft_entry__.build()`).
"""
import os
import subprocess

import numpy as np
import pytest

from paper_2403_01161_amd.inputs import box_center, icosphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2403_01161_amd", "csrc")
OBJS = ["lattice_f64", "lattice_f32", "lattice_f16", "lattice_bf16", "kernels", "ib_patch", "indicator", "adjoint"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_host_validation_under_sanitizers(tmp_path):
    objs = [os.path.join(CSRC, "_build", o + ".o") for o in OBJS]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("library objects not built")
    api = str(tmp_path / "api_san.o")
    r = subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *HOST_SAN,
                        "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, "api.hip"),
                        "-o", api], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_sanitize_check")
    r = subprocess.run(["/opt/rocm/llvm/bin/clang++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
                        os.path.join(ROOT, "tests", "abi_sanitize_check.cpp"), api, *objs,
                        "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    L = (16, 16, 16)
    V, T = icosphere(2, 3.0, box_center(L))
    mesh = tmp_path / "mesh.txt"
    with open(mesh, "w") as f:
        f.write(f"{len(V)} {len(T)}\n")
        np.savetxt(f, V, fmt="%.17g")
        np.savetxt(f, T, fmt="%d")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe, str(mesh)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ran clean" in r.stdout
