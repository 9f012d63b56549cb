"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This module holds no arithmetic of the IB-LB method itself: it only builds
the triangulated droplet mesh and the velocity-gradient time series that both
implementations consume as inputs.

* ``icosphere`` — the closed triangular droplet mesh. The paper uses "a
  structured mesh composed of 20480 triangles" (Sec. 3.2); a level-5
  icosphere has exactly that many triangles (10242 vertices).
* ``ou_gradient_table`` — a seeded, traceless Ornstein-Uhlenbeck stand-in for
  the turbulent velocity-gradient samples A(t) = grad u(t) of the TURB-Lagr
  trajectories (Sec. 3.2), which are not available here.
* ``simple_shear`` — the steady shear gradient A = [[0, g, 0], [0, 0, 0],
  [0, 0, 0]], i.e. u_x = g (y - y_c) (Eq. linearized velocity).

Gradient convention: A is row-major with A[3a+b] = d u_a / d x_b, so the
far-field velocity is u = A (x - x_c).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

__all__ = ["icosphere", "icosphere_counts", "ou_gradient_table", "simple_shear",
           "box_center"]


def box_center(L):
    """Centre of a box of L[a] nodes at 0..L[a]-1 per axis."""
    return np.array([(float(n) - 1.0) / 2.0 for n in L], dtype=np.float64)


def icosphere_counts(level: int):
    """(n_vertices, n_triangles) of a level-`level` icosphere."""
    return 10 * 4 ** level + 2, 20 * 4 ** level


def _icosahedron():
    g = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * g))
            v.append((s1, s2 * g, 0.0))
            v.append((s2 * g, 0.0, s1))
    v = np.array(v, dtype=np.float64)
    # faces: triples of mutually adjacent vertices (edge length 2)
    faces = []
    for i, j, k in itertools.combinations(range(12), 3):
        if (abs(np.linalg.norm(v[i] - v[j]) - 2.0) < 1e-9
                and abs(np.linalg.norm(v[j] - v[k]) - 2.0) < 1e-9
                and abs(np.linalg.norm(v[i] - v[k]) - 2.0) < 1e-9):
            n = np.cross(v[j] - v[i], v[k] - v[i])
            if np.dot(n, v[i] + v[j] + v[k]) < 0.0:
                faces.append((i, k, j))
            else:
                faces.append((i, j, k))
    assert len(faces) == 20
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, faces


def icosphere(level: int, radius: float, center=(0.0, 0.0, 0.0)):
    """Closed, outward-oriented (counter-clockwise seen from outside) icosphere.

    Midpoint-subdivides an icosahedron `level` times, projecting new vertices
    onto the unit sphere, then scales by `radius` and translates to `center`.

    Returns (vertices float64 [nv, 3], triangles int32 [nt, 3]).
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    v, faces = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(level):
        cache = {}
        new_faces = []

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                p = np.add(verts[a], verts[b])
                p = p / np.linalg.norm(p)
                verts.append(tuple(p))
                idx = len(verts) - 1
                cache[key] = idx
            return idx

        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    V = np.asarray(verts, dtype=np.float64) * float(radius)
    V += np.asarray(center, dtype=np.float64)[None, :]
    T = np.asarray(faces, dtype=np.int32)
    return V, T


def simple_shear(gamma: float):
    """Row-major gradient of the simple shear u_x = gamma (y - y_c)."""
    A = np.zeros(9, dtype=np.float64)
    A[1] = gamma
    return A


def ou_gradient_table(nsteps: int, corr_steps: float, rms: float, seed: int):
    """Seeded traceless Ornstein-Uhlenbeck velocity-gradient table.

    Per step n: B_{n+1} = e^{-1/T} B_n + sqrt(1 - e^{-2/T}) s Xi_n with
    Xi_n nine iid N(0, 1) entries and B_0 entries iid N(0, s^2); the output
    row is B_n projected traceless, B_n - tr(B_n)/3 I. The projection keeps
    8 of the 9 degrees of freedom, so E ||A||_F^2 = 8 s^2 and s = rms/sqrt(8)
    gives an rms Frobenius norm `rms`.

    Returns float64 [nsteps, 9] (row-major A per step).
    """
    if nsteps < 0:
        raise ValueError("nsteps must be >= 0")
    rng = np.random.default_rng(seed)
    s = float(rms) / math.sqrt(8.0)
    a = math.exp(-1.0 / float(corr_steps))
    b = math.sqrt(max(0.0, 1.0 - a * a))
    out = np.empty((nsteps, 9), dtype=np.float64)
    B = rng.standard_normal(9) * s
    eye = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1], dtype=np.float64)
    for n in range(nsteps):
        tr = B[0] + B[4] + B[8]
        out[n] = B - (tr / 3.0) * eye
        B = a * B + b * s * rng.standard_normal(9)
    return out


def dns_gradient_frames(nframes: int, seed: int, tau_eta: float = 2.3e-2, dt: float = 2.25e-3):
    """Synthetic stand-in for a Lagrangian velocity-gradient trajectory of
    homogeneous isotropic turbulence, in DNS units, one frame every `dt`: the
    traceless Ornstein-Uhlenbeck table above with correlation time tau_eta
    (tau_eta / dt frames) and rms Frobenius norm 1 / tau_eta (in such flows
    the mean of |grad u|^2 is epsilon / nu = 1 / tau_eta^2).

    Returns float64 [nframes, 9]."""
    return ou_gradient_table(nframes, tau_eta / dt, 1.0 / tau_eta, seed)
