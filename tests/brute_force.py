"""Dense NumPy re-implementation of the IB-LB step for tiny boxes (test pin).

A second, structurally different implementation used only to pin the oracle
on 8^3 boxes:
  * the D3Q19 set is enumerated from {-1, 0, 1}^3 (its own ordering);
  * streaming is an explicit gather-index permutation per direction;
  * spreading and interpolation use the dense vertex x node weight matrix
    (all pairs, minimum image on periodic axes);
  * surface-tension forces are the complex-step derivative of the total
    mesh area (no hand-derived gradient);
  * the smoothing uses the dense neighbour-averaging matrix.
Arithmetic follows arXiv 2403.01161 Sec. 3.1 and Sec. 3.3 with the readings
stated in the oracle (standard equilibrium, link-wise moving bounce-back).
"""
import itertools

import numpy as np

CS2 = 1.0 / 3.0


def d3q19():
    c = np.array([v for v in itertools.product((-1, 0, 1), repeat=3) if sum(x * x for x in v) <= 2])
    n2 = (c * c).sum(axis=1)
    w = np.where(n2 == 0, 1 / 3, np.where(n2 == 1, 1 / 18, 1 / 36))
    opp = np.array([int(np.flatnonzero((c == -v).all(axis=1))[0]) for v in c])
    return c, w, opp


def peskin(r):
    a = np.abs(r)
    inner = (3 - 2 * a + np.sqrt(np.clip(1 + 4 * a - 4 * a * a, 0, None))) / 8
    outer = (5 - 2 * a - np.sqrt(np.clip(-7 + 12 * a - 4 * a * a, 0, None))) / 8
    return np.where(a < 1, inner, np.where(a < 2, outer, 0.0))


class Dense:
    def __init__(self, L, periodic, tau, sigma, verts, tris, A0, rho0=1.0,
                 alpha=0.1, gamma=0.51, tol=0.01, max_iter=50, sign=1):
        self.L = np.array(L)
        self.per = np.array(periodic, dtype=bool)
        self.tau, self.sigma, self.rho0 = tau, sigma, rho0
        self.c, self.w, self.opp = d3q19()
        Lx, Ly, Lz = L
        z, y, x = np.meshgrid(np.arange(Lz), np.arange(Ly), np.arange(Lx), indexing="ij")
        self.X = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1).astype(float)
        self.xc = (self.L - 1) / 2.0
        self.r = np.array(verts, dtype=float)
        self.T = np.array(tris)
        self.alpha, self.gamma, self.tol, self.max_iter, self.sign = alpha, gamma, tol, max_iter, sign
        nv = len(self.r)
        M = np.zeros((nv, nv))
        for t in self.T:
            for j in range(3):
                M[t[j], t[(j + 1) % 3]] = M[t[(j + 1) % 3], t[j]] = 1.0
        self.M = M / M.sum(axis=1, keepdims=True)
        # gather index per direction: source node x - c_i, or -1 beyond a wall
        N = len(self.X)
        self.src = np.full((19, N), -1, dtype=np.int64)
        for i, ci in enumerate(self.c):
            s = self.X - ci
            ok = np.ones(N, dtype=bool)
            for a in range(3):
                if self.per[a]:
                    s[:, a] = np.mod(s[:, a], L[a])
                else:
                    ok &= (s[:, a] >= 0) & (s[:, a] < L[a])
            idx = (s[:, 0] + Lx * (s[:, 1] + Ly * s[:, 2])).astype(np.int64)
            self.src[i, ok] = idx[ok]
        A0 = np.asarray(A0, dtype=float).reshape(3, 3)
        u0 = (self.X - self.xc) @ A0.T
        Q = np.einsum("ia,ib->iab", self.c, self.c) - CS2 * np.eye(3)
        self.f = (self.feq(np.full(N, rho0), u0)
                  - 3 * tau * rho0 * self.w[:, None] * np.einsum("iab,ab->i", Q, A0)[:, None])

    def feq(self, rho, u):
        cu = u @ self.c.T  # [N, 19]
        uu = (u * u).sum(axis=1)
        return (self.w[None, :] * rho[:, None]
                * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - uu[:, None] / (2 * CS2))).T

    def weights(self):
        d = self.r[:, None, :] - self.X[None, :, :]
        for a in range(3):
            if self.per[a]:
                d[..., a] -= self.L[a] * np.round(d[..., a] / self.L[a])
        return peskin(d[..., 0]) * peskin(d[..., 1]) * peskin(d[..., 2])  # [nv, N]

    def area(self, r):
        e1 = r[self.T[:, 1]] - r[self.T[:, 0]]
        e2 = r[self.T[:, 2]] - r[self.T[:, 0]]
        n = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                      e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                      e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], axis=1)
        return 0.5 * np.sqrt((n * n).sum(axis=1)).sum()

    def forces(self):
        h = 1e-30
        g = np.zeros_like(self.r)
        for k in range(len(self.r)):
            for a in range(3):
                rc = self.r.astype(complex)
                rc[k, a] += 1j * h
                g[k, a] = self.area(rc).imag / h
        return -self.sigma * g

    def smooth(self, o):
        p = o.copy()
        for it in range(1, self.max_iter + 1):
            q = p
            pp = self.alpha * o + (1 - self.alpha) * (self.M @ q)
            b = pp - (self.alpha * o + (1 - self.alpha) * q)
            p = pp - (self.gamma * b + self.sign * (1 - self.gamma) * (self.M @ b))
            if np.sqrt(((p - q) ** 2).sum(axis=1)).max() < self.tol:
                break
        return p

    def step(self, A):
        A = np.asarray(A, dtype=float).reshape(3, 3)
        W = self.weights()
        F = W.T @ self.forces()
        rho = self.f.sum(axis=0)
        u = (self.f.T @ self.c + F / 2) / rho[:, None]
        U = W @ u
        cu = u @ self.c.T
        S = ((1 - 1 / (2 * self.tau)) * self.w[None, :] / CS2
             * ((cu / CS2 + 1) * (F @ self.c.T) - (u * F).sum(axis=1)[:, None])).T
        fs = self.f - (self.f - self.feq(rho, u)) / self.tau + S
        new = np.empty_like(fs)
        for i, ci in enumerate(self.c):
            ok = self.src[i] >= 0
            new[i, ok] = fs[i, self.src[i, ok]]
            xw = self.X[~ok] - 0.5 * ci - self.xc
            new[i, ~ok] = fs[self.opp[i], ~ok] + 2 * self.w[i] * self.rho0 * ((xw @ A.T) @ ci) / CS2
        self.f = new
        self.r = self.smooth(self.r + U)
