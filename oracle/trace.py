"""Plain FP64 oracle of path backtracking on S (Section 6, path planning).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Paths follow
dx/dt = -grad S / |grad S| (eq. PathPlanning-backTrackOnS) from each start
point until they come within a radius of a source.  The paper leaves the
discretisation open; this module takes these readings, step by step:

* node gradient: central difference of S along each axis, one-sided at the
  first and last node, in units of one grid spacing;
* gradient at a point x: multilinear interpolation of the node gradients of
  the 2^D nodes of x's cell (cell index clamped to [0, n-2]);
* step: classical fourth-order Runge-Kutta of length ``step`` on the unit
  field u = -g/|g|, each stage position and each new point clamped to the box
  [0, n_d - 1];
* stop: within ``radius`` of a source (status 0), after ``max_steps`` steps
  (1), where the gradient vanishes or is not finite (2); a start outside the
  box records no point (3).

Paths are advanced together with numpy (one vector lane per path), masked
once they stop.  Everything is float64.
"""
from __future__ import annotations

import numpy as np


def _node_grad(S: np.ndarray, idx: np.ndarray, d: int) -> np.ndarray:
    """Central difference of S along axis d at integer nodes idx [P, D]."""
    n = S.shape[d]
    m = idx[:, d]
    up = idx.copy()
    dn = idx.copy()
    up[:, d] = np.minimum(m + 1, n - 1)
    dn[:, d] = np.maximum(m - 1, 0)
    s_up = S[tuple(up.T)]
    s_dn = S[tuple(dn.T)]
    s_0 = S[tuple(idx.T)]
    interior = (m > 0) & (m < n - 1)
    g = np.where(m == 0, s_up - s_0, s_0 - s_dn)
    return np.where(interior, 0.5 * (s_up - s_dn), g)


def gradient(S: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Multilinearly interpolated node gradient of S at points x [P, D]."""
    D = S.ndim
    n = np.array(S.shape)
    i = np.clip(np.floor(x).astype(np.int64), 0, n - 2)
    t = x - i
    g = np.zeros_like(x)
    for corner in range(1 << D):
        bits = np.array([(corner >> (D - 1 - d)) & 1 for d in range(D)])
        node = i + bits
        w = np.prod(np.where(bits == 1, t, 1.0 - t), axis=1)
        for d in range(D):
            g[:, d] += w * _node_grad(S, node, d)
    return g


def _direction(S, x):
    g = gradient(S, x)
    nrm = np.sqrt(np.sum(g * g, axis=1))
    ok = (nrm > 0) & np.isfinite(nrm)
    with np.errstate(invalid="ignore", divide="ignore"):
        u = -g / nrm[:, None]
    return u, ok


def backtrack(S: np.ndarray, src: np.ndarray, start: np.ndarray, step: float = 0.5,
              radius: float = 1.0, max_steps: int = 4096):
    """Returns (path [P, max_steps+1, D], n_points [P], status [P])."""
    S = np.asarray(S, np.float64)
    D = S.ndim
    src = np.asarray(src, np.float64).reshape(-1, D)
    x = np.array(start, np.float64).reshape(-1, D)
    P = x.shape[0]
    hi = np.array(S.shape, np.float64) - 1.0
    path = np.zeros((P, max_steps + 1, D))
    n_points = np.zeros(P, np.int32)
    status = np.full(P, -1, np.int32)
    inside = np.all((x >= 0) & (x <= hi), axis=1)  # False for NaN
    status[~inside] = 3
    active = inside.copy()
    path[:, 0] = np.where(inside[:, None], x, 0.0)
    k = np.zeros(P, np.int64)

    def clamp(y):
        return np.minimum(np.maximum(y, 0.0), hi)

    while active.any():
        a = np.nonzero(active)[0]
        xa = x[a]
        if len(src):
            d2 = np.min(np.sum((xa[:, None, :] - src[None, :, :]) ** 2, axis=2), axis=1)
        else:
            d2 = np.full(len(a), np.inf)
        near = d2 < radius * radius
        status[a[near]] = 0
        done = near | (k[a] == max_steps)
        status[a[~near & (k[a] == max_steps)]] = 1
        go = a[~done]
        active[a[done]] = False
        if len(go) == 0:
            continue
        xg = x[go]
        k1, ok1 = _direction(S, xg)
        k2, ok2 = _direction(S, clamp(xg + 0.5 * step * k1))
        k3, ok3 = _direction(S, clamp(xg + 0.5 * step * k2))
        k4, ok4 = _direction(S, clamp(xg + step * k3))
        ok = ok1 & ok2 & ok3 & ok4
        stuck = go[~ok]
        status[stuck] = 2
        active[stuck] = False
        mv = go[ok]
        xn = xg[ok] + step / 6.0 * (k1[ok] + 2.0 * k2[ok] + 2.0 * k3[ok] + k4[ok])
        x[mv] = clamp(xn)
        k[mv] += 1
        path[mv, k[mv]] = x[mv]
    n_points[inside] = (k[inside] + 1).astype(np.int32)
    return path, n_points, status
