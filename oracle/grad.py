"""Plain FP64 oracle of the full gradient of a loss L(S) of the 2D or 3D solve.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Not in the paper: the
derivative of the steps of Table 1 with respect to all of their inputs,

  beta = ftilde h / hbar,  gamma = f^2 / ftilde^2 - 1,  w_k = exp(-s_k / hbar),
  phi_0 = sum_k w_k exp(-beta |m - y_k|)                 (eq. phi_0Solution)
  phi_i = kappa_beta (*) (gamma phi_{i-1})               (eq. phiRecRelation)
  phi = sum_i (-1)^i phi_i,  S = -hbar ln phi            (eqs. phiSolution, SfromPhi)

with ftilde a function of f (nu = sqrt((fmin^2 + fmax^2)/2), or sup f, or a
constant: Section 5.1).  dL/df is the adjoint with ftilde fixed plus
dL/dftilde times a subgradient of ftilde(f): the derivative with respect to
fmin (fmax) goes to the first grid point, in C order, where f attains it.

The three scalar paths (beta through the kernel and phi_0, ftilde through
gamma, hbar through the weights) are propagated forward: one tangent series
per path, each convolution done by the oracle's convolution (own FFT) or, for
the kernel's beta-derivative, by a numpy FFT of its even extension.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

import oracle


def kappa_dbeta(dims, beta: float) -> np.ndarray:
    """d kappa / d beta on the orthant 0 <= m_d < n_d.
    2D: (beta/pi) K0(beta r) - (beta^2 r / 2 pi) K1(beta r) off the origin;
    at the origin the beta-derivative of the ball average 1 - a K1(a),
    a = beta/sqrt(pi), which is (beta/pi) K0(beta/sqrt(pi)).
    3D: kappa = beta^2 exp(-beta r) / (4 pi r) gives
    beta exp(-beta r) (2 - beta r) / (4 pi r); at the origin the ball
    average 1 - (1 + a) exp(-a), a = c beta, c = (3/(4 pi))^(1/3), has the
    derivative c a exp(-a)."""
    dims = tuple(int(d) for d in dims)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims], indexing="ij")
    r = np.sqrt(sum(g * g for g in grids))
    out = np.zeros(dims)
    nz = r > 0
    if len(dims) == 2:
        x = beta * r[nz]
        out[nz] = beta / np.pi * oracle.k0(x) - beta * beta * r[nz] / (2 * np.pi) * oracle.k1(x)
        out[(0,) * 2] = beta / np.pi * float(oracle.k0(beta / np.sqrt(np.pi)))
    elif len(dims) == 3:
        rr = r[nz]
        out[nz] = beta * np.exp(-beta * rr) * (2.0 - beta * rr) / (4 * np.pi * rr)
        c = (3.0 / (4.0 * np.pi)) ** (1.0 / 3.0)
        out[(0,) * 3] = c * c * beta * np.exp(-c * beta)
    else:
        raise ValueError("2D or 3D")
    return out


def conv_table(x: np.ndarray, table: np.ndarray) -> np.ndarray:
    """Linear convolution of x with the even extension of an orthant table,
    by numpy FFTs on the zero-padded grid."""
    dims = x.shape
    M = oracle.pad_sizes(dims)
    K = np.zeros(M)
    for signs in np.ndindex(*(2,) * len(dims)):
        idx = [((1 - 2 * s) * np.arange(n)) % m for s, n, m in zip(signs, dims, M)]
        K[np.ix_(*idx)] = table
    X = np.zeros(M)
    X[tuple(slice(0, n) for n in dims)] = x
    y = np.fft.ifftn(np.fft.fftn(X) * np.fft.fftn(K)).real
    return y[tuple(slice(0, n) for n in dims)]


def full_gradient(f: np.ndarray, src: np.ndarray, h: float, hbar: float, T: int,
                  dLdS: np.ndarray, ft_mode: str = "nu", ftilde: Optional[float] = None,
                  src_s: Optional[np.ndarray] = None) -> dict:
    f = np.asarray(f, np.float64)
    dims = f.shape
    nd = f.ndim
    src = np.asarray(src, np.int32).reshape(-1, nd)
    dLdS = np.asarray(dLdS, np.float64)
    lo, hi = float(f.min()), float(f.max())
    ft = {"nu": np.sqrt(0.5 * (lo * lo + hi * hi)), "fmax": hi, "given": ftilde}[ft_mode]
    beta = ft * h / hbar
    gam = (f - ft) * (f + ft) / (ft * ft)
    s = np.zeros(len(src)) if src_s is None else np.asarray(src_s, np.float64)
    w = np.exp(-s / hbar)

    # forward series
    phis = [oracle.phi0(dims, beta, src, w)]
    for _ in range(T):
        phis.append(oracle.conv(gam * phis[-1], beta))
    sgn = [(-1.0) ** i for i in range(T + 1)]
    phi = sum(sg * p for sg, p in zip(sgn, phis))
    S = -hbar * np.log(phi)
    lam = -hbar * dLdS / phi

    # reverse sweep with ftilde fixed: a_i = dL/dphi_i
    a = sgn[T] * lam
    dLdg = np.zeros(dims)
    for i in range(T, 0, -1):
        b = oracle.conv(a, beta)
        dLdg += phis[i - 1] * b
        a = sgn[i - 1] * lam + gam * b
    dLdf = dLdg * 2.0 * f / (ft * ft)

    # forward tangents of the three scalar paths
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in dims], indexing="ij")
    dist = [np.sqrt(sum((g - yd) ** 2 for g, yd in zip(grids, y))) for y in src]
    ex = [np.exp(-beta * d) for d in dist]
    dkap = kappa_dbeta(dims, beta)
    dgam = -2.0 * f * f / ft ** 3
    t = [-sum(wk * d * e for wk, d, e in zip(w, dist, ex))]            # d phi_i / d beta
    u = [np.zeros(dims)]                                                # d phi_i / d ftilde (gamma)
    v = [sum(wk * sk / hbar ** 2 * e for wk, sk, e in zip(w, s, ex))]  # d phi_i / d hbar (weights)
    for i in range(1, T + 1):
        t.append(conv_table(gam * phis[i - 1], dkap) + oracle.conv(gam * t[-1], beta))
        u.append(oracle.conv(dgam * phis[i - 1] + gam * u[-1], beta))
        v.append(oracle.conv(gam * v[-1], beta))
    dLdbeta = float(np.sum(lam * sum(sg * x for sg, x in zip(sgn, t))))
    dLdft_gamma = float(np.sum(lam * sum(sg * x for sg, x in zip(sgn, u))))
    dLdhbar_w = float(np.sum(lam * sum(sg * x for sg, x in zip(sgn, v))))

    dLdhbar = float(np.sum(dLdS * S / hbar)) - beta / hbar * dLdbeta + dLdhbar_w
    dLdft = h / hbar * dLdbeta + dLdft_gamma
    flat = dLdf.reshape(-1)
    if ft_mode == "nu":
        flat[int(np.argmin(f))] += dLdft * lo / (2.0 * ft)
        flat[int(np.argmax(f))] += dLdft * hi / (2.0 * ft)
    elif ft_mode == "fmax":
        flat[int(np.argmax(f))] += dLdft
    return {"dLdf": dLdf, "dLdhbar": dLdhbar, "dLdftilde": dLdft, "dLdbeta": dLdbeta,
            "S": S, "ftilde": ft, "beta": beta}
