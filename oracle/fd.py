"""Plain FP64 oracle of the paper's second method: the finite-difference
screened Poisson system (Section 6, eq. sparse-system).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The wave function obeys -hbar^2 lap(phi) + f^2 phi = 0 (eq. phiEquation)
away from the sources.  With the standard (2D: five-point, 3D: seven-point)
Laplacian on the grid and phi = 0 outside it, multiplying by h^2/hbar^2 gives
the sparse system of eq. sparse-system,

    (2D + (h f_m / hbar)^2) phi_m - sum_{neighbours n of m} phi_n = b_m,

b = the Kronecker delta of the point set (eq. deltakron), and then
S = -hbar ln phi (eq. SfromPhi).  Readings: the diagonal term that the
printed system writes as f(X_i) is taken as (h f(X_i) / hbar)^2, the only
form consistent with eq. phiEquation; the right-hand side is used as printed
(1 at the sources), so phi at a source is a value of the discrete Green's
function rather than 1, and S there is O(hbar).

The system is assembled with scipy.sparse and solved by a sparse direct
factorisation (scipy.sparse.linalg.spsolve), the counterpart of the paper's
direct sparse solve.  Small grids only.
"""
from __future__ import annotations

import numpy as np


def _lap1d(n: int):
    import scipy.sparse as sp
    return sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])


def matrix(f: np.ndarray, h: float, hbar: float):
    """A = discrete Laplacian (Dirichlet zero outside the grid) + diag((h f / hbar)^2)."""
    import scipy.sparse as sp
    f = np.asarray(f, np.float64)
    dims = f.shape
    L = None
    for d in range(len(dims)):
        term = None
        for e in range(len(dims)):
            m = _lap1d(dims[e]) if e == d else sp.identity(dims[e])
            term = m if term is None else sp.kron(term, m)
        L = term if L is None else L + term
    return (L + sp.diags(((h / hbar) * f).ravel() ** 2)).tocsc()


def rhs(dims, src: np.ndarray) -> np.ndarray:
    """Kronecker delta of the point set (eq. deltakron)."""
    b = np.zeros(dims)
    src = np.asarray(src).reshape(-1, len(dims))
    b[tuple(src.T)] = 1.0
    return b


def solve(f: np.ndarray, src: np.ndarray, h: float, hbar: float) -> dict:
    """phi = A^-1 b and S = -hbar ln phi (+inf where phi <= 0)."""
    from scipy.sparse.linalg import spsolve
    f = np.asarray(f, np.float64)
    A = matrix(f, h, hbar)
    phi = spsolve(A, rhs(f.shape, src).ravel()).reshape(f.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        S = np.where(phi > 0, -hbar * np.log(np.where(phi > 0, phi, 1.0)), np.inf)
    return {"phi": phi, "S": S}
