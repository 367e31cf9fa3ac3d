"""Shared helpers for the GPU parity tests (no solver arithmetic here).

Resolvable sets.  FFT convolution has an absolute error of about
eps * max|psi| spread over the grid while phi falls off like exp(-S/hbar),
so the relative error of S at x grows like c eps exp(Lambda(x)) / Lambda(x)
with Lambda(x) = ln(max phi / phi(x)) from the FP64 oracle; the measured
constant c lies between 0.05 and 0.2 for both precisions.  The paper meets
the same limit (Section 5.3).  Parity is claimed where the law with c = 1
guarantees the stated tolerance: R64 = {Lambda <= 16} for the FP64 path
(rel <= 1e-10) and R32 = {Lambda <= 9} for the FP32-scaled path
(rel <= 1e-4), with rel = |S - S_oracle| / max(|S_oracle|, hbar).  Beyond
those sets every point up to Lambda = 30 (FP64) or 14 (FP32) is checked
against the envelope tol + eps exp(Lambda) / max(Lambda, 1).
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TOL = {"fp64": 1e-10, "fp32": 1e-4}
LAMBDA_MAX = {"fp64": 16.0, "fp32": 9.0}
EPS = {"fp64": 2.0 ** -52, "fp32": 2.0 ** -23}


def ensure_built():
    """Build the HIP library only if nothing is built yet."""
    import paper_1403_1937_amd as pk
    if not os.path.exists(pk.lib_path()):
        from paper_1403_1937_amd import build
        build.build()


def lam(phi_oracle: np.ndarray) -> np.ndarray:
    phi = np.asarray(phi_oracle, np.float64)
    out = np.full(phi.shape, np.inf)
    pos = phi > 0
    out[pos] = np.log(phi[pos].max() / phi[pos])
    return out


def rel_err(S, S_o, hbar):
    S = np.asarray(S, np.float64)
    return np.abs(S - S_o) / np.maximum(np.abs(S_o), hbar)


def resolvable(phi_oracle, prec):
    return lam(phi_oracle) <= LAMBDA_MAX[prec]


def report(S, out_o, hbar, prec):
    """(max rel error on the resolvable set, fraction of the set, max rel on
    the whole grid where both are finite)."""
    m = resolvable(out_o["phi"], prec)
    e = rel_err(S, out_o["S"], hbar)
    fin = np.isfinite(S) & np.isfinite(out_o["S"])
    return float(e[m].max()) if m.any() else 0.0, float(m.mean()), float(e[fin].max())


LAMBDA_ENVELOPE = {"fp64": 30.0, "fp32": 14.0}


def envelope_violations(S, out_o, hbar, prec, lam_cap=None, ulps=1.0):
    """Points with Lambda <= lam_cap whose error exceeds the conditioning
    envelope TOL + ulps EPS exp(Lambda) / max(Lambda, 1) (an absolute
    rounding error of ulps units of max phi, seen relative to phi)."""
    L = lam(out_o["phi"])
    e = rel_err(S, out_o["S"], hbar)
    m = L <= (LAMBDA_ENVELOPE[prec] if lam_cap is None else lam_cap)
    bound = TOL[prec] + ulps * EPS[prec] * np.exp(np.minimum(L, 700)) / np.maximum(L, 1.0)
    bad = m & ~(e <= bound)
    return int(bad.sum())
