"""Plain FP64 CPU oracle for the linearised eikonal solve (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline of the benchmark may import this package.  It shares no code with
the GPU path: its arithmetic lives in ``oracle.c`` (own FFT, own Bessel
functions), compiled here with gcc and FP contraction off.

What is computed, and which passage each step follows, is listed in
``oracle.h``: reference forcing (Section 5.1), kernel from the Green's
functions (Section 3.2), phi_0 (eq. phi_0Solution), the recurrence
(eqs. phiRecRelation / phi_i_Solution), the alternating sum (eq.
phiSolution) and the logarithm (eq. SfromPhi); steps as in Table 1.

Two numpy modules cover Section 6: ``oracle.trace`` (path backtracking on S)
and ``oracle.fd`` (the finite-difference screened Poisson system, solved by a
sparse direct factorisation).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

FT_MODES = {"nu": 0, "fmax": 1, "given": 2}
CONV = {"fft": 0, "direct": 1}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (-O2, no FP contraction, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra",
           os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Problem(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("dims", C.c_int64 * 3), ("h", C.c_double),
                ("hbar", C.c_double), ("T", C.c_int32), ("ft_mode", C.c_int32),
                ("ftilde_given", C.c_double), ("conv", C.c_int32),
                ("nthreads", C.c_int32), ("src_s", C.c_void_p)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int32)
    lp = C.POINTER(C.c_int64)
    lib.orc_fft.argtypes = [C.c_int64, dp, C.c_int]
    lib.orc_bessel_k0.argtypes = [C.c_double]
    lib.orc_bessel_k0.restype = C.c_double
    lib.orc_bessel_k1.argtypes = [C.c_double]
    lib.orc_bessel_k1.restype = C.c_double
    lib.orc_kappa0.argtypes = [C.c_int, C.c_double]
    lib.orc_kappa0.restype = C.c_double
    lib.orc_kappa.argtypes = [C.c_int, lp, C.c_double, dp]
    lib.orc_ghat.argtypes = [C.c_int, lp, C.c_double, dp]
    lib.orc_ghat.restype = C.c_int64
    lib.orc_phi0.argtypes = [C.c_int, lp, C.c_double, C.c_int32, ip, dp]
    lib.orc_phi0_weighted.argtypes = [C.c_int, lp, C.c_double, C.c_int32, ip, dp, dp]
    lib.orc_conv.argtypes = [C.c_int, lp, C.c_double, dp, dp, C.c_int32,
                             C.c_int32]
    lib.orc_solve.argtypes = [C.POINTER(_Problem), dp, C.c_int32, ip, dp, dp,
                              dp, dp]
    lib.orc_adjoint.argtypes = [C.POINTER(_Problem), dp, C.c_int32, ip, dp, dp,
                                dp]
    lib.orc_solve_logdirect.argtypes = [C.POINTER(_Problem), dp, C.c_int32, ip, dp, dp, dp]
    lib.orc_log_kappa.argtypes = [C.c_int, lp, C.c_double, dp]
    _lib = lib
    return lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def _dims(shape):
    d = (C.c_int64 * 3)(*([int(s) for s in shape] + [1] * (3 - len(shape))))
    return d


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle {what} rejected its arguments (rc={rc})")


def fft(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """Own radix-2 FFT of a 1D complex array (power-of-two length)."""
    lib = _load()
    a = np.ascontiguousarray(np.asarray(x, np.complex128)).copy()
    buf = a.view(np.float64)
    _check(lib.orc_fft(a.size, _dp(buf), int(inverse)), "fft")
    return a


def k0(x) -> np.ndarray:
    lib = _load()
    x = np.asarray(x, np.float64)
    return np.vectorize(lambda v: lib.orc_bessel_k0(float(v)))(x)


def k1(x) -> np.ndarray:
    lib = _load()
    x = np.asarray(x, np.float64)
    return np.vectorize(lambda v: lib.orc_bessel_k1(float(v)))(x)


def kappa0(ndim: int, beta: float) -> float:
    return float(_load().orc_kappa0(int(ndim), float(beta)))


def kappa(dims, beta: float) -> np.ndarray:
    """Normalised kernel on the orthant 0 <= m_d < n_d."""
    lib = _load()
    out = np.empty(tuple(int(d) for d in dims), np.float64)
    _check(lib.orc_kappa(len(dims), _dims(dims), float(beta), _dp(out)), "kappa")
    return out


def pad_sizes(dims):
    return tuple(1 << int(np.ceil(np.log2(max(2 * int(n) - 1, 1)))) for n in dims)


def ghat(dims, beta: float) -> np.ndarray:
    """Real kernel spectrum on the unique orthant [0..M_d/2]."""
    lib = _load()
    M = pad_sizes(dims)
    out = np.empty(tuple(m // 2 + 1 for m in M), np.float64)
    rc = lib.orc_ghat(len(dims), _dims(dims), float(beta), _dp(out))
    _check(rc, "ghat")
    return out


def phi0(dims, beta: float, src: np.ndarray, weights: Optional[np.ndarray] = None) -> np.ndarray:
    """sum_k w_k exp(-beta |m - y_k|) (eq. phi_0Solution; w_k = 1 by default)."""
    lib = _load()
    src = np.ascontiguousarray(np.asarray(src, np.int32))
    out = np.empty(tuple(int(d) for d in dims), np.float64)
    if weights is None:
        rc = lib.orc_phi0(len(dims), _dims(dims), float(beta), len(src), _ip(src), _dp(out))
    else:
        w = np.ascontiguousarray(np.asarray(weights, np.float64))
        rc = lib.orc_phi0_weighted(len(dims), _dims(dims), float(beta), len(src), _ip(src),
                                   _dp(w), _dp(out))
    _check(rc, "phi0")
    return out


def conv(x: np.ndarray, beta: float, method: str = "fft",
         nthreads: int = 0) -> np.ndarray:
    """kappa (*) x, linear convolution over the grid."""
    lib = _load()
    x = np.ascontiguousarray(np.asarray(x, np.float64))
    out = np.empty_like(x)
    _check(lib.orc_conv(x.ndim, _dims(x.shape), float(beta), _dp(x), _dp(out),
                        CONV[method], int(nthreads)), "conv")
    return out


def _problem(f, h, hbar, T, ft_mode, ftilde, method, nthreads, src_s=None) -> _Problem:
    p = _Problem()
    p.ndim = f.ndim
    p.dims = _dims(f.shape)
    p.h = float(h)
    p.hbar = float(hbar)
    p.T = int(T)
    p.ft_mode = FT_MODES[ft_mode]
    p.ftilde_given = float(ftilde) if ftilde is not None else 0.0
    p.conv = CONV[method]
    p.nthreads = int(nthreads)
    if src_s is not None:
        p._src_s = np.ascontiguousarray(np.asarray(src_s, np.float64))  # kept alive with p
        p.src_s = p._src_s.ctypes.data
    return p


def _info(v) -> dict:
    return {"ftilde": v[0], "beta": v[1], "fmin": v[2], "fmax": v[3],
            "c0_bound": v[4], "n_nonpositive_phi": int(v[5]),
            "padded_points": int(v[6])}


def solve(f: np.ndarray, src: np.ndarray, h: float, hbar: float, T: int,
          ft_mode: str = "nu", ftilde: Optional[float] = None,
          method: str = "fft", nthreads: int = 0, want_terms: bool = False,
          src_s: Optional[np.ndarray] = None):
    """Full T-term solve.  Returns dict(S, phi, terms?, info).  src_s: values
    of S at the sources (default 0)."""
    lib = _load()
    f = np.ascontiguousarray(np.asarray(f, np.float64))
    src = np.ascontiguousarray(np.asarray(src, np.int32))
    p = _problem(f, h, hbar, T, ft_mode, ftilde, method, nthreads, src_s)
    S = np.empty_like(f)
    phi = np.empty_like(f)
    terms = np.empty((int(T) + 1,) + f.shape, np.float64) if want_terms else None
    info = np.zeros(8, np.float64)
    rc = lib.orc_solve(C.byref(p), _dp(f), len(src), _ip(src), _dp(S), _dp(phi),
                       _dp(terms) if terms is not None else None, _dp(info))
    _check(rc, "solve")
    out = {"S": S, "phi": phi, "info": _info(info)}
    if terms is not None:
        out["terms"] = terms
    return out


def solve_logdirect(f: np.ndarray, src: np.ndarray, h: float, hbar: float, T: int,
                    nthreads: int = 0, src_s: Optional[np.ndarray] = None):
    """The T-term series with ftilde = sup f by direct sums in the log
    domain (every term is non-negative then): S with full relative accuracy
    at any distance from the sources, where phi underflows double precision.
    O(N^2) per term.  Returns dict(S, logphi, info)."""
    lib = _load()
    f = np.ascontiguousarray(np.asarray(f, np.float64))
    src = np.ascontiguousarray(np.asarray(src, np.int32))
    p = _problem(f, h, hbar, T, "fmax", None, "direct", nthreads, src_s)
    S = np.empty_like(f)
    lphi = np.empty_like(f)
    info = np.zeros(8, np.float64)
    _check(lib.orc_solve_logdirect(C.byref(p), _dp(f), len(src), _ip(src), _dp(S), _dp(lphi),
                                   _dp(info)), "solve_logdirect")
    return {"S": S, "logphi": lphi, "info": _info(info)}


def log_kappa(dims, beta: float) -> np.ndarray:
    """ln kappa on the orthant 0 <= m_d < n_d."""
    lib = _load()
    out = np.empty(tuple(dims), np.float64)
    _check(lib.orc_log_kappa(len(dims), _dims(dims), float(beta), _dp(out)), "log_kappa")
    return out


def adjoint(f: np.ndarray, src: np.ndarray, h: float, hbar: float, T: int,
            dLdS: np.ndarray, ft_mode: str = "nu", ftilde: Optional[float] = None,
            method: str = "fft", nthreads: int = 0):
    """dL/df of a loss L(S) given dL/dS, with ftilde held fixed."""
    lib = _load()
    f = np.ascontiguousarray(np.asarray(f, np.float64))
    src = np.ascontiguousarray(np.asarray(src, np.int32))
    g = np.ascontiguousarray(np.asarray(dLdS, np.float64))
    p = _problem(f, h, hbar, T, ft_mode, ftilde, method, nthreads)
    out = np.empty_like(f)
    info = np.zeros(8, np.float64)
    rc = lib.orc_adjoint(C.byref(p), _dp(f), len(src), _ip(src), _dp(g),
                         _dp(out), _dp(info))
    _check(rc, "adjoint")
    return out, _info(info)


def dense_limit(f: np.ndarray, src: np.ndarray, h: float, hbar: float,
                ft_mode: str = "nu", ftilde: Optional[float] = None):
    """Limit of the series, phi_inf = (I + K diag(gamma))^-1 phi_0, by a dense
    LU solve (eq. phiandphi_0Equation with the discrete operator).  Tiny grids
    only (N <= ~2000).  Returns (phi_inf, phi_0, K, gamma)."""
    f = np.asarray(f, np.float64)
    dims = f.shape
    lo, hi = float(f.min()), float(f.max())
    ft = {"nu": np.sqrt(0.5 * (lo * lo + hi * hi)), "fmax": hi,
          "given": ftilde}[ft_mode]
    beta = ft * h / hbar
    kap = kappa(dims, beta)
    idx = np.stack(np.unravel_index(np.arange(f.size), dims), axis=1)
    diff = np.abs(idx[:, None, :] - idx[None, :, :])
    K = kap[tuple(diff[..., d] for d in range(len(dims)))]
    gam = (f * f / (ft * ft) - 1.0).ravel()
    p0 = phi0(dims, beta, src).ravel()
    A = np.eye(f.size) + K * gam[None, :]
    return np.linalg.solve(A, p0).reshape(dims), p0.reshape(dims), K, gam.reshape(dims)
