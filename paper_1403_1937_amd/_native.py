"""ctypes marshalling for libsweik.so (C ABI in include/sweik.h).

Argument conversion only: tensors are passed as device pointers, the stream
as torch's current HIP stream, and status codes become exceptions
(ValueError for argument errors, RuntimeError for device errors).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsweik.so")

MAX_TERMS = 64
STATUS = {0: "ok", 1: "invalid argument", 2: "unsupported problem",
          3: "workspace too small", 4: "HIP error", 5: "out of host memory"}
PREC = {"fp32": 0, "fp64": 1}
FT_MODES = {"nu": 0, "fmax": 1, "given": 2}
INFO_FLAGS = {"f_nonfinite": 1, "f_nonpositive": 2, "c0_ge_1": 4, "bad_source": 8}


class SweikError(RuntimeError):
    pass


class _Problem(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("dims", C.c_int64 * 3), ("h", C.c_double),
                ("hbar", C.c_double), ("T", C.c_int32), ("n_src", C.c_int32),
                ("prec", C.c_int32), ("ft_mode", C.c_int32), ("ftilde", C.c_double)]


class _Schedule(C.Structure):
    _fields_ = [("row_e", C.c_int32), ("col_e", C.c_int32), ("phi0_fft", C.c_int32),
                ("reserved", C.c_int32 * 5)]


class _Info(C.Structure):
    _fields_ = [("f_min", C.c_double), ("f_max", C.c_double), ("ftilde", C.c_double),
                ("beta", C.c_double), ("c0_bound", C.c_double),
                ("n_nonpositive_phi", C.c_int64), ("flags", C.c_int32), ("T", C.c_int32),
                ("scale_exp", C.c_int32 * (MAX_TERMS + 1))]


class _FdInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32),
                ("rel_residual", C.c_double), ("n_nonpositive_phi", C.c_int64),
                ("flags", C.c_int32), ("n_sources", C.c_int32)]


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libsweik.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is not built (run paper_1403_1937_amd/build.py)")
    lib = C.CDLL(_LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    P = C.POINTER(_Problem)
    lib.sweik_plan_create.argtypes = [P, C.POINTER(vp)]
    lib.sweik_plan_destroy.argtypes = [vp]
    lib.sweik_plan_destroy.restype = None
    lib.sweik_workspace_bytes.argtypes = [vp]
    lib.sweik_workspace_bytes.restype = sz
    lib.sweik_checkpoint_bytes.argtypes = [vp]
    lib.sweik_checkpoint_bytes.restype = sz
    lib.sweik_plan_padded_dims.argtypes = [vp, C.POINTER(C.c_int64)]
    lib.sweik_check_sources.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.sweik_solve.argtypes = [vp, vp, vp, vp, vp, sz, vp, vp, vp]
    lib.sweik_solve_seeded.argtypes = [vp, vp, vp, vp, vp, vp, sz, vp, vp, vp]
    lib.sweik_solve_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sweik_tilted_workspace_bytes.argtypes = [vp, C.c_int32]
    lib.sweik_tilted_workspace_bytes.restype = sz
    lib.sweik_solve_tilted.argtypes = [vp, vp, vp, vp, vp, C.POINTER(C.c_double), C.c_int32,
                                       C.c_int32, vp, sz, vp, vp]
    lib.sweik_noalloc_scratch_bytes.restype = sz
    lib.sweik_solve_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.sweik_solve_timed.argtypes = [vp, vp, vp, vp, vp, sz, vp, C.POINTER(C.c_float),
                                      C.POINTER(C.c_int32)]
    lib.sweik_batch_create.argtypes = [P, C.c_int32, C.POINTER(vp)]
    lib.sweik_batch_prepare.argtypes = [vp]
    lib.sweik_batch_destroy.argtypes = [vp]
    lib.sweik_batch_destroy.restype = None
    lib.sweik_resource_count.restype = C.c_int64
    lib.sweik_batch_workspace_bytes.argtypes = [vp]
    lib.sweik_batch_workspace_bytes.restype = sz
    PP = C.POINTER(vp)
    lib.sweik_batch_solve.argtypes = [vp, PP, PP, PP, vp, sz, vp, vp]
    lib.sweik_batch_solve_graph.argtypes = [vp, PP, PP, PP, vp, sz, vp, vp]
    lib.sweik_autotune.argtypes = [vp, vp, sz, vp]
    lib.sweik_plan_get_schedule.argtypes = [vp, C.POINTER(_Schedule)]
    lib.sweik_plan_set_schedule.argtypes = [vp, C.POINTER(_Schedule)]
    lib.sweik_backtrack.argtypes = [C.c_int32, C.POINTER(C.c_int64), C.c_int, vp, vp, C.c_int32,
                                    vp, C.c_int32, C.c_int32, C.c_double, C.c_double, vp, vp,
                                    vp, vp]
    lib.sweik_adjoint_full_workspace_bytes.argtypes = [vp]
    lib.sweik_adjoint_full_workspace_bytes.restype = sz
    lib.sweik_solve_adjoint_full.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    lib.sweik_fd_workspace_bytes.argtypes = [vp]
    lib.sweik_fd_workspace_bytes.restype = sz
    lib.sweik_fd_solve.argtypes = [vp, vp, vp, vp, vp, sz, C.c_int32, C.c_double, vp,
                                   C.POINTER(_FdInfo)]
    lib.sweik_status_string.argtypes = [C.c_int]
    lib.sweik_status_string.restype = C.c_char_p
    lib.sweik_abi_version.restype = C.c_int32
    lib.sweik_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc: int, what: str):
    if rc == 0:
        return
    msg = f"{what}: {STATUS.get(rc, rc)}"
    if rc == 4:
        detail = _lib.sweik_last_error().decode() if _lib is not None else ""
        raise SweikError(f"{msg} ({detail})" if detail else msg)
    raise ValueError(msg)


def _stream_ptr(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _prec_of(dtype) -> str:
    if dtype == torch.float32:
        return "fp32"
    if dtype == torch.float64:
        return "fp64"
    raise ValueError(f"f must be float32 or float64, got {dtype}")


def _info_dict(raw: _Info) -> dict:
    return {"f_min": raw.f_min, "f_max": raw.f_max, "ftilde": raw.ftilde,
            "beta": raw.beta, "c0_bound": raw.c0_bound,
            "n_nonpositive_phi": int(raw.n_nonpositive_phi), "flags": int(raw.flags),
            "T": int(raw.T), "scale_exp": [int(v) for v in raw.scale_exp[: raw.T + 1]]}


def _read_info(buf: torch.Tensor) -> dict:
    host = buf.cpu().numpy().tobytes()
    return _info_dict(_Info.from_buffer_copy(host[: C.sizeof(_Info)]))


class Plan:
    """An immutable solve plan (sweik_plan) for one problem shape."""

    def __init__(self, dims: Sequence[int], h: float, hbar: float, T: int, n_src: int,
                 precision: str = "fp32", ftilde_mode: str = "nu",
                 ftilde: Optional[float] = None):
        lib = load_library()
        p = _Problem()
        p.ndim = len(dims)
        p.dims = (C.c_int64 * 3)(*([int(d) for d in dims] + [1] * (3 - len(dims))))
        p.h, p.hbar, p.T, p.n_src = float(h), float(hbar), int(T), int(n_src)
        if precision not in PREC:
            raise ValueError(f"precision must be one of {list(PREC)}")
        if ftilde_mode not in FT_MODES:
            raise ValueError(f"ftilde_mode must be one of {list(FT_MODES)}")
        p.prec = PREC[precision]
        p.ft_mode = FT_MODES[ftilde_mode]
        p.ftilde = float(ftilde) if ftilde is not None else 0.0
        handle = C.c_void_p()
        _check(lib.sweik_plan_create(C.byref(p), C.byref(handle)), "sweik_plan_create")
        self._lib = lib
        self._h = handle
        self.problem = p
        self.dims = tuple(int(d) for d in dims)
        self.precision = precision
        self.T = int(T)
        self.n_src = int(n_src)
        self.workspace_bytes = int(lib.sweik_workspace_bytes(handle))
        self.checkpoint_bytes = int(lib.sweik_checkpoint_bytes(handle))
        pad = (C.c_int64 * 3)()
        lib.sweik_plan_padded_dims(handle, pad)
        self.padded = tuple(int(v) for v in pad[: len(dims)])

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.sweik_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def check_sources(self, src_host: np.ndarray):
        a = np.ascontiguousarray(np.asarray(src_host, np.int32))
        if a.shape != (self.n_src, len(self.dims)):
            raise ValueError(f"src must have shape ({self.n_src}, {len(self.dims)})")
        _check(self._lib.sweik_check_sources(self._h, a.ctypes.data_as(C.POINTER(C.c_int32))),
               "sources")

    def workspace(self, device) -> torch.Tensor:
        return torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    def checkpoint(self, device) -> torch.Tensor:
        return torch.empty(self.checkpoint_bytes, dtype=torch.uint8, device=device)

    def solve(self, f: torch.Tensor, src: torch.Tensor, S: torch.Tensor, ws: torch.Tensor,
              ckpt: Optional[torch.Tensor] = None, info: Optional[torch.Tensor] = None,
              stream=None, src_s: Optional[torch.Tensor] = None):
        """Enqueue a solve with caller-owned buffers (no allocation).  src_s:
        device values of S at the sources (dtype of f), default 0."""
        if src_s is not None and (src_s.dtype != f.dtype or src_s.numel() != self.n_src
                                  or not src_s.is_contiguous()):
            raise ValueError("src_s must be a contiguous tensor of n_src values of f's dtype")
        _check(self._lib.sweik_solve_seeded(
            self._h, f.data_ptr(), src.data_ptr(),
            src_s.data_ptr() if src_s is not None else None, S.data_ptr(), ws.data_ptr(),
            ws.numel(), ckpt.data_ptr() if ckpt is not None else None,
            _stream_ptr(stream), info.data_ptr() if info is not None else None),
            "sweik_solve")

    def tilted_workspace_bytes(self, n_tilt: int) -> int:
        """Workspace bytes of a tilted solve with n_tilt tilts (0 in 3D)."""
        return int(self._lib.sweik_tilted_workspace_bytes(self._h, int(n_tilt)))

    def solve_tilted(self, f: torch.Tensor, src: torch.Tensor, S: torch.Tensor, ws: torch.Tensor,
                     tilts, info: Optional[torch.Tensor] = None, stream=None,
                     per_source: bool = False, src_s: Optional[torch.Tensor] = None):
        """Enqueue the far-field stabilised solve (sweik_solve_tilted):
        tilts is a host sequence of (tilt0, tilt1) pairs in units of beta;
        per_source splits the solve over the sources; src_s: device values
        of S at the sources (dtype of f); ws must hold
        tilted_workspace_bytes(len(tilts))."""
        if src_s is not None and (src_s.dtype != f.dtype or src_s.numel() != self.n_src
                                  or not src_s.is_contiguous()):
            raise ValueError("src_s must be a contiguous tensor of n_src values of f's dtype")
        t = np.ascontiguousarray(np.asarray(tilts, np.float64).reshape(-1, 2))
        _check(self._lib.sweik_solve_tilted(
            self._h, f.data_ptr(), src.data_ptr(),
            src_s.data_ptr() if src_s is not None else None, S.data_ptr(),
            t.ctypes.data_as(C.POINTER(C.c_double)), len(t), int(bool(per_source)), ws.data_ptr(),
            ws.numel(), _stream_ptr(stream), info.data_ptr() if info is not None else None),
            "sweik_solve_tilted")

    KERNEL_CLASSES = ("prep", "ghat_row", "ghat_col", "phi0_row", "conv_col", "term_row",
                      "last_row", "y_fwd", "y_inv", "ghat_z", "phi0_fft")

    def solve_timed(self, f, src, S, ws, stream=None) -> dict:
        """Solve with HIP events around every kernel (synchronises); returns
        {class: (total ms, launches)}."""
        n = len(self.KERNEL_CLASSES)
        ms = (C.c_float * n)()
        cnt = (C.c_int32 * n)()
        _check(self._lib.sweik_solve_timed(self._h, f.data_ptr(), src.data_ptr(), S.data_ptr(),
                                           ws.data_ptr(), ws.numel(), _stream_ptr(stream), ms,
                                           cnt), "sweik_solve_timed")
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(self.KERNEL_CLASSES)}

    def adjoint(self, f, src, ckpt, dLdS, dLdf, ws, stream=None):
        _check(self._lib.sweik_solve_adjoint(
            self._h, f.data_ptr(), src.data_ptr(), ckpt.data_ptr(), dLdS.data_ptr(),
            dLdf.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)),
            "sweik_solve_adjoint")

    def adjoint_full(self, f, src, ckpt, dLdS, dLdf, grads, ws, src_s=None, stream=None):
        """Full gradient (dLdf with the ftilde path; grads: 4 float64 device
        values dL/dhbar, dL/dftilde, dL/dbeta, 0) into caller buffers; ws
        must hold adjoint_full_workspace_bytes."""
        _check(self._lib.sweik_solve_adjoint_full(
            self._h, f.data_ptr(), src.data_ptr(),
            src_s.data_ptr() if src_s is not None else None, ckpt.data_ptr(), dLdS.data_ptr(),
            dLdf.data_ptr(), grads.data_ptr() if grads is not None else None, ws.data_ptr(),
            ws.numel(), _stream_ptr(stream)), "sweik_solve_adjoint_full")

    @property
    def adjoint_full_workspace_bytes(self) -> int:
        return int(self._lib.sweik_adjoint_full_workspace_bytes(self._h))

    def autotune(self, ws: torch.Tensor, stream=None) -> int:
        """Time the candidate schedules on `ws` (overwritten) and keep the
        fastest; returns the number of schedules timed."""
        n = int(self._lib.sweik_autotune(self._h, ws.data_ptr(), ws.numel(),
                                         _stream_ptr(stream)))
        if n < 0:
            raise SweikError("sweik_autotune failed")
        return n

    @property
    def schedule(self) -> dict:
        sc = _Schedule()
        _check(self._lib.sweik_plan_get_schedule(self._h, C.byref(sc)), "schedule")
        return {"row_e": int(sc.row_e), "col_e": int(sc.col_e), "phi0_fft": int(sc.phi0_fft)}

    def set_schedule(self, row_e: int = 16, col_e: int = 16, phi0_fft: Optional[int] = None):
        """Set the schedule; phi0_fft None keeps the plan's phi_0 route."""
        sc = _Schedule()
        sc.row_e, sc.col_e = int(row_e), int(col_e)
        sc.phi0_fft = self.schedule["phi0_fft"] if phi0_fft is None else int(phi0_fft)
        _check(self._lib.sweik_plan_set_schedule(self._h, C.byref(sc)), "set_schedule")


_plan_cache: Dict[Tuple, Plan] = {}


def _plan_for(f: torch.Tensor, n_src: int, h, hbar, T, ftilde_mode, ftilde) -> Plan:
    key = (tuple(f.shape), float(h), float(hbar), int(T), int(n_src), _prec_of(f.dtype),
           ftilde_mode, None if ftilde is None else float(ftilde))
    pl = _plan_cache.get(key)
    if pl is None:
        pl = Plan(f.shape, h, hbar, T, n_src, _prec_of(f.dtype), ftilde_mode, ftilde)
        _plan_cache[key] = pl
    return pl


def _src_to_device(src, plan: Plan, device) -> torch.Tensor:
    if isinstance(src, torch.Tensor):
        host = src.detach().cpu().numpy()
    else:
        host = np.asarray(src)
    plan.check_sources(host)
    return torch.as_tensor(np.ascontiguousarray(host.astype(np.int32)), device=device)


def _check_f(f: torch.Tensor):
    if not isinstance(f, torch.Tensor) or not f.is_cuda:
        raise ValueError("f must be a CUDA (HIP) tensor")
    if not f.is_contiguous():
        raise ValueError("f must be contiguous")


def solve(f: torch.Tensor, src, h: float, hbar: float, T: int, ftilde_mode: str = "nu",
          ftilde: Optional[float] = None, return_info: bool = False, stream=None,
          src_s=None):
    """S = -hbar ln phi of the T-term series for forcing f (float32 or
    float64 CUDA tensor, 2D or 3D) and point sources src (int [n_src, ndim])
    with values src_s there (default 0)."""
    _check_f(f)
    n_src = len(src)
    pl = _plan_for(f, n_src, h, hbar, T, ftilde_mode, ftilde)
    d_src = _src_to_device(src, pl, f.device)
    d_s = None
    if src_s is not None:
        d_s = torch.as_tensor(np.asarray(src_s, np.float64)).to(f.device, f.dtype).contiguous()
    S = torch.empty_like(f)
    ws = pl.workspace(f.device)
    info = torch.zeros(C.sizeof(_Info), dtype=torch.uint8, device=f.device) if return_info else None
    pl.solve(f, d_src, S, ws, None, info, stream, src_s=d_s)
    if return_info:
        return S, _read_info(info)
    return S


def default_tilts(directions: int = 8, strength: float = 0.9):
    """The plain solve (0, 0) and `directions` tilts of the given strength
    (a fraction of beta) evenly spaced in angle."""
    th = 2.0 * np.pi * np.arange(directions) / directions
    return [(0.0, 0.0)] + [(strength * np.cos(a), strength * np.sin(a)) for a in th]


def solve_tilted(f: torch.Tensor, src, h: float, hbar: float, T: int, tilts=None,
                 ftilde_mode: str = "nu", ftilde: Optional[float] = None,
                 return_info: bool = False, stream=None, per_source: bool = False,
                 src_s=None):
    """Far-field stabilised S (2D): the series solved once per tilt, each
    point from the best-conditioned tilt (sweik_solve_tilted).  tilts:
    (tilt0, tilt1) pairs in units of beta, default default_tilts();
    per_source: one tilted solve per source, summed (n_src times the cost);
    src_s: values of S at the sources (default 0)."""
    _check_f(f)
    pl = _plan_for(f, len(src), h, hbar, T, ftilde_mode, ftilde)
    d_src = _src_to_device(src, pl, f.device)
    S = torch.empty_like(f)
    tilts = default_tilts() if tilts is None else tilts
    ws = torch.empty(pl.tilted_workspace_bytes(len(tilts)), dtype=torch.uint8, device=f.device)
    info = torch.zeros(C.sizeof(_Info), dtype=torch.uint8, device=f.device) if return_info else None
    d_s = None
    if src_s is not None:
        d_s = torch.as_tensor(np.asarray(src_s, np.float64)).to(f.device, f.dtype).contiguous()
    pl.solve_tilted(f, d_src, S, ws, tilts, info, stream, per_source=per_source, src_s=d_s)
    if return_info:
        return S, _read_info(info)
    return S


def fd_solve(f: torch.Tensor, src, h: float, hbar: float, max_iter: int = 50000,
             rtol: float = 1e-12, return_info: bool = False, stream=None):
    """The paper's second method (Section 6): S = -hbar ln phi with phi from
    the finite-difference screened Poisson system (eq. sparse-system), solved
    by diagonally preconditioned conjugate gradients on the GPU in float64.
    Synchronises the stream.  With return_info, also a dict with the
    iteration count, convergence and the final relative residual."""
    lib = load_library()
    _check_f(f)
    n_src = len(src)
    pl = _plan_for(f, n_src, h, hbar, 0, "nu", None)
    d_src = _src_to_device(src, pl, f.device)
    S = torch.empty_like(f)
    nb = int(lib.sweik_fd_workspace_bytes(pl.handle))
    ws = torch.empty(nb, dtype=torch.uint8, device=f.device)
    info = _FdInfo()
    rc = lib.sweik_fd_solve(pl.handle, f.data_ptr(), d_src.data_ptr(), S.data_ptr(),
                            ws.data_ptr(), nb, int(max_iter), float(rtol), _stream_ptr(stream),
                            C.byref(info))
    _check(rc, "sweik_fd_solve")
    if return_info:
        return S, {k: getattr(info, k) for k, _ in _FdInfo._fields_}
    return S


TRACE_STATUS = {0: "reached a source", 1: "max_steps", 2: "no gradient", 3: "start outside"}


def backtrack(S: torch.Tensor, src, start, step: float = 0.5, radius: float = 1.0,
              max_steps: int = 4096, stream=None):
    """Paths of steepest descent on S (Section 6, path planning) from each
    start point (grid coordinates, [n_paths, ndim]) to the sources (int
    [n_src, ndim]).  Returns (path [n_paths, max_steps+1, ndim] float64,
    n_points [n_paths] int32, status [n_paths] int32) on S's device; path p
    holds n_points[p] valid points (status codes: TRACE_STATUS)."""
    lib = load_library()
    _check_f(S)
    if S.dtype not in (torch.float32, torch.float64):
        raise ValueError("S must be float32 or float64")
    dev = S.device
    ndim = S.dim()
    d_src = torch.as_tensor(np.ascontiguousarray(np.asarray(src, np.int32).reshape(-1, ndim))).to(dev)
    d_start = torch.as_tensor(np.asarray(start, np.float64).reshape(-1, ndim)).to(dev).contiguous()
    n_paths = d_start.shape[0]
    path = torch.empty((n_paths, max_steps + 1, ndim), dtype=torch.float64, device=dev)
    n_points = torch.empty(n_paths, dtype=torch.int32, device=dev)
    status = torch.empty(n_paths, dtype=torch.int32, device=dev)
    dims = (C.c_int64 * 3)(*S.shape, *([0] * (3 - ndim)))
    prec = 1 if S.dtype == torch.float64 else 0
    rc = lib.sweik_backtrack(ndim, dims, prec, S.data_ptr(), d_src.data_ptr(), d_src.shape[0],
                             d_start.data_ptr(), n_paths, int(max_steps), float(step),
                             float(radius), path.data_ptr(), n_points.data_ptr(),
                             status.data_ptr(), _stream_ptr(stream))
    _check(rc, "sweik_backtrack")
    return path, n_points, status


def solve_with_checkpoint(f: torch.Tensor, src, h, hbar, T, ftilde_mode="nu", ftilde=None,
                          stream=None):
    """Forward solve that keeps what the adjoint needs.  Returns (S, ckpt,
    plan, d_src, ws, info_tensor)."""
    _check_f(f)
    pl = _plan_for(f, len(src), h, hbar, T, ftilde_mode, ftilde)
    d_src = _src_to_device(src, pl, f.device)
    S = torch.empty_like(f)
    ws = pl.workspace(f.device)
    ck = pl.checkpoint(f.device)
    info = torch.zeros(C.sizeof(_Info), dtype=torch.uint8, device=f.device)
    pl.solve(f, d_src, S, ws, ck, info, stream)
    return S, ck, pl, d_src, ws, info


def solve_adjoint(f: torch.Tensor, src, h, hbar, T, dLdS: torch.Tensor, ftilde_mode="nu",
                  ftilde=None, stream=None):
    """dL/df (ftilde held fixed) for a loss with gradient dLdS w.r.t. S."""
    S, ck, pl, d_src, ws, _ = solve_with_checkpoint(f, src, h, hbar, T, ftilde_mode, ftilde,
                                                    stream)
    g = torch.empty_like(f)
    pl.adjoint(f, d_src, ck, dLdS.contiguous(), g, ws, stream)
    return g


def solve_gradient(f: torch.Tensor, src, h, hbar, T, dLdS: torch.Tensor, ftilde_mode="nu",
                   ftilde=None, src_s=None, stream=None):
    """Full gradient of a loss with gradient dLdS w.r.t. S (2D or 3D): returns
    (dL/df including the dependence of ftilde on f, {"dLdhbar", "dLdftilde",
    "dLdbeta"}).  src_s: values of S at the sources (default 0)."""
    _check_f(f)
    pl = _plan_for(f, len(src), h, hbar, T, ftilde_mode, ftilde)
    d_src = _src_to_device(src, pl, f.device)
    d_s = None
    if src_s is not None:
        d_s = torch.as_tensor(np.asarray(src_s, np.float64)).to(f.device, f.dtype).contiguous()
    S = torch.empty_like(f)
    ws = torch.empty(pl.adjoint_full_workspace_bytes, dtype=torch.uint8, device=f.device)
    ck = pl.checkpoint(f.device)
    pl.solve(f, d_src, S, ws, ck, None, stream, src_s=d_s)
    g = torch.empty_like(f)
    grads = torch.zeros(4, dtype=torch.float64, device=f.device)
    pl.adjoint_full(f, d_src, ck, dLdS.contiguous(), g, grads, ws, d_s, stream)
    v = grads.cpu().tolist()
    return g, {"dLdhbar": v[0], "dLdftilde": v[1], "dLdbeta": v[2]}


class EikonalFn(torch.autograd.Function):
    """S = solve(f) with a hand-written adjoint: backward convolves back
    through the same (even) Green's kernel using the checkpointed terms."""

    @staticmethod
    def forward(ctx, f, src, h, hbar, T, ftilde_mode="nu", ftilde=None):
        S, ck, pl, d_src, ws, _ = solve_with_checkpoint(f.detach().contiguous(), src, h, hbar,
                                                        T, ftilde_mode, ftilde)
        ctx.plan, ctx.d_src, ctx.ck, ctx.ws = pl, d_src, ck, ws
        ctx.save_for_backward(f)
        return S

    @staticmethod
    def backward(ctx, gS):
        (f,) = ctx.saved_tensors
        g = torch.empty_like(f)
        ctx.plan.adjoint(f.detach().contiguous(), ctx.d_src, ctx.ck, gS.contiguous(), g,
                         ctx.ws)
        return g, None, None, None, None, None, None


def eikonal(f, src, h, hbar, T, ftilde_mode="nu", ftilde=None):
    return EikonalFn.apply(f, src, h, hbar, T, ftilde_mode, ftilde)


class Batch:
    """Uneven batch of independent 2D problems (sweik_batch)."""

    def __init__(self, problems: Sequence[dict], precision: str = "fp32", prepare: bool = True):
        """prepare=False only validates and lays out the batch (host only):
        such a batch cannot be solved."""
        lib = load_library()
        arr = (_Problem * len(problems))()
        for i, q in enumerate(problems):
            p = arr[i]
            dims = q["dims"]
            p.ndim = len(dims)
            p.dims = (C.c_int64 * 3)(*([int(d) for d in dims] + [1] * (3 - len(dims))))
            p.h, p.hbar, p.T, p.n_src = float(q["h"]), float(q["hbar"]), int(q["T"]), int(q["n_src"])
            p.prec = PREC[precision]
            p.ft_mode = FT_MODES[q.get("ftilde_mode", "nu")]
            p.ftilde = float(q.get("ftilde") or 0.0)
        handle = C.c_void_p()
        _check(lib.sweik_batch_create(arr, len(problems), C.byref(handle)), "sweik_batch_create")
        self._lib, self._h, self.count = lib, handle, len(problems)
        self.workspace_bytes = int(lib.sweik_batch_workspace_bytes(handle))
        # streams, events and pinned staging on the current device, once
        if prepare:
            _check(lib.sweik_batch_prepare(handle), "sweik_batch_prepare")

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.sweik_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def _ptrs(self, ts):
        return (C.c_void_p * len(ts))(*[t.data_ptr() for t in ts])

    def solve(self, fs, srcs, Ss, ws, infos: Optional[torch.Tensor] = None, graph=False,
              stream=None):
        fn = self._lib.sweik_batch_solve_graph if graph else self._lib.sweik_batch_solve
        _check(fn(self._h, self._ptrs(fs), self._ptrs(srcs), self._ptrs(Ss), ws.data_ptr(),
                  ws.numel(), _stream_ptr(stream),
                  infos.data_ptr() if infos is not None else None), "sweik_batch_solve")


def batch_solve(fs: Sequence[torch.Tensor], srcs, hs, hbars, T: int, graph: bool = False):
    probs = [{"dims": tuple(f.shape), "h": h, "hbar": hb, "T": T, "n_src": len(s)}
             for f, s, h, hb in zip(fs, srcs, hs, hbars)]
    prec = _prec_of(fs[0].dtype)
    b = Batch(probs, prec)
    d_srcs = [torch.as_tensor(np.ascontiguousarray(np.asarray(
        s.cpu() if isinstance(s, torch.Tensor) else s, np.int32)), device=fs[0].device)
        for s in srcs]
    Ss = [torch.empty_like(f) for f in fs]
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device=fs[0].device)
    b.solve(fs, d_srcs, Ss, ws, graph=graph)
    return Ss


def resource_count() -> int:
    """HIP resources the library has created so far in this process."""
    return int(load_library().sweik_resource_count())


def info_struct_size() -> int:
    return C.sizeof(_Info)
