"""CPU checks of the C ABI: the library loads, exports every symbol that
include/sweik.h declares, and rejects invalid arguments on the host before
any HIP call (plan creation and source checks make no device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from common import ROOT, ensure_built

HEADER = os.path.join(ROOT, "include", "sweik.h")


@pytest.fixture(scope="module")
def lib():
    ensure_built()
    import paper_1403_1937_amd as pk
    return pk.load_library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sweik_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_abi_version(lib):
    assert lib.sweik_abi_version() == 1
    assert lib.sweik_status_string(1) == b"invalid argument"


def _plan(**kw):
    from paper_1403_1937_amd import Plan
    args = dict(dims=(64, 64), h=1 / 64, hbar=0.05, T=4, n_src=1)
    args.update(kw)
    return Plan(**args)


@pytest.mark.parametrize("bad", [
    dict(dims=(1, 64)), dict(dims=(64, 0)), dict(h=0.0), dict(h=-1.0), dict(hbar=0.0),
    dict(hbar=float("nan")), dict(T=-1), dict(T=65), dict(n_src=0),
    dict(ftilde_mode="given", ftilde=0.0), dict(ftilde_mode="given", ftilde=-2.0),
])
def test_plan_rejects_invalid(lib, bad):
    with pytest.raises(ValueError):
        _plan(**bad)


def test_plan_rejects_unknown_modes(lib):
    with pytest.raises(ValueError):
        _plan(precision="fp16")
    with pytest.raises(ValueError):
        _plan(ftilde_mode="mean")


def test_unsupported_sizes(lib):
    with pytest.raises(ValueError, match="unsupported"):
        _plan(dims=(4097, 64))      # column FFT length 16384
    _plan(dims=(4096, 64), precision="fp64")  # float64 column FFT length 8192
    with pytest.raises(ValueError, match="unsupported"):
        _plan(dims=(64, 8193))      # row FFT length 32768
    _plan(dims=(4096, 8192))        # largest 2D grid (float32)
    _plan(dims=(4096, 8192), precision="fp64")  # largest float64 grid
    with pytest.raises(ValueError, match="unsupported"):
        _plan(dims=(64, 8193), precision="fp64")  # float64 row FFT length 32768
    wide = _plan(dims=(40, 5000))   # 8192-point complex rows: radix 16 only
    assert wide.schedule["row_e"] == 16
    with pytest.raises(ValueError, match="unsupported"):
        wide.set_schedule(8, 16)
    for prec in ("fp32", "fp64"):
        _plan(dims=(1024, 1024, 1024), precision=prec)  # largest 3D grid
        with pytest.raises(ValueError, match="unsupported"):
            _plan(dims=(1025, 8, 8), precision=prec)


def test_workspace_sizes_scale_with_grid(lib):
    a = _plan(dims=(256, 256))
    b = _plan(dims=(512, 512))
    assert b.workspace_bytes > 3.5 * a.workspace_bytes
    c = _plan(dims=(256, 256), precision="fp64")
    assert c.workspace_bytes > a.workspace_bytes
    assert a.padded == (512, 512)
    assert _plan(dims=(100, 7)).padded == (256, 64)
    # checkpoint: T float terms + float64 phi
    assert a.checkpoint_bytes >= 256 * 256 * (4 * 4 + 8)


def test_source_checks(lib):
    p = _plan(n_src=2)
    p.check_sources(np.array([[0, 0], [63, 63]]))
    with pytest.raises(ValueError):
        p.check_sources(np.array([[0, 0], [64, 3]]))
    with pytest.raises(ValueError):
        p.check_sources(np.array([[0, -1], [3, 3]]))
    with pytest.raises(ValueError):
        p.check_sources(np.array([[5, 5], [5, 5]]))
    with pytest.raises(ValueError):
        p.check_sources(np.array([[5, 5]]))


def test_solve_rejects_null_and_small_workspace(lib):
    p = _plan()
    vp = C.c_void_p
    rc = lib.sweik_solve(p.handle, None, None, None, None, 0, None, None, None)
    assert rc == 1
    rc = lib.sweik_solve(p.handle, vp(16), vp(16), vp(16), vp(16), 10, None, None, None)
    assert rc == 3


def test_batch_create_checks_and_layout(lib):
    from paper_1403_1937_amd import Batch
    base = {"dims": (64, 64), "h": 1 / 64, "hbar": 0.1, "T": 4, "n_src": 1}
    with pytest.raises(ValueError):
        Batch([], "fp32", prepare=False)
    with pytest.raises(ValueError):
        Batch([base, dict(base, T=5)], "fp32", prepare=False)          # T must agree
    with pytest.raises(ValueError):
        Batch([base, dict(base, dims=(8, 8, 8))], "fp32", prepare=False)  # 2D only
    with pytest.raises(ValueError):
        Batch([base, dict(base, hbar=-1.0)], "fp32", prepare=False)
    probs = [base, dict(base, dims=(100, 76)), dict(base, dims=(7, 300)), base]
    b = Batch(probs, "fp32", prepare=False)
    singles = sum(_plan(dims=q["dims"], T=4).workspace_bytes for q in probs)
    # per-instance regions plus the work lists at the head
    assert singles < b.workspace_bytes < singles + 64 * 1024


def test_tall_grids(lib):
    # n0 up to 4096 takes 8192-point columns (radix 16 only), in both precisions
    p = _plan(dims=(3000, 40))
    assert p.padded == (8192, 128)
    assert p.schedule["col_e"] == 16
    with pytest.raises(ValueError, match="unsupported"):
        p.set_schedule(16, 8)
    p.set_schedule(8, 16)
    q = _plan(dims=(3000, 40), precision="fp64")
    assert q.schedule["col_e"] == 16
    with pytest.raises(ValueError, match="unsupported"):
        q.set_schedule(16, 8)
    with pytest.raises(ValueError, match="unsupported"):
        _plan(dims=(4097, 40))


def test_phi0_route_defaults_and_checks(lib):
    few = _plan(n_src=8)
    assert few.schedule["phi0_fft"] == 0
    many = _plan(n_src=100)
    assert many.schedule["phi0_fft"] == 1
    many.set_schedule(16, 16, phi0_fft=0)
    assert many.schedule["phi0_fft"] == 0
    with pytest.raises(ValueError):
        many.set_schedule(16, 16, phi0_fft=2)
    # 3D: the measured crossovers, 128 sources in float32 and 32 in float64
    cube = _plan(dims=(16, 16, 16), n_src=200)
    assert cube.schedule["phi0_fft"] == 1
    cube.set_schedule(16, 16, phi0_fft=0)
    assert cube.schedule["phi0_fft"] == 0
    assert _plan(dims=(16, 16, 16), n_src=100).schedule["phi0_fft"] == 0
    assert _plan(dims=(16, 16, 16), n_src=40, precision="fp64").schedule["phi0_fft"] == 1
    assert _plan(dims=(16, 16, 16), n_src=32, precision="fp64").schedule["phi0_fft"] == 0
    with pytest.raises(ValueError, match="unsupported"):
        cube.set_schedule(8, 16, phi0_fft=1)


def test_backtrack_rejects_invalid_arguments(lib):
    # every argument error returns SWEIK_EINVAL before any HIP call; a
    # zero-path call is a no-op
    vp = C.c_void_p
    dims = (C.c_int64 * 3)(64, 64, 0)
    ok = dict(ndim=2, dims=dims, prec=0, S=vp(16), src=vp(16), n_src=1, start=vp(16),
              n_paths=4, max_steps=10, step=0.5, radius=1.0, path=vp(16), n_points=vp(16),
              status=vp(16), stream=None)

    def call(**kw):
        a = dict(ok, **kw)
        return lib.sweik_backtrack(a["ndim"], a["dims"], a["prec"], a["S"], a["src"], a["n_src"],
                                   a["start"], a["n_paths"], a["max_steps"], a["step"],
                                   a["radius"], a["path"], a["n_points"], a["status"],
                                   a["stream"])
    bad = [dict(ndim=1), dict(ndim=4), dict(dims=None), dict(prec=7),
           dict(dims=(C.c_int64 * 3)(1, 64, 0)), dict(n_src=-1), dict(n_paths=-1),
           dict(max_steps=-1), dict(max_steps=(1 << 20) + 1), dict(step=0.0),
           dict(step=float("nan")), dict(radius=-1.0), dict(radius=float("inf")),
           dict(S=None), dict(src=None), dict(start=None), dict(path=None),
           dict(n_points=None), dict(status=None)]
    for kw in bad:
        assert call(**kw) == 1, kw
    assert call(n_paths=0, S=None, start=None, path=None) == 0


def test_full_gradient_entry_checks(lib):
    # host-side rejections before any device call; the full gradient needs
    # more workspace than a solve (a second spectrum and partial sums)
    p = _plan()
    vp = C.c_void_p
    assert lib.sweik_adjoint_full_workspace_bytes(p.handle) > lib.sweik_workspace_bytes(p.handle)
    rc = lib.sweik_solve_adjoint_full(p.handle, None, None, None, None, None, None, None, None,
                                      0, None)
    assert rc == 1
    need = lib.sweik_adjoint_full_workspace_bytes(p.handle)
    rc = lib.sweik_solve_adjoint_full(p.handle, vp(16), vp(16), None, vp(16), vp(16), vp(16),
                                      None, vp(16), need - 1, None)
    assert rc == 3  # SWEIK_EWORKSPACE
    # 3D: the kernel's beta-derivative spectrum and a second x-pass spectrum
    # come after the solve's workspace as well
    p3 = _plan(dims=(20, 18, 22), T=4)
    need3 = lib.sweik_adjoint_full_workspace_bytes(p3.handle)
    assert need3 > lib.sweik_workspace_bytes(p3.handle)
    rc = lib.sweik_solve_adjoint_full(p3.handle, vp(16), vp(16), None, vp(16), vp(16), vp(16),
                                      None, vp(16), need3 - 1, None)
    assert rc == 3


def test_batch_solve_before_prepare_is_rejected(lib):
    # a batch that was only created (host only) has no streams or staging:
    # its solves return SWEIK_EINVAL before any HIP call
    from paper_1403_1937_amd import Batch
    base = {"dims": (64, 64), "h": 1 / 64, "hbar": 0.1, "T": 4, "n_src": 1}
    b = Batch([base, dict(base, dims=(40, 90))], "fp32", prepare=False)
    vp = C.c_void_p
    P = vp * 2
    ptrs = P(vp(256), vp(512))
    for fn in (lib.sweik_batch_solve, lib.sweik_batch_solve_graph):
        assert fn(b._h, ptrs, ptrs, ptrs, vp(4096), b.workspace_bytes, None, None) == 1
    assert lib.sweik_batch_prepare(None) == 1


def test_noalloc_entry_checks(lib):
    # argument errors and plans larger than the static array are rejected
    # before any HIP call
    vp = C.c_void_p
    small = _plan()
    assert lib.sweik_noalloc_scratch_bytes() == 64 << 20
    assert lib.sweik_solve_noalloc(small.handle, None, vp(16), vp(16), None, None) == 1
    assert lib.sweik_solve_noalloc(None, vp(16), vp(16), vp(16), None, None) == 1
    big = _plan(dims=(1024, 1024), T=16, n_src=16)
    assert big.workspace_bytes > lib.sweik_noalloc_scratch_bytes()
    assert lib.sweik_solve_noalloc(big.handle, vp(16), vp(16), vp(16), None, None) == 3


def test_host_only_calls_create_no_hip_resource(lib):
    # plans, batches and argument checks make no HIP call
    from paper_1403_1937_amd import Batch
    n = lib.sweik_resource_count()
    _plan()
    Batch([{"dims": (64, 64), "h": 1 / 64, "hbar": 0.1, "T": 4, "n_src": 1}], "fp32",
          prepare=False)
    assert lib.sweik_resource_count() == n


def test_tilted_entry_checks(lib):
    # argument errors return before any HIP call; 3D is unsupported
    vp = C.c_void_p
    p = _plan(T=4)
    need = lib.sweik_tilted_workspace_bytes(p.handle, 1)
    assert need > lib.sweik_workspace_bytes(p.handle)
    # one slice per tilt: the workspace grows linearly with the tilt count
    w2, w9 = (lib.sweik_tilted_workspace_bytes(p.handle, n) for n in (2, 9))
    assert need < w2 < w9
    assert abs((w9 - w2) - 7 * (w2 - need)) <= 4096  # up to the alignment of the work lists
    assert lib.sweik_tilted_workspace_bytes(p.handle, 0) == 0
    assert lib.sweik_tilted_workspace_bytes(p.handle, 65) == 0
    D = C.POINTER(C.c_double)

    def call(tilts, n=None, ws_bytes=None, plan=p):
        t = np.ascontiguousarray(np.asarray(tilts, np.float64).reshape(-1, 2))
        return lib.sweik_solve_tilted(plan.handle, vp(16), vp(16), None, vp(16),
                                      t.ctypes.data_as(D), len(t) if n is None else n, 0, vp(16),
                                      need if ws_bytes is None else ws_bytes, None, None)
    assert call([(0.0, 0.0)], n=0) == 1
    assert call([(0.0, 0.0)] * 65) == 1
    assert call([(1.0, 0.0)]) == 1
    assert call([(0.8, 0.7)]) == 1
    assert call([(float("nan"), 0.0)]) == 1
    assert call([(0.0, 0.0)], ws_bytes=need - 1) == 3
    assert lib.sweik_solve_tilted(p.handle, None, vp(16), None, vp(16), None, 1, 0, vp(16), need,
                                  None, None) == 1
    cube = _plan(dims=(16, 16, 16))
    assert lib.sweik_tilted_workspace_bytes(cube.handle, 1) == 0
    assert call([(0.0, 0.0)], plan=cube) == 2
