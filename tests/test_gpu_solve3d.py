"""GPU parity of the 3D forward solve against the FP64 CPU oracle.

The 3D path uses an odd-frequency real transform along the last axis and
full transforms along the other two; the oracle uses its own complex
radix-2 FFT over the whole padded box.  Tolerances are claimed on the
resolvable sets of tests/common.py.

Every compiled line length is compared element by element with the oracle:
thin grids pad one or two axes to 512 or 1024 points (the x pass with 256
or 512 odd-frequency bins, the axis-1 and axis-0 column passes of length
512 and 1024) while the oracle's padded box stays small, and the 256^3
blob workload itself (the benchmark's launch configuration, T = 16) is
solved by the oracle at full size.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from common import (EPS, LAMBDA_MAX, TOL, ensure_built, envelope_violations, rel_err, report,
                    resolvable)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _supported(dims, h, hbar, T, n_src, prec):
    """The planner's decision (host only): False when it rejects the sizes."""
    import paper_1403_1937_amd as pk
    try:
        pk.Plan(dims, h, hbar, T, n_src, prec)
    except ValueError as e:
        if "unsupported" in str(e):
            return False
        raise
    return True


def _run(f32, src, h, hbar, T, prec, ft_mode="nu", ftilde=None):
    import paper_1403_1937_amd as pk
    dt = torch.float32 if prec == "fp32" else torch.float64
    f = torch.as_tensor(f32.astype(np.float64)).to("cuda", dt)
    S, info = pk.solve(f, src, h, hbar, T, ftilde_mode=ft_mode, ftilde=ftilde, return_info=True)
    torch.cuda.synchronize()
    return S.double().cpu().numpy(), info


CASES = [
    # (name, dims, h, hbar, T, n_src, seed)
    ("cube16", (16, 16, 16), 1 / 16, 0.1, 6, 2, 21),
    ("ragged5x6x7", (5, 6, 7), 1 / 7, 0.15, 4, 1, 22),
    ("ragged20x9x33", (20, 9, 33), 1 / 33, 0.08, 5, 3, 23),
    ("full32", (32, 32, 32), 1 / 32, 0.1, 8, 2, 24),
    ("mixed16x48x64", (16, 48, 64), 1 / 64, 0.06, 6, 4, 25),
    ("rect40x33x65", (40, 33, 65), 1 / 65, 0.1, 5, 2, 26),
    # thin grids whose padded lengths reach the benchmark's 512 and the
    # largest supported 1024 along one or two axes
    ("thin130x6x130", (130, 6, 130), 1 / 130, 0.1, 4, 2, 41),
    ("thin6x130x6", (6, 130, 6), 1 / 130, 0.1, 4, 2, 42),
    ("thin300x5x5", (300, 5, 5), 1 / 300, 0.1, 4, 2, 43),
    ("thin5x300x5", (5, 300, 5), 1 / 300, 0.1, 4, 2, 44),
    ("thin5x5x300", (5, 5, 300), 1 / 300, 0.1, 4, 2, 45),
    # padded length 2048 (x pass with 1024 odd-frequency bins, 2048-point
    # column passes): the largest supported axis, 1024
    ("thin600x5x5", (600, 5, 5), 1 / 600, 0.1, 4, 2, 46),
    ("thin5x600x5", (5, 600, 5), 1 / 600, 0.1, 4, 2, 47),
    ("thin5x5x600", (5, 5, 600), 1 / 600, 0.1, 4, 2, 48),
    ("thin1024x4x4", (1024, 4, 4), 1 / 1024, 0.1, 3, 2, 49),
    ("thin4x4x1024", (4, 4, 1024), 1 / 1024, 0.1, 3, 2, 50),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forward_parity_3d(case, prec):
    name, dims, h, hbar, T, n_src, seed = case
    if not _supported(dims, h, hbar, T, n_src, prec):
        pytest.skip(f"{dims} {prec}: padded lengths beyond the planner's limits")
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 3.0, 0.5, 2.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, n_src, rng)
    print(f"case {name} prec {prec} dims {dims}", flush=True)
    S, info = _run(f, src, h, hbar, T, prec)
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    assert info["flags"] == 0
    assert abs(info["ftilde"] - o["info"]["ftilde"]) <= 1e-14 * o["info"]["ftilde"]
    worst, frac, _ = report(S, o, hbar, prec)
    nbad = envelope_violations(S, o, hbar, prec)
    print(f"  max rel on resolvable set {worst:.3e} (fraction {frac:.3f}); "
          f"envelope violations {nbad}", flush=True)
    assert frac > 0.1
    assert worst <= TOL[prec]
    assert nbad == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_blobs_workload_reduced(prec):
    """The 256^3 blob workload's recipe at 48^3 (h = 1/48, hbar = 0.1,
    one source at the centre, T = 16)."""
    p = workloads.problem(3, 48)
    S, info = _run(p.f, p.src, p.h, p.hbar, p.T, prec)
    o = oracle.solve(p.f.astype(np.float64), p.src, p.h, p.hbar, p.T)
    worst, frac, _ = report(S, o, p.hbar, prec)
    print(f"blobs48 {prec}: max rel {worst:.3e} on {frac:.3f}", flush=True)
    assert worst <= TOL[prec]
    assert envelope_violations(S, o, p.hbar, prec) == 0


def _closed_form(dims, src, c, h, hbar):
    g = np.stack(np.meshgrid(*[np.arange(n) for n in dims], indexing="ij"), -1)
    acc = np.zeros(dims)
    for s in src:
        acc += np.exp(-c * np.linalg.norm(g - s, axis=-1) * h / hbar)
    return -hbar * np.log(acc)


def test_constant_forcing_closed_form_3d():
    """f = c => gamma = 0 => phi = phi_0 exactly (eq. phi_0Solution)."""
    dims = (12, 17, 30)
    src = np.array([[1, 2, 3], [10, 15, 20]], np.int32)
    f = np.full(dims, 1.25, np.float32)
    S, info = _run(f, src, 0.05, 0.1, 4, "fp64")
    assert info["c0_bound"] == 0.0
    assert np.max(np.abs(S - _closed_form(dims, src, 1.25, 0.05, 0.1))) < 1e-12


def test_full_size_256_closed_form():
    """At 256^3: the constant-forcing closed form on a sample of points."""
    n = 256
    p = workloads.problem(3, n)
    f = np.full((n, n, n), 1.3, np.float32)
    print("256^3 constant forcing, fp32", flush=True)
    S, info = _run(f, p.src, p.h, p.hbar, 3, "fp32")
    rng = np.random.default_rng(31)
    idx = rng.integers(0, n, (4096, 3))
    d = np.linalg.norm(idx - p.src[0], axis=-1) * p.h
    ref = 1.3 * d  # one source: S = ftilde |x - y|
    got = S[idx[:, 0], idx[:, 1], idx[:, 2]]
    assert np.max(np.abs(got - ref) / np.maximum(ref, p.hbar)) < 1e-5


@pytest.mark.timeout(600)
def test_blobs_workload_full_size_against_oracle():
    """The 256^3 blob workload (h = 1/256, hbar = 0.1, centre source,
    T = 16) in both precisions, element by element over the whole grid
    against the FP64 oracle's full-size solve, in the plan the benchmark
    times."""
    p = workloads.problem(3)
    print("256^3 blobs: oracle solve (T = 16)", flush=True)
    o = oracle.solve(p.f.astype(np.float64), p.src, p.h, p.hbar, p.T)
    for prec in ("fp32", "fp64"):
        print(f"256^3 blobs: GPU {prec}", flush=True)
        S, info = _run(p.f, p.src, p.h, p.hbar, p.T, prec)
        assert info["flags"] == 0
        assert abs(info["ftilde"] - o["info"]["ftilde"]) <= 1e-14 * o["info"]["ftilde"]
        worst, frac, _ = report(S, o, p.hbar, prec)
        nbad = envelope_violations(S, o, p.hbar, prec)
        print(f"  max rel {worst:.3e} on {frac:.3f} of the grid; envelope violations {nbad}; "
              f"+inf {info['n_nonpositive_phi']} (oracle {o['info']['n_nonpositive_phi']})",
              flush=True)
        assert frac > 0.9
        assert worst <= TOL[prec]
        assert nbad == 0
        assert info["n_nonpositive_phi"] == int(np.isinf(S).sum())
        del S


def test_zero_terms_3d():
    rng = np.random.default_rng(32)
    dims = (9, 10, 11)
    f = rng.uniform(1, 2, dims).astype(np.float32)
    src = np.array([[4, 5, 5]], np.int32)
    S, _ = _run(f, src, 0.1, 0.2, 0, "fp64")
    o = oracle.solve(f.astype(np.float64), src, 0.1, 0.2, 0)
    assert np.max(rel_err(S, o["S"], 0.2)) < 1e-13


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_seed_values_parity_3d(prec):
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(82)
    dims, h, hbar, T = (20, 24, 28), 1 / 28, 0.1, 5
    f = workloads.smoothed_noise(dims, 3.0, 0.5, 2.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 3, rng)
    s = rng.uniform(0.0, 0.2, len(src))
    dt = torch.float32 if prec == "fp32" else torch.float64
    S = pk.solve(torch.as_tensor(f.astype(np.float64)).to("cuda", dt), src, h, hbar, T,
                 src_s=s).double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T,
                     src_s=np.asarray(s, np.float32 if prec == "fp32" else np.float64))
    worst, frac, _ = report(S, o, hbar, prec)
    assert frac > 0.1 and worst <= TOL[prec]


def _sphere_sources(dims, count, rng):
    """Distinct grid points near a sphere (a dense seed surface)."""
    c = np.array(dims, np.float64) / 2
    rad = 0.3 * min(dims)
    v = rng.standard_normal((4 * count, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    pts = np.unique(np.round(c + rad * v).astype(np.int32), axis=0)
    return np.ascontiguousarray(pts[rng.permutation(len(pts))[:count]])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("seeded", [False, True], ids=["plain", "seed_values"])
def test_phi0_by_fft_many_sources_3d(prec, seeded):
    """300 sources on a sphere: the 3D plan takes the FFT route of phi_0
    (Table 1 steps 1-5), checked against the oracle's direct sum."""
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(93)
    dims, h, hbar, T = (40, 44, 36), 1 / 44, 0.06, 4
    f = workloads.smoothed_noise(dims, 3.0, 1.0, 2.0, rng).astype(np.float32)
    src = _sphere_sources(dims, 300, rng)
    assert len(src) == 300
    s = rng.uniform(0.0, 0.05, len(src)) if seeded else None
    pl = pk.Plan(dims, h, hbar, T, len(src), prec)
    assert pl.schedule["phi0_fft"] == 1
    dt = torch.float32 if prec == "fp32" else torch.float64
    print(f"3D phi0 by FFT {prec} {'seeded' if seeded else 'plain'}", flush=True)
    S = pk.solve(torch.as_tensor(f.astype(np.float64)).to("cuda", dt), src, h, hbar, T,
                 src_s=s).double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T,
                     src_s=None if s is None else
                     np.asarray(s, np.float32 if prec == "fp32" else np.float64))
    worst, frac, _ = report(S, o, hbar, prec)
    print(f"  max rel {worst:.3e} on {frac:.3f}", flush=True)
    assert frac > 0.1 and worst <= TOL[prec]
    assert envelope_violations(S, o, hbar, prec) == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dims,T", [((20, 9, 33), 5), ((33, 12, 40), 0), ((16, 16, 16), 3)])
def test_phi0_routes_agree_3d(prec, dims, T):
    """Few sources, both routes of phi_0 forced: each against the oracle
    (ragged grids, T = 0 where S comes from phi_0 alone)."""
    import paper_1403_1937_amd as pk
    from paper_1403_1937_amd._native import _read_info, info_struct_size
    rng = np.random.default_rng(94 + T)
    h, hbar = 1 / max(dims), 0.1
    f = workloads.smoothed_noise(dims, 3.0, 1.0, 2.5, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 3, rng)
    dt = torch.float32 if prec == "fp32" else torch.float64
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    for route in (0, 1):
        pl = pk.Plan(dims, h, hbar, T, len(src), prec)
        pl.set_schedule(16, 16, phi0_fft=route)
        ft = torch.as_tensor(f.astype(np.float64)).to("cuda", dt)
        S = torch.empty_like(ft)
        info = torch.zeros(info_struct_size(), dtype=torch.uint8, device="cuda")
        print(f"3D phi0 route {route} {prec} {dims} T={T}", flush=True)
        pl.solve(ft, torch.as_tensor(src).cuda(), S, pl.workspace("cuda"), None, info)
        torch.cuda.synchronize()
        worst, frac, _ = report(S.double().cpu().numpy(), o, hbar, prec)
        print(f"  max rel {worst:.3e} on {frac:.3f}", flush=True)
        assert _read_info(info)["flags"] == 0
        assert frac > 0.1 and worst <= TOL[prec]


def test_full_size_256_phi0_fft_closed_form():
    """At 256^3 with 400 sources on a sphere and constant forcing (phi =
    phi_0): the FFT route of phi_0 against the closed form
    -hbar ln sum_k exp(-c |x - y_k| h / hbar) on a sample of points."""
    import paper_1403_1937_amd as pk
    n, c, hbar, T = 256, 1.3, 0.1, 2
    rng = np.random.default_rng(33)
    src = _sphere_sources((n, n, n), 400, rng)
    f = torch.full((n, n, n), c, dtype=torch.float32, device="cuda")
    pl = pk.Plan((n, n, n), 1 / n, hbar, T, len(src), "fp32")
    assert pl.schedule["phi0_fft"] == 1
    print("256^3 phi0 by FFT, 400 sources, fp32", flush=True)
    S = pk.solve(f, src, 1 / n, hbar, T)
    idx = np.concatenate([rng.integers(0, n, (4096, 3)), src[:64]])
    phi = np.exp(-c * np.linalg.norm(idx[:, None, :] - src[None, :, :], axis=-1) / n / hbar)
    phi = phi.sum(axis=1)
    ref = -hbar * np.log(phi)
    got = S[tuple(torch.as_tensor(idx.T).cuda().long())].double().cpu().numpy()
    err = np.abs(got - ref) / np.maximum(np.abs(ref), hbar)
    # Lambda against the largest phi of the sample (sources included): the
    # FP32 tolerance on the resolvable set, the conditioning envelope beyond
    L = np.log(phi.max() / phi)
    m = L <= LAMBDA_MAX["fp32"]
    print(f"  max rel {err[m].max():.3e} on {m.mean():.3f} of the sample (Lambda up to "
          f"{L.max():.1f})", flush=True)
    assert m.mean() > 0.5 and err[m].max() <= TOL["fp32"]
    env = TOL["fp32"] + EPS["fp32"] * np.exp(L) / np.maximum(L, 1.0)
    assert np.all(err <= env)
