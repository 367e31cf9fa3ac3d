"""GPU parity of the 2D forward solve against the FP64 CPU oracle.

Inputs are seeded synthetic fields from `workloads`; the oracle runs the
same algorithm (Table 1) with its own FFT.  Tolerances are claimed on the
resolvable sets described in tests/common.py.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from common import (LAMBDA_ENVELOPE, LAMBDA_MAX, TOL, ensure_built, envelope_violations, lam,
                    rel_err, report, resolvable)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(f32, src, h, hbar, T, prec, ft_mode="nu", ftilde=None):
    import paper_1403_1937_amd as pk
    dt = torch.float32 if prec == "fp32" else torch.float64
    f = torch.as_tensor(f32.astype(np.float32 if prec == "fp32" else np.float64)).to("cuda", dt)
    S, info = pk.solve(f, src, h, hbar, T, ftilde_mode=ft_mode, ftilde=ftilde, return_info=True)
    torch.cuda.synchronize()
    return S.double().cpu().numpy(), info


def _oracle(f32, src, h, hbar, T, ft_mode="nu", ftilde=None):
    return oracle.solve(f32.astype(np.float64), src, h, hbar, T, ft_mode=ft_mode, ftilde=ftilde)


CASES = [
    # (name, dims, h, hbar, T, n_src, seed)
    ("square64", (64, 64), 1 / 64, 0.05, 8, 3, 1),
    ("ragged100x76", (100, 76), 1 / 100, 0.2, 6, 5, 2),
    ("ragged33x130", (33, 130), 1 / 130, 0.06, 5, 2, 3),
    ("thin7x300", (7, 300), 1 / 300, 0.3, 4, 2, 4),
    ("tall257x20", (257, 20), 1 / 257, 0.25, 4, 2, 5),
    ("square256", (256, 256), 1 / 256, 0.05, 10, 16, 6),
    ("rect200x513", (200, 513), 1 / 513, 0.1, 7, 4, 7),
    ("wide24x3000", (24, 3000), 1 / 3000, 0.3, 4, 2, 8),  # row FFT length 8192
]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forward_parity_2d(case, prec):
    name, dims, h, hbar, T, n_src, seed = case
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, n_src, rng)
    print(f"case {name} prec {prec} dims {dims}", flush=True)
    S, info = _run(f, src, h, hbar, T, prec)
    o = _oracle(f, src, h, hbar, T)
    assert info["flags"] == 0
    assert abs(info["ftilde"] - o["info"]["ftilde"]) <= 1e-14 * o["info"]["ftilde"]
    assert abs(info["beta"] - o["info"]["beta"]) <= 1e-14 * o["info"]["beta"]
    worst, frac, _ = report(S, o, hbar, prec)
    nbad = envelope_violations(S, o, hbar, prec)
    print(f"  max rel on resolvable set {worst:.3e} (fraction {frac:.3f}); "
          f"envelope violations {nbad}", flush=True)
    assert frac > 0.1
    assert worst <= TOL[prec]
    assert nbad == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_workload1_bumps64(prec):
    """64x64, h = 1, hbar = 0.5 (beta ~ 2.6): phi spans ~100 e-folds, so
    the FFT result is only resolvable near the source (Section 5.3)."""
    p = workloads.problem(1)
    S, info = _run(p.f, p.src, p.h, p.hbar, p.T, prec)
    o = _oracle(p.f, p.src, p.h, p.hbar, p.T)
    worst, frac, _ = report(S, o, p.hbar, prec)
    print(f"bumps64 {prec}: max rel {worst:.3e} on {frac:.3f} of grid", flush=True)
    assert worst <= TOL[prec]
    assert envelope_violations(S, o, p.hbar, prec) == 0
    # +inf where phi <= 0 (FFT noise far from the source).  The reported count
    # is the number of +inf points written; no +inf lies where the oracle
    # resolves phi, and every GPU +inf lies where the oracle's phi is
    # non-positive or deep in its noise.
    n_inf = int(np.isinf(S).sum())
    n_o = int(o["info"]["n_nonpositive_phi"])
    print(f"  +inf: GPU {info['n_nonpositive_phi']} ({n_inf} written), oracle {n_o}", flush=True)
    assert info["n_nonpositive_phi"] == n_inf
    L = lam(o["phi"])
    assert not np.isinf(S[L <= LAMBDA_ENVELOPE[prec]]).any()
    assert (L[np.isinf(S)] > {"fp64": 25.0, "fp32": 12.0}[prec]).all()
    # where the oracle's phi <= 0 the GPU value is noise as well: +inf or a
    # Lambda (from the GPU's own S) beyond its resolvable set
    fin = np.isfinite(S)
    lam_gpu = np.full(S.shape, np.inf)
    lam_gpu[fin] = (S[fin] - S[fin].min()) / p.hbar
    assert (lam_gpu[~(o["phi"] > 0)] > LAMBDA_MAX[prec]).all()
    if prec == "fp64":
        # both sides' noise-dominated points take the sign of independent
        # rounding noise, about half of them negative on each side: the
        # counts agree to a few standard deviations (sqrt(n)/2 each)
        assert abs(n_inf - n_o) <= 0.1 * n_o + 50


@pytest.mark.parametrize("ft_mode", ["fmax", "given"])
def test_ftilde_modes(ft_mode):
    rng = np.random.default_rng(9)
    dims = (80, 96)
    f = workloads.smoothed_noise(dims, 5.0, 1.0, 2.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 3, rng)
    ft = 1.77 if ft_mode == "given" else None
    S, info = _run(f, src, 1 / 96, 0.05, 6, "fp64", ft_mode, ft)
    o = _oracle(f, src, 1 / 96, 0.05, 6, ft_mode, ft)
    assert abs(info["ftilde"] - o["info"]["ftilde"]) <= 1e-14
    worst, frac, _ = report(S, o, 0.05, "fp64")
    assert worst <= TOL["fp64"]
    assert envelope_violations(S, o, 0.05, "fp64") == 0


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-13), ("fp32", 1e-5)])
@pytest.mark.parametrize("a", [0.5, 2.5, 10.0, 40.0, 150.0])
def test_kernel_origin_value(a, prec, tol):
    """The kernel's value at the origin, 1 - a K1(a) with a = beta / sqrt(pi)
    (the ball average at the singular point), through a solve that isolates
    it: ftilde given as 1 and f = 1 everywhere except at the single source,
    where gamma = g, so every term at the source is phi_i = (kappa(0) g)^i
    and S there is -hbar ln sum_i (-kappa(0) g)^i.  kappa(0) is the oracle's
    (pinned to scipy); a spans the ascending series (a <= 2) and the
    integral route of K1 above it."""
    dims, y = (7, 7), (3, 3)
    beta = a * np.sqrt(np.pi)
    hbar = 1.0 / beta  # h = 1, ftilde = 1
    f = np.ones(dims)
    f[y] = np.sqrt(1.5)
    if prec == "fp32":  # the solve sees f in float32 and stores gamma in float32
        f[y] = float(np.float32(f[y]))
    g = (f[y] - 1.0) * (f[y] + 1.0)
    if prec == "fp32":
        g = float(np.float32(g))
    T = 6
    k0 = oracle.kappa0(2, beta)
    expect = -hbar * np.log(sum((-k0 * g) ** i for i in range(T + 1)))
    S, info = _run(f, np.array([y], np.int32), 1.0, hbar, T, prec, "given", 1.0)
    assert abs(info["beta"] - beta) <= 1e-14 * beta
    err = abs(S[y] - expect) / hbar
    print(f"a = {a} {prec}: kappa(0) = {k0:.16f}, S at the source {S[y]:.15e}, "
          f"closed form {expect:.15e}, |dS|/hbar {err:.1e}", flush=True)
    assert err <= tol


def test_constant_forcing_closed_form_gpu():
    """f = c => phi = phi_0 exactly: S = -hbar ln sum_k exp(-c|x-y_k|/hbar)."""
    dims = (50, 70)
    f = np.full(dims, 1.5, np.float32)
    src = np.array([[3, 4], [40, 60]], np.int32)
    S, info = _run(f, src, 0.02, 0.05, 5, "fp64")
    g = np.stack(np.meshgrid(np.arange(50), np.arange(70), indexing="ij"), -1)
    d = np.stack([np.linalg.norm(g - s, axis=-1) for s in src]) * 0.02
    ref = -0.05 * np.log(np.exp(-1.5 * d / 0.05).sum(0))
    assert np.max(np.abs(S - ref)) < 1e-12
    assert info["c0_bound"] == 0.0


def test_zero_terms():
    rng = np.random.default_rng(12)
    dims = (40, 40)
    f = rng.uniform(1, 2, dims).astype(np.float32)
    src = np.array([[20, 20]], np.int32)
    S, _ = _run(f, src, 1 / 40, 0.05, 0, "fp64")
    o = _oracle(f, src, 1 / 40, 0.05, 0)
    assert np.max(rel_err(S, o["S"], 0.05)) < 1e-13


def test_scale_exponents_track_decay():
    """With f close to ftilde the terms decay fast; the stored exponents
    must follow so that mantissas stay representable."""
    rng = np.random.default_rng(13)
    dims = (64, 64)
    f = (1.0 + 1e-3 * rng.uniform(0, 1, dims)).astype(np.float32)
    src = np.array([[32, 32]], np.int32)
    S, info = _run(f, src, 1 / 64, 0.05, 30, "fp32")
    o = _oracle(f, src, 1 / 64, 0.05, 30)
    assert info["scale_exp"][-1] < -150  # far below float32's range
    worst, frac, _ = report(S, o, 0.05, "fp32")
    assert worst <= TOL["fp32"]


def _run_sched(f32, src, h, hbar, T, prec, sched):
    """Solve through an explicit plan with schedule (row_e, col_e)."""
    import paper_1403_1937_amd as pk
    from paper_1403_1937_amd._native import _read_info, info_struct_size
    dims = f32.shape
    pl = pk.Plan(dims, h, hbar, T, len(src), prec)
    pl.set_schedule(*sched)
    assert pl.schedule["row_e"] == sched[0] and pl.schedule["col_e"] == sched[1]
    dt = torch.float32 if prec == "fp32" else torch.float64
    f = torch.as_tensor(f32.astype(np.float64)).to("cuda", dt)
    d_src = torch.as_tensor(np.ascontiguousarray(src, np.int32)).to("cuda")
    S = torch.empty_like(f)
    info = torch.zeros(info_struct_size(), dtype=torch.uint8, device="cuda")
    pl.solve(f, d_src, S, pl.workspace("cuda"), None, info)
    torch.cuda.synchronize()
    return S.double().cpu().numpy(), _read_info(info)


SCHED_CASES = [c for c in CASES if c[0] in ("ragged100x76", "tall257x20", "thin7x300",
                                                "square256", "rect200x513")]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("sched", [(8, 8), (16, 8), (8, 16), (4, 4), (4, 16), (16, 4)],
                         ids=["r8c8", "r16c8", "r8c16", "r4c4", "r4c16", "r16c4"])
@pytest.mark.parametrize("case", SCHED_CASES, ids=[c[0] for c in SCHED_CASES])
def test_schedules_parity_2d(case, sched, prec):
    """Radix-8 (512-thread) and radix-4 (1024-thread, float32 only) team
    FFTs, against the oracle."""
    name, dims, h, hbar, T, n_src, seed = case
    if prec == "fp64" and 4 in sched:
        pytest.skip("radix 4 is a float32 schedule")
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, n_src, rng)
    print(f"case {name} sched {sched} prec {prec}", flush=True)
    S, info = _run_sched(f, src, h, hbar, T, prec, sched)
    o = _oracle(f, src, h, hbar, T)
    assert info["flags"] == 0
    worst, frac, _ = report(S, o, hbar, prec)
    print(f"  max rel {worst:.3e} on {frac:.3f}", flush=True)
    assert worst <= TOL[prec]
    assert envelope_violations(S, o, hbar, prec) == 0


def test_autotune_picks_a_schedule_and_stays_correct():
    import paper_1403_1937_amd as pk
    # lengths no other test uses: the tuned entries go to the process table
    dims, h, hbar, T = (150, 2000), 1 / 2000, 0.05, 6
    rng = np.random.default_rng(41)
    f32 = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 3, rng)
    pl = pk.Plan(dims, h, hbar, T, len(src), "fp32")
    ws = pl.workspace("cuda")
    n = pl.autotune(ws)
    print(f"autotune timed {n} schedules -> {pl.schedule}", flush=True)
    assert n == 9
    assert pl.schedule["row_e"] in (4, 8, 16) and pl.schedule["col_e"] in (4, 8, 16)
    # later plans of the same lengths start from the tuned entries
    assert pk.Plan(dims, h, hbar, T, len(src), "fp32").schedule == pl.schedule  # same lengths
    f = torch.as_tensor(f32).cuda()
    d_src = torch.as_tensor(src).cuda()
    S = torch.empty_like(f)
    pl.solve(f, d_src, S, ws)  # the workspace was overwritten by the tuner
    torch.cuda.synchronize()
    o = _oracle(f32, src, h, hbar, T)
    worst, _, _ = report(S.double().cpu().numpy(), o, hbar, "fp32")
    assert worst <= TOL["fp32"]


def test_data_flags_reported():
    """Errors in the data are reported in sweik_info.flags (asynchronously):
    a non-finite f, f <= 0, and sup|gamma| >= 1 with a given ftilde; a
    valid problem reports none."""
    import paper_1403_1937_amd as pk
    from paper_1403_1937_amd import INFO_FLAGS
    dims = (40, 48)
    src = np.array([[10, 12]], np.int32)
    base = np.full(dims, 1.5, np.float64)

    def flags(f, **kw):
        _, info = pk.solve(torch.as_tensor(f).cuda(), src, 0.02, 0.1, 3, return_info=True, **kw)
        return info["flags"]

    assert flags(base) == 0
    f = base.copy()
    f[3, 4] = np.nan
    assert flags(f) & INFO_FLAGS["f_nonfinite"]
    f = base.copy()
    f[5, 6] = -1.0
    assert flags(f) & INFO_FLAGS["f_nonpositive"]
    f = base.copy()
    f[7, 8] = 3.0  # gamma = (3/1.5)^2 - 1 = 3 with ftilde given as 1.5
    assert flags(f, ftilde_mode="given", ftilde=1.5) & INFO_FLAGS["c0_ge_1"]


def test_sources_validated_on_the_host():
    import paper_1403_1937_amd as pk
    f = torch.full((30, 30), 1.2, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        pk.solve(f, np.array([[30, 0]], np.int32), 0.1, 0.1, 2)
    with pytest.raises(ValueError):
        pk.solve(f, np.array([[1, 1], [1, 1]], np.int32), 0.1, 0.1, 2)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_seed_values_parity(prec):
    """Sources with prescribed values S(y_k) = s_k against the oracle."""
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(81)
    dims, h, hbar, T = (90, 70), 1 / 90, 0.08, 6
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 5, rng)
    s = rng.uniform(0.0, 0.3, len(src))
    dt = torch.float32 if prec == "fp32" else torch.float64
    S = pk.solve(torch.as_tensor(f.astype(np.float64)).to("cuda", dt), src, h, hbar, T,
                 src_s=s).double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T,
                     src_s=np.asarray(s, np.float32 if prec == "fp32" else np.float64))
    worst, frac, _ = report(S, o, hbar, prec)
    print(f"seeded {prec}: max rel {worst:.3e} on {frac:.3f}", flush=True)
    assert frac > 0.1 and worst <= TOL[prec]
    assert envelope_violations(S, o, hbar, prec) == 0


def _circle_sources(dims, count, rng):
    """`count` distinct grid points on a circle (a dense seed curve)."""
    c0, c1, rad = dims[0] / 2, dims[1] / 2, 0.35 * min(dims)
    th = np.sort(rng.uniform(0, 2 * np.pi, 4 * count))
    pts = np.stack([np.round(c0 + rad * np.cos(th)), np.round(c1 + rad * np.sin(th))], 1)
    pts = np.unique(pts.astype(np.int32), axis=0)
    return np.ascontiguousarray(pts[rng.permutation(len(pts))[:count]])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("seeded", [False, True], ids=["plain", "seed_values"])
def test_phi0_by_fft_many_sources(prec, seeded):
    """200 sources on a circle: the plan takes the FFT route of phi_0
    (Table 1 steps 1-5), checked against the oracle's direct sum."""
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(91)
    dims, h, hbar, T = (128, 160), 1 / 160, 0.05, 6
    f = workloads.smoothed_noise(dims, 6.0, 1.0, 2.0, rng).astype(np.float32)
    src = _circle_sources(dims, 200, rng)
    s = rng.uniform(0.0, 0.05, len(src)) if seeded else None
    pl = pk.Plan(dims, h, hbar, T, len(src), prec)
    assert pl.schedule["phi0_fft"] == 1
    dt = torch.float32 if prec == "fp32" else torch.float64
    S = pk.solve(torch.as_tensor(f.astype(np.float64)).to("cuda", dt), src, h, hbar, T,
                 src_s=s).double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T,
                     src_s=None if s is None else
                     np.asarray(s, np.float32 if prec == "fp32" else np.float64))
    worst, frac, _ = report(S, o, hbar, prec)
    print(f"phi0 by FFT {prec} {'seeded' if seeded else 'plain'}: max rel {worst:.3e} "
          f"on {frac:.3f}", flush=True)
    assert frac > 0.1 and worst <= TOL[prec]
    assert envelope_violations(S, o, hbar, prec) == 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_phi0_routes_agree(prec):
    """Few sources, the FFT route forced: against the oracle like the
    direct route (ragged grid, partial tiles)."""
    import paper_1403_1937_amd as pk
    from paper_1403_1937_amd._native import _read_info, info_struct_size
    rng = np.random.default_rng(92)
    dims, h, hbar, T = (100, 76), 1 / 100, 0.1, 5
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 4, rng)
    dt = torch.float32 if prec == "fp32" else torch.float64
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    for route in (0, 1):
        pl = pk.Plan(dims, h, hbar, T, len(src), prec)
        pl.set_schedule(16, 16, phi0_fft=route)
        ft = torch.as_tensor(f.astype(np.float64)).to("cuda", dt)
        S = torch.empty_like(ft)
        info = torch.zeros(info_struct_size(), dtype=torch.uint8, device="cuda")
        pl.solve(ft, torch.as_tensor(src).cuda(), S, pl.workspace("cuda"), None, info)
        torch.cuda.synchronize()
        worst, frac, _ = report(S.double().cpu().numpy(), o, hbar, prec)
        print(f"route {route} {prec}: max rel {worst:.3e} on {frac:.3f}", flush=True)
        assert _read_info(info)["flags"] == 0
        assert worst <= TOL[prec]


@pytest.mark.parametrize("cfg", [2, 5], ids=["noise1024_T16_src16", "noise2048_T12_src4"])
def test_benchmark_workloads_full_size(cfg):
    """The 1024^2 workload the benchmark times (T = 16, 16 sources) and the
    forward solve of the 2048^2 differentiation workload (T = 12, 4 sources),
    at full size through a plan in the schedule the autotuner picks, against
    the FP64 oracle over the whole grid: FP32-scaled and FP64 on their
    resolvable sets, and no point outside the conditioning envelope."""
    import paper_1403_1937_amd as pk
    p = workloads.problem(cfg)
    print(f"workload {cfg}: {p.dims} T={p.T} n_src={len(p.src)}: oracle", flush=True)
    o = oracle.solve(p.f.astype(np.float64), p.src, p.h, p.hbar, p.T)
    src = torch.as_tensor(np.ascontiguousarray(p.src, np.int32)).to("cuda")
    for prec, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        plan = pk.Plan(p.dims, p.h, p.hbar, p.T, len(p.src), prec)
        ws = plan.workspace("cuda")
        plan.autotune(ws)
        f = torch.as_tensor(p.f.astype(np.float64)).to("cuda", dt)
        S = torch.empty_like(f)
        plan.solve(f, src, S, ws)
        torch.cuda.synchronize()
        Sh = S.double().cpu().numpy()
        worst, frac, _ = report(Sh, o, p.hbar, prec)
        nbad = envelope_violations(Sh, o, p.hbar, prec)
        print(f"  {prec} schedule {plan.schedule}: max rel {worst:.3e} on {frac:.3f} of the grid; "
              f"envelope violations {nbad}", flush=True)
        assert frac > 0.4
        assert worst <= TOL[prec]
        assert nbad == 0
