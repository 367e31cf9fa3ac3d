"""GPU adjoint (dL/df with ftilde held fixed) against the FP64 oracle's
reverse sweep, against central finite differences of the GPU forward solve,
and through torch.autograd.

Loss: L = sum_r w_r (S(x_r) - t_r)^2 over receivers near the sources, where
the wave function is far above rounding noise (Section 5.3)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from common import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _setup(dims, n_src, n_rec, seed, hbar):
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, n_src, rng)
    rec = workloads.receivers_near_sources(dims, src, n_rec, 0.1 * max(dims), rng)
    w = rng.uniform(0.5, 1.5, n_rec)
    return f, src, rec, w


def _dLdS_dense(dims, rec, w, S, target):
    g = np.zeros(dims)
    for k, (i, j) in enumerate(rec):
        g[i, j] = 2.0 * w[k] * (S[i, j] - target[k])
    return g


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
@pytest.mark.parametrize("dims,T", [((64, 64), 6), ((100, 76), 8), ((256, 256), 12)])
def test_adjoint_matches_oracle(prec, tol, dims, T):
    import paper_1403_1937_amd as pk
    f, src, rec, w = _setup(dims, 3, 32, sum(dims) + T, 0.08)
    h = 1.0 / max(dims)
    o = oracle.solve(f.astype(np.float64), src, h, 0.08, T)
    target = np.array([o["S"][i, j] for i, j in rec]) * 0.97
    dLdS = _dLdS_dense(dims, rec, w, o["S"], target)
    g_o, _ = oracle.adjoint(f.astype(np.float64), src, h, 0.08, T, dLdS)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ft = torch.as_tensor(f.astype(np.float64)).to("cuda", dt)
    g = pk.solve_adjoint(ft, src, h, 0.08, T, torch.as_tensor(dLdS).to("cuda", dt))
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - g_o) / np.linalg.norm(g_o)
    print(f"adjoint {prec} {dims} T={T}: normwise rel {err:.3e}", flush=True)
    assert err <= tol


def test_adjoint_zero_terms():
    import paper_1403_1937_amd as pk
    f, src, rec, w = _setup((40, 40), 1, 8, 3, 0.1)
    ft = torch.as_tensor(f.astype(np.float64)).cuda()
    g = pk.solve_adjoint(ft, src, 1 / 40, 0.1, 0, torch.ones_like(ft))
    assert torch.count_nonzero(g).item() == 0


def test_adjoint_finite_differences_gpu():
    """Directional derivatives and single-point partials of the GPU loss
    (FP64, ftilde given so that it does not move with f) against the
    adjoint: rel <= 1e-5."""
    import paper_1403_1937_amd as pk
    dims, T, hbar = (48, 56), 8, 0.1
    h = 1.0 / 56
    f, src, rec, w = _setup(dims, 2, 24, 77, hbar)
    f64 = f.astype(np.float64)
    ftil = float(np.sqrt(0.5 * (f64.min() ** 2 + f64.max() ** 2)))
    kw = dict(ftilde_mode="given", ftilde=ftil)
    S0 = pk.solve(torch.as_tensor(f64).cuda(), src, h, hbar, T, **kw).cpu().numpy()
    target = np.array([S0[i, j] for i, j in rec]) * 0.95

    def loss(ff):
        S = pk.solve(torch.as_tensor(ff).cuda(), src, h, hbar, T, **kw).cpu().numpy()
        return float(sum(w[k] * (S[i, j] - target[k]) ** 2 for k, (i, j) in enumerate(rec)))

    dLdS = _dLdS_dense(dims, rec, w, S0, target)
    g = pk.solve_adjoint(torch.as_tensor(f64).cuda(), src, h, hbar, T,
                         torch.as_tensor(dLdS).cuda(), **kw).cpu().numpy()
    rng = np.random.default_rng(5)
    for _ in range(4):
        d = rng.standard_normal(dims)
        eps = 1e-6
        fd = (loss(f64 + eps * d) - loss(f64 - eps * d)) / (2 * eps)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-5 * abs(an), (fd, an)
    big = np.argsort(-np.abs(g).ravel())[:6]
    for flat in big:
        idx = np.unravel_index(flat, dims)
        e = np.zeros(dims)
        e[idx] = 1.0
        eps = 1e-6
        fd = (loss(f64 + eps * e) - loss(f64 - eps * e)) / (2 * eps)
        assert abs(fd - g[idx]) <= 1e-5 * abs(g[idx]) + 1e-12, (idx, fd, g[idx])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_autograd_function(prec):
    import paper_1403_1937_amd as pk
    dims, T, hbar = (64, 80), 6, 0.08
    f, src, rec, w = _setup(dims, 2, 16, 91, hbar)
    dt = torch.float64 if prec == "fp64" else torch.float32
    ft = torch.as_tensor(f.astype(np.float64)).to("cuda", dt).requires_grad_(True)
    S = pk.eikonal(ft, src, 1 / 80, hbar, T)
    ri = torch.as_tensor(rec[:, 0]).cuda().long()
    rj = torch.as_tensor(rec[:, 1]).cuda().long()
    wt = torch.as_tensor(w).to("cuda", dt)
    L = (wt * (S[ri, rj] - 0.1) ** 2).sum()
    L.backward()
    dLdS = torch.zeros_like(S)
    dLdS[ri, rj] = 2 * wt * (S[ri, rj].detach() - 0.1)
    g = pk.solve_adjoint(ft.detach(), src, 1 / 80, hbar, T, dLdS)
    torch.cuda.synchronize()
    assert torch.allclose(ft.grad, g, rtol=1e-6 if prec == "fp32" else 1e-12, atol=0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
def test_adjoint_radix8_schedule(prec, tol):
    """The adjoint sweep with radix-8 team FFTs (512-thread work-groups)."""
    import paper_1403_1937_amd as pk
    dims, T, hbar = (100, 76), 8, 0.08
    f, src, rec, w = _setup(dims, 3, 32, 91, hbar)
    h = 1.0 / max(dims)
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    target = np.array([o["S"][i, j] for i, j in rec]) * 0.97
    dLdS = _dLdS_dense(dims, rec, w, o["S"], target)
    g_o, _ = oracle.adjoint(f.astype(np.float64), src, h, hbar, T, dLdS)
    dt = torch.float64 if prec == "fp64" else torch.float32
    pl = pk.Plan(dims, h, hbar, T, len(src), prec)
    pl.set_schedule(8, 8)
    ft = torch.as_tensor(f.astype(np.float64)).to("cuda", dt)
    d_src = torch.as_tensor(np.ascontiguousarray(src, np.int32)).cuda()
    S, ws, ck = torch.empty_like(ft), pl.workspace("cuda"), pl.checkpoint("cuda")
    g = torch.empty_like(ft)
    pl.solve(ft, d_src, S, ws, ck)
    pl.adjoint(ft, d_src, ck, torch.as_tensor(dLdS).to("cuda", dt), g, ws)
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - g_o) / np.linalg.norm(g_o)
    print(f"adjoint radix-8 {prec}: normwise rel {err:.3e}", flush=True)
    assert err <= tol


@pytest.mark.timeout(600)
def test_differentiation_workload_full_size():
    """The 2048^2 differentiation workload at full size (T = 12, 4 sources,
    256 receivers near the sources, target from the perturbed forcing,
    ftilde given as nu of f).  dL/dS is formed from the FP64 oracle's
    forward solves, and the FP64 and FP32-scaled GPU gradients are compared
    with the oracle's adjoint over the whole grid (normwise rel <= 1e-9 and
    <= 1e-3); then the FP64 gradient against central differences of the GPU
    loss along two smooth directions (rel <= 1e-5)."""
    import paper_1403_1937_amd as pk
    p = workloads.problem(5)
    rec, f_t = workloads.loss_setup(p)
    f64 = p.f.astype(np.float64)
    ftil = float(np.sqrt(0.5 * (f64.min() ** 2 + f64.max() ** 2)))
    kw = dict(ftilde_mode="given", ftilde=ftil)
    okw = dict(ft_mode="given", ftilde=ftil)
    print("2048^2: oracle target and forward solves", flush=True)
    tgt_o = oracle.solve(f_t.astype(np.float64), p.src, p.h, p.hbar, p.T, **okw)["S"]
    S_o = oracle.solve(f64, p.src, p.h, p.hbar, p.T, **okw)["S"]
    dLdS = np.zeros(p.dims)
    dLdS[rec[:, 0], rec[:, 1]] = 2.0 * (S_o[rec[:, 0], rec[:, 1]] - tgt_o[rec[:, 0], rec[:, 1]])
    print("2048^2: oracle adjoint", flush=True)
    g_o, _ = oracle.adjoint(f64, p.src, p.h, p.hbar, p.T, dLdS, **okw)
    print("2048^2: GPU adjoints", flush=True)
    g64 = pk.solve_adjoint(torch.as_tensor(f64).cuda(), p.src, p.h, p.hbar, p.T,
                           torch.as_tensor(dLdS).cuda(), **kw).cpu().numpy()
    g32 = pk.solve_adjoint(torch.as_tensor(p.f).cuda(), p.src, p.h, p.hbar, p.T,
                           torch.as_tensor(dLdS.astype(np.float32)).cuda(),
                           **kw).double().cpu().numpy()
    e64 = np.linalg.norm(g64 - g_o) / np.linalg.norm(g_o)
    e32 = np.linalg.norm(g32 - g_o) / np.linalg.norm(g_o)
    print(f"  against the oracle gradient: fp64 normwise rel {e64:.3e}, fp32 {e32:.3e}",
          flush=True)
    assert np.isfinite(g64).all() and np.isfinite(g32).all()
    assert e64 <= 1e-9
    assert e32 <= 1e-3

    # the loss of the GPU's own FP64 forward solve, for the differences
    tgt = pk.solve(torch.as_tensor(f_t.astype(np.float64)).cuda(), p.src, p.h, p.hbar, p.T,
                   **kw).cpu().numpy()[rec[:, 0], rec[:, 1]]
    S64 = pk.solve(torch.as_tensor(f64).cuda(), p.src, p.h, p.hbar, p.T, **kw).cpu().numpy()
    dLdS_g = np.zeros(p.dims)
    dLdS_g[rec[:, 0], rec[:, 1]] = 2.0 * (S64[rec[:, 0], rec[:, 1]] - tgt)
    g64 = pk.solve_adjoint(torch.as_tensor(f64).cuda(), p.src, p.h, p.hbar, p.T,
                           torch.as_tensor(dLdS_g).cuda(), **kw).cpu().numpy()

    def loss(ff):
        S = pk.solve(torch.as_tensor(ff).cuda(), p.src, p.h, p.hbar, p.T, **kw).cpu().numpy()
        return float(np.sum((S[rec[:, 0], rec[:, 1]] - tgt) ** 2))

    rng = np.random.default_rng(17)
    for k in range(2):
        d = workloads.smoothed_noise(p.dims, 32.0, -1.0, 1.0, rng)
        eps = 1e-5
        fd = (loss(f64 + eps * d) - loss(f64 - eps * d)) / (2 * eps)
        an = float(np.sum(g64 * d))
        print(f"  direction {k}: fd {fd:.9e} adjoint {an:.9e}", flush=True)
        assert abs(fd - an) <= 1e-5 * abs(an)


@pytest.mark.parametrize("phi0_fft", [0, 1], ids=["phi0_direct", "phi0_fft"])
def test_solve_and_adjoint_graph_replays(phi0_fft):
    """A solve and its adjoint enqueue only kernels on the caller's stream
    (no allocation, no memset), so they can be captured into a HIP graph:
    every replay, with unrelated eager work and synchronisations between
    the replays, equals the eager result bit for bit."""
    import paper_1403_1937_amd as pk
    dims, T, hbar = (96, 80), 6, 0.08
    f, src, rec, w = _setup(dims, 3, 16, 93, hbar)
    h = 1.0 / 96
    pl = pk.Plan(dims, h, hbar, T, len(src), "fp32")
    pl.set_schedule(16, 16, phi0_fft=phi0_fft)
    ft = torch.as_tensor(f).cuda()
    d_src = torch.as_tensor(src).cuda()
    ws, ck = pl.workspace("cuda"), pl.checkpoint("cuda")
    dLdS = torch.zeros(dims, device="cuda")
    dLdS[torch.as_tensor(rec[:, 0]).long(), torch.as_tensor(rec[:, 1]).long()] = 1.0
    S, g = torch.empty_like(ft), torch.empty_like(ft)
    pl.solve(ft, d_src, S, ws, ck)
    pl.adjoint(ft, d_src, ck, dLdS, g, ws)
    torch.cuda.synchronize()
    S_ref, g_ref = S.clone(), g.clone()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph):
            pl.solve(ft, d_src, S, ws, ck)
            pl.adjoint(ft, d_src, ck, dLdS, g, ws)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(4):
        S.fill_(float("nan"))
        g.fill_(float("nan"))
        ws.random_(0, 255)  # the workspace holds nothing between solves
        torch.randn(1 << 18, device="cuda").sum().item()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(S, S_ref), f"replay {rep}: S"
        assert torch.equal(g, g_ref), f"replay {rep}: dL/df"
