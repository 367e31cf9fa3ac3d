"""Full gradient of the 3D solve on the GPU (dL/df with the reference
forcing's dependence on f, dL/dhbar and dL/dftilde) against the FP64
oracle's forward tangents, and at the 256^3 blob workload against central
differences of the GPU's own forward solve.

Loss: L = sum_r w_r (S(x_r) - t_r)^2 over receivers near the sources."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from common import ensure_built
from oracle import grad

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


def _setup(dims, n_src, n_rec, seed):
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 2.0, 1.0, 3.0, rng).astype(np.float32).astype(np.float64)
    src = workloads.distinct_sources(dims, n_src, rng)
    rec = workloads.receivers_near_sources(dims, src, n_rec, 0.2 * max(dims), rng)
    w = rng.uniform(0.5, 1.5, n_rec)
    s = rng.uniform(0.0, 0.05, n_src)
    return f, src, rec, w, s


def _dLdS(dims, rec, w, S, target):
    g = np.zeros(dims)
    for k, r in enumerate(rec):
        g[tuple(r)] += 2.0 * w[k] * (S[tuple(r)] - target[k])
    return g


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
@pytest.mark.parametrize("dims,T,mode", [((20, 18, 22), 4, "nu"), ((16, 24, 20), 5, "fmax"),
                                         ((18, 18, 18), 3, "given"), ((20, 16, 18), 0, "nu"),
                                         ((40, 36, 44), 6, "nu"), ((33, 12, 40), 5, "fmax")])
def test_full_gradient_3d_matches_oracle(prec, tol, dims, T, mode):
    import paper_1403_1937_amd as pk
    f, src, rec, w, s = _setup(dims, 3, 24, sum(dims) + T)
    h, hbar = 1.0 / max(dims), 0.12
    ft = 2.1 if mode == "given" else None
    o = oracle.solve(f, src, h, hbar, T, ft_mode=mode, ftilde=ft, src_s=s)
    target = np.array([o["S"][tuple(r)] for r in rec]) * 0.97
    dLdS = _dLdS(dims, rec, w, o["S"], target)
    go = grad.full_gradient(f, src, h, hbar, T, dLdS, ft_mode=mode, ftilde=ft, src_s=s)
    dt = torch.float64 if prec == "fp64" else torch.float32
    print(f"3D full gradient {prec} {dims} T={T} {mode}", flush=True)
    g, sc = pk.solve_gradient(torch.as_tensor(f).to("cuda", dt), src, h, hbar, T,
                              torch.as_tensor(dLdS).to("cuda", dt), ftilde_mode=mode,
                              ftilde=ft, src_s=s)
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - go["dLdf"]) / np.linalg.norm(go["dLdf"])
    eh = abs(sc["dLdhbar"] - go["dLdhbar"]) / abs(go["dLdhbar"])
    ef = abs(sc["dLdftilde"] - go["dLdftilde"]) / max(abs(go["dLdftilde"]), 1e-300)
    eb = abs(sc["dLdbeta"] - go["dLdbeta"]) / max(abs(go["dLdbeta"]), 1e-300)
    print(f"  dLdf {err:.2e}, dLdhbar {eh:.2e} ({sc['dLdhbar']:.6e} vs {go['dLdhbar']:.6e}), "
          f"dLdftilde {ef:.2e}, dLdbeta {eb:.2e}", flush=True)
    assert err <= tol and eh <= tol and eb <= tol
    if mode != "given":
        assert ef <= tol
    # the reference-forcing path shows at the extreme points of f
    if mode in ("nu", "fmax"):
        i = int(np.argmax(f))
        assert abs(g.reshape(-1)[i] - go["dLdf"].reshape(-1)[i]) <= tol * np.abs(go["dLdf"]).max()


def test_full_gradient_3d_given_equals_adjoint():
    """With a given reference forcing dL/df is the fixed-forcing adjoint."""
    import paper_1403_1937_amd as pk
    dims, T = (24, 20, 30), 5
    f, src, rec, w, s = _setup(dims, 2, 16, 77)
    h, hbar = 1.0 / 30, 0.12
    o = oracle.solve(f, src, h, hbar, T, ft_mode="given", ftilde=2.2)
    target = np.array([o["S"][tuple(r)] for r in rec]) * 0.97
    dLdS = torch.as_tensor(_dLdS(dims, rec, w, o["S"], target)).cuda()
    ft = torch.as_tensor(f).cuda()
    print("3D full gradient vs adjoint, given ftilde", flush=True)
    g, _ = pk.solve_gradient(ft, src, h, hbar, T, dLdS, ftilde_mode="given", ftilde=2.2)
    ga = pk.solve_adjoint(ft, src, h, hbar, T, dLdS, ftilde_mode="given", ftilde=2.2)
    np.testing.assert_allclose(g.cpu().numpy(), ga.cpu().numpy(), rtol=1e-12,
                               atol=1e-14 * float(ga.abs().max()))


def test_blob_workload_3d_against_differences():
    """256^3, T = 16 (the 3D workload) in FP64: dL/dhbar and a directional
    derivative in f (moving fmin and fmax too) against central differences of
    the GPU forward solve.  The blob field in float32 takes its minimum 0.5
    at several hundred points, where nu(f) has only one-sided derivatives;
    the first minimum is lowered and the first maximum raised by 1e-3 so
    that both extremes are unique and the loss is differentiable in f."""
    import paper_1403_1937_amd as pk
    p = workloads.problem(3)
    f64 = p.f.astype(np.float64).reshape(-1)
    f64[int(np.argmin(f64))] -= 1e-3
    f64[int(np.argmax(f64))] += 1e-3
    f = torch.as_tensor(f64.reshape(p.dims)).cuda()
    rng = np.random.default_rng(11)
    rec = workloads.receivers_near_sources(p.dims, p.src, 256, 0.25 * p.dims[0], rng)
    ridx = torch.as_tensor(np.ravel_multi_index(tuple(rec.T), p.dims).astype(np.int64)).cuda()
    print("3D full gradient 256^3 against differences", flush=True)
    S0 = pk.solve(f, p.src, p.h, p.hbar, p.T)
    tgt = 0.97 * S0.view(-1)[ridx]

    def loss(ff, hb):
        S = pk.solve(ff, p.src, p.h, hb, p.T)
        v = S.view(-1)[ridx]
        return float(((v - tgt) ** 2).sum()), v

    L0, v = loss(f, p.hbar)
    dLdS = torch.zeros(f.numel(), dtype=torch.float64, device=f.device)
    dLdS.index_put_((ridx,), 2.0 * (v - tgt), accumulate=True)
    g, sc = pk.solve_gradient(f, p.src, p.h, p.hbar, p.T, dLdS.view(p.dims))
    dh = 1e-5 * p.hbar
    num = (loss(f, p.hbar + dh)[0] - loss(f, p.hbar - dh)[0]) / (2 * dh)
    print(f"256^3 dL/dhbar {sc['dLdhbar']:.8e} vs differences {num:.8e}", flush=True)
    assert abs(sc["dLdhbar"] - num) <= 1e-5 * abs(num)
    # a smooth direction of unit size (sum of a few random plane waves)
    ax = [torch.arange(n, dtype=torch.float64, device=f.device) / n for n in p.dims]
    x0, x1, x2 = torch.meshgrid(*ax, indexing="ij")
    d = torch.zeros_like(f)
    for k, ph in zip(rng.integers(1, 4, (4, 3)), rng.uniform(0, 2 * np.pi, 4)):
        d += 0.25 * torch.cos(2 * np.pi * (int(k[0]) * x0 + int(k[1]) * x1 + int(k[2]) * x2) + ph)
    eps = 1e-6
    num = (loss(f + eps * d, p.hbar)[0] - loss(f - eps * d, p.hbar)[0]) / (2 * eps)
    ana = float((g * d).sum())
    print(f"256^3 directional dL/df {ana:.8e} vs differences {num:.8e}", flush=True)
    assert abs(ana - num) <= 1e-5 * abs(num)


@pytest.mark.parametrize("dims,phi0_fft", [((24, 20, 30), 0), ((24, 20, 30), 1), ((96, 80), 0)],
                         ids=["3d_phi0_direct", "3d_phi0_fft", "2d"])
def test_solve_and_full_gradient_graph_replays(dims, phi0_fft):
    """A solve with its checkpoint and the full gradient enqueue only
    kernels on the caller's stream, so they can be captured into a HIP
    graph: every replay, with a scrambled workspace and unrelated eager work
    between the replays, equals the eager result bit for bit."""
    import paper_1403_1937_amd as pk
    f, src, rec, w, s = _setup(dims, 3, 16, 95)
    h, hbar, T = 1.0 / max(dims), 0.12, 4
    pl = pk.Plan(dims, h, hbar, T, len(src), "fp32")
    pl.set_schedule(16, 16, phi0_fft=phi0_fft)
    ft = torch.as_tensor(f, dtype=torch.float32).cuda()
    d_src = torch.as_tensor(src.astype(np.int32)).cuda()
    d_s = torch.as_tensor(s, dtype=torch.float32).cuda()
    ws = torch.empty(pl.adjoint_full_workspace_bytes, dtype=torch.uint8, device="cuda")
    ck = pl.checkpoint("cuda")
    dLdS = torch.zeros(dims, device="cuda")
    for r in rec:
        dLdS[tuple(int(v) for v in r)] = 1.0
    S, g = torch.empty_like(ft), torch.empty_like(ft)
    grads = torch.zeros(4, dtype=torch.float64, device="cuda")
    print(f"full-gradient graph {dims} phi0_fft={phi0_fft}", flush=True)
    pl.solve(ft, d_src, S, ws, ck, src_s=d_s)
    pl.adjoint_full(ft, d_src, ck, dLdS, g, grads, ws, d_s)
    torch.cuda.synchronize()
    S_ref, g_ref, gr_ref = S.clone(), g.clone(), grads.clone()
    assert torch.isfinite(g_ref).all() and torch.isfinite(gr_ref[:3]).all()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph):
            pl.solve(ft, d_src, S, ws, ck, src_s=d_s)
            pl.adjoint_full(ft, d_src, ck, dLdS, g, grads, ws, d_s)
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(4):
        S.fill_(float("nan"))
        g.fill_(float("nan"))
        grads.fill_(float("nan"))
        ws.random_(0, 255)  # the workspace holds nothing between calls
        torch.randn(1 << 18, device="cuda").sum().item()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(S, S_ref), f"replay {rep}: S"
        assert torch.equal(g, g_ref), f"replay {rep}: dL/df"
        assert torch.equal(grads[:3], gr_ref[:3]), f"replay {rep}: scalars"
