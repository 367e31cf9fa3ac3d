"""GPU adjoint of the 3D solve (dL/df with ftilde held fixed) against the
FP64 oracle's reverse sweep and against central finite differences of the
GPU forward solve.

Loss: L = sum_r w_r (S(x_r) - t_r)^2 over receivers near the sources (where
phi is far above rounding noise), as for the 2D adjoint."""
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


def _setup(dims, n_src, n_rec, seed):
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 2.0, 1.0, 2.0, rng)
    src = workloads.distinct_sources(dims, n_src, rng)
    rec = workloads.receivers_near_sources(dims, src, n_rec, 0.15 * max(dims), rng)
    w = rng.uniform(0.5, 1.5, n_rec)
    return f, src, rec, w


def _dLdS(dims, rec, w, S, target):
    g = np.zeros(dims)
    for k, r in enumerate(rec):
        g[tuple(r)] = 2.0 * w[k] * (S[tuple(r)] - target[k])
    return g


# padded lengths 64 (the smallest), 128 and 256 along some axes, ragged sizes;
# 2048 (the largest) along the contiguous axis and along axis 0
CASES = [((20, 18, 22), 4), ((33, 12, 40), 5), ((16, 50, 16), 3), ((96, 80, 64), 6),
         ((6, 5, 700), 3), ((700, 5, 6), 3)]


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
@pytest.mark.parametrize("dims,T", CASES)
def test_adjoint3d_matches_oracle(prec, tol, dims, T):
    import paper_1403_1937_amd as pk
    f, src, rec, w = _setup(dims, 2, 24, sum(dims) + T)
    h, hbar = 1.0 / max(dims), 0.12
    o = oracle.solve(f, src, h, hbar, T)
    target = np.array([o["S"][tuple(r)] for r in rec]) * 0.97
    dLdS = _dLdS(dims, rec, w, o["S"], target)
    g_o, _ = oracle.adjoint(f, src, h, hbar, T, dLdS)
    dt = torch.float64 if prec == "fp64" else torch.float32
    print(f"3D adjoint {prec} {dims} T={T}", flush=True)
    g = pk.solve_adjoint(torch.as_tensor(f).to("cuda", dt), src, h, hbar, T,
                         torch.as_tensor(dLdS).to("cuda", dt))
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - g_o) / np.linalg.norm(g_o)
    print(f"  normwise rel {err:.3e}", flush=True)
    assert np.isfinite(g).all()
    assert err <= tol


def test_adjoint3d_zero_terms():
    import paper_1403_1937_amd as pk
    f, src, rec, w = _setup((12, 14, 16), 1, 8, 3)
    ft = torch.as_tensor(f).cuda()
    g = pk.solve_adjoint(ft, src, 1 / 16, 0.1, 0, torch.ones_like(ft))
    assert torch.count_nonzero(g).item() == 0


def test_adjoint3d_finite_differences():
    """Directional derivative of the GPU loss (FP64, ftilde given so that it
    does not move with f) along two random directions: central differences
    against <dL/df, d>, rel <= 1e-5."""
    import paper_1403_1937_amd as pk
    dims, T, hbar = (18, 20, 24), 5, 0.12
    h = 1.0 / 24
    f, src, rec, w = _setup(dims, 2, 16, 91)
    ftil = float(np.sqrt(0.5 * (f.min() ** 2 + f.max() ** 2)))
    kw = dict(ftilde_mode="given", ftilde=ftil)
    S0 = pk.solve(torch.as_tensor(f).cuda(), src, h, hbar, T, **kw).cpu().numpy()
    target = np.array([S0[tuple(r)] for r in rec]) * 0.95

    def loss(ff):
        S = pk.solve(torch.as_tensor(ff).cuda(), src, h, hbar, T, **kw).cpu().numpy()
        return sum(w[k] * (S[tuple(r)] - target[k]) ** 2 for k, r in enumerate(rec))

    dLdS = _dLdS(dims, rec, w, S0, target)
    g = pk.solve_adjoint(torch.as_tensor(f).cuda(), src, h, hbar, T,
                         torch.as_tensor(dLdS).cuda(), **kw).cpu().numpy()
    rng = np.random.default_rng(5)
    for _ in range(2):
        d = rng.standard_normal(dims)
        eps = 1e-4
        fd = (loss(f + eps * d) - loss(f - eps * d)) / (2 * eps)
        an = float((g * d).sum())
        print(f"3D directional: fd {fd:.10e} adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-5 * abs(an)


def test_autograd_3d():
    """torch.autograd through the 3D solve gives the adjoint's gradient."""
    import paper_1403_1937_amd as pk
    dims, T, hbar = (14, 16, 18), 4, 0.12
    f, src, rec, w = _setup(dims, 1, 8, 17)
    ft = torch.as_tensor(f).cuda().requires_grad_(True)
    S = pk.eikonal(ft, src, 1 / 18, hbar, T)
    idx = torch.as_tensor(np.asarray(rec)).cuda()
    loss = (torch.as_tensor(w).cuda() * S[idx[:, 0], idx[:, 1], idx[:, 2]] ** 2).sum()
    loss.backward()
    dLdS = torch.zeros_like(S.detach())
    dLdS[idx[:, 0], idx[:, 1], idx[:, 2]] = 2 * torch.as_tensor(w).cuda() * S.detach()[idx[:, 0], idx[:, 1], idx[:, 2]]
    g = pk.solve_adjoint(ft.detach(), src, 1 / 18, hbar, T, dLdS)
    assert torch.allclose(ft.grad, g, rtol=1e-12, atol=0)
