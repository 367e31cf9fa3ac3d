"""Full gradient on the GPU (dL/df with the reference forcing's dependence
on f, and dL/dhbar) against the FP64 oracle's forward tangents, and at the
2048^2 differentiation workload against central differences of the GPU's
own forward solve.

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
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32).astype(np.float64)
    src = workloads.distinct_sources(dims, n_src, rng)
    rec = workloads.receivers_near_sources(dims, src, n_rec, 0.1 * max(dims), rng)
    w = rng.uniform(0.5, 1.5, n_rec)
    s = rng.uniform(0.0, 0.05, n_src)
    return f, src, rec, w, s


def _dLdS(dims, rec, w, S, target):
    g = np.zeros(dims)
    for k, (i, j) in enumerate(rec):
        g[i, j] += 2.0 * w[k] * (S[i, j] - target[k])
    return g


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
@pytest.mark.parametrize("dims,T,mode", [((40, 48), 6, "nu"), ((37, 50), 6, "fmax"),
                                         ((64, 64), 8, "given"), ((48, 40), 0, "nu"),
                                         ((100, 76), 10, "nu")])
def test_full_gradient_matches_oracle(prec, tol, dims, T, mode):
    import paper_1403_1937_amd as pk
    f, src, rec, w, s = _setup(dims, 3, 24, sum(dims) + T)
    h, hbar = 1.0 / max(dims), 0.08
    ft = 2.1 if mode == "given" else None
    o = oracle.solve(f, src, h, hbar, T, ft_mode=mode, ftilde=ft, src_s=s)
    target = np.array([o["S"][i, j] for i, j in rec]) * 0.97
    dLdS = _dLdS(dims, rec, w, o["S"], target)
    go = grad.full_gradient(f, src, h, hbar, T, dLdS, ft_mode=mode, ftilde=ft, src_s=s)
    dt = torch.float64 if prec == "fp64" else torch.float32
    g, sc = pk.solve_gradient(torch.as_tensor(f).to("cuda", dt), src, h, hbar, T,
                              torch.as_tensor(dLdS).to("cuda", dt), ftilde_mode=mode,
                              ftilde=ft, src_s=s)
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - go["dLdf"]) / np.linalg.norm(go["dLdf"])
    eh = abs(sc["dLdhbar"] - go["dLdhbar"]) / abs(go["dLdhbar"])
    ef = abs(sc["dLdftilde"] - go["dLdftilde"]) / max(abs(go["dLdftilde"]), 1e-300)
    print(f"{prec} {dims} T={T} {mode}: dLdf {err:.2e}, dLdhbar {eh:.2e} "
          f"({sc['dLdhbar']:.6e} vs {go['dLdhbar']:.6e}), dLdftilde {ef:.2e}", flush=True)
    assert err <= tol and eh <= tol
    if mode != "given":
        assert ef <= tol
    # the reference-forcing path shows at the extreme points of f
    if mode == "nu":
        i = int(np.argmax(f))
        assert abs(g.reshape(-1)[i] - go["dLdf"].reshape(-1)[i]) <= tol * np.abs(go["dLdf"]).max()


def test_differentiation_workload_against_differences():
    """2048^2, T = 12 (the fwd+bwd workload) in FP64: dL/dhbar and a
    directional derivative in f (moving fmin and fmax too) against central
    differences of the GPU forward solve."""
    import paper_1403_1937_amd as pk
    p = workloads.problem(5, 2048)
    rec, f_target = workloads.loss_setup(p)
    f = torch.as_tensor(p.f.astype(np.float64)).cuda()
    rec_t = torch.as_tensor(rec).cuda().long()
    St = pk.solve(torch.as_tensor(f_target.astype(np.float64)).cuda(), p.src, p.h, p.hbar, p.T)
    tgt = St[rec_t[:, 0], rec_t[:, 1]]

    def loss(ff, hb):
        S = pk.solve(ff, p.src, p.h, hb, p.T)
        v = S[rec_t[:, 0], rec_t[:, 1]]
        return float(((v - tgt) ** 2).sum()), S, v

    L0, S, v = loss(f, p.hbar)
    dLdS = torch.zeros_like(f)
    dLdS.index_put_((rec_t[:, 0], rec_t[:, 1]), 2.0 * (v - tgt), accumulate=True)
    g, sc = pk.solve_gradient(f, p.src, p.h, p.hbar, p.T, dLdS)
    dh = 1e-5 * p.hbar
    num = (loss(f, p.hbar + dh)[0] - loss(f, p.hbar - dh)[0]) / (2 * dh)
    print(f"2048^2 dL/dhbar {sc['dLdhbar']:.8e} vs differences {num:.8e}", flush=True)
    assert abs(sc["dLdhbar"] - num) <= 1e-5 * abs(num)
    rng = np.random.default_rng(5)
    d = torch.as_tensor(workloads.smoothed_noise((2048, 2048), 32.0, -1.0, 1.0, rng)).cuda()
    eps = 1e-6
    num = (loss(f + eps * d, p.hbar)[0] - loss(f - eps * d, p.hbar)[0]) / (2 * eps)
    ana = float((g * d).sum())
    print(f"2048^2 directional dL/df {ana:.8e} vs differences {num:.8e}", flush=True)
    assert abs(ana - num) <= 1e-5 * abs(num)
