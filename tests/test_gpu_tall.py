"""2D grids beyond 2048 rows or 4096 columns (float32): the column passes
transform 8192-point columns and the row passes 8192-point complex rows
(16384 real points), one per work-group.  Forward, adjoint, full gradient,
tilted and batched solves against the FP64 oracle or the single solve."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from common import LAMBDA_MAX, TOL, ensure_built, envelope_violations, lam, rel_err, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()


TALL = [
    # (name, dims, h, hbar, T, n_src, seed)
    ("tall3000x24", (3000, 24), 1 / 3000, 0.3, 4, 2, 9),     # partial last row block
    ("tall4096x96", (4096, 96), 1 / 4096, 0.2, 6, 3, 10),    # every column work-group full
    ("tall2049x130", (2049, 130), 1 / 2049, 0.15, 5, 4, 11),  # smallest n0 past 2048
    ("wide24x5000", (24, 5000), 1 / 5000, 0.3, 4, 2, 15),     # 8192-point complex rows
    ("wide40x8192", (40, 8192), 1 / 8192, 0.2, 4, 3, 16),     # every row full
    ("both2100x4200", (2100, 4200), 1 / 4200, 0.1, 3, 4, 17),  # both long axes
]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("case", TALL, ids=[c[0] for c in TALL])
def test_forward_parity_tall(case, prec):
    import paper_1403_1937_amd as pk
    name, dims, h, hbar, T, n_src, seed = case
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, n_src, rng)
    s = rng.uniform(0.0, 0.05, n_src)
    print(f"tall case {name} {dims} {prec}", flush=True)
    pl = pk.Plan(dims, h, hbar, T, n_src, prec)
    assert pl.padded[0] == 8192 or pl.padded[1] == 16384
    dt = torch.float32 if prec == "fp32" else torch.float64
    ft = torch.as_tensor(f.astype(np.float64)).to("cuda", dt)
    S, info = pk.solve(ft, src, h, hbar, T, src_s=s, return_info=True)
    S = S.double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T,
                     src_s=np.asarray(s, np.float32 if prec == "fp32" else np.float64))
    assert info["flags"] == 0
    worst, frac, _ = report(S, o, hbar, prec)
    nbad = envelope_violations(S, o, hbar, prec)
    print(f"  max rel {worst:.3e} on {frac:.3f}; envelope violations {nbad}", flush=True)
    assert frac > 0.1 and worst <= TOL[prec] and nbad == 0


def test_adjoint_tall():
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(12)
    dims, h, hbar, T = (3000, 40), 1 / 3000, 0.2, 5
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 2, rng)
    rec = workloads.receivers_near_sources(dims, src, 32, 200.0, rng)
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    dLdS = np.zeros(dims)
    for r in rec:
        dLdS[tuple(r)] += 2.0 * 0.03 * o["S"][tuple(r)]
    ref, _ = oracle.adjoint(f.astype(np.float64), src, h, hbar, T, dLdS)
    print("tall adjoint (3000, 40) fp32", flush=True)
    g = pk.solve_adjoint(torch.as_tensor(f).cuda(), src, h, hbar, T,
                         torch.as_tensor(dLdS, dtype=torch.float32).cuda())
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - ref) / np.linalg.norm(ref)
    print(f"  normwise rel {err:.3e}", flush=True)
    assert err <= 1e-3


def test_full_gradient_wide():
    """The full gradient's row passes at 8192-point complex rows."""
    import paper_1403_1937_amd as pk
    from oracle import grad
    rng = np.random.default_rng(18)
    dims, h, hbar, T = (20, 5000), 1 / 5000, 0.3, 3
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32).astype(np.float64)
    src = workloads.distinct_sources(dims, 2, rng)
    rec = workloads.receivers_near_sources(dims, src, 24, 300.0, rng)
    o = oracle.solve(f, src, h, hbar, T)
    dLdS = np.zeros(dims)
    for r in rec:
        dLdS[tuple(r)] += 0.06 * o["S"][tuple(r)]
    go = grad.full_gradient(f, src, h, hbar, T, dLdS)
    print("wide full gradient (20, 5000) fp32", flush=True)
    g, sc = pk.solve_gradient(torch.as_tensor(f, dtype=torch.float32).cuda(), src, h, hbar, T,
                              torch.as_tensor(dLdS, dtype=torch.float32).cuda())
    g = g.double().cpu().numpy()
    err = np.linalg.norm(g - go["dLdf"]) / np.linalg.norm(go["dLdf"])
    eh = abs(sc["dLdhbar"] - go["dLdhbar"]) / abs(go["dLdhbar"])
    # the same without the two extreme points of f, whose reference-forcing
    # part (formed in float64) can dominate the norm
    bulk = np.ones(dims, bool)
    bulk.reshape(-1)[[int(np.argmin(f)), int(np.argmax(f))]] = False
    eb = np.linalg.norm((g - go["dLdf"])[bulk]) / np.linalg.norm(go["dLdf"][bulk])
    print(f"  dLdf {err:.3e} (without the extreme points {eb:.3e}), dLdhbar {eh:.3e}", flush=True)
    assert err <= 1e-3 and eb <= 1e-3 and eh <= 1e-3


def test_tilted_tall():
    """The tilted column passes (complex kernel spectrum) at 8192 points."""
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(13)
    dims, h, hbar, T = (2200, 12), 1 / 2200, 0.02, 4
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 2.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 1, rng)
    print("tall tilted (2200, 12) fp32", flush=True)
    S = pk.solve_tilted(torch.as_tensor(f).cuda(), src, h, hbar, T,
                        tilts=[(0.0, 0.0), (0.7, 0.0), (-0.7, 0.0)]).double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    ref = oracle.solve(f.astype(np.float64), src, h, hbar, T, method="direct")["S"]
    e = rel_err(S, ref, hbar)
    m = lam(o["phi"]) <= LAMBDA_MAX["fp32"]
    ok = e <= TOL["fp32"]
    print(f"  plain-resolvable {m.mean():.3f}, resolved {ok.mean():.3f}", flush=True)
    assert ok[m].all()
    # the tilts along the long axis resolve more than the plain solve's set
    assert ok.mean() > m.mean()


def test_tilted_wide():
    """The tilted row passes (tilted kernel table, last pass) at 8192-point
    complex rows."""
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(19)
    dims, h, hbar, T = (8, 4500), 1 / 4500, 0.02, 4
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 2.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, 1, rng)
    print("wide tilted (8, 4500) fp32", flush=True)
    S = pk.solve_tilted(torch.as_tensor(f).cuda(), src, h, hbar, T,
                        tilts=[(0.0, 0.0), (0.0, 0.7), (0.0, -0.7)]).double().cpu().numpy()
    o = oracle.solve(f.astype(np.float64), src, h, hbar, T)
    ref = oracle.solve(f.astype(np.float64), src, h, hbar, T, method="direct")["S"]
    e = rel_err(S, ref, hbar)
    m = lam(o["phi"]) <= LAMBDA_MAX["fp32"]
    ok = e <= TOL["fp32"]
    print(f"  plain-resolvable {m.mean():.3f}, resolved {ok.mean():.3f}", flush=True)
    assert ok[m].all()
    assert ok.mean() > m.mean()


def test_batch_with_tall_instance():
    import paper_1403_1937_amd as pk
    rng = np.random.default_rng(14)
    probs, fs, srcs = [], [], []
    for dims, n_src in (((3000, 24), 2), ((100, 76), 3), ((2100, 40), 1)):
        f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
        src = workloads.distinct_sources(dims, n_src, rng)
        probs.append({"dims": dims, "h": 1 / max(dims), "hbar": 0.2, "T": 4, "n_src": n_src})
        fs.append(torch.as_tensor(f).cuda())
        srcs.append(torch.as_tensor(src.astype(np.int32)).cuda())
    print("batch with 8192-point columns fp32", flush=True)
    b = pk.Batch(probs, "fp32")
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    Ss = [torch.full_like(f, -1.0) for f in fs]
    b.solve(fs, srcs, Ss, ws)
    torch.cuda.synchronize()
    for q, f, src, S in zip(probs, fs, srcs, Ss):
        R = pk.solve(f, src.cpu().numpy(), q["h"], q["hbar"], q["T"])
        assert torch.equal(S, R), q["dims"]
