"""Backtracking on the GPU (Section 6, eq. PathPlanning-backTrackOnS) against
the float64 oracle path by path: the same discretisation on both sides, all
in float64, so the paths agree to rounding and their lengths and status
codes agree exactly (the radius test can flip only where a point lies
within rounding of the radius, which the comparison allows)."""
import numpy as np
import pytest
import torch

from common import ensure_built

pytestmark = [pytest.mark.gpu, pytest.mark.filterwarnings("ignore::RuntimeWarning")]

TOL = 1e-9  # grid units, after thousands of RK4 steps in float64


@pytest.fixture(scope="module")
def pk():
    ensure_built()
    import paper_1403_1937_amd as pk
    return pk


def _compare(pk, S, src, start, step, radius, max_steps):
    from oracle import trace
    dev = "cuda:0"
    St = torch.as_tensor(S).to(dev)
    path, npts, st = pk.backtrack(St, src, start, step=step, radius=radius, max_steps=max_steps)
    torch.cuda.synchronize()
    path, npts, st = path.cpu().numpy(), npts.cpu().numpy(), st.cpu().numpy()
    opath, onpts, ost = trace.backtrack(np.asarray(S, np.float64), src, start, step=step,
                                        radius=radius, max_steps=max_steps)
    print(f"paths {len(start)}: status counts {np.bincount(st, minlength=4)}, "
          f"points {int(npts.sum())}", flush=True)
    np.testing.assert_array_equal(st, ost)
    assert np.all(np.abs(npts.astype(int) - onpts) <= 1)
    for q in range(len(start)):
        n = min(npts[q], onpts[q])
        if n:
            err = np.abs(path[q, :n] - opath[q, :n]).max()
            assert err < TOL, (q, err)
    return st, npts


def _solved(pk, n, src, dtype):
    import workloads
    rng = np.random.default_rng(5)
    f = workloads.smoothed_noise((n, n), 8.0, 1.0, 3.0, rng)
    S = pk.solve(torch.as_tensor(f).to("cuda:0", dtype), src, 1.0 / n, 0.05, 12)
    return S.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_paths_on_solved_field(pk, dtype):
    n = 256
    rng = np.random.default_rng(11)
    src = rng.choice(n * n, 16, replace=False)
    src = np.stack([src // n, src % n], axis=1).astype(np.int32)
    S = _solved(pk, n, src, dtype)
    start = rng.uniform(0, n - 1, size=(97, 2))  # not a multiple of the 64-thread group
    st, _ = _compare(pk, S, src, start, 0.5, 1.0, 3000)
    assert np.mean(st == 0) > 0.95


def test_paths_3d(pk):
    n = 40
    rng = np.random.default_rng(3)
    g = np.meshgrid(*[np.arange(n, dtype=np.float64)] * 3, indexing="ij")
    y = np.array([[12, 20, 30], [30, 8, 10]])
    S = np.minimum(np.sqrt(sum((g[d] - y[0, d]) ** 2 for d in range(3))),
                   np.sqrt(sum((g[d] - y[1, d]) ** 2 for d in range(3))) + 2.0)
    start = rng.uniform(0, n - 1, size=(70, 3))
    for dt in (np.float32, np.float64):
        st, _ = _compare(pk, S.astype(dt), y, start, 0.5, 1.0, 400)
        assert np.all(st == 0)


def test_plane_wave_exact(pk):
    g = np.meshgrid(np.arange(64.0), np.arange(80.0), indexing="ij")
    S = 0.6 * g[0] + 0.8 * g[1]
    start = np.array([[40.0, 50.0]])
    path, npts, st = pk.backtrack(torch.as_tensor(S).to("cuda:0"), [[28, 34]], start, 0.5, 1.0, 100)
    path = path.cpu().numpy()
    assert int(st[0]) == 0 and int(npts[0]) == 40
    k = np.arange(40)[:, None]
    np.testing.assert_allclose(path[0, :40], start - 0.5 * k * np.array([0.6, 0.8]), atol=1e-12)


def test_edge_cases(pk):
    g = np.meshgrid(np.arange(16.0), np.arange(16.0), indexing="ij")
    S = g[0] + g[1]
    S[5:7, :] = np.inf
    start = np.array([[8.0, 8.0], [3.2, 3.1], [-1.0, 4.0], [4.0, 15.5], [np.nan, 1.0],
                      [12.0, 12.0], [15.0, 15.0], [0.0, 0.0]])
    st, npts = _compare(pk, S, np.array([[3, 3]]), start, 0.5, 1.0, 50)
    assert list(st[2:5]) == [3, 3, 3] and list(npts[2:5]) == [0, 0, 0]
    assert st[1] == 0 and npts[1] == 1
    assert st[5] == 2  # runs into S = +inf
    # flat field, no sources, max_steps = 0
    st, npts = _compare(pk, np.ones((16, 16)), np.zeros((0, 2), np.int32), start[:2], 0.5, 1.0, 0)
    assert list(st) == [1, 1] and list(npts) == [1, 1]
    st, npts = _compare(pk, np.ones((16, 16)), np.array([[3, 3]]), start[:1], 0.5, 1.0, 5)
    assert st[0] == 2
    # no paths
    path, npts, st = pk.backtrack(torch.ones(8, 8, device="cuda:0"), [[1, 1]], np.zeros((0, 2)))
    assert path.shape == (0, 4097, 2)


def test_many_sources_beyond_lds(pk):
    # 600 sources: the first 512 are kept in LDS, the rest read from memory
    n = 128
    rng = np.random.default_rng(9)
    idx = rng.choice(n * n, 600, replace=False)
    src = np.stack([idx // n, idx % n], axis=1).astype(np.int32)
    g = np.meshgrid(np.arange(float(n)), np.arange(float(n)), indexing="ij")
    # distance to the last source only: paths must end there
    S = np.hypot(g[0] - src[-1, 0], g[1] - src[-1, 1])
    start = rng.uniform(0, n - 1, size=(64, 2))
    st, _ = _compare(pk, S, src, start, 0.5, 0.3, 1000)
    assert np.all(st == 0)
