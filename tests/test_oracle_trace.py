"""Pins of the backtracking oracle (Section 6, eq. PathPlanning-backTrackOnS)
against closed forms and invariants; CPU only."""
import numpy as np
import pytest

from oracle import trace

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _grid(shape):
    return np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")


def test_plane_wave_2d_exact():
    # S = 0.6 m0 + 0.8 m1: every difference and interpolation is exact, so the
    # path is x_k = start - k step (0.6, 0.8) until it is within the radius
    m0, m1 = _grid((64, 80))
    S = 0.6 * m0 + 0.8 * m1
    start = np.array([[40.0, 50.0]])
    src = np.array([[28, 34]])  # start - 20 (0.6, 0.8)
    path, npts, st = trace.backtrack(S, src, start, step=0.5, radius=1.0, max_steps=100)
    # distance to the source is 20 - k/2 < 1 first at k = 39
    assert st[0] == 0 and npts[0] == 40
    k = np.arange(40)[:, None]
    want = start + (-0.5 * k) * np.array([0.6, 0.8])
    np.testing.assert_allclose(path[0, :40], want, atol=1e-12)


def test_plane_wave_3d_exact():
    m0, m1, m2 = _grid((20, 24, 28))
    a = np.array([2.0, -3.0, 6.0]) / 7.0
    S = a[0] * m0 + a[1] * m1 + a[2] * m2
    start = np.array([[10.0, 5.0, 20.0]])
    src = (start[0] - 14.0 * a).round().astype(int)[None, :]  # 14 a = (4, -6, 12): integral
    path, npts, st = trace.backtrack(S, src, start, step=0.25, radius=0.5, max_steps=200)
    assert st[0] == 0 and npts[0] == 56  # 14 - k/4 < 0.5 first at k = 55
    k = np.arange(56)[:, None]
    np.testing.assert_allclose(path[0, :56], start - 0.25 * k * a, atol=1e-12)


def test_curved_paths_fourth_order():
    # S = x0^2 + 4 x1^2 about the centre: differences and interpolation of the
    # node gradients are exact for a quadratic, and the normalised gradient
    # flow follows x1 = C x0^4.  RK4 error drops 16x when the step halves.
    n, c = 201, 100.0
    m0, m1 = _grid((n, n))
    S = (m0 - c) ** 2 + 4 * (m1 - c) ** 2
    start = np.array([[c + 80, c + 30], [c - 70, c + 40], [c + 90, c - 20]])
    errs = []
    for step in (1.0, 0.5):
        path, npts, st = trace.backtrack(S, np.array([[100, 100]]), start, step=step,
                                         radius=3.0, max_steps=2000)
        assert np.all(st == 0)
        e = 0.0
        for q in range(len(start)):
            pts = path[q, :npts[q]] - c
            C0 = pts[0, 1] / pts[0, 0] ** 4
            far = np.abs(pts[:, 0]) > 20
            e = max(e, float(np.max(np.abs(pts[far, 1] / pts[far, 0] ** 4 / C0 - 1))))
        errs.append(e)
    assert errs[0] < 3e-5
    assert 10.0 < errs[0] / errs[1] < 25.0


def test_cone_paths_are_straight():
    # S = |m - y|: the paths run straight to the source, one step per `step`
    n = 65
    m0, m1 = _grid((n, n))
    y = np.array([32.0, 32.0])
    S = np.hypot(m0 - y[0], m1 - y[1])
    ang = np.linspace(0.1, 2 * np.pi, 12, endpoint=False)
    start = y + 25.0 * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    path, npts, st = trace.backtrack(S, y[None, :].astype(int), start, step=0.5, radius=1.5,
                                     max_steps=500)
    assert np.all(st == 0)
    for q in range(len(start)):
        pts = path[q, :npts[q]]
        d = start[q] - y
        d /= np.linalg.norm(d)
        rel = pts - y
        perp = np.abs(rel[:, 0] * d[1] - rel[:, 1] * d[0])
        assert perp.max() < 0.05
        # about (25 - 1.5) / 0.5 steps
        assert abs(npts[q] - 1 - (25.0 - 1.5) / 0.5) <= 2


def test_degenerate_cases():
    S = np.ones((16, 16))
    src = np.array([[3, 3]])
    start = np.array([[8.0, 8.0], [3.2, 3.1], [-1.0, 4.0], [4.0, 15.5], [np.nan, 1.0]])
    path, npts, st = trace.backtrack(S, src, start, step=0.5, radius=1.0, max_steps=10)
    # flat S: no direction; on the source: done; outside the box or NaN: rejected
    np.testing.assert_array_equal(st, [2, 0, 3, 3, 3])
    np.testing.assert_array_equal(npts, [1, 1, 0, 0, 0])
    m0, m1 = _grid((16, 16))
    path, npts, st = trace.backtrack(m0 + m1, src, start[:1], step=0.5, radius=1.0, max_steps=0)
    assert st[0] == 1 and npts[0] == 1
    # S = +inf somewhere on the way: the gradient is not finite there
    S2 = (m0 + m1).copy()
    S2[5:7, :] = np.inf
    path, npts, st = trace.backtrack(S2, src, np.array([[12.0, 12.0]]), step=0.5, radius=1.0,
                                     max_steps=100)
    assert st[0] == 2


def test_paths_on_a_solved_field_reach_sources():
    # the value function has no local minima (Section 6): every path from a
    # smooth-forcing solve ends at a source
    import oracle
    rng = np.random.default_rng(7)
    n = 64
    m0, m1 = _grid((n, n))
    f = 1.0 + 0.5 * np.exp(-((m0 - 20) ** 2 + (m1 - 40) ** 2) / 200.0)
    src = np.array([[10, 10], [50, 45], [30, 60]], np.int32)
    o = oracle.solve(f, src, 1.0 / n, 0.03, 8)
    S = o["S"]
    assert np.all(np.isfinite(S))
    start = rng.uniform(2, n - 3, size=(40, 2))
    path, npts, st = trace.backtrack(S, src, start, step=0.25, radius=1.0, max_steps=4000)
    assert np.all(st == 0)
    # ... and the interpolated S does not rise along a path (beyond 0.1 % of
    # its range: the steps follow the interpolated node gradients, not the
    # gradient of the interpolated S)
    from scipy.ndimage import map_coordinates
    for q in range(len(start)):
        s = map_coordinates(S, path[q, :npts[q]].T, order=1)
        assert np.all(np.diff(s) < 1e-3 * np.abs(s[:-1]).max())
