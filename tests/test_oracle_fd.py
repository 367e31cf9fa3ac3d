"""Pins of the finite-difference oracle (Section 6, eq. sparse-system); CPU only.

With constant f the matrix is diagonalised by the orthonormal type-I sine
transform (one per axis, eigenvalues 2 - 2 cos(pi k / (n + 1)) of the
Dirichlet second difference): an independent closed form of A^-1 b.  With
variable f, A is an M-matrix: phi > 0, a larger f gives a smaller phi, and
mirror symmetry of (f, sources) carries over to phi."""
import numpy as np
import pytest
from scipy.fft import dstn

from oracle import fd


def _dst_solve(dims, src, d):
    b = fd.rhs(dims, src)
    lam = d
    for ax, n in enumerate(dims):
        k = np.arange(1, n + 1)
        shape = [1] * len(dims)
        shape[ax] = n
        lam = lam + (2.0 - 2.0 * np.cos(np.pi * k / (n + 1))).reshape(shape)
    return dstn(dstn(b, type=1, norm="ortho") / lam, type=1, norm="ortho")


@pytest.mark.parametrize("dims,src", [((24, 31), [[5, 7], [20, 3], [11, 30]]),
                                      ((10, 12, 14), [[2, 3, 4], [9, 0, 13]])])
def test_constant_forcing_matches_sine_transform(dims, src):
    h, hbar, c = 0.05, 0.1, 1.7
    f = np.full(dims, c)
    o = fd.solve(f, np.array(src), h, hbar)
    want = _dst_solve(dims, np.array(src), (h * c / hbar) ** 2)
    # the transform route rounds at ~1e-16 of the largest value
    np.testing.assert_allclose(o["phi"], want, rtol=1e-11, atol=1e-15 * want.max())
    big = want > 1e-6 * want.max()
    np.testing.assert_allclose(o["S"][big], -hbar * np.log(want[big]), rtol=1e-11)


def test_m_matrix_properties():
    rng = np.random.default_rng(4)
    n0, n1 = 30, 26
    f = rng.uniform(1.0, 3.0, size=(n0 // 2, n1))
    f = np.concatenate([f, f[::-1]], axis=0)  # mirror symmetric in axis 0
    src = np.array([[4, 5], [n0 - 1 - 4, 5], [9, 20], [n0 - 1 - 9, 20]])
    h, hbar = 1.0 / 32, 0.05
    phi = fd.solve(f, src, h, hbar)["phi"]
    assert np.all(phi > 0)
    np.testing.assert_allclose(phi, phi[::-1], rtol=1e-12)
    phi2 = fd.solve(f * 1.3, src, h, hbar)["phi"]
    assert np.all(phi2 <= phi) and np.all(phi2[phi2 > 1e-300] < phi[phi2 > 1e-300])
    # at a source phi >= (A^-1)_ss >= 1 / A_ss (A symmetric positive definite;
    # the other sources only add positive terms)
    d = (h * f / hbar) ** 2
    assert np.all(phi[tuple(src.T)] >= 1.0 / (4.0 + d[tuple(src.T)]))


@pytest.mark.filterwarnings("ignore::RuntimeWarning")
def test_fd_and_series_agree_to_order_hbar():
    # the FD system and the perturbation series discretise the same screened
    # Poisson problem differently (and normalise phi differently at the
    # source), so their S agree up to O(hbar): the gap divided by hbar stays
    # bounded as hbar shrinks, on the set the FP64 series resolves
    import oracle
    n = 96
    h = 1.0 / n
    m0, m1 = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    f = 1.0 + 0.4 * np.exp(-((m0 - 40) ** 2 + (m1 - 60) ** 2) / 300.0)
    src = np.array([[48, 30]], np.int32)
    far = np.hypot(m0 - 48, m1 - 30) > 6
    gaps = []
    for hbar in (0.08, 0.04, 0.02):
        o = oracle.solve(f, src, h, hbar, 20)
        lam = np.log(o["phi"].max() / np.where(o["phi"] > 0, o["phi"], 1e-300))
        mk = far & (lam < 9)
        gap = np.abs(fd.solve(f, src, h, hbar)["S"] - o["S"])[mk].max() / hbar
        gaps.append(gap)
    assert max(gaps) < 8.0
    assert gaps[-1] < gaps[0]
