"""Pins of the full-gradient oracle (dL/df with the reference forcing's
dependence on f, and dL/dhbar) against central differences of the C oracle's
forward solve, and of its pieces against the oracle's kernel and
convolution; CPU only."""
import numpy as np
import pytest

import oracle
from oracle import grad


def _setup(seed=3, shape=(20, 24)):
    rng = np.random.default_rng(seed)
    import workloads
    f = workloads.smoothed_noise(shape, 2.0, 1.0, 2.0, rng)
    src = np.array([[4, 5], [15, 18], [9, 20]], np.int32)
    s = np.array([0.0, 0.03, 0.05])
    target = oracle.solve(f * 1.05, src, 1.0 / 24, 0.08, 6, src_s=s)["S"]
    wgt = rng.uniform(0.5, 1.5, size=shape)
    return f, src, s, target, wgt


def _loss(f, src, s, target, wgt, hbar, mode, ftilde=None, T=6):
    S = oracle.solve(f, src, 1.0 / 24, hbar, T, ft_mode=mode, ftilde=ftilde, src_s=s)["S"]
    return float(np.sum(wgt * (S - target) ** 2)), 2.0 * wgt * (S - target)


def test_kernel_beta_derivative_matches_differences():
    dims, beta, db = (12, 15), 0.37, 1e-5
    num = (oracle.kappa(dims, beta + db) - oracle.kappa(dims, beta - db)) / (2 * db)
    np.testing.assert_allclose(grad.kappa_dbeta(dims, beta), num, rtol=1e-7, atol=1e-12)


def test_table_convolution_matches_oracle_convolution():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((13, 21))
    beta = 0.6
    np.testing.assert_allclose(grad.conv_table(x, oracle.kappa(x.shape, beta)),
                               oracle.conv(x, beta), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("mode", ["nu", "fmax", "given"])
def test_hbar_derivative_matches_differences(mode):
    f, src, s, target, wgt = _setup()
    hbar, dh = 0.08, 1e-5
    ft = 1.6 if mode == "given" else None
    L0, dLdS = _loss(f, src, s, target, wgt, hbar, mode, ft)
    g = grad.full_gradient(f, src, 1.0 / 24, hbar, 6, dLdS, ft_mode=mode, ftilde=ft, src_s=s)
    Lp = _loss(f, src, s, target, wgt, hbar + dh, mode, ft)[0]
    Lm = _loss(f, src, s, target, wgt, hbar - dh, mode, ft)[0]
    num = (Lp - Lm) / (2 * dh)
    assert abs(g["dLdhbar"] - num) <= 1e-6 * abs(num), (g["dLdhbar"], num)


@pytest.mark.parametrize("mode", ["nu", "fmax"])
def test_f_derivative_with_reference_forcing_matches_differences(mode):
    # a direction that moves the extreme values of f (and so ftilde) as well
    f, src, s, target, wgt = _setup()
    hbar = 0.08
    L0, dLdS = _loss(f, src, s, target, wgt, hbar, mode)
    g = grad.full_gradient(f, src, 1.0 / 24, hbar, 6, dLdS, ft_mode=mode, src_s=s)
    rng = np.random.default_rng(9)
    d = rng.standard_normal(f.shape)
    eps = 1e-6
    num = (_loss(f + eps * d, src, s, target, wgt, hbar, mode)[0]
           - _loss(f - eps * d, src, s, target, wgt, hbar, mode)[0]) / (2 * eps)
    ana = float(np.sum(g["dLdf"] * d))
    assert abs(ana - num) <= 1e-6 * abs(num), (ana, num)
    # the reference-forcing part is not negligible here
    assert abs(g["dLdftilde"]) > 1e-3 * np.abs(g["dLdf"]).max()


def test_given_ftilde_reduces_to_the_fixed_adjoint():
    f, src, s, target, wgt = _setup()
    hbar = 0.08
    L0, dLdS = _loss(f, src, None, target, wgt, hbar, "given", 1.6)
    g = grad.full_gradient(f, src, 1.0 / 24, hbar, 6, dLdS, ft_mode="given", ftilde=1.6)
    ref, _ = oracle.adjoint(f, src, 1.0 / 24, hbar, 6, dLdS, ft_mode="given", ftilde=1.6)
    np.testing.assert_allclose(g["dLdf"], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


# ---- 3D ----------------------------------------------------------------------

H3, HBAR3, T3 = 1.0 / 12, 0.15, 4


def _setup3(seed=5, shape=(10, 12, 9)):
    rng = np.random.default_rng(seed)
    import workloads
    f = workloads.smoothed_noise(shape, 1.5, 1.0, 2.0, rng)
    src = np.array([[2, 3, 4], [7, 9, 2]], np.int32)
    s = np.array([0.0, 0.04])
    target = oracle.solve(f * 1.05, src, H3, HBAR3, T3, src_s=s)["S"]
    wgt = rng.uniform(0.5, 1.5, size=shape)
    return f, src, s, target, wgt


def _loss3(f, src, s, target, wgt, hbar, mode, ftilde=None):
    S = oracle.solve(f, src, H3, hbar, T3, ft_mode=mode, ftilde=ftilde, src_s=s)["S"]
    return float(np.sum(wgt * (S - target) ** 2)), 2.0 * wgt * (S - target)


@pytest.mark.parametrize("beta", [0.37, 1.3])  # both branches of the 3D origin value
def test_kernel_beta_derivative_matches_differences_3d(beta):
    dims, db = (7, 9, 6), 1e-5
    num = (oracle.kappa(dims, beta + db) - oracle.kappa(dims, beta - db)) / (2 * db)
    np.testing.assert_allclose(grad.kappa_dbeta(dims, beta), num, rtol=1e-7, atol=1e-12)


def test_table_convolution_matches_oracle_convolution_3d():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((9, 6, 11))
    beta = 0.8
    np.testing.assert_allclose(grad.conv_table(x, oracle.kappa(x.shape, beta)),
                               oracle.conv(x, beta), rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("mode", ["nu", "fmax", "given"])
def test_hbar_derivative_matches_differences_3d(mode):
    f, src, s, target, wgt = _setup3()
    dh = 1e-5
    ft = 1.7 if mode == "given" else None
    L0, dLdS = _loss3(f, src, s, target, wgt, HBAR3, mode, ft)
    g = grad.full_gradient(f, src, H3, HBAR3, T3, dLdS, ft_mode=mode, ftilde=ft, src_s=s)
    num = (_loss3(f, src, s, target, wgt, HBAR3 + dh, mode, ft)[0]
           - _loss3(f, src, s, target, wgt, HBAR3 - dh, mode, ft)[0]) / (2 * dh)
    assert abs(g["dLdhbar"] - num) <= 1e-6 * abs(num), (g["dLdhbar"], num)


@pytest.mark.parametrize("mode", ["nu", "fmax"])
def test_f_derivative_with_reference_forcing_matches_differences_3d(mode):
    f, src, s, target, wgt = _setup3()
    L0, dLdS = _loss3(f, src, s, target, wgt, HBAR3, mode)
    g = grad.full_gradient(f, src, H3, HBAR3, T3, dLdS, ft_mode=mode, src_s=s)
    d = np.random.default_rng(11).standard_normal(f.shape)
    eps = 1e-6
    num = (_loss3(f + eps * d, src, s, target, wgt, HBAR3, mode)[0]
           - _loss3(f - eps * d, src, s, target, wgt, HBAR3, mode)[0]) / (2 * eps)
    ana = float(np.sum(g["dLdf"] * d))
    assert abs(ana - num) <= 1e-6 * abs(num), (ana, num)
    assert abs(g["dLdftilde"]) > 1e-3 * np.abs(g["dLdf"]).max()


def test_given_ftilde_reduces_to_the_fixed_adjoint_3d():
    f, src, s, target, wgt = _setup3()
    L0, dLdS = _loss3(f, src, None, target, wgt, HBAR3, "given", 1.7)
    g = grad.full_gradient(f, src, H3, HBAR3, T3, dLdS, ft_mode="given", ftilde=1.7)
    ref, _ = oracle.adjoint(f, src, H3, HBAR3, T3, dLdS, ft_mode="given", ftilde=1.7)
    np.testing.assert_allclose(g["dLdf"], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
