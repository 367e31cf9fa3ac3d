"""The finite-difference screened Poisson solve on the GPU (Section 6, eq.
sparse-system) against the sparse direct oracle, the sine-transform closed
form for constant f, and (at the benchmark size, where no direct solve is
practical) the true residual of the linear system."""
import numpy as np
import pytest
import torch

from common import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    ensure_built()
    import paper_1403_1937_amd as pk
    return pk


def _smooth(shape, seed, lo, hi):
    import workloads
    return workloads.smoothed_noise(shape, 3.0, lo, hi, np.random.default_rng(seed))


def _sources(shape, k, seed):
    rng = np.random.default_rng(seed)
    idx = rng.choice(int(np.prod(shape)), k, replace=False)
    return np.stack(np.unravel_index(idx, shape), axis=1).astype(np.int32)


def _residual(f, src, h, hbar, phi):
    """||A phi - b|| / ||b|| with the five/seven-point stencil, in float64."""
    from oracle import fd
    A = fd.matrix(f, h, hbar)
    b = fd.rhs(f.shape, src).ravel()
    return np.linalg.norm(A @ phi.ravel() - b) / np.linalg.norm(b)


@pytest.mark.parametrize("shape", [(64, 80), (20, 24, 28)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_matches_direct_solve(pk, shape, dtype):
    from oracle import fd
    h, hbar = 1.0 / 64, 0.05
    f = _smooth(shape, 1, 1.0, 3.0)
    src = _sources(shape, 5, 2)
    ft = torch.as_tensor(f).to("cuda:0", dtype)
    S, info = pk.fd_solve(ft, src, h, hbar, rtol=1e-13, return_info=True)
    print(shape, dtype, info, flush=True)
    assert info["converged"] == 1 and info["rel_residual"] <= 1e-13
    assert info["flags"] == 0 and info["n_sources"] == 5 and info["n_nonpositive_phi"] == 0
    f64 = ft.double().cpu().numpy()  # the forcing the GPU saw
    o = fd.solve(f64, src, h, hbar)
    S = S.double().cpu().numpy()
    # CG leaves an error of about rtol (times the condition number) relative
    # to the largest phi, so phi is compared against its maximum; S = -hbar
    # ln phi only where phi is within 1e-4 of it.  A float32 S adds one
    # rounding: 6e-8 S / hbar relative in phi.
    f32 = dtype == torch.float32
    phi = np.exp(-S / hbar)
    err = np.abs(phi - o["phi"]).max() / o["phi"].max()
    assert err < (1e-5 if f32 else 1e-11), err
    ok = o["phi"] > 1e-4 * o["phi"].max()
    rel = np.abs(S[ok] - o["S"][ok]) / np.maximum(np.abs(o["S"][ok]), hbar)
    assert rel.max() < (1e-6 if f32 else 1e-8), rel.max()


def test_constant_forcing_closed_form(pk):
    from scipy.fft import dstn
    from oracle import fd
    shape, h, hbar, c = (50, 37), 0.02, 0.05, 1.3
    src = _sources(shape, 3, 5)
    S = pk.fd_solve(torch.full(shape, c, dtype=torch.float64, device="cuda:0"), src, h, hbar,
                    rtol=1e-14).cpu().numpy()
    lam = (h * c / hbar) ** 2
    for ax, n in enumerate(shape):
        k = np.arange(1, n + 1)
        sh = [1, 1]
        sh[ax] = n
        lam = lam + (2.0 - 2.0 * np.cos(np.pi * k / (n + 1))).reshape(sh)
    phi = dstn(dstn(fd.rhs(shape, src), type=1, norm="ortho") / lam, type=1, norm="ortho")
    assert np.abs(np.exp(-S / hbar) - phi).max() < 1e-11 * phi.max()
    ok = phi > 1e-4 * phi.max()
    np.testing.assert_allclose(S[ok], -hbar * np.log(phi[ok]), rtol=1e-8)


def test_iteration_limit_and_no_iterations(pk):
    shape = (32, 32)
    f = torch.as_tensor(_smooth(shape, 3, 1.0, 2.0)).to("cuda:0")
    src = _sources(shape, 2, 4)
    S, info = pk.fd_solve(f, src, 1.0 / 32, 0.05, max_iter=0, return_info=True)
    assert info["iterations"] == 0 and info["converged"] == 0
    assert info["n_nonpositive_phi"] == 32 * 32 and torch.isinf(S).all()
    S, info = pk.fd_solve(f, src, 1.0 / 32, 0.05, max_iter=5, return_info=True)
    assert info["iterations"] == 5 and info["converged"] == 0 and info["rel_residual"] > 1e-6
    # more than one chunk of iterations, converged inside the last one
    # (a large hbar: weak screening, slow convergence)
    S, info = pk.fd_solve(f, src, 1.0 / 32, 0.5, rtol=1e-12, return_info=True)
    assert info["converged"] == 1 and info["iterations"] > 64


def test_benchmark_size_true_residual(pk):
    import workloads
    p = workloads.problem(2, 1024)
    f = torch.as_tensor(p.f).to("cuda:0", torch.float64)
    S, info = pk.fd_solve(f, p.src, p.h, p.hbar, rtol=1e-10, return_info=True)
    print("1024^2:", info, flush=True)
    assert info["converged"] == 1
    S = S.cpu().numpy()
    phi = np.exp(-S / p.hbar)
    # the residual of the recursion tracks the true one
    assert _residual(p.f.astype(np.float64), p.src, p.h, p.hbar, phi) < 1e-8
