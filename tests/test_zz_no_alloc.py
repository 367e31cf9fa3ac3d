"""GPU test of sweik_solve_noalloc, the solve for callers that cannot
allocate: its workspace is the library's static device array.  Called
through the C ABI (ctypes), its results are compared with sweik_solve's on
the same inputs (the same kernels in the same order: bit-identical), on
two calls in a row, the second with a smaller grid, then a 3D call; after
the first call nothing is allocated and no HIP resource is created.  A plan
whose workspace exceeds the array is rejected before anything runs."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads
from common import ensure_built

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _inputs(dims, n_src, prec, seed):
    rng = np.random.default_rng(seed)
    f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
    src = workloads.distinct_sources(dims, n_src, rng)
    dt = torch.float32 if prec == "fp32" else torch.float64
    return (torch.as_tensor(f.astype(np.float64)).to("cuda", dt),
            torch.as_tensor(src).to("cuda"), src)


def _both(pk, lib, dims, h, hbar, T, n_src, prec, seed):
    """(S and info of sweik_solve_noalloc, S and info of sweik_solve)."""
    f, d_src, src = _inputs(dims, n_src, prec, seed)
    pl = pk.Plan(dims, h, hbar, T, n_src, prec)
    pl.check_sources(src)
    assert pl.workspace_bytes <= lib.sweik_noalloc_scratch_bytes()
    info_sz = pk._native.info_struct_size()
    S_na = torch.full_like(f, float("nan"))
    info_na = torch.zeros(info_sz, dtype=torch.uint8, device="cuda")
    print(f"noalloc solve {dims} {prec} T={T}", flush=True)
    rc = lib.sweik_solve_noalloc(pl._h, f.data_ptr(), d_src.data_ptr(), S_na.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream, info_na.data_ptr())
    assert rc == 0, rc
    torch.cuda.synchronize()
    S_ref = torch.full_like(f, float("nan"))
    info_ref = torch.zeros(info_sz, dtype=torch.uint8, device="cuda")
    ws = pl.workspace("cuda")
    pl.solve(f, d_src, S_ref, ws, info=info_ref)
    torch.cuda.synchronize()
    return S_na, info_na, S_ref, info_ref


def test_noalloc_matches_solve_twice_then_smaller():
    import paper_1403_1937_amd as pk
    lib = pk.load_library()
    # first call on this device: looks up the array's address
    S1, i1, R1, j1 = _both(pk, lib, (256, 256), 1 / 256, 0.05, 8, 4, "fp32", 71)
    assert torch.equal(S1, R1)
    assert torch.equal(i1, j1)
    assert torch.isfinite(S1).float().mean().item() > 0.5
    # later calls: no allocation, no HIP resource
    free0 = torch.cuda.mem_get_info()[0]
    n0 = pk._native.resource_count()
    f, d_src, _ = _inputs((256, 256), 4, "fp32", 71)
    pl = pk.Plan((256, 256), 1 / 256, 0.05, 8, 4, "fp32")
    S = torch.empty_like(f)
    st = torch.cuda.current_stream().cuda_stream
    for _ in range(3):
        assert lib.sweik_solve_noalloc(pl._h, f.data_ptr(), d_src.data_ptr(), S.data_ptr(),
                                       st, None) == 0
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert pk._native.resource_count() == n0
    assert torch.equal(S, R1)
    # second shape, smaller, in float64: the array keeps the larger call's
    # contents, which the solve must not depend on
    S2, i2, R2, j2 = _both(pk, lib, (96, 80), 1 / 96, 0.08, 6, 3, "fp64", 72)
    assert torch.equal(S2, R2)
    assert torch.equal(i2, j2)
    # a 3D problem through the same entry point
    S3, i3, R3, j3 = _both(pk, lib, (20, 24, 28), 1 / 28, 0.1, 5, 2, "fp32", 73)
    assert torch.equal(S3, R3)


def test_noalloc_rejects_plans_beyond_the_array():
    import paper_1403_1937_amd as pk
    lib = pk.load_library()
    pl = pk.Plan((1024, 1024), 1 / 1024, 0.05, 16, 16, "fp32")
    assert pl.workspace_bytes > lib.sweik_noalloc_scratch_bytes()
    f = torch.ones((1024, 1024), device="cuda")
    src = torch.zeros((16, 2), dtype=torch.int32, device="cuda")
    S = torch.empty_like(f)
    rc = lib.sweik_solve_noalloc(pl._h, f.data_ptr(), src.data_ptr(), S.data_ptr(),
                                 torch.cuda.current_stream().cuda_stream, None)
    assert rc == 3  # SWEIK_EWORKSPACE
