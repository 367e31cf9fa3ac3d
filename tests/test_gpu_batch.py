"""GPU tests of the uneven batch (sweik_batch_*): one launch per pass and
size class over a device work list, eager and captured into a HIP graph.

Every instance of a batch must equal the same problem solved alone (the
batched kernels run the single-solve code per work-group, so the results
are bit-identical), and two instances are checked against the FP64 oracle.
Graph replays are checked against the eager result, with unrelated eager
work and synchronisations between the replays.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads
from common import TOL, ensure_built, envelope_violations, report

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


# (dims, hbar, n_src, ftilde_mode): five size classes, ragged edges, two
# instances sharing a class with different row counts
INSTANCES = [
    ((64, 64), 0.05, 3, "nu"),
    ((100, 76), 0.2, 5, "nu"),
    ((60, 50), 0.1, 1, "fmax"),
    ((33, 130), 0.06, 2, "nu"),
    ((7, 300), 0.3, 2, "nu"),
    ((128, 128), 0.08, 8, "nu"),
    ((40, 64), 0.12, 4, "nu"),
]
T = 6


def _make(prec, seed=11):
    rng = np.random.default_rng(seed)
    dt = torch.float32 if prec == "fp32" else torch.float64
    probs, fs, srcs, hosts = [], [], [], []
    for dims, hbar, n_src, ftm in INSTANCES:
        f = workloads.smoothed_noise(dims, 4.0, 1.0, 3.0, rng).astype(np.float32)
        src = workloads.distinct_sources(dims, n_src, rng)
        h = 1.0 / max(dims)
        probs.append({"dims": dims, "h": h, "hbar": hbar, "T": T, "n_src": n_src,
                      "ftilde_mode": ftm})
        fs.append(torch.as_tensor(f.astype(np.float64)).to("cuda", dt))
        srcs.append(torch.as_tensor(src.astype(np.int32)).to("cuda"))
        hosts.append((f, src, h, hbar, ftm))
    return probs, fs, srcs, hosts


def _single(prec, fs, hosts):
    import paper_1403_1937_amd as pk
    out, infos = [], []
    for f, (_, src, h, hbar, ftm) in zip(fs, hosts):
        S, info = pk.solve(f, src, h, hbar, T, ftilde_mode=ftm, return_info=True)
        out.append(S)
        infos.append(info)
    torch.cuda.synchronize()
    return out, infos


def _info_list(buf, n):
    import ctypes as C
    from paper_1403_1937_amd._native import _Info, _info_dict
    raw = buf.cpu().numpy().tobytes()
    sz = C.sizeof(_Info)
    return [_info_dict(_Info.from_buffer_copy(raw[i * sz:(i + 1) * sz])) for i in range(n)]


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_matches_single_and_oracle(prec):
    import paper_1403_1937_amd as pk
    from paper_1403_1937_amd._native import info_struct_size
    probs, fs, srcs, hosts = _make(prec)
    print(f"batch eager prec {prec}: {len(probs)} instances", flush=True)
    b = pk.Batch(probs, prec)
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    Ss = [torch.full_like(f, -1.0) for f in fs]
    infos = torch.zeros(len(probs) * info_struct_size(), dtype=torch.uint8, device="cuda")
    b.solve(fs, srcs, Ss, ws, infos=infos)
    torch.cuda.synchronize()
    ref, ref_info = _single(prec, fs, hosts)
    got_info = _info_list(infos, len(probs))
    for i, (S, R) in enumerate(zip(Ss, ref)):
        assert torch.equal(S, R), f"instance {i} {INSTANCES[i][0]} differs from its single solve"
        gi, ri = got_info[i], ref_info[i]
        assert gi["ftilde"] == ri["ftilde"] and gi["scale_exp"] == ri["scale_exp"]
        assert gi["flags"] == ri["flags"] == 0
    for i in (1, 3):
        f, src, h, hbar, ftm = hosts[i]
        o = oracle.solve(f.astype(np.float64), src, h, hbar, T, ft_mode=ftm)
        S = Ss[i].double().cpu().numpy()
        worst, frac, _ = report(S, o, hbar, prec)
        print(f"  instance {i}: max rel {worst:.3e} on {frac:.3f}", flush=True)
        assert worst <= TOL[prec]
        assert envelope_violations(S, o, hbar, prec) == 0


def test_batch_graph_replays():
    import paper_1403_1937_amd as pk
    prec = "fp32"
    probs, fs, srcs, hosts = _make(prec, seed=12)
    print("batch graph: eager reference", flush=True)
    b = pk.Batch(probs, prec)
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    eager = [torch.empty_like(f) for f in fs]
    b.solve(fs, srcs, eager, ws)
    torch.cuda.synchronize()
    Ss = [torch.empty_like(f) for f in fs]
    for rep in range(4):
        print(f"  replay {rep}", flush=True)
        for S in Ss:
            S.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()  # unrelated eager work, then a sync
        b.solve(fs, srcs, Ss, ws, graph=True)
        torch.cuda.synchronize()
        for i, (S, E) in enumerate(zip(Ss, eager)):
            assert torch.equal(S, E), f"replay {rep} instance {i} differs from eager"
    # other output buffers: the batch re-captures
    Ss2 = [torch.empty_like(f) for f in fs]
    b.solve(fs, srcs, Ss2, ws, graph=True)
    torch.cuda.synchronize()
    for i, (S, E) in enumerate(zip(Ss2, eager)):
        assert torch.equal(S, E), f"re-captured graph instance {i} differs from eager"


def test_batch_rejects_mixed_and_bad_args():
    import paper_1403_1937_amd as pk
    base = {"dims": (64, 64), "h": 1 / 64, "hbar": 0.1, "T": 4, "n_src": 1}
    with pytest.raises(ValueError):
        pk.Batch([base, dict(base, T=5)], "fp32")
    with pytest.raises(ValueError):
        pk.Batch([base, dict(base, dims=(8, 8, 8))], "fp32")
    b = pk.Batch([base], "fp32")
    f = torch.ones(64, 64, device="cuda")
    src = torch.zeros(1, 2, dtype=torch.int32, device="cuda")
    S = torch.empty_like(f)
    small = torch.empty(b.workspace_bytes - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        b.solve([f], [src], [S], small)


def test_benchmark_batch_full_size_sampled():
    """The 64-instance batch the benchmark times (edges 256..2048, T = 12,
    FP32-scaled), solved by one graph replay at full size; one instance of
    each edge length is checked against the FP64 oracle over its whole grid
    (resolvable set and envelope)."""
    import paper_1403_1937_amd as pk
    probs = workloads.batch_problems()
    b = pk.Batch([{"dims": q.dims, "h": q.h, "hbar": q.hbar, "T": q.T, "n_src": len(q.src)}
                  for q in probs], "fp32")
    fs = [torch.as_tensor(q.f).cuda() for q in probs]
    srcs = [torch.as_tensor(q.src).cuda() for q in probs]
    Ss = [torch.empty_like(f) for f in fs]
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    print(f"batch of {len(probs)}, sum N = {sum(q.dims[0] * q.dims[1] for q in probs)}", flush=True)
    b.solve(fs, srcs, Ss, ws, graph=True)
    torch.cuda.synchronize()
    seen = set()
    for i, q in enumerate(probs):
        if q.dims[0] in seen:
            continue
        seen.add(q.dims[0])
        o = oracle.solve(q.f.astype(np.float64), q.src, q.h, q.hbar, q.T)
        S = Ss[i].double().cpu().numpy()
        worst, frac, _ = report(S, o, q.hbar, "fp32")
        nbad = envelope_violations(S, o, q.hbar, "fp32")
        print(f"  instance {i} {q.dims} hbar {q.hbar:.3f} n_src {len(q.src)}: max rel "
              f"{worst:.3e} on {frac:.3f}; envelope violations {nbad}", flush=True)
        assert frac > 0.05
        assert worst <= TOL["fp32"]
        assert nbad == 0
    assert len(seen) >= 3


def test_batch_solves_create_nothing():
    """After sweik_batch_prepare, eager batch solves create no HIP resource
    and allocate no device memory; the graph variant creates one graph
    executable on its first call and nothing on replays."""
    import paper_1403_1937_amd as pk
    probs, fs, srcs, _ = _make("fp32", seed=12)
    b = pk.Batch(probs, "fp32")  # prepares
    Ss = [torch.empty_like(f) for f in fs]
    ws = torch.empty(b.workspace_bytes, dtype=torch.uint8, device="cuda")
    b.solve(fs, srcs, Ss, ws)
    torch.cuda.synchronize()
    ref = [S.clone() for S in Ss]
    free0, _ = torch.cuda.mem_get_info()
    n0 = pk._native.resource_count()
    for _ in range(6):  # more calls than the staging ring has slots
        b.solve(fs, srcs, Ss, ws)
    torch.cuda.synchronize()
    assert pk._native.resource_count() == n0
    assert torch.cuda.mem_get_info()[0] == free0
    assert all(torch.equal(S, R) for S, R in zip(Ss, ref))
    b.solve(fs, srcs, Ss, ws, graph=True)
    torch.cuda.synchronize()
    assert pk._native.resource_count() == n0 + 1
    n1 = pk._native.resource_count()
    for _ in range(3):
        b.solve(fs, srcs, Ss, ws, graph=True)
    torch.cuda.synchronize()
    assert pk._native.resource_count() == n1
    assert all(torch.equal(S, R) for S, R in zip(Ss, ref))


def test_batch_solve_needs_prepare():
    """A batch that was not prepared is rejected before anything is
    enqueued."""
    import ctypes as C
    import paper_1403_1937_amd as pk
    probs, fs, srcs, _ = _make("fp32", seed=13)
    lib = pk.load_library()
    arr = (pk._native._Problem * len(probs))()
    for i, q in enumerate(probs):
        arr[i].ndim = 2
        arr[i].dims = (C.c_int64 * 3)(q["dims"][0], q["dims"][1], 1)
        arr[i].h, arr[i].hbar, arr[i].T, arr[i].n_src = q["h"], q["hbar"], q["T"], q["n_src"]
        arr[i].prec, arr[i].ft_mode = 0, 0
    h = C.c_void_p()
    assert lib.sweik_batch_create(arr, len(probs), C.byref(h)) == 0
    try:
        Ss = [torch.empty_like(f) for f in fs]
        ws = torch.empty(int(lib.sweik_batch_workspace_bytes(h)), dtype=torch.uint8,
                         device="cuda")
        P = C.c_void_p * len(fs)
        rc = lib.sweik_batch_solve(h, P(*[f.data_ptr() for f in fs]),
                                   P(*[s.data_ptr() for s in srcs]),
                                   P(*[S.data_ptr() for S in Ss]), ws.data_ptr(), ws.numel(),
                                   None, None)
        assert rc == 1  # SWEIK_EINVAL
    finally:
        lib.sweik_batch_destroy(h)
