"""Seeded synthetic inputs for the linearised eikonal solve.

This module is the only code shared between the CPU oracle and the GPU path.
It draws forcing fields f, point sources and receivers; it contains none of
the solver's arithmetic (no Green's function, no series, no logarithm of a
wave function).  Everything is deterministic in the seed.

Workload recipes (grid, spacing h, forcing, sources, hbar, number of series
terms T) follow the paper's setting: f positive and bounded on a regular grid
(problem statement in Section 1 and the convergence argument of Section 5.1),
a finite point set with S = 0 on it (Section 3.2), hbar small against the
domain size (Section 5.4 uses hbar/L between 0.02 and 0.06).  Grids of the
large workloads are unit boxes with h = 1/n.

The canonical forcing is float32: it is drawn in float64, rounded once, and
every consumer (FP32 path, FP64 path, oracle) reads those same values.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Problem", "gaussian_bumps_2d", "smoothed_noise", "gaussian_blobs_3d",
    "distinct_sources", "receivers_near_sources", "problem", "batch_problems",
    "WORKLOADS",
]


@dataclasses.dataclass
class Problem:
    """One eikonal instance: forcing f on a grid, sources, spacing, hbar, T."""
    f: np.ndarray            # float32, C order, shape = grid dims
    src: np.ndarray          # int32 [n_src, ndim], distinct grid indices
    h: float                 # isotropic grid spacing
    hbar: float
    T: int                   # number of series correction terms
    name: str = ""

    @property
    def dims(self) -> Tuple[int, ...]:
        return tuple(int(d) for d in self.f.shape)

    @property
    def ndim(self) -> int:
        return self.f.ndim

    @property
    def npoints(self) -> int:
        return int(self.f.size)


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def _affine(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    """Map min(x)..max(x) affinely onto lo..hi (float64)."""
    x = np.asarray(x, dtype=np.float64)
    a, b = float(x.min()), float(x.max())
    if b <= a:
        return np.full_like(x, 0.5 * (lo + hi))
    return lo + (hi - lo) * (x - a) / (b - a)


def gaussian_bumps_2d(n0: int, n1: int, count: int, amp: Tuple[float, float],
                      sigma_px: Tuple[float, float], rng: np.random.Generator
                      ) -> np.ndarray:
    """f = 1 + sum_j a_j exp(-|x - c_j|^2 / (2 sigma_j^2)), pixel units."""
    a = rng.uniform(amp[0], amp[1], count)
    s = rng.uniform(sigma_px[0], sigma_px[1], count)
    c0 = rng.uniform(0.0, n0, count)
    c1 = rng.uniform(0.0, n1, count)
    i0 = np.arange(n0, dtype=np.float64)[:, None]
    i1 = np.arange(n1, dtype=np.float64)[None, :]
    f = np.ones((n0, n1), dtype=np.float64)
    for j in range(count):
        r2 = (i0 - c0[j]) ** 2 + (i1 - c1[j]) ** 2
        f += a[j] * np.exp(-r2 / (2.0 * s[j] ** 2))
    return f


def smoothed_noise(shape: Sequence[int], sigma_px: float, lo: float, hi: float,
                   rng: np.random.Generator) -> np.ndarray:
    """iid N(0,1) noise, Gaussian-filtered (periodic wrap, truncated at 4
    sigma), then mapped affinely onto [lo, hi]."""
    from scipy.ndimage import gaussian_filter
    w = rng.standard_normal(tuple(int(s) for s in shape))
    sm = gaussian_filter(w, sigma=float(sigma_px), mode="wrap", truncate=4.0)
    return _affine(sm, lo, hi)


def gaussian_blobs_3d(n: int, count: int, lo: float, hi: float,
                      rng: np.random.Generator,
                      sigma_px: Tuple[float, float] = (8.0, 32.0)) -> np.ndarray:
    """Sum of `count` Gaussian blobs (amplitude U[0,1], sigma U[8,32] px,
    centres uniform in the cube), mapped affinely onto [lo, hi]."""
    a = rng.uniform(0.0, 1.0, count)
    s = rng.uniform(sigma_px[0] * n / 256.0, sigma_px[1] * n / 256.0, count)
    c = rng.uniform(0.0, n, (count, 3))
    ax = np.arange(n, dtype=np.float64)
    f = np.zeros((n, n, n), dtype=np.float64)
    for j in range(count):
        g0 = np.exp(-(ax - c[j, 0]) ** 2 / (2 * s[j] ** 2))
        g1 = np.exp(-(ax - c[j, 1]) ** 2 / (2 * s[j] ** 2))
        g2 = np.exp(-(ax - c[j, 2]) ** 2 / (2 * s[j] ** 2))
        f += a[j] * (g0[:, None, None] * g1[None, :, None] * g2[None, None, :])
    return _affine(f, lo, hi)


def distinct_sources(shape: Sequence[int], n_src: int,
                     rng: np.random.Generator) -> np.ndarray:
    """n_src distinct grid points drawn uniformly, as int32 [n_src, ndim]."""
    N = int(np.prod(shape))
    flat = rng.choice(N, size=n_src, replace=False)
    idx = np.stack(np.unravel_index(flat, tuple(shape)), axis=1)
    return np.ascontiguousarray(idx.astype(np.int32))


def receivers_near_sources(shape: Sequence[int], src: np.ndarray, count: int,
                           radius_px: float, rng: np.random.Generator
                           ) -> np.ndarray:
    """`count` distinct grid points, not sources, each within `radius_px`
    (Euclidean, pixels) of some source.  Points near the sources are where
    the wave function is well above rounding noise."""
    shape = tuple(int(s) for s in shape)
    taken = {tuple(int(v) for v in s) for s in src}
    out: List[Tuple[int, ...]] = []
    guard = 0
    while len(out) < count:
        guard += 1
        if guard > 1000 * count:
            raise RuntimeError("could not place receivers")
        k = int(rng.integers(0, len(src)))
        d = rng.standard_normal(len(shape))
        d *= rng.uniform(0.0, radius_px) / max(np.linalg.norm(d), 1e-12)
        p = tuple(int(np.clip(round(src[k][a] + d[a]), 0, shape[a] - 1))
                  for a in range(len(shape)))
        if p in taken:
            continue
        taken.add(p)
        out.append(p)
    return np.asarray(out, dtype=np.int32)


def _pack(f64: np.ndarray, src, h, hbar, T, name) -> Problem:
    f32 = np.ascontiguousarray(f64.astype(np.float32))
    return Problem(f=f32, src=np.ascontiguousarray(np.asarray(src, np.int32)),
                   h=float(h), hbar=float(hbar), T=int(T), name=name)


# ---------------------------------------------------------------------------
# The five workload recipes.  `n` overrides the grid edge (parity tests use
# reduced sizes); the physical setup (unit box, hbar, value ranges) is kept.
# ---------------------------------------------------------------------------

def _w1(n: Optional[int] = None) -> Problem:
    """2D 64x64, h = 1, f = 1 + 8 Gaussian bumps (amp U[0,.5], sigma U[3,10]
    px), one source at the centre, hbar = 0.5, T = 8."""
    n = 64 if n is None else int(n)
    rng = _rng(1001)
    f = gaussian_bumps_2d(n, n, 8, (0.0, 0.5), (3.0, 10.0), rng)
    src = np.array([[n // 2, n // 2]], np.int32)
    return _pack(f, src, 1.0, 0.5, 8, f"bumps2d_{n}")


def _w2(n: Optional[int] = None) -> Problem:
    """2D 1024x1024 unit box, f smoothed noise (sigma 16 px) in [1,3],
    16 sources, hbar = 0.05, T = 16."""
    n = 1024 if n is None else int(n)
    rng = _rng(1002)
    f = smoothed_noise((n, n), 16.0 * n / 1024.0, 1.0, 3.0, rng)
    src = distinct_sources((n, n), 16, rng)
    return _pack(f, src, 1.0 / n, 0.05, 16, f"noise2d_{n}")


def _w3(n: Optional[int] = None) -> Problem:
    """3D 256^3 unit cube, f from 32 Gaussian blobs in [0.5,2], one source at
    the centre, hbar = 0.1, T = 16."""
    n = 256 if n is None else int(n)
    rng = _rng(1003)
    f = gaussian_blobs_3d(n, 32, 0.5, 2.0, rng)
    src = np.array([[n // 2, n // 2, n // 2]], np.int32)
    return _pack(f, src, 1.0 / n, 0.1, 16, f"blobs3d_{n}")


def _w5(n: Optional[int] = None) -> Problem:
    """2D 2048x2048 unit box, f smoothed noise (sigma 16 px) in [1,3],
    4 sources, hbar = 0.05, T = 12 (the differentiation workload)."""
    n = 2048 if n is None else int(n)
    rng = _rng(1005)
    f = smoothed_noise((n, n), 16.0 * n / 2048.0, 1.0, 3.0, rng)
    src = distinct_sources((n, n), 4, rng)
    return _pack(f, src, 1.0 / n, 0.05, 12, f"noise2d_grad_{n}")


WORKLOADS = {1: _w1, 2: _w2, 3: _w3, 5: _w5}


def problem(cfg: int, n: Optional[int] = None) -> Problem:
    """Workload `cfg` (1, 2, 3 or 5) at grid edge `n` (default: full size)."""
    return WORKLOADS[int(cfg)](n)


def batch_problems(count: int = 64, sizes: Sequence[int] = (256, 512, 1024, 2048),
                   seed: int = 1004, T: int = 12) -> List[Problem]:
    """Uneven batch: `count` independent 2D instances; square edge drawn from
    `sizes`, h = 1/n, f smoothed noise (sigma 16 px) in [1,4], 1..8 sources,
    hbar U[0.02, 0.2], common T."""
    seqs = np.random.SeedSequence(seed).spawn(count)
    out = []
    for j, ss in enumerate(seqs):
        rng = _rng(ss)
        n = int(rng.choice(np.asarray(sizes)))
        n_src = int(rng.integers(1, 9))
        hbar = float(rng.uniform(0.02, 0.2))
        f = smoothed_noise((n, n), 16.0, 1.0, 4.0, rng)
        src = distinct_sources((n, n), n_src, rng)
        out.append(_pack(f, src, 1.0 / n, hbar, T, f"batch{j}_{n}"))
    return out


def loss_setup(p: Problem, count: int = 256, seed: int = 1105,
               radius_frac: float = 0.1):
    """Receivers and a perturbed forcing for the differentiation workload.

    Receivers: `count` distinct non-source points within radius_frac of the
    domain edge of some source.  Perturbed forcing f_t = clip(f + 0.1 p, lo,
    hi) with p smoothed noise (sigma 64 px at 2048) in [-1, 1]."""
    rng = _rng(seed)
    n = max(p.dims)
    rec = receivers_near_sources(p.dims, p.src, count, radius_frac * n, rng)
    pert = smoothed_noise(p.dims, 64.0 * n / 2048.0, -1.0, 1.0, rng)
    f64 = p.f.astype(np.float64)
    ft = np.clip(f64 + 0.1 * pert, float(f64.min()), float(f64.max()))
    return rec, np.ascontiguousarray(ft.astype(np.float32))
