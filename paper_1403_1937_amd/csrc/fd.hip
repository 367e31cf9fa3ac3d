// fd.hip -- the paper's second method (Section 6, eq. sparse-system): the
// finite-difference screened Poisson system
//
//   (2D + c f_m^2) phi_m - sum_{grid neighbours n of m} phi_n = b_m,
//   c = (h / hbar)^2,  b = Kronecker delta of the point set (eq. deltakron),
//
// (five-point Laplacian in 2D, seven-point in 3D, phi = 0 outside the grid),
// then S = -hbar ln phi (eq. SfromPhi).  The matrix is symmetric positive
// definite (an M-matrix), so it is solved matrix-free by conjugate gradients
// with the diagonal as preconditioner, in float64 whatever the type of f and
// S.
//
// The iteration is the Chronopoulos-Gear form of preconditioned CG (one
// pair of inner products per iteration, both formed after the update), so
// that one iteration is one kernel over the grid:
//   p = u + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
//   u = r / diag,  w = A u,  gamma = (r, u),  delta = (w, u),  (r, r)
// with beta = gamma / gamma_prev and alpha = gamma / (delta - beta gamma /
// alpha_prev).  The stencil w = A u needs the new u at the neighbours; each
// thread recomputes it there from the old r, w, s (read-only in the
// kernel), so the old and new r, w and s live in two buffers each, by
// iteration parity.  Every block first sums the per-block partials of the
// kernel before it (a fixed number of blocks and a fixed order:
// deterministic) and derives alpha and beta itself; block 0 keeps the
// scalars the next iteration needs.  A convergence test on (r, r) raises a
// flag that makes every later kernel return at once; the host checks the
// flag between chunks of iterations.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "plan.hpp"

namespace sweik {
namespace {

constexpr int kFdThreads = 256;
constexpr int kFdBlocks = 1024;
constexpr int kFdChunk = 64;  // iterations enqueued between two convergence checks
// partial-sum slots, two parities each: (r, u), (w, u), (r, r)
enum { P_G = 0, P_D = 1, P_RR = 2, P_COUNT = 3 };

struct FdArgs {
  int n[3];
  long long st[3];
  long long N;
  int D;
  double c;        // (h / hbar)^2
  double tol2;     // rtol^2
  double *dinv, *x, *p, *r[2], *w[2], *s[2];
  double *part;    // [2][P_COUNT][kFdBlocks]
  double *hist;    // [2][2]: gamma and alpha of the last iterations, by parity
  double *scal;    // [0] ||b||^2, [1] r.r at exit
  int *state;      // [0] converged, [1] iterations, [2] flags
  unsigned long long *nbad;
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sums of up to three values over the block (every thread gets them)
template <int K> __device__ __forceinline__ void block_sums(double (&v)[K]) {
  __shared__ double s[K][kFdThreads / 64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    v[k] = wave_sum(v[k]);
    if (l == 0) s[k][w] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
#pragma unroll
    for (int i = 0; i < kFdThreads / 64; ++i) t += s[k][i];
    v[k] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ double *part_of(const FdArgs &a, int parity, int slot) {
  return a.part + ((size_t)parity * P_COUNT + slot) * kFdBlocks;
}

// the three partial sums of one parity
__device__ __forceinline__ void reduce_parts(const FdArgs &a, int parity, double (&out)[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double *pp = part_of(a, parity, k);
    double t = 0.0;
    for (int i = threadIdx.x; i < kFdBlocks; i += kFdThreads) t += pp[i];
    out[k] = t;
  }
  block_sums(out);
}

__global__ void __launch_bounds__(kFdThreads) k_fd_init(FdArgs a) {
  if (threadIdx.x < 4) a.state[threadIdx.x] = 0;
  if (threadIdx.x < 2) a.scal[threadIdx.x] = 0.0;
  if (threadIdx.x < 4) a.hist[threadIdx.x] = 0.0;
  if (threadIdx.x == 0) *a.nbad = 0ull;
}

template <typename R>
__global__ void __launch_bounds__(kFdThreads) k_fd_setup(FdArgs a, const R *__restrict__ f) {
  int fl = 0;
  for (long long i = (long long)blockIdx.x * kFdThreads + threadIdx.x; i < a.N;
       i += (long long)kFdBlocks * kFdThreads) {
    const double fv = (double)f[i];
    if (!isfinite(fv)) fl |= SWEIK_FLAG_F_NONFINITE;
    else if (!(fv > 0.0)) fl |= SWEIK_FLAG_F_NONPOSITIVE;
    a.dinv[i] = 1.0 / (2.0 * a.D + a.c * fv * fv);
    a.x[i] = 0.0;
    a.p[i] = 0.0;
    a.r[0][i] = 0.0;
    a.s[1][i] = 0.0;  // s of iteration -1
  }
  if (fl) atomicOr(&a.state[2], fl);
}

// b = delta at the sources: r_0 = b (one thread: the list is short)
__global__ void k_fd_seed(FdArgs a, const int32_t *__restrict__ src, int n_src) {
  if (threadIdx.x != 0) return;
  double cnt = 0.0;
  int fl = 0;
  for (int k = 0; k < n_src; ++k) {
    long long o = 0;
    bool ok = true;
    for (int e = 0; e < a.D; ++e) {
      const int y = src[(size_t)k * a.D + e];
      ok = ok && y >= 0 && y < a.n[e];
      o += (long long)y * a.st[e];
    }
    if (!ok) {
      fl |= SWEIK_FLAG_BAD_SOURCE;
      continue;
    }
    if (a.r[0][o] == 0.0) {  // a repeated source counts once (b is an indicator)
      a.r[0][o] = 1.0;
      cnt += 1.0;
    }
  }
  a.scal[0] = cnt;
  if (fl) atomicOr(&a.state[2], fl);
}

// Grid lines along the last axis, one per block at a time: the line's
// coordinates on the other axes cost one division per line.
template <int D, typename F>
__device__ __forceinline__ void for_points(const FdArgs &a, F &&fn) {
  const int nl = a.n[D - 1];
  const long long lines = a.N / nl;
  for (long long line = blockIdx.x; line < lines; line += kFdBlocks) {
    int m[D];
    long long rem = line;
#pragma unroll
    for (int e = D - 2; e >= 0; --e) {
      const long long qd = rem / a.n[e];
      m[e] = (int)(rem - qd * a.n[e]);
      rem = qd;
    }
    const long long base = line * nl;
    for (int c = threadIdx.x; c < nl; c += kFdThreads) {
      m[D - 1] = c;
      fn(base + c, m);
    }
  }
}

// w_0 = A u_0 with u_0 = r_0 / diag, and the partials of iteration 0
template <int D>
__global__ void __launch_bounds__(kFdThreads) k_fd_start(FdArgs a) {
  const double *__restrict__ r = a.r[0];
  double g = 0.0, dl = 0.0, rr = 0.0;
  for_points<D>(a, [&](long long i, const int (&m)[D]) {
    const double u = r[i] * a.dinv[i];
    double w = r[i];  // diag u
#pragma unroll
    for (int e = 0; e < D; ++e) {
      if (m[e] > 0) w -= r[i - a.st[e]] * a.dinv[i - a.st[e]];
      if (m[e] < a.n[e] - 1) w -= r[i + a.st[e]] * a.dinv[i + a.st[e]];
    }
    a.w[0][i] = w;
    g += r[i] * u;
    dl += w * u;
    rr += r[i] * r[i];
  });
  double t[3] = {g, dl, rr};
  block_sums(t);
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) part_of(a, 0, k)[blockIdx.x] = t[k];
}

template <int D>
__global__ void __launch_bounds__(kFdThreads) k_fd_iter(FdArgs a, int k) {
  if (a.state[0]) return;
  const int cur = k & 1, nxt = cur ^ 1;
  double sc[3];
  reduce_parts(a, cur, sc);
  const double gam = sc[0], del = sc[1], rr = sc[2], bb = a.scal[0];
  if (rr <= a.tol2 * bb) {  // converged (also when there is no source: b = 0)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.state[0] = 1;
      a.state[1] = k;
      a.scal[1] = rr;
    }
    return;
  }
  double beta = 0.0, alpha = gam / del;
  if (k > 0) {
    beta = gam / a.hist[2 * nxt];
    alpha = gam / (del - beta * gam / a.hist[2 * nxt + 1]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // read by the next iteration only
    a.hist[2 * cur] = gam;
    a.hist[2 * cur + 1] = alpha;
  }
  const double *__restrict__ r0 = a.r[cur];
  const double *__restrict__ w0 = a.w[cur];
  const double *__restrict__ s0 = a.s[nxt];  // s of the previous iteration
  double *__restrict__ r1 = a.r[nxt];
  double *__restrict__ w1 = a.w[nxt];
  double *__restrict__ s1 = a.s[cur];
  const double *__restrict__ dinv = a.dinv;
  // the new residual's preconditioned value at any point
  auto unew = [&](long long j) { return (r0[j] - alpha * (w0[j] + beta * s0[j])) * dinv[j]; };
  double g = 0.0, dl = 0.0, rs = 0.0;
  for_points<D>(a, [&](long long i, const int (&m)[D]) {
    const double di = dinv[i];
    const double p = r0[i] * di + beta * a.p[i];
    const double s = w0[i] + beta * s0[i];
    a.p[i] = p;
    s1[i] = s;
    a.x[i] += alpha * p;
    const double rn = r0[i] - alpha * s;
    const double u = rn * di;
    double w = rn;  // diag u
#pragma unroll
    for (int e = 0; e < D; ++e) {
      if (m[e] > 0) w -= unew(i - a.st[e]);
      if (m[e] < a.n[e] - 1) w -= unew(i + a.st[e]);
    }
    r1[i] = rn;
    w1[i] = w;
    g += rn * u;
    dl += w * u;
    rs += rn * rn;
  });
  double t[3] = {g, dl, rs};
  block_sums(t);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part_of(a, nxt, q)[blockIdx.x] = t[q];
}

// 2D form of the same step on tiles of kFdTileRows x kFdThreads points: the
// new preconditioned residual is formed once per point of the tile and its
// one-point halo into LDS, and the stencil reads it there (a point's four
// neighbours then cost no extra global reads).
constexpr int kFdTileRows = 4;
__global__ void __launch_bounds__(kFdThreads) k_fd_iter_2d(FdArgs a, int k) {
  if (a.state[0]) return;
  const int cur = k & 1, nxt = cur ^ 1;
  double sc[3];
  reduce_parts(a, cur, sc);
  const double gam = sc[0], del = sc[1], rr = sc[2], bb = a.scal[0];
  if (rr <= a.tol2 * bb) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.state[0] = 1;
      a.state[1] = k;
      a.scal[1] = rr;
    }
    return;
  }
  double beta = 0.0, alpha = gam / del;
  if (k > 0) {
    beta = gam / a.hist[2 * nxt];
    alpha = gam / (del - beta * gam / a.hist[2 * nxt + 1]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.hist[2 * cur] = gam;
    a.hist[2 * cur + 1] = alpha;
  }
  const double *__restrict__ r0 = a.r[cur];
  const double *__restrict__ w0 = a.w[cur];
  const double *__restrict__ s0 = a.s[nxt];
  double *__restrict__ r1 = a.r[nxt];
  double *__restrict__ w1 = a.w[nxt];
  double *__restrict__ s1 = a.s[cur];
  const double *__restrict__ dinv = a.dinv;
  constexpr int TR = kFdTileRows;
  __shared__ double su[TR + 2][kFdThreads + 2];  // new u on the tile and its halo (0 outside)
  const int n0 = a.n[0], n1 = a.n[1];
  const int tiles1 = (n1 + kFdThreads - 1) / kFdThreads;
  const long long ntiles = (long long)((n0 + TR - 1) / TR) * tiles1;
  const int t = threadIdx.x;
  auto unew = [&](int row, int col) -> double {
    if (row < 0 || row >= n0 || col < 0 || col >= n1) return 0.0;
    const long long j = (long long)row * n1 + col;
    return (r0[j] - alpha * (w0[j] + beta * s0[j])) * dinv[j];
  };
  double g = 0.0, dl = 0.0, rs = 0.0;
  for (long long tile = blockIdx.x; tile < ntiles; tile += kFdBlocks) {
    const int tr = (int)(tile / tiles1), tc = (int)(tile - (long long)tr * tiles1);
    const int row0 = tr * TR, col0 = tc * kFdThreads, c = col0 + t;
    double rv[TR], wv[TR], sv[TR], dv[TR];
#pragma unroll
    for (int q = 0; q < TR; ++q) {  // the tile's own points: keep the old values
      const int row = row0 + q;
      rv[q] = wv[q] = sv[q] = dv[q] = 0.0;
      double u = 0.0;
      if (row < n0 && c < n1) {
        const long long i = (long long)row * n1 + c;
        rv[q] = r0[i];
        wv[q] = w0[i];
        sv[q] = s0[i];
        dv[q] = dinv[i];
        u = (rv[q] - alpha * (wv[q] + beta * sv[q])) * dv[q];
      }
      su[q + 1][t + 1] = u;
    }
    su[0][t + 1] = unew(row0 - 1, c);
    su[TR + 1][t + 1] = unew(row0 + TR, c);
    if (t < 2 * (TR + 2)) {  // halo columns
      const int side = t / (TR + 2), q = t - side * (TR + 2);
      su[q][side ? kFdThreads + 1 : 0] = unew(row0 - 1 + q, side ? col0 + kFdThreads : col0 - 1);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < TR; ++q) {
      const int row = row0 + q;
      if (row < n0 && c < n1) {
        const long long i = (long long)row * n1 + c;
        const double p = rv[q] * dv[q] + beta * a.p[i];
        const double s = wv[q] + beta * sv[q];
        a.p[i] = p;
        s1[i] = s;
        a.x[i] += alpha * p;
        const double rn = rv[q] - alpha * s;
        const double u = rn * dv[q];
        const double w = rn - (su[q][t + 1] + su[q + 2][t + 1] + su[q + 1][t] + su[q + 1][t + 2]);
        r1[i] = rn;
        w1[i] = w;
        g += rn * u;
        dl += w * u;
        rs += rn * rn;
      }
    }
    __syncthreads();  // before the next tile overwrites su
  }
  double tt[3] = {g, dl, rs};
  block_sums(tt);
  if (threadIdx.x == 0)
    for (int q = 0; q < 3; ++q) part_of(a, nxt, q)[blockIdx.x] = tt[q];
}

template <typename R>
__global__ void __launch_bounds__(kFdThreads) k_fd_finish(FdArgs a, R *__restrict__ S, double hbar,
                                                          int iters_run) {
  if (blockIdx.x == 0) {
    double s[3];
    reduce_parts(a, iters_run & 1, s);
    if (threadIdx.x == 0 && !a.state[0]) {
      a.state[1] = iters_run;
      a.scal[1] = s[2];
    }
  }
  unsigned long long bad = 0;
  for (long long i = (long long)blockIdx.x * kFdThreads + threadIdx.x; i < a.N;
       i += (long long)kFdBlocks * kFdThreads) {
    const double ph = a.x[i];
    double v;
    if (ph > 0.0 && isfinite(ph)) {
      v = -hbar * log(ph);
    } else {
      v = INFINITY;
      ++bad;
    }
    S[i] = (R)v;
  }
  double t[1] = {(double)bad};
  block_sums(t);
  if (threadIdx.x == 0 && t[0] > 0) atomicAdd(a.nbad, (unsigned long long)t[0]);
}

struct FdLayout {
  size_t vec, part, hist, scal, state, nbad, total;
};

FdLayout fd_layout(long long N) {
  FdLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.vec = take((size_t)9 * N * sizeof(double));
  L.part = take((size_t)2 * P_COUNT * kFdBlocks * sizeof(double));
  L.hist = take(4 * sizeof(double));
  L.scal = take(4 * sizeof(double));
  L.state = take(4 * sizeof(int));
  L.nbad = take(sizeof(unsigned long long));
  L.total = off;
  return L;
}

long long grid_points(const sweik_plan_s *pl) {
  long long N = 1;
  for (int e = 0; e < pl->p.ndim; ++e) N *= pl->p.dims[e];
  return N;
}

template <typename R>
sweik_status fd_run(const sweik_plan_s *pl, const void *f, const int32_t *src, void *S, char *ws,
                    int32_t max_iter, double rtol, hipStream_t st, sweik_fd_info *info) {
  const long long N = grid_points(pl);
  const FdLayout L = fd_layout(N);
  FdArgs a;
  a.D = pl->p.ndim;
  long long stride = 1;
  for (int e = 2; e >= 0; --e) {
    a.n[e] = e < a.D ? (int)pl->p.dims[e] : 1;
    a.st[e] = stride;
    if (e < a.D) stride *= pl->p.dims[e];
  }
  a.N = N;
  a.c = (pl->p.h / pl->p.hbar) * (pl->p.h / pl->p.hbar);
  a.tol2 = rtol * rtol;
  double *v = (double *)(ws + L.vec);
  a.dinv = v;
  a.x = v + N;
  a.p = v + 2 * N;
  for (int q = 0; q < 2; ++q) {
    a.r[q] = v + (3 + q) * N;
    a.w[q] = v + (5 + q) * N;
    a.s[q] = v + (7 + q) * N;
  }
  a.part = (double *)(ws + L.part);
  a.hist = (double *)(ws + L.hist);
  a.scal = (double *)(ws + L.scal);
  a.state = (int *)(ws + L.state);
  a.nbad = (unsigned long long *)(ws + L.nbad);
  const dim3 grid(kFdBlocks), blk(kFdThreads);

  hipLaunchKernelGGL(k_fd_init, dim3(1), blk, 0, st, a);
  hipLaunchKernelGGL((k_fd_setup<R>), grid, blk, 0, st, a, (const R *)f);
  hipLaunchKernelGGL(k_fd_seed, dim3(1), dim3(64), 0, st, a, src, pl->p.n_src);
  if (a.D == 2) hipLaunchKernelGGL((k_fd_start<2>), grid, blk, 0, st, a);
  else hipLaunchKernelGGL((k_fd_start<3>), grid, blk, 0, st, a);
  if (hipGetLastError() != hipSuccess) return SWEIK_EDEVICE;
  int it = 0;
  while (it < max_iter) {
    const int chunk = max_iter - it < kFdChunk ? max_iter - it : kFdChunk;
    for (int j = 0; j < chunk; ++j) {
      if (a.D == 2) hipLaunchKernelGGL(k_fd_iter_2d, grid, blk, 0, st, a, it + j);
      else hipLaunchKernelGGL((k_fd_iter<3>), grid, blk, 0, st, a, it + j);
    }
    it += chunk;
    int done = 0;
    if (hipMemcpyAsync(&done, a.state, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return SWEIK_EDEVICE;
    if (done) break;
  }
  hipLaunchKernelGGL((k_fd_finish<R>), grid, blk, 0, st, a, (R *)S, pl->p.hbar, it);
  if (hipGetLastError() != hipSuccess) return SWEIK_EDEVICE;
  int state[4];
  double scal[4];
  unsigned long long nbad = 0;
  if (hipMemcpyAsync(state, a.state, sizeof(state), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(scal, a.scal, sizeof(scal), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&nbad, a.nbad, sizeof(nbad), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return SWEIK_EDEVICE;
  if (info) {
    info->iterations = state[1];
    info->converged = state[0];
    info->rel_residual = scal[0] > 0 ? sqrt(scal[1] / scal[0]) : 0.0;
    info->n_nonpositive_phi = (int64_t)nbad;
    info->flags = state[2];
    info->n_sources = (int32_t)scal[0];
  }
  return SWEIK_OK;
}

}  // namespace
}  // namespace sweik

extern "C" size_t sweik_fd_workspace_bytes(sweik_plan plan) {
  if (!plan) return 0;
  return sweik::fd_layout(sweik::grid_points(plan)).total;
}

extern "C" sweik_status sweik_fd_solve(sweik_plan plan, const void *f, const int32_t *src, void *S,
                                       void *ws, size_t ws_bytes, int32_t max_iter, double rtol,
                                       void *stream, sweik_fd_info *info) {
  using namespace sweik;
  if (!plan || !f || !src || !S || !ws) return SWEIK_EINVAL;
  if (max_iter < 0 || max_iter > (1 << 24) || !(rtol >= 0.0) || !__builtin_isfinite(rtol))
    return SWEIK_EINVAL;
  if (ws_bytes < fd_layout(grid_points(plan)).total) return SWEIK_EWORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  return plan->p.prec == SWEIK_F64
             ? fd_run<double>(plan, f, src, S, (char *)ws, max_iter, rtol, st, info)
             : fd_run<float>(plan, f, src, S, (char *)ws, max_iter, rtol, st, info);
}
