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
// One CG iteration is two kernels over the grid:
//   apply   p = z + beta p_prev (at the point and at its neighbours, read
//           from the previous direction buffer) and q = A p; partial sums of
//           p.q
//   update  x += alpha p, r -= alpha q, z = r / diag; partial sums of r.z
//           and r.r
// Every block of a kernel first sums the per-block partials of the kernel
// before it (a fixed number of blocks and a fixed order: deterministic), so
// the scalars alpha and beta need no separate launch.  The partials of r.z
// alternate between two buffers by iteration parity, and so do the search
// directions, so that no kernel overwrites what another block of the same
// kernel still reads.  The apply kernel also tests ||r|| <= rtol ||b|| and
// raises a flag that makes every later kernel return at once; the host
// checks the flag between chunks of iterations.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "plan.hpp"

namespace sweik {
namespace {

constexpr int kFdThreads = 256;
constexpr int kFdBlocks = 1024;
constexpr int kFdChunk = 64;  // iterations enqueued between two convergence checks
enum { P_RZ0 = 0, P_RZ1 = 1, P_RR = 2, P_PQ = 3, P_COUNT = 4 };

struct FdArgs {
  int n[3];
  long long st[3];
  long long N;
  int D;
  double c;        // (h / hbar)^2
  double tol2;     // rtol^2
  double *d, *x, *r, *z, *q, *p[2];
  double *part;    // [P_COUNT][kFdBlocks]
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

// sums of the per-block partials of the listed slots
template <int K> __device__ __forceinline__ void reduce_parts(const FdArgs &a, const int (&slot)[K],
                                                             double (&out)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
    for (int i = threadIdx.x; i < kFdBlocks; i += kFdThreads) t += a.part[slot[k] * kFdBlocks + i];
    out[k] = t;
  }
  block_sums(out);
}

__global__ void __launch_bounds__(kFdThreads) k_fd_init(FdArgs a) {
  if (threadIdx.x < 4) a.state[threadIdx.x] = 0;
  if (threadIdx.x < 2) a.scal[threadIdx.x] = 0.0;
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
    a.d[i] = 2.0 * a.D + a.c * fv * fv;
    a.x[i] = 0.0;
    a.r[i] = 0.0;
    a.z[i] = 0.0;
    a.p[0][i] = 0.0;
  }
  if (threadIdx.x < P_COUNT) a.part[threadIdx.x * kFdBlocks + blockIdx.x] = 0.0;
  if (fl) atomicOr(&a.state[2], fl);
}

// b = delta at the sources: r = b, z = b / diag; the partials of r.z and r.r
// of the first iteration (one thread: the list is short)
__global__ void k_fd_seed(FdArgs a, const int32_t *__restrict__ src, int n_src) {
  if (threadIdx.x != 0) return;
  double rz = 0.0, cnt = 0.0;
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
    if (a.r[o] == 0.0) {  // a repeated source counts once (b is an indicator)
      a.r[o] = 1.0;
      a.z[o] = 1.0 / a.d[o];
      rz += a.z[o];
      cnt += 1.0;
    }
  }
  a.part[P_RZ0 * kFdBlocks] = rz;
  a.part[P_RR * kFdBlocks] = cnt;
  a.scal[0] = cnt;
  if (fl) atomicOr(&a.state[2], fl);
}

template <int D>
__global__ void __launch_bounds__(kFdThreads) k_fd_apply(FdArgs a, int k) {
  if (a.state[0]) return;
  double s[3];
  const int slots[3] = {(k & 1) ? P_RZ1 : P_RZ0, (k & 1) ? P_RZ0 : P_RZ1, P_RR};
  reduce_parts(a, slots, s);
  const double rz = s[0], rz_prev = s[1], rr = s[2], bb = a.scal[0];
  if (rr <= a.tol2 * bb) {  // converged (also when there is no source: b = 0)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.state[0] = 1;
      a.state[1] = k;
      a.scal[1] = rr;
    }
    return;
  }
  const double beta = k == 0 ? 0.0 : rz / rz_prev;
  const double *__restrict__ pin = a.p[k & 1];
  double *__restrict__ pout = a.p[(k + 1) & 1];
  const double *__restrict__ z = a.z;
  auto dirv = [&](long long j) { return z[j] + beta * pin[j]; };
  // one grid line (along the last axis) per block at a time: the line's
  // coordinates on the other axes cost one division per line, not per point
  const int nl = a.n[D - 1];
  const long long lines = a.N / nl;
  double acc = 0.0;
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
      const long long i = base + c;
      m[D - 1] = c;
      const double pc = dirv(i);
      double v = a.d[i] * pc;
#pragma unroll
      for (int e = 0; e < D; ++e) {
        if (m[e] > 0) v -= dirv(i - a.st[e]);
        if (m[e] < a.n[e] - 1) v -= dirv(i + a.st[e]);
      }
      pout[i] = pc;
      a.q[i] = v;
      acc += pc * v;
    }
  }
  double t[1] = {acc};
  block_sums(t);
  if (threadIdx.x == 0) a.part[P_PQ * kFdBlocks + blockIdx.x] = t[0];
}

__global__ void __launch_bounds__(kFdThreads) k_fd_update(FdArgs a, int k) {
  if (a.state[0]) return;
  double s[2];
  const int slots[2] = {(k & 1) ? P_RZ1 : P_RZ0, P_PQ};
  reduce_parts(a, slots, s);
  const double alpha = s[0] / s[1];
  const double *__restrict__ p = a.p[(k + 1) & 1];
  double rz = 0.0, rr = 0.0;
  for (long long i = (long long)blockIdx.x * kFdThreads + threadIdx.x; i < a.N;
       i += (long long)kFdBlocks * kFdThreads) {
    a.x[i] += alpha * p[i];
    const double r = a.r[i] - alpha * a.q[i];
    const double z = r / a.d[i];
    a.r[i] = r;
    a.z[i] = z;
    rz += r * z;
    rr += r * r;
  }
  double t[2] = {rz, rr};
  block_sums(t);
  if (threadIdx.x == 0) {
    a.part[((k & 1) ? P_RZ0 : P_RZ1) * kFdBlocks + blockIdx.x] = t[0];
    a.part[P_RR * kFdBlocks + blockIdx.x] = t[1];
  }
}

template <typename R>
__global__ void __launch_bounds__(kFdThreads) k_fd_finish(FdArgs a, R *__restrict__ S, double hbar,
                                                          int iters_run) {
  if (blockIdx.x == 0) {
    double s[1];
    const int slots[1] = {P_RR};
    reduce_parts(a, slots, s);
    if (threadIdx.x == 0 && !a.state[0]) {
      a.state[1] = iters_run;
      a.scal[1] = s[0];
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
  size_t vec, part, scal, state, nbad, total;
};

FdLayout fd_layout(long long N) {
  FdLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.vec = take((size_t)7 * N * sizeof(double));
  L.part = take((size_t)P_COUNT * kFdBlocks * sizeof(double));
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
  a.d = v;
  a.x = v + N;
  a.r = v + 2 * N;
  a.z = v + 3 * N;
  a.q = v + 4 * N;
  a.p[0] = v + 5 * N;
  a.p[1] = v + 6 * N;
  a.part = (double *)(ws + L.part);
  a.scal = (double *)(ws + L.scal);
  a.state = (int *)(ws + L.state);
  a.nbad = (unsigned long long *)(ws + L.nbad);
  const dim3 grid(kFdBlocks), blk(kFdThreads);

  hipLaunchKernelGGL(k_fd_init, dim3(1), blk, 0, st, a);
  hipLaunchKernelGGL((k_fd_setup<R>), grid, blk, 0, st, a, (const R *)f);
  hipLaunchKernelGGL(k_fd_seed, dim3(1), dim3(64), 0, st, a, src, pl->p.n_src);
  if (hipGetLastError() != hipSuccess) return SWEIK_EDEVICE;
  int it = 0;
  while (it < max_iter) {
    const int chunk = max_iter - it < kFdChunk ? max_iter - it : kFdChunk;
    for (int j = 0; j < chunk; ++j) {
      if (a.D == 2) hipLaunchKernelGGL((k_fd_apply<2>), grid, blk, 0, st, a, it + j);
      else hipLaunchKernelGGL((k_fd_apply<3>), grid, blk, 0, st, a, it + j);
      hipLaunchKernelGGL(k_fd_update, grid, blk, 0, st, a, it + j);
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
