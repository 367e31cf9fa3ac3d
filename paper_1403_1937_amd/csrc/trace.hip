// trace.hip -- path backtracking on a computed S (Section 6, path planning):
// from each start point, integrate dx/dt = -grad S / |grad S| (eq.
// PathPlanning-backTrackOnS) until the path comes within a radius of a
// source.
//
// Discretisation (the paper leaves it open):
//   node gradient   central differences of S along each axis, one-sided at
//                   the first and last node (units: per grid spacing)
//   gradient at x   multilinear interpolation of the node gradients of the
//                   2^D nodes of x's cell (cells clamped to the grid)
//   step            classical fourth-order Runge-Kutta step of length `step`
//                   (grid units) on the unit direction field -g/|g|; every
//                   stage position and every new point is clamped to the box
//                   [0, n_d - 1]
//   stop            within `radius` of a source (status 0), after max_steps
//                   steps (1), where the gradient vanishes or is not finite
//                   (2); a start outside the box or not finite is rejected
//                   (3, no point recorded)
// One thread per path: paths are independent and each step depends on the
// previous one, so the kernel is bound by the latency of its (cached) reads
// of S.  All arithmetic in float64, whatever the type of S.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "sweik.h"

namespace sweik {
namespace {

constexpr int kTraceThreads = 64;
constexpr int kTraceSrcLds = 512;  // sources kept in LDS; the rest are read from memory
constexpr int32_t kTraceMaxSteps = 1 << 20;

template <typename R, int D> struct TraceField {
  const R *S;
  int n[D];
  long long st[D];

  __device__ __forceinline__ double val(long long o) const { return (double)S[o]; }
  // central difference along axis d at node offset o (index m along d)
  __device__ __forceinline__ double node_grad(long long o, int m, int d) const {
    if (m == 0) return val(o + st[d]) - val(o);
    if (m == n[d] - 1) return val(o) - val(o - st[d]);
    return 0.5 * (val(o + st[d]) - val(o - st[d]));
  }
  __device__ __forceinline__ void clamp(double (&x)[D]) const {
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = fmin(fmax(x[d], 0.0), (double)(n[d] - 1));
  }
  // interpolated gradient at x (inside the box)
  __device__ __forceinline__ void grad(const double (&x)[D], double (&g)[D]) const {
    int i[D];
    double t[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int c = (int)floor(x[d]);
      i[d] = c < 0 ? 0 : (c > n[d] - 2 ? n[d] - 2 : c);
      t[d] = x[d] - (double)i[d];
      g[d] = 0.0;
    }
#pragma unroll
    for (int corner = 0; corner < (1 << D); ++corner) {
      double w = 1.0;
      long long o = 0;
      int m[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int b = (corner >> (D - 1 - d)) & 1;
        m[d] = i[d] + b;
        w *= b ? t[d] : 1.0 - t[d];
        o += (long long)m[d] * st[d];
      }
#pragma unroll
      for (int d = 0; d < D; ++d) g[d] += w * node_grad(o, m[d], d);
    }
  }
  // unit descent direction at x; false where the gradient vanishes or is not finite
  __device__ __forceinline__ bool dir(const double (&x)[D], double (&u)[D]) const {
    double g[D];
    grad(x, g);
    double s = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) s += g[d] * g[d];
    const double nrm = sqrt(s);
    if (!(nrm > 0.0) || !isfinite(nrm)) return false;
#pragma unroll
    for (int d = 0; d < D; ++d) u[d] = -g[d] / nrm;
    return true;
  }
};

template <typename R, int D>
__global__ void __launch_bounds__(kTraceThreads)
    k_backtrack(TraceField<R, D> fld, const int32_t *__restrict__ src, int n_src,
                const double *__restrict__ start, int n_paths, int max_steps, double step,
                double radius, double *__restrict__ path, int32_t *__restrict__ n_points,
                int32_t *__restrict__ status) {
  __shared__ double s_src[D * kTraceSrcLds];
  const int nl = n_src < kTraceSrcLds ? n_src : kTraceSrcLds;
  for (int i = threadIdx.x; i < D * nl; i += blockDim.x) s_src[i] = (double)src[i];
  __syncthreads();
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n_paths) return;

  const double r2 = radius * radius;
  auto near_source = [&](const double (&x)[D]) -> bool {
    double best = INFINITY;
    for (int k = 0; k < nl; ++k) {
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double e = x[d] - s_src[D * k + d];
        s += e * e;
      }
      best = fmin(best, s);
    }
    for (int k = nl; k < n_src; ++k) {
      double s = 0.0;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double e = x[d] - (double)src[D * k + d];
        s += e * e;
      }
      best = fmin(best, s);
    }
    return best < r2;
  };

  double x[D];
  bool inside = true;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    x[d] = start[(size_t)p * D + d];
    inside = inside && x[d] >= 0.0 && x[d] <= (double)(fld.n[d] - 1);
  }
  if (!inside) {  // also catches NaN
    n_points[p] = 0;
    status[p] = 3;
    return;
  }
  double *out = path + (size_t)p * (size_t)(max_steps + 1) * D;
#pragma unroll
  for (int d = 0; d < D; ++d) out[d] = x[d];
  int k = 0, st = 1;
  while (true) {
    if (near_source(x)) {
      st = 0;
      break;
    }
    if (k == max_steps) {
      st = 1;
      break;
    }
    double k1[D], k2[D], k3[D], k4[D], y[D];
    bool ok = fld.dir(x, k1);
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] + 0.5 * step * k1[d];
    fld.clamp(y);
    ok = ok && fld.dir(y, k2);
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] + 0.5 * step * k2[d];
    fld.clamp(y);
    ok = ok && fld.dir(y, k3);
#pragma unroll
    for (int d = 0; d < D; ++d) y[d] = x[d] + step * k3[d];
    fld.clamp(y);
    ok = ok && fld.dir(y, k4);
    if (!ok) {
      st = 2;
      break;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] += step / 6.0 * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
    fld.clamp(x);
    ++k;
#pragma unroll
    for (int d = 0; d < D; ++d) out[(size_t)k * D + d] = x[d];
  }
  n_points[p] = k + 1;
  status[p] = st;
}

template <typename R, int D>
hipError_t launch_backtrack(const int64_t *dims, const void *S, const int32_t *src, int n_src,
                            const double *start, int n_paths, int max_steps, double step,
                            double radius, double *path, int32_t *n_points, int32_t *status,
                            hipStream_t st) {
  TraceField<R, D> fld;
  fld.S = (const R *)S;
  long long stride = 1;
  for (int d = D - 1; d >= 0; --d) {
    fld.n[d] = (int)dims[d];
    fld.st[d] = stride;
    stride *= dims[d];
  }
  const int blocks = (n_paths + kTraceThreads - 1) / kTraceThreads;
  hipLaunchKernelGGL((k_backtrack<R, D>), dim3(blocks), dim3(kTraceThreads), 0, st, fld, src,
                     n_src, start, n_paths, max_steps, step, radius, path, n_points, status);
  return hipGetLastError();
}

}  // namespace
}  // namespace sweik

extern "C" sweik_status sweik_backtrack(int32_t ndim, const int64_t *dims, sweik_precision prec,
                                        const void *S, const int32_t *src, int32_t n_src,
                                        const double *start, int32_t n_paths,
                                        int32_t max_steps, double step, double radius,
                                        double *path, int32_t *n_points, int32_t *status,
                                        void *stream) {
  using namespace sweik;
  if (!dims || (ndim != 2 && ndim != 3)) return SWEIK_EINVAL;
  if (prec != SWEIK_F32_SCALED && prec != SWEIK_F64) return SWEIK_EINVAL;
  for (int d = 0; d < ndim; ++d)
    if (dims[d] < 2 || dims[d] > (1 << 20)) return SWEIK_EINVAL;
  if (ndim == 2 ? dims[0] * dims[1] > (1LL << 31) : dims[0] * dims[1] * dims[2] > (1LL << 31))
    return SWEIK_EUNSUPPORTED;
  if (n_src < 0 || n_paths < 0 || max_steps < 0 || max_steps > kTraceMaxSteps) return SWEIK_EINVAL;
  if (!(step > 0.0) || !(radius >= 0.0) || !__builtin_isfinite(step) || !__builtin_isfinite(radius))
    return SWEIK_EINVAL;
  if (n_paths == 0) return SWEIK_OK;
  if (!S || (n_src > 0 && !src) || !start || !path || !n_points || !status) return SWEIK_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (ndim == 2)
    e = prec == SWEIK_F64
            ? launch_backtrack<double, 2>(dims, S, src, n_src, start, n_paths, max_steps, step,
                                          radius, path, n_points, status, st)
            : launch_backtrack<float, 2>(dims, S, src, n_src, start, n_paths, max_steps, step,
                                         radius, path, n_points, status, st);
  else
    e = prec == SWEIK_F64
            ? launch_backtrack<double, 3>(dims, S, src, n_src, start, n_paths, max_steps, step,
                                          radius, path, n_points, status, st)
            : launch_backtrack<float, 3>(dims, S, src, n_src, start, n_paths, max_steps, step,
                                         radius, path, n_points, status, st);
  return e == hipSuccess ? SWEIK_OK : SWEIK_EDEVICE;
}
