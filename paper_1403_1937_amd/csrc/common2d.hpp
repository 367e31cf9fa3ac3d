// common2d.hpp -- gfx950 kernels of the 2D perturbation-series eikonal solve:
// shared definitions, the reduction of f and block-level helpers.
//
// Per correction term i (Table 1, steps 9-13) the 2D linear convolution
// phi_i = kappa (*) (gamma phi_{i-1}) is evaluated on the zero-padded grid
// M0 x M1 (M_d >= 2 n_d - 1) in two passes:
//   column pass  for each spectral column k1: forward FFT of length M0 over
//                the (zero-padded) rows, product with the real kernel
//                spectrum Ghat[k0][k1], inverse FFT, keep the first rows
//   row pass     for each grid row: inverse real FFT of length M1 (a complex
//                FFT of length M1/2 plus a split step), crop to n1 columns,
//                rescale, accumulate (-1)^i phi_i in float64, form
//                gamma * phi_i for the next term and take its forward real
//                FFT; after the last term write S = -hbar ln phi instead.
// The half spectrum (H1+1 = M1/2+1 columns, rows 0..n0-1) lives in a
// blocked transposed layout spec[b][k1][rr] with RB rows per block b: a row
// pass work-group reads and writes whole contiguous blocks, and a column
// pass reads RB contiguous rows of CPW neighbouring columns per block.
// Every pass issues all of its global reads (spectrum, kernel spectrum,
// twiddles, forcing, accumulator) before its first barrier, so that a pass
// costs one memory latency rather than one per operand.
//
// The same two kernels build the kernel spectrum (mode GHAT): the row pass
// evaluates the evenly extended kernel table row by row and takes its real
// FFT; the column pass extends each column evenly, transforms it and keeps
// the real part.  phi_0 (mode PHI0) is evaluated directly from the sources
// (eq. phi_0Solution) in the first row pass.
//
// Scaling: term i is stored as a mantissa field m_i and an exponent E_i
// (phi_i = 2^E_i m_i).  The exponent step applied to m_i is the binary
// exponent of max|m_{i-1}|, known from the previous pass, so the stored
// values stay near the contraction factor instead of decaying like c0^i.
#pragma once

#include "geom2d.hpp"
#include "green.hpp"
#include "sweik.h"

#include <climits>
#include <type_traits>

namespace sweik {

constexpr int kRedBlocks = 1024;  // partial reductions of f (work-groups of the prep)

struct Params {      // device-side scalars shared by the kernels of a solve
  double ftilde, beta, hbar, inv_ft2, kappa0, fmin, fmax, c0;
  int flags, pad_;
};

template <typename R> struct Args2 {
  // geometry
  int n0, n1;      // grid
  int H1, ldk;     // M1/2, H1 stored spectral columns (bins 0 and H1 share column 0)
  int M0, H0, ldg; // column FFT length, M0/2, H0+1
  int nb;          // spectral row blocks (spec_rb rows each)
  int nbr;         // number of row-pass WGs
  int ncw;         // number of column-pass WGs
  int lmax_log;    // log2 of the twiddle table length
  int T, n_src, ft_mode;
  int table;     // kernel table of the ROW_GHAT pass: 0 kappa, 1 exp(-beta |m|)
  int phi0_fft;  // phi_0 from the transform of the source grid (in the spectrum)
  int own_par;   // ROW_PHI0 forms the reference forcing itself (paired with ROW_GHAT)
  double ftilde_given, h, hbar;
  // data
  const R *f;
  const int *src;
  const R *src_s;  // nullable: S at the sources
  R *S;
  // workspace
  Params *par;
  double *red;   // kRedBlocks x 3 (min, max, flags)
  double *mu;    // (T+1) x nbr partial max |m_i|
  int *expo;     // T+1 exponents
  const cplx<R> *tw;
  cplx<R> *spec;
  R *g;          // (H1+1) x (H0+1) kernel spectrum orthant, pre-scaled
  double *acc;   // n0 x n1 adjoint accumulator of dL/dgamma
  R *terms;      // T x n0 x n1 mantissas of phi_0..phi_{T-1} (the checkpoint's when kept)
  R *gam;        // n0 x n1 gamma = f^2/ftilde^2 - 1
  ChebK0 k0tab;  // K0 for x > 2
  // adjoint
  const R *dLdS;
  R *dLdf;
  R *lam;        // n0 x n1 lambda mantissas
  // optional
  sweik_info *info;
  int *ck_expo;  // T+1
  double *ck_phi;// n0 x n1
  R *ck_terms;   // T x n0 x n1 series-term mantissas (read by the adjoint)
  // full gradient
  cplx<R> *spec2;  // spectrum convolved with the kernel's beta-derivative
  double *gpart;   // kGradSlots x nbr per-work-group partial sums
  // far-field stabilised (tilted) solve: the convolution runs on
  // phi_i exp(a . x) with the kernel kappa(m) exp(a . m), a = beta (tilt0, tilt1)
  // per grid index (|tilt| < 1); tmax: 0 when not tilted
  double tilt0, tilt1;
  int tsign;         // ROW_GHATT: +1 kernel rows m0 >= 0, -1 rows m0 <= 0
  int tfirst, tlast; // ROW_LASTT: first / last tilt of the solve
  cplx<R> *gc;       // tilted kernel spectrum, (H1 + 1) x M0 complex, column k1 contiguous
  cplx<R> *spec_neg; // COL_GHATC: row transforms of the kernel rows m0 <= 0
  float *best;       // per point: score of the tilt whose S is stored
  double *tmax;      // T + 2: max |phi_i| per stored term, then the tilt's offset A
};

// Per-work-group partial sums of the full gradient (each slot nbr long):
//   G_S   sum dL/dS * S / hbar                  (hbar in S = -hbar ln phi)
//   G_C   sum over terms of <c_i, gamma phi_{i-1}>, c_i = dkappa/dbeta (*) a_i
//   G_B0  <a_0, d phi_0 / d beta>
//   G_H0  <a_0, d phi_0 / d hbar> through the weights exp(-s_k / hbar)
//   G_GF  sum dL/dgamma * f^2                   (gamma = f^2 / ftilde^2 - 1)
enum { G_S = 0, G_C = 1, G_B0 = 2, G_H0 = 3, G_GF = 4, kGradSlots = 5 };

// ---------------------------------------------------------------------------
// prep: partial min / max / validity of f, and the twiddle table
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void prep_fold(double v, double &lo, double &hi, int &fl) {
  if (!isfinite(v)) {
    fl |= SWEIK_FLAG_F_NONFINITE;
    return;
  }
  if (!(v > 0.0)) fl |= SWEIK_FLAG_F_NONPOSITIVE;
  lo = v < lo ? v : lo;
  hi = v > hi ? v : hi;
}

template <typename R>
__device__ __forceinline__ void prep_block(const R *__restrict__ f, long long N,
                                           double *__restrict__ red, cplx<R> *__restrict__ tw,
                                           int lmax, int bid, int nblk) {
  __shared__ double smin[16], smax[16];  // up to 1024 threads
  __shared__ int sfl[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
  int fl = 0;
  // pairs of consecutive values (vector loads when f is aligned to a pair),
  // four pairs in flight per thread and iteration; then the tail
  using V = cplx<R>;  // two R
  const long long G = N / 2, stride = (long long)nblk * blockDim.x;
  const long long g0 = (long long)bid * blockDim.x + threadIdx.x;
  if ((reinterpret_cast<uintptr_t>(f) & (sizeof(V) - 1)) == 0) {
    const V *f2 = reinterpret_cast<const V *>(f);
    for (long long g = g0; g < G; g += 4 * stride) {
      V x[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const long long gu = g + u * stride;
        x[u] = f2[gu < G ? gu : g];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        prep_fold<R>((double)x[u].x, lo, hi, fl);
        prep_fold<R>((double)x[u].y, lo, hi, fl);
      }
    }
    for (long long i = 2 * G + g0; i < N; i += stride) prep_fold<R>((double)f[i], lo, hi, fl);
  } else {
    for (long long i = g0; i < N; i += stride) prep_fold<R>((double)f[i], lo, hi, fl);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  fl = wave_or(fl);
  if (lane == 0) {
    smin[wid] = lo;
    smax[wid] = hi;
    sfl[wid] = fl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      lo = smin[w] < lo ? smin[w] : lo;
      hi = smax[w] > hi ? smax[w] : hi;
      fl |= sfl[w];
    }
    lo = smin[0] < lo ? smin[0] : lo;
    hi = smax[0] > hi ? smax[0] : hi;
    fl |= sfl[0];
    red[3 * bid + 0] = lo;
    red[3 * bid + 1] = hi;
    red[3 * bid + 2] = (double)fl;
  }
  // twiddles exp(-2 pi i j / lmax) from an exact argument
  for (int j = bid * blockDim.x + threadIdx.x; j < lmax; j += nblk * blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)j / (double)lmax, &s, &c);
    cplx<R> w;
    w.x = (R)c;
    w.y = (R)(-s);
    tw[j] = w;
  }
}

template <typename R>
__global__ void __launch_bounds__(256) k_prep(const R *__restrict__ f, long long N,
                                              double *__restrict__ red,
                                              cplx<R> *__restrict__ tw, int lmax) {
  prep_block(f, N, red, tw, lmax, (int)blockIdx.x, (int)gridDim.x);
}

// Reduce the prep partials into the reference forcing (Section 5.1).
// Every work-group of the first row pass does this; block 0 publishes it.
__device__ inline void reduce_forcing(const double *__restrict__ red, int ft_mode,
                                      double ft_given, double *out_lo,
                                      double *out_hi, int *out_fl) {
  __shared__ double slo[16], shi[16];
  __shared__ int sfl[16];
  double lo = __builtin_huge_val(), hi = -__builtin_huge_val();
  int fl = 0;
  // the partials of the first kIt rounds are all read before any is used
  // (a loop that folds as it reads waits once per round); the tail loop
  // serves work-groups of fewer than kRedBlocks / kIt threads
  constexpr int kIt = 4;
  double rl[kIt], rh[kIt], rf[kIt];
#pragma unroll
  for (int u = 0; u < kIt; ++u) {
    const int i = (int)threadIdx.x + u * (int)blockDim.x;
    const int k = i < kRedBlocks ? i : 0;
    rl[u] = red[3 * k];
    rh[u] = red[3 * k + 1];
    rf[u] = i < kRedBlocks ? red[3 * k + 2] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kIt; ++u) {
    lo = rl[u] < lo ? rl[u] : lo;
    hi = rh[u] > hi ? rh[u] : hi;
    fl |= (int)rf[u];
  }
  for (int i = threadIdx.x + kIt * blockDim.x; i < kRedBlocks; i += blockDim.x) {
    lo = red[3 * i] < lo ? red[3 * i] : lo;
    hi = red[3 * i + 1] > hi ? red[3 * i + 1] : hi;
    fl |= (int)red[3 * i + 2];
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  fl = wave_or(fl);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    slo[wid] = lo;
    shi[wid] = hi;
    sfl[wid] = fl;
  }
  __syncthreads();
  lo = slo[0];
  hi = shi[0];
  fl = sfl[0];
  for (int w = 1; w < nw; ++w) {
    lo = slo[w] < lo ? slo[w] : lo;
    hi = shi[w] > hi ? shi[w] : hi;
    fl |= sfl[w];
  }
  *out_lo = lo;
  *out_hi = hi;
  *out_fl = fl;
}

// block reductions for up to 1024 threads (16 waves)
__device__ inline double block_max(double x) {
  __shared__ double s[16];
  x = wave_max(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) s[wid] = x;
  __syncthreads();
  x = s[0];
  for (int w = 1; w < nw; ++w) x = s[w] > x ? s[w] : x;
  return x;
}

// sums of K doubles over the block (every thread gets them)
template <int K> __device__ inline void block_sums_d(double (&v)[K]) {
  __shared__ double s[K][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) s[k][wid] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = s[k][0];
    for (int w = 1; w < nw; ++w) x += s[k][w];
    v[k] = x;
  }
}

__device__ inline long long block_sum_ll(long long x) {
  __shared__ long long s[16];
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) s[wid] = x;
  __syncthreads();
  x = s[0];
  for (int w = 1; w < nw; ++w) x += s[w];
  return x;
}

// binary exponent step for a measured maximum (0 when it is 0 or not finite)
__device__ inline int exp_step(double mu) {
  if (!(mu > 0.0) || !isfinite(mu)) return 0;
  return ilogb(mu);
}

// S = -hbar ln phi (eq. SfromPhi); phi <= 0 or not finite -> +inf.
// Returns 1 for such a point.
template <typename A>
__device__ __forceinline__ int write_S(const A &a, size_t i, double phi) {
  const bool ok = phi > 0.0 && isfinite(phi);
  using R = typename std::remove_pointer<decltype(a.S)>::type;
  a.S[i] = ok ? (R)(-a.hbar * log(phi)) : (R)__builtin_huge_val();
  return ok ? 0 : 1;
}

// Tilted solve, last pass: phi~ = phi exp(a . x - A) at point i (ax =
// a . x - A).  The result replaces the stored one when its score
// ln phi~ - ln B (B the tilt's noise scale: FFT rounding is about eps B in
// phi~ everywhere, so exp(-score) is the relative error to expect) beats the
// score stored by an earlier tilt (prev), or on the first tilt.  Returns 1,
// on the last tilt, for a point that no tilt resolved (phi~ <= 0 in every
// tilt: S = +inf).
template <typename A>
__device__ __forceinline__ int write_S_tilt(const A &a, size_t i, double phit, double ax,
                                            double lnB, float prev) {
  using R = typename std::remove_pointer<decltype(a.S)>::type;
  const bool ok = phit > 0.0 && isfinite(phit);
  const double lp = ok ? log(phit) : 0.0;
  const float sc = ok ? (float)(lp - lnB) : -__builtin_huge_valf();
  const bool take = a.tfirst || sc > prev;
  if (take) {
    a.S[i] = ok ? (R)(-a.hbar * (lp - ax)) : (R)__builtin_huge_val();
    a.best[i] = sc;
  }
  const float now = take ? sc : prev;
  return (a.tlast && !(now > -__builtin_huge_valf())) ? 1 : 0;
}

// Tilted solve split over the sources (phi = sum_k phi^(k) at a fixed
// reference forcing: the series is linear in phi_0): acc = ln sum over the
// sources solved so far of exp(-S_k / hbar), S_k the source's result in S
// (+inf contributes nothing).  The last source's call writes S = -hbar acc
// and counts the points that no source resolved.
template <typename R>
__global__ void __launch_bounds__(256) k_source_lse(R *__restrict__ S, double *__restrict__ acc,
                                                    long long N, double hbar, int first, int last,
                                                    sweik_info *info) {
  const double ninf = -__builtin_huge_val();
  long long nbad = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const double s = (double)S[i];
    const double l = s < __builtin_huge_val() ? -s / hbar : ninf;  // +inf and NaN: nothing
    double a = l;
    if (!first) {
      const double b = acc[i];
      const double m = fmax(a, b);
      a = m > ninf ? m + log1p(exp(-fabs(a - b))) : ninf;
    }
    if (last) {
      const bool ok = a > ninf;
      S[i] = ok ? (R)(-hbar * a) : (R)__builtin_huge_val();
      nbad += ok ? 0 : 1;
    } else {
      acc[i] = a;
    }
  }
  if (last && info) {
    const long long nb = block_sum_ll(nbad);
    if (threadIdx.x == 0 && nb)
      atomicAdd((unsigned long long *)&info->n_nonpositive_phi, (unsigned long long)nb);
  }
}

// One instance of an uneven batch: its arguments and the first work-group
// of its share of a batched launch.
template <typename R> struct BatchItem {
  Args2<R> a;
  int begin;
  int pad_;
};

// Far-field stabilised solve, all tilts in one launch per pass: each tilt
// owns a slice of the workspace (its spectra, kernel spectrum, terms,
// scales, result and scores) at these byte offsets, and the passes run as
// uneven batches over the tilts' work lists.
struct TiltTable {
  double t[2 * SWEIK_MAX_TILTS];  // (tilt0, tilt1) per tilt, in units of beta
};
struct TiltSlice {
  size_t spec, spec_neg, gc, terms, mu, expo, tmax, S, best, bytes;
};

// The work lists of the tilts' passes from the solve's arguments: rows and
// cols for the row and column passes, negs for the kernel-table rows
// m0 <= 0 (into spec_neg).  Every tilt stores its own S and scores (tfirst);
// only tilt 0 reports into info, and k_tilt_select counts.
template <typename R>
__global__ void __launch_bounds__(64) k_tilt_items(Args2<R> base, TiltTable tt, int n_tilt,
                                                   unsigned char *slices, TiltSlice sl,
                                                   BatchItem<R> *rows, BatchItem<R> *negs,
                                                   BatchItem<R> *cols) {
  const int d = threadIdx.x;
  if (d >= n_tilt) return;
  unsigned char *s = slices + (size_t)d * sl.bytes;
  Args2<R> a = base;
  a.spec = reinterpret_cast<cplx<R> *>(s + sl.spec);
  a.spec_neg = reinterpret_cast<cplx<R> *>(s + sl.spec_neg);
  a.gc = reinterpret_cast<cplx<R> *>(s + sl.gc);
  a.terms = reinterpret_cast<R *>(s + sl.terms);
  a.mu = reinterpret_cast<double *>(s + sl.mu);
  a.expo = reinterpret_cast<int *>(s + sl.expo);
  a.tmax = reinterpret_cast<double *>(s + sl.tmax);
  a.S = reinterpret_cast<R *>(s + sl.S);
  a.best = reinterpret_cast<float *>(s + sl.best);
  a.tilt0 = tt.t[2 * d];
  a.tilt1 = tt.t[2 * d + 1];
  a.tsign = 1;
  a.tfirst = 1;
  a.tlast = 0;
  if (d > 0) a.info = nullptr;
  rows[d].a = a;
  rows[d].begin = d * a.nbr;
  rows[d].pad_ = 0;
  cols[d].a = a;
  cols[d].begin = d * a.ncw;
  cols[d].pad_ = 0;
  a.tsign = -1;
  a.spec = a.spec_neg;
  negs[d].a = a;
  negs[d].begin = d * a.nbr;
  negs[d].pad_ = 0;
}

// Per point the tilt with the highest score (the first on ties, as if the
// tilts had been solved in turn): its S into the result; with count, the
// points no tilt resolved (S = +inf) into info.
template <typename R>
__global__ void __launch_bounds__(256) k_tilt_select(R *__restrict__ S,
                                                     const unsigned char *__restrict__ slices,
                                                     TiltSlice sl, int n_tilt, long long N,
                                                     int count, sweik_info *info) {
  long long nbad = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    float best = -__builtin_huge_valf();
    R v = (R)0;
    for (int d = 0; d < n_tilt; ++d) {
      const unsigned char *p = slices + (size_t)d * sl.bytes;
      const float b = reinterpret_cast<const float *>(p + sl.best)[i];
      if (d == 0 || b > best) {
        best = b;
        v = reinterpret_cast<const R *>(p + sl.S)[i];
      }
    }
    S[i] = v;
    nbad += best > -__builtin_huge_valf() ? 0 : 1;
  }
  if (count && info) {
    const long long nb = block_sum_ll(nbad);
    if (threadIdx.x == 0 && nb)
      atomicAdd((unsigned long long *)&info->n_nonpositive_phi, (unsigned long long)nb);
  }
}

// Pointers read from a work list in memory are generic to the compiler (flat
// loads and stores).  Rebuilding each one as a global-address-space pointer
// from its integer value lets it use global memory instructions (a plain
// generic -> global -> generic cast is folded away).
template <typename T> __device__ __forceinline__ T *as_global(T *p) {
  using G = __attribute__((address_space(1))) T;
  return (T *)(G *)(unsigned long)p;
}
template <typename R> __device__ __forceinline__ Args2<R> item_args(const BatchItem<R> &it) {
  Args2<R> a = it.a;
  a.f = as_global(a.f);
  a.src = as_global(a.src);
  a.src_s = as_global(a.src_s);
  a.S = as_global(a.S);
  a.par = as_global(a.par);
  a.red = as_global(a.red);
  a.mu = as_global(a.mu);
  a.expo = as_global(a.expo);
  a.tw = as_global(a.tw);
  a.spec = as_global(a.spec);
  a.g = as_global(a.g);
  a.acc = as_global(a.acc);
  a.terms = as_global(a.terms);
  a.gam = as_global(a.gam);
  a.dLdS = as_global(a.dLdS);
  a.dLdf = as_global(a.dLdf);
  a.lam = as_global(a.lam);
  a.info = as_global(a.info);
  a.ck_expo = as_global(a.ck_expo);
  a.ck_phi = as_global(a.ck_phi);
  a.ck_terms = as_global(a.ck_terms);
  a.spec2 = as_global(a.spec2);
  a.gpart = as_global(a.gpart);
  a.gc = as_global(a.gc);
  a.spec_neg = as_global(a.spec_neg);
  a.best = as_global(a.best);
  a.tmax = as_global(a.tmax);
  return a;
}

// Instance owning work-group g (items sorted by begin; small lists).
template <typename R>
__device__ __forceinline__ int find_item(const BatchItem<R> *items, int n, int g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].begin <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename R>
__global__ void __launch_bounds__(256) k_prep_batch(const BatchItem<R> *__restrict__ items) {
  const int i = blockIdx.x / kRedBlocks, bid = blockIdx.x % kRedBlocks;
  const Args2<R> a = item_args(items[i]);
  prep_block(a.f, (long long)a.n0 * a.n1, a.red, const_cast<cplx<R> *>(a.tw),
             1 << a.lmax_log, bid, kRedBlocks);
}

// Source grid of phi_0 by FFT: the weight exp(-s_k/hbar) (1 without values)
// at every source of a zeroed grid (n0 x n1, or n0 x n1 x n2 when n2 > 0).
template <typename R>
__global__ void __launch_bounds__(256) k_seed_scatter(R *__restrict__ grid, const int *__restrict__ src,
                                                      const R *__restrict__ src_s, int n_src,
                                                      double hbar, int n0, int n1, int n2) {
  const int nd = n2 > 0 ? 3 : 2;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_src; k += gridDim.x * blockDim.x) {
    const int y0 = src[nd * k], y1 = src[nd * k + 1], y2 = nd == 3 ? src[nd * k + 2] : 0;
    // sources outside the grid are flagged by the kernel-table pass
    if (y0 < 0 || y0 >= n0 || y1 < 0 || y1 >= n1 || (nd == 3 && (y2 < 0 || y2 >= n2))) continue;
    const size_t at = nd == 3 ? ((size_t)y0 * n1 + y1) * n2 + y2 : (size_t)y0 * n1 + y1;
    grid[at] = src_s ? (R)exp(-(double)src_s[k] / hbar) : (R)1;
  }
}

// Work-group index -> tile index such that consecutive tiles run on the same
// XCD (blocks are dispatched round-robin over the 8 XCDs, each with its own
// L2): tiles sharing cache lines then share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  constexpr int kXcd = 8;
  const int q = nblocks / kXcd, rem = nblocks % kXcd;
  const int x = b % kXcd, m = b / kXcd;
  return x * q + min(x, rem) + m;
}

}  // namespace sweik
