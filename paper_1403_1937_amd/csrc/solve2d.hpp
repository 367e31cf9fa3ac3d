// solve2d.hpp -- gfx950 kernels of the 2D perturbation-series eikonal solve.
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

#include "fft_team.hpp"
#include "green.hpp"
#include "../../include/sweik.h"

namespace sweik {

enum RowMode { ROW_GHAT = 0, ROW_PHI0 = 1, ROW_TERM = 2 };
enum ColMode { COL_GHAT = 0, COL_CONV = 1 };

constexpr int kRedBlocks = 256;  // partial reductions of f

struct Params {      // device-side scalars shared by the kernels of a solve
  double ftilde, beta, hbar, inv_ft2, kappa0, fmin, fmax, c0;
  int flags, pad_;
};

template <typename R> struct Args2 {
  // geometry
  int n0, n1;      // grid
  int H1, ldk;     // M1/2, H1+1 spectral columns
  int M0, H0, ldg; // column FFT length, M0/2, H0+1
  int RB, nb;      // rows per spectral block, number of blocks
  int rpw, cpw;    // rows per row-pass WG, columns per column-pass WG
  int nbr;         // number of row-pass WGs
  int lmax_log;    // log2 of the twiddle table length
  int T, n_src, ft_mode;
  double ftilde_given, h, hbar;
  // data
  const R *f;
  const int *src;
  R *S;
  // workspace
  Params *par;
  double *red;   // kRedBlocks x 3 (min, max, flags)
  double *mu;    // (T+1) x nbr partial max |m_i|
  int *expo;     // T+1 exponents
  const cplx<R> *tw;
  cplx<R> *spec;
  R *g;          // (H1+1) x (H0+1) kernel spectrum, pre-scaled
  double *acc;   // n0 x n1
  // optional
  sweik_info *info;
  int *ck_expo;  // T+1
  double *ck_phi;// n0 x n1
  R *ck_terms;   // T x n0 x n1
};

// ---------------------------------------------------------------------------
// prep: partial min / max / validity of f, and the twiddle table
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) k_prep(const R *__restrict__ f, long long N,
                                              double *__restrict__ red,
                                              cplx<R> *__restrict__ tw, int lmax) {
  __shared__ double smin[4], smax[4];
  __shared__ int sfl[4];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double lo = 1.0 / 0.0, hi = -1.0 / 0.0;
  int fl = 0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (double)f[i];
    if (!isfinite(v)) {
      fl |= SWEIK_FLAG_F_NONFINITE;
      continue;
    }
    if (!(v > 0.0)) fl |= SWEIK_FLAG_F_NONPOSITIVE;
    lo = v < lo ? v : lo;
    hi = v > hi ? v : hi;
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
    red[3 * blockIdx.x + 0] = lo;
    red[3 * blockIdx.x + 1] = hi;
    red[3 * blockIdx.x + 2] = (double)fl;
  }
  // twiddles exp(-2 pi i j / lmax) from an exact argument
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < lmax; j += gridDim.x * blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)j / (double)lmax, &s, &c);
    cplx<R> w;
    w.x = (R)c;
    w.y = (R)(-s);
    tw[j] = w;
  }
}

// Reduce the prep partials into the reference forcing (Section 5.1).
// Every work-group of the first row pass does this; block 0 publishes it.
__device__ inline void reduce_forcing(const double *__restrict__ red, int ft_mode,
                                      double ft_given, double *out_lo,
                                      double *out_hi, int *out_fl) {
  __shared__ double slo[4], shi[4];
  __shared__ int sfl[4];
  double lo = 1.0 / 0.0, hi = -1.0 / 0.0;
  int fl = 0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) {
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

__device__ inline double block_max(double x) {
  __shared__ double s[4];
  x = wave_max(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) s[wid] = x;
  __syncthreads();
  x = s[0];
  for (int w = 1; w < nw; ++w) x = s[w] > x ? s[w] : x;
  return x;
}

__device__ inline long long block_sum_ll(long long x) {
  __shared__ long long s[4];
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

// tile of `rows` spectral rows starting at row0: element e -> (row_local, k1)
struct TileMap {
  int rows, RB, ldk, rr0;
  __device__ __forceinline__ void map(int e, int &rl, int &k1) const {
    if (rows >= RB) {
      const int per = ldk * RB;
      const int bl = e / per;
      const int rem = e - bl * per;
      k1 = rem / RB;
      rl = bl * RB + (rem - k1 * RB);
    } else {
      k1 = e / rows;
      rl = e - k1 * rows;
    }
  }
  // global offset (in elements) of the tile element relative to the tile base
  __device__ __forceinline__ long long goff(int e, int rl, int k1) const {
    if (rows >= RB) return e;
    return (long long)k1 * RB + rl;  // base already includes rr0
  }
};

// ---------------------------------------------------------------------------
// row pass
// ---------------------------------------------------------------------------
template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_row2(Args2<R> a, int term) {
  using C = cplx<R>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *smem = reinterpret_cast<C *>(smem_raw);
  __shared__ double s_par[4];
  __shared__ int s_E;

  const int H = a.H1, P = H >> 4;
  const int logH = 31 - __clz(H);
  const int tw_sh = a.lmax_log - (logH + 1);  // table stride for exp(-2 pi i k / 2H)
  const int tid = threadIdx.x;
  const int team = tid / P, t = tid - team * P;
  const int row0 = blockIdx.x * a.rpw;
  const int r = row0 + team;
  const int LL = lds_line_len(H);
  C *line = smem + team * LL;
  const int spec_rows = a.nb * a.RB;
  const int tile_rows = min(a.rpw, spec_rows - row0);
  const bool row_ok = r < a.n0;
  const bool last = (MODE == ROW_TERM && term == a.T) || (MODE == ROW_PHI0 && a.T == 0);

  // ---- scalars --------------------------------------------------------------
  double beta, inv_ft2, ft;
  if (MODE == ROW_GHAT) {
    double lo, hi;
    int fl;
    reduce_forcing(a.red, a.ft_mode, a.ftilde_given, &lo, &hi, &fl);
    ft = a.ft_mode == SWEIK_FT_NU ? sqrt(0.5 * (lo * lo + hi * hi))
                : a.ft_mode == SWEIK_FT_FMAX ? hi : a.ftilde_given;
    beta = ft * a.h / a.hbar;
    inv_ft2 = 1.0 / (ft * ft);
    if (tid == 0) {
      s_par[0] = kappa0_2d(beta);
      const double c0 = fmax((hi - ft) * (hi + ft), (ft - lo) * (ft + lo)) * inv_ft2;
      if (!(c0 < 1.0)) fl |= SWEIK_FLAG_C0_GE_1;
      for (int k = 0; k < a.n_src; ++k) {
        const int y0 = a.src[2 * k], y1 = a.src[2 * k + 1];
        if (y0 < 0 || y0 >= a.n0 || y1 < 0 || y1 >= a.n1) fl |= SWEIK_FLAG_BAD_SOURCE;
      }
      if (blockIdx.x == 0) {
        Params p;
        p.ftilde = ft;
        p.beta = beta;
        p.hbar = a.hbar;
        p.inv_ft2 = inv_ft2;
        p.kappa0 = s_par[0];
        p.fmin = lo;
        p.fmax = hi;
        p.c0 = c0;
        p.flags = fl;
        p.pad_ = 0;
        *a.par = p;
        if (a.info) {
          a.info->f_min = lo;
          a.info->f_max = hi;
          a.info->ftilde = ft;
          a.info->beta = beta;
          a.info->c0_bound = c0;
          a.info->n_nonpositive_phi = 0;
          a.info->flags = fl;
          a.info->T = a.T;
        }
      }
    }
    __syncthreads();
  } else {
    beta = a.par->beta;
    inv_ft2 = a.par->inv_ft2;
    ft = a.par->ftilde;
  }

  // exponent bookkeeping (phi_i = 2^E_i m_i)
  int dstep = 0, E = 0;
  if (MODE == ROW_TERM) {
    double mu = 0.0;
    for (int i = tid; i < a.nbr; i += blockDim.x) {
      const double v = a.mu[(size_t)(term - 1) * a.nbr + i];
      mu = v > mu ? v : mu;
    }
    mu = block_max(mu);
    dstep = exp_step(mu);
    E = a.expo[term - 1] + dstep;
  }
  if (MODE != ROW_GHAT && blockIdx.x == 0 && tid == 0) {
    const int e = MODE == ROW_TERM ? E : 0;
    a.expo[MODE == ROW_TERM ? term : 0] = e;
    if (a.info) a.info->scale_exp[MODE == ROW_TERM ? term : 0] = e;
    if (a.ck_expo) a.ck_expo[MODE == ROW_TERM ? term : 0] = e;
  }

  C v[16];
  const TileMap tm{tile_rows, a.RB, a.ldk, 0};
  C *gtile = a.spec + (size_t)row0 * a.ldk;  // base of this WG's rows
  if (tile_rows < a.RB) {
    const int b = row0 / a.RB, rr0 = row0 - b * a.RB;
    gtile = a.spec + ((size_t)b * a.ldk * a.RB + rr0);
  }

  if (MODE == ROW_TERM) {
    // ---- load the spectral tile into LDS lines (contiguous in memory)
    const int total = tile_rows * a.ldk;
    for (int e = tid; e < total; e += blockDim.x) {
      int rl, k1;
      tm.map(e, rl, k1);
      smem[rl * LL + lpad(k1)] = gtile[tm.goff(e, rl, k1)];
    }
    __syncthreads();
    // ---- split step of the inverse real FFT: Z = E + iO
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = t + P * j;
      C xk = line[lpad(k)];
      C xc = cconj(line[lpad(H - k)]);
      C w = a.tw[k << tw_sh];
      C e = cadd(xk, xc);
      C o = cmulc(csub(xk, xc), w);
      v[j] = cmake<C>(e.x - o.y, e.y + o.x);
    }
    team_fft<true>(v, t, P, H, line, a.tw, a.lmax_log, true);
  }

  // ---- pointwise step over this thread's columns 2k, 2k+1 (k = t + P j)
  const size_t rowoff = (size_t)r * a.n1;
  double mloc = 0.0;
  long long nbad = 0;
  const double scale_m = ldexp(1.0, -dstep);
  const double scale_E = ldexp(1.0, E);
  const double sgn = (MODE == ROW_TERM && (term & 1)) ? -1.0 : 1.0;
  double k0v = 0.0;
  if (MODE == ROW_GHAT) k0v = s_par[0];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int kk = t + P * j;
    const int c0 = 2 * kk;
    R z0 = 0, z1 = 0;
    if (MODE == ROW_GHAT) {
      // evenly extended kernel row: x[m] = kappa(r, min(m, 2H - m)), zero
      // for offsets >= n1
      if (row_ok) {
        const int m0 = c0 <= H ? c0 : 2 * H - c0;
        const int m1 = c0 + 1 <= H ? c0 + 1 : 2 * H - c0 - 1;
        const long long rr = (long long)r * r;
        if (m0 < a.n1) z0 = (R)kappa_2d(beta, rr + (long long)m0 * m0, k0v);
        if (m1 < a.n1) z1 = (R)kappa_2d(beta, rr + (long long)m1 * m1, k0v);
      }
    } else if (row_ok && c0 < a.n1) {
      const bool ok1 = c0 + 1 < a.n1;
      double p0, p1 = 0.0;      // phi_i contributions (true scale)
      R m0, m1 = 0;             // stored mantissas
      if (MODE == ROW_PHI0) {
        double s0 = 0.0, s1 = 0.0;
        for (int k = 0; k < a.n_src; ++k) {
          const double d0 = (double)(r - a.src[2 * k]);
          const double d1 = (double)(c0 - a.src[2 * k + 1]);
          if (sizeof(R) == 4) {
            const float q0 = (float)(d0 * d0);
            s0 += (double)expf(-(float)beta * sqrtf(q0 + (float)(d1 * d1)));
            s1 += (double)expf(-(float)beta * sqrtf(q0 + (float)((d1 + 1) * (d1 + 1))));
          } else {
            s0 += exp(-beta * sqrt(d0 * d0 + d1 * d1));
            s1 += exp(-beta * sqrt(d0 * d0 + (d1 + 1) * (d1 + 1)));
          }
        }
        m0 = (R)s0;
        m1 = (R)s1;
        p0 = s0;
        p1 = s1;
        a.acc[rowoff + c0] = p0;
        if (ok1) a.acc[rowoff + c0 + 1] = p1;
      } else {
        m0 = (R)((double)v[j].x * scale_m);
        m1 = (R)((double)v[j].y * scale_m);
        p0 = (double)m0 * scale_E;
        p1 = (double)m1 * scale_E;
        double a0 = a.acc[rowoff + c0] + sgn * p0;
        double a1 = ok1 ? a.acc[rowoff + c0 + 1] + sgn * p1 : 0.0;
        if (!last) {
          a.acc[rowoff + c0] = a0;
          if (ok1) a.acc[rowoff + c0 + 1] = a1;
        } else {
          p0 = a0;
          p1 = a1;
        }
      }
      if (last) {
        // S = -hbar ln phi (eq. SfromPhi); phi <= 0 -> +inf
        const double inf = 1.0 / 0.0;
        const double s0 = (p0 > 0.0 && isfinite(p0)) ? -a.hbar * log(p0) : inf;
        nbad += !(p0 > 0.0 && isfinite(p0));
        a.S[rowoff + c0] = (R)s0;
        if (a.ck_phi) a.ck_phi[rowoff + c0] = p0;
        if (ok1) {
          const double s1 = (p1 > 0.0 && isfinite(p1)) ? -a.hbar * log(p1) : inf;
          nbad += !(p1 > 0.0 && isfinite(p1));
          a.S[rowoff + c0 + 1] = (R)s1;
          if (a.ck_phi) a.ck_phi[rowoff + c0 + 1] = p1;
        }
      } else {
        if (a.ck_terms) {
          const int slot = MODE == ROW_TERM ? term : 0;
          R *ck = a.ck_terms + (size_t)slot * a.n0 * a.n1 + rowoff;
          ck[c0] = m0;
          if (ok1) ck[c0 + 1] = m1;
        }
        // gamma = f^2/ftilde^2 - 1, exactly 0 where f = ftilde
        const double fa = (double)a.f[rowoff + c0];
        z0 = (R)((fa - ft) * (fa + ft) * inv_ft2) * m0;
        if (ok1) {
          const double fb = (double)a.f[rowoff + c0 + 1];
          z1 = (R)((fb - ft) * (fb + ft) * inv_ft2) * m1;
        }
        double am = fabs((double)m0);
        if (ok1) am = fmax(am, fabs((double)m1));
        mloc = am > mloc ? am : mloc;
      }
    }
    v[j] = cmake<C>(z0, z1);
  }

  if (MODE != ROW_GHAT) {
    if (last) {
      const long long nb = block_sum_ll(nbad);
      if (tid == 0 && a.info && nb) atomicAdd((unsigned long long *)&a.info->n_nonpositive_phi,
                                              (unsigned long long)nb);
      return;
    }
    const double bm = block_max(mloc);
    if (tid == 0) a.mu[(size_t)(MODE == ROW_TERM ? term : 0) * a.nbr + blockIdx.x] = bm;
  }

  // ---- forward real FFT of the next forcing term, split step, store ---------
  team_fft<false>(v, t, P, H, line, a.tw, a.lmax_log, true);
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) line[lpad(t + P * j)] = v[j];
  __syncthreads();
  C x[16];
  C xH = cmake<C>((R)0, (R)0);
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int k = t + P * j;
    C zk = line[lpad(k)];
    C zc = cconj(line[lpad((H - k) & (H - 1))]);
    C e = cadd(zk, zc);
    C d = csub(zk, zc);
    C o = cmake<C>(d.y, -d.x);  // d / i
    x[j] = cadd(e, cmul(a.tw[k << tw_sh], o));
    if (k == 0) xH = cmake<C>((R)2 * (zk.x - zk.y), (R)0);
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 16; ++j) line[lpad(t + P * j)] = x[j];
  if (t == 0) line[lpad(H)] = xH;
  __syncthreads();
  const int total = tile_rows * a.ldk;
  for (int e = tid; e < total; e += blockDim.x) {
    int rl, k1;
    tm.map(e, rl, k1);
    gtile[tm.goff(e, rl, k1)] = smem[rl * LL + lpad(k1)];
  }
}

// ---------------------------------------------------------------------------
// column pass
// ---------------------------------------------------------------------------
template <typename R, int MODE>
__global__ void __launch_bounds__(256) k_col2(Args2<R> a) {
  using C = cplx<R>;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *smem = reinterpret_cast<C *>(smem_raw);
  const int L = a.M0, P = L >> 4, H0 = a.H0;
  const int tid = threadIdx.x;
  // lanes interleave the teams in groups of RB so that one wave reads RB
  // contiguous rows of CPW neighbouring columns
  const int grp = tid / a.RB, rr = tid - grp * a.RB;
  const int team = grp % a.cpw;
  const int t = (grp / a.cpw) * a.RB + rr;
  const int k1 = blockIdx.x * a.cpw + team;
  const bool active = k1 < a.ldk;
  const int LL = lds_line_len(L);
  C *line = smem + team * LL;
  const int spec_rows = a.nb * a.RB;
  const size_t cstride = (size_t)a.ldk * a.RB;  // elements between blocks
  C *col = a.spec + (size_t)k1 * a.RB;
  C v[16];

  if (MODE == COL_CONV) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int rho = t + P * j;
      C x = cmake<C>((R)0, (R)0);
      if (j < 8 && active && rho < spec_rows) {
        const int b = rho / a.RB;
        x = col[b * cstride + (rho - b * a.RB)];
      }
      v[j] = x;
    }
    team_fft<false>(v, t, P, L, line, a.tw, a.lmax_log, false);
    if (active) {
      const R *gcol = a.g + (size_t)k1 * a.ldg;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k0 = t + P * j;
        const R gv = gcol[k0 <= H0 ? k0 : L - k0];
        v[j] = cscale(v[j], gv);
      }
    }
    team_fft<true>(v, t, P, L, line, a.tw, a.lmax_log, true);
    if (active) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int rho = t + P * j;
        if (rho < spec_rows) {
          const int b = rho / a.RB;
          col[b * cstride + (rho - b * a.RB)] = v[j];
        }
      }
    }
  } else {
    // even extension of the column: x[rho] = x[M0 - rho]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int rho = t + P * j;
      const int sr = rho <= H0 ? rho : L - rho;
      C x = cmake<C>((R)0, (R)0);
      if (active && sr < spec_rows) {
        const int b = sr / a.RB;
        x = col[b * cstride + (sr - b * a.RB)];
      }
      v[j] = x;
    }
    team_fft<false>(v, t, P, L, line, a.tw, a.lmax_log, false);
    if (active) {
      // the row step's split transform is twice the DFT; the column and row
      // round trips contribute M0 and 2 M1: store Ghat / (2 M0 M1)
      const double sc = 1.0 / (4.0 * (double)a.M0 * (double)(2 * a.H1));
      R *gcol = a.g + (size_t)k1 * a.ldg;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k0 = t + P * j;
        if (k0 <= H0) gcol[k0] = (R)((double)v[j].x * sc);
      }
    }
  }
}

}  // namespace sweik
