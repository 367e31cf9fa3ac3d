/*
 * oracle.c -- plain FP64 CPU oracle for the linearised eikonal solve.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written for clarity, not speed:
 * an iterative radix-2 FFT over full complex arrays, a direct O(N^2)
 * convolution with compensated summation, Bessel functions from their series
 * and integral representations.  Build with FP contraction off.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const double PI = 3.14159265358979323846264338327950288;
static const double EULER_GAMMA = 0.57721566490153286060651209008240243;

/* ------------------------------------------------------------------------ */
/* FFT: iterative radix-2 Cooley-Tukey, bit-reversed input order.            */
/* ------------------------------------------------------------------------ */

static int is_pow2(int64_t m) { return m > 0 && (m & (m - 1)) == 0; }

static int64_t next_pow2(int64_t m) {
  int64_t p = 1;
  while (p < m) p <<= 1;
  return p;
}

/* Twiddles w[j] = exp(-2 pi i j / M), j < M/2, each from an exact argument. */
static double *make_twiddles(int64_t M) {
  int64_t half = M / 2 > 0 ? M / 2 : 1;
  double *w = (double *)malloc(sizeof(double) * 2 * half);
  for (int64_t j = 0; j < half; ++j) {
    double a = 2.0 * PI * (double)j / (double)M;
    w[2 * j] = cos(a);
    w[2 * j + 1] = -sin(a);
  }
  return w;
}

static void fft_line(double *x, int64_t M, const double *tw, int inverse) {
  /* bit reversal permutation */
  for (int64_t i = 1, j = 0; i < M; ++i) {
    int64_t bit = M >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double tr = x[2 * i], ti = x[2 * i + 1];
      x[2 * i] = x[2 * j];
      x[2 * i + 1] = x[2 * j + 1];
      x[2 * j] = tr;
      x[2 * j + 1] = ti;
    }
  }
  for (int64_t len = 2; len <= M; len <<= 1) {
    int64_t half = len / 2, step = M / len;
    for (int64_t s = 0; s < M; s += len) {
      for (int64_t k = 0; k < half; ++k) {
        double wr = tw[2 * k * step];
        double wi = inverse ? -tw[2 * k * step + 1] : tw[2 * k * step + 1];
        double *a = x + 2 * (s + k), *b = x + 2 * (s + k + half);
        double br = b[0] * wr - b[1] * wi;
        double bi = b[0] * wi + b[1] * wr;
        b[0] = a[0] - br;
        b[1] = a[1] - bi;
        a[0] = a[0] + br;
        a[1] = a[1] + bi;
      }
    }
  }
  if (inverse) {
    double s = 1.0 / (double)M;
    for (int64_t i = 0; i < 2 * M; ++i) x[i] *= s;
  }
}

int orc_fft(int64_t M, double *data, int inverse) {
  if (!is_pow2(M) || !data) return -1;
  double *tw = make_twiddles(M);
  fft_line(data, M, tw, inverse);
  free(tw);
  return 0;
}

/* N-D complex FFT over an array of shape M[0..ndim), applied axis by axis. */
static void fft_nd(double *a, int ndim, const int64_t *M, int inverse) {
  int64_t total = 1;
  for (int d = 0; d < ndim; ++d) total *= M[d];
  for (int d = 0; d < ndim; ++d) {
    int64_t len = M[d];
    int64_t stride = 1;
    for (int e = d + 1; e < ndim; ++e) stride *= M[e];
    int64_t nlines = total / len;
    double *tw = make_twiddles(len);
#pragma omp parallel
    {
      double *buf = (double *)malloc(sizeof(double) * 2 * len);
#pragma omp for schedule(static)
      for (int64_t l = 0; l < nlines; ++l) {
        int64_t outer = l / stride, inner = l % stride;
        int64_t base = outer * len * stride + inner;
        for (int64_t j = 0; j < len; ++j) {
          buf[2 * j] = a[2 * (base + j * stride)];
          buf[2 * j + 1] = a[2 * (base + j * stride) + 1];
        }
        fft_line(buf, len, tw, inverse);
        for (int64_t j = 0; j < len; ++j) {
          a[2 * (base + j * stride)] = buf[2 * j];
          a[2 * (base + j * stride) + 1] = buf[2 * j + 1];
        }
      }
      free(buf);
    }
    free(tw);
  }
}

/* ------------------------------------------------------------------------ */
/* Modified Bessel functions of the second kind, orders 0 and 1.            */
/*   x <= 2: power series (Abramowitz & Stegun 9.6.13 and 9.6.11).          */
/*   x  > 2: trapezoid rule on e^x K_nu(x) = int_0^inf exp(-x(cosh t - 1))  */
/*           cosh(nu t) dt (A&S 9.6.24); the integrand is analytic in the    */
/*           strip |Im t| < pi/2, so the rule converges geometrically; the   */
/*           step pi^2/(x+45) keeps the discretisation error below 1e-17.   */
/* ------------------------------------------------------------------------ */

static double k_integral_scaled(double x, int nu) {
  double eta = PI * PI / (x + 45.0);
  double sum = 0.5; /* g(0) = 1 */
  for (int j = 1; j < 100000; ++j) {
    double t = eta * (double)j;
    double sh = sinh(0.5 * t);
    double g = exp(-x * 2.0 * sh * sh); /* cosh t - 1 = 2 sinh^2(t/2) */
    if (nu) g *= cosh(t);
    sum += g;
    if (g < 1e-18 * sum) break;
  }
  return eta * sum;
}

double orc_bessel_k0(double x) {
  if (isnan(x) || x < 0.0) return NAN;
  if (x == 0.0) return INFINITY;
  if (x <= 2.0) {
    double q = 0.25 * x * x, term = 1.0, i0 = 1.0, sh = 0.0, hk = 0.0;
    for (int k = 1; k < 80; ++k) {
      term *= q / ((double)k * (double)k);
      hk += 1.0 / (double)k;
      i0 += term;
      sh += term * hk;
      if (term < 1e-19 * i0) break;
    }
    return -(log(0.5 * x) + EULER_GAMMA) * i0 + sh;
  }
  return exp(-x) * k_integral_scaled(x, 0);
}

/* The parts of x K1(x) = 1 + x ln(x/2) I1(x) - (x^2/4) sum_k c_k (x^2/4)^k
 * with c_k = (psi(k+1) + psi(k+2)) / (k! (k+1)!)  (A&S 9.6.11, n = 1). */
static void k1_series_parts(double x, double *xlnI1, double *tail) {
  double q = 0.25 * x * x;
  double term = 1.0;  /* q^k / (k! (k+1)!) */
  double psi1 = -EULER_GAMMA;               /* psi(k+1) */
  double psi2 = -EULER_GAMMA + 1.0;         /* psi(k+2) */
  double i1s = 0.0, s = 0.0;
  for (int k = 0; k < 80; ++k) {
    if (k > 0) {
      term *= q / ((double)k * (double)(k + 1));
      psi1 += 1.0 / (double)k;
      psi2 += 1.0 / (double)(k + 1);
    }
    i1s += term;
    s += (psi1 + psi2) * term;
    if (term < 1e-19 * (i1s > 1.0 ? i1s : 1.0) && k > 2) break;
  }
  /* I1(x) = (x/2) i1s */
  *xlnI1 = x * log(0.5 * x) * (0.5 * x) * i1s;
  *tail = q * s;
}

double orc_bessel_k1(double x) {
  if (isnan(x) || x < 0.0) return NAN;
  if (x == 0.0) return INFINITY;
  if (x <= 2.0) {
    double a, b;
    k1_series_parts(x, &a, &b);
    return (1.0 + a - b) / x;
  }
  return exp(-x) * k_integral_scaled(x, 1);
}

/* ------------------------------------------------------------------------ */
/* Normalised Green's kernel (eqs. GreensFunction2D / GreensFunction3D).   */
/* ------------------------------------------------------------------------ */

double orc_kappa0(int ndim, double beta) {
  if (ndim == 2) {
    /* ball radius r0 = h/sqrt(pi); kappa(0) = int_0^a t K0(t) dt
       = 1 - a K1(a), a = beta/sqrt(pi) */
    double a = beta / sqrt(PI);
    if (a <= 2.0) {
      double p, t;
      k1_series_parts(a, &p, &t);
      return -p + t; /* 1 - a K1(a) without the cancelling leading 1 */
    }
    return 1.0 - a * orc_bessel_k1(a);
  }
  if (ndim == 3) {
    /* r0 = h (3/(4 pi))^(1/3); kappa(0) = int_0^a t e^-t dt = 1-(1+a)e^-a */
    double a = beta * cbrt(3.0 / (4.0 * PI));
    if (a < 0.5) {
      /* sum_{k>=2} (-a)^k (k-1)/k! */
      double s = 0.0, p = 1.0;
      for (int k = 1; k < 40; ++k) {
        p *= -a / (double)k; /* (-a)^k / k! */
        if (k >= 2) s += p * (double)(k - 1);
      }
      return s;
    }
    return 1.0 - (1.0 + a) * exp(-a);
  }
  return NAN;
}

static double kappa_at(int ndim, double beta, double r) {
  if (r == 0.0) return orc_kappa0(ndim, beta);
  if (ndim == 2) return beta * beta / (2.0 * PI) * orc_bessel_k0(beta * r);
  return beta * beta * exp(-beta * r) / (4.0 * PI * r);
}

int orc_kappa(int ndim, const int64_t *dims, double beta, double *kappa) {
  if ((ndim != 2 && ndim != 3) || !dims || !kappa || !(beta > 0)) return -1;
  int64_t n0 = dims[0], n1 = dims[1], n2 = ndim == 3 ? dims[2] : 1;
#pragma omp parallel for schedule(static) collapse(2)
  for (int64_t a = 0; a < n0; ++a)
    for (int64_t b = 0; b < n1; ++b)
      for (int64_t c = 0; c < n2; ++c) {
        double r = sqrt((double)(a * a + b * b + c * c));
        kappa[(a * n1 + b) * n2 + c] = kappa_at(ndim, beta, r);
      }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Convolution plan: padded grid M_d >= 2 n_d - 1, kernel spectrum.         */
/* ------------------------------------------------------------------------ */

typedef struct {
  int ndim;
  int64_t n[3], M[3];
  int64_t N, Np;
  double *kap;   /* orthant kernel table, N entries */
  double *ghat;  /* complex, Np */
  double *work;  /* complex, Np */
} conv_plan;

static void conv_plan_free(conv_plan *c) {
  free(c->kap);
  free(c->ghat);
  free(c->work);
  memset(c, 0, sizeof(*c));
}

static int conv_plan_init(conv_plan *c, int ndim, const int64_t *dims,
                          double beta, int need_fft) {
  memset(c, 0, sizeof(*c));
  c->ndim = ndim;
  c->N = 1;
  c->Np = 1;
  for (int d = 0; d < 3; ++d) {
    c->n[d] = d < ndim ? dims[d] : 1;
    c->M[d] = d < ndim ? next_pow2(2 * dims[d] - 1) : 1;
    c->N *= c->n[d];
    c->Np *= c->M[d];
  }
  c->kap = (double *)malloc(sizeof(double) * c->N);
  if (!c->kap) return -1;
  orc_kappa(ndim, dims, beta, c->kap);
  if (!need_fft) return 0;
  c->ghat = (double *)calloc((size_t)(2 * c->Np), sizeof(double));
  c->work = (double *)calloc((size_t)(2 * c->Np), sizeof(double));
  if (!c->ghat || !c->work) return -1;
  /* place kappa(|m|) at m mod M for |m_d| <= n_d - 1 */
  for (int64_t a = -(c->n[0] - 1); a <= c->n[0] - 1; ++a)
    for (int64_t b = -(c->n[1] - 1); b <= c->n[1] - 1; ++b)
      for (int64_t e = -(c->n[2] - 1); e <= c->n[2] - 1; ++e) {
        int64_t ia = (a + c->M[0]) % c->M[0];
        int64_t ib = (b + c->M[1]) % c->M[1];
        int64_t ie = (e + c->M[2]) % c->M[2];
        int64_t src = (llabs(a) * c->n[1] + llabs(b)) * c->n[2] + llabs(e);
        c->ghat[2 * ((ia * c->M[1] + ib) * c->M[2] + ie)] = c->kap[src];
      }
  fft_nd(c->ghat, ndim, c->M, 0);
  return 0;
}

/* out = kappa (*) in by zero padding, FFT, product, inverse FFT, crop. */
static void conv_fft(conv_plan *c, const double *in, double *out) {
  memset(c->work, 0, sizeof(double) * 2 * c->Np);
  for (int64_t a = 0; a < c->n[0]; ++a)
    for (int64_t b = 0; b < c->n[1]; ++b)
      for (int64_t e = 0; e < c->n[2]; ++e)
        c->work[2 * ((a * c->M[1] + b) * c->M[2] + e)] =
            in[(a * c->n[1] + b) * c->n[2] + e];
  fft_nd(c->work, c->ndim, c->M, 0);
  for (int64_t k = 0; k < c->Np; ++k) {
    double xr = c->work[2 * k], xi = c->work[2 * k + 1];
    double gr = c->ghat[2 * k], gi = c->ghat[2 * k + 1];
    c->work[2 * k] = xr * gr - xi * gi;
    c->work[2 * k + 1] = xr * gi + xi * gr;
  }
  fft_nd(c->work, c->ndim, c->M, 1);
  for (int64_t a = 0; a < c->n[0]; ++a)
    for (int64_t b = 0; b < c->n[1]; ++b)
      for (int64_t e = 0; e < c->n[2]; ++e)
        out[(a * c->n[1] + b) * c->n[2] + e] =
            c->work[2 * ((a * c->M[1] + b) * c->M[2] + e)];
}

/* out(x) = sum_y kappa(x - y) in(y), compensated (Kahan) summation. */
static void conv_direct(conv_plan *c, const double *in, double *out) {
  int64_t n1 = c->n[1], n2 = c->n[2];
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t x = 0; x < c->N; ++x) {
    int64_t xa = x / (n1 * n2), xb = (x / n2) % n1, xe = x % n2;
    double s = 0.0, comp = 0.0;
    for (int64_t y = 0; y < c->N; ++y) {
      int64_t ya = y / (n1 * n2), yb = (y / n2) % n1, ye = y % n2;
      int64_t k = (llabs(xa - ya) * n1 + llabs(xb - yb)) * n2 + llabs(xe - ye);
      double term = c->kap[k] * in[y] - comp;
      double t = s + term;
      comp = (t - s) - term;
      s = t;
    }
    out[x] = s;
  }
}

static void conv_apply(conv_plan *c, int method, const double *in,
                       double *out) {
  if (method == ORC_CONV_DIRECT)
    conv_direct(c, in, out);
  else
    conv_fft(c, in, out);
}

int64_t orc_ghat(int ndim, const int64_t *dims, double beta, double *ghat) {
  if ((ndim != 2 && ndim != 3) || !dims || !ghat || !(beta > 0)) return -1;
  conv_plan c;
  if (conv_plan_init(&c, ndim, dims, beta, 1)) {
    conv_plan_free(&c);
    return -2;
  }
  int64_t h0 = c.M[0] / 2 + 1, h1 = c.M[1] / 2 + 1;
  int64_t h2 = ndim == 3 ? c.M[2] / 2 + 1 : 1;
  for (int64_t a = 0; a < h0; ++a)
    for (int64_t b = 0; b < h1; ++b)
      for (int64_t e = 0; e < h2; ++e)
        ghat[(a * h1 + b) * h2 + e] =
            c.ghat[2 * ((a * c.M[1] + b) * c.M[2] + e)];
  conv_plan_free(&c);
  return h0 * h1 * h2;
}

int orc_phi0(int ndim, const int64_t *dims, double beta, int32_t n_src,
             const int32_t *src, double *phi0) {
  return orc_phi0_weighted(ndim, dims, beta, n_src, src, NULL, phi0);
}

/* Sources with prescribed values S(y_k) = s_k: the source term of the
 * screened Poisson problem for a point whose wave function is exp(-s_k/hbar)
 * there is that multiple of the unit one, so each exponential of eq.
 * phi_0Solution carries the weight w_k = exp(-s_k / hbar) (superposition). */
int orc_phi0_weighted(int ndim, const int64_t *dims, double beta, int32_t n_src,
                      const int32_t *src, const double *w, double *phi0) {
  if ((ndim != 2 && ndim != 3) || !dims || !phi0 || n_src < 1 || !src)
    return -1;
  int64_t n0 = dims[0], n1 = dims[1], n2 = ndim == 3 ? dims[2] : 1;
  int64_t N = n0 * n1 * n2;
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; ++x) {
    int64_t c[3] = {x / (n1 * n2), (x / n2) % n1, x % n2};
    double s = 0.0;
    for (int k = 0; k < n_src; ++k) {
      double r2 = 0.0;
      for (int d = 0; d < ndim; ++d) {
        double dd = (double)(c[d] - src[k * ndim + d]);
        r2 += dd * dd;
      }
      s += (w ? w[k] : 1.0) * exp(-beta * sqrt(r2));
    }
    phi0[x] = s;
  }
  return 0;
}

int orc_conv(int ndim, const int64_t *dims, double beta, const double *in,
             double *out, int32_t method, int32_t nthreads) {
  if ((ndim != 2 && ndim != 3) || !dims || !in || !out || !(beta > 0))
    return -1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  conv_plan c;
  if (conv_plan_init(&c, ndim, dims, beta, method != ORC_CONV_DIRECT)) {
    conv_plan_free(&c);
    return -2;
  }
  conv_apply(&c, method, in, out);
  conv_plan_free(&c);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The solve (Table 1).                                                      */
/* ------------------------------------------------------------------------ */

static int check_problem(const orc_problem *p, const double *f, int32_t n_src,
                         const int32_t *src) {
  if (!p || !f || !src || n_src < 1) return -1;
  if (p->ndim != 2 && p->ndim != 3) return -1;
  for (int d = 0; d < p->ndim; ++d)
    if (p->dims[d] < 1) return -1;
  if (!(p->h > 0) || !(p->hbar > 0) || p->T < 0) return -1;
  for (int k = 0; k < n_src; ++k)
    for (int d = 0; d < p->ndim; ++d)
      if (src[k * p->ndim + d] < 0 || src[k * p->ndim + d] >= p->dims[d])
        return -1;
  return 0;
}

static int64_t grid_size(const orc_problem *p) {
  int64_t N = 1;
  for (int d = 0; d < p->ndim; ++d) N *= p->dims[d];
  return N;
}

/* Reference forcing (Section 5.1) and the derived quantities. */
static int reference_forcing(const orc_problem *p, const double *f, int64_t N,
                             double *ftilde, double *fmin, double *fmax) {
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t i = 0; i < N; ++i) {
    if (!(f[i] > 0) || !isfinite(f[i])) return -3;
    if (f[i] < lo) lo = f[i];
    if (f[i] > hi) hi = f[i];
  }
  *fmin = lo;
  *fmax = hi;
  if (p->ft_mode == ORC_FT_NU)
    *ftilde = sqrt(0.5 * (lo * lo + hi * hi));
  else if (p->ft_mode == ORC_FT_FMAX)
    *ftilde = hi;
  else if (p->ft_mode == ORC_FT_GIVEN)
    *ftilde = p->ftilde_given;
  else
    return -1;
  return (*ftilde > 0 && isfinite(*ftilde)) ? 0 : -1;
}

/* Forward series.  terms (T+1)*N may be NULL; phi (N) required. */
static int forward(const orc_problem *p, const double *f, int32_t n_src,
                   const int32_t *src, double *phi, double *terms,
                   double *gamma_out, conv_plan *c, double *info) {
  int64_t N = grid_size(p);
  double ft, lo, hi;
  int rc = reference_forcing(p, f, N, &ft, &lo, &hi);
  if (rc) return rc;
  double beta = ft * p->h / p->hbar;
  double c0 = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    gamma_out[i] = f[i] * f[i] / (ft * ft) - 1.0;
    if (fabs(gamma_out[i]) > c0) c0 = fabs(gamma_out[i]);
  }
  if (conv_plan_init(c, p->ndim, p->dims, beta, p->conv != ORC_CONV_DIRECT))
    return -2;
  double *prev = (double *)malloc(sizeof(double) * N);
  double *cur = (double *)malloc(sizeof(double) * N);
  double *psi = (double *)malloc(sizeof(double) * N);
  if (!prev || !cur || !psi) {
    free(prev);
    free(cur);
    free(psi);
    return -2;
  }
  double *w = NULL;
  if (p->src_s) {
    w = (double *)malloc(sizeof(double) * n_src);
    if (!w) {
      free(prev);
      free(cur);
      free(psi);
      return -2;
    }
    for (int k = 0; k < n_src; ++k) w[k] = exp(-p->src_s[k] / p->hbar);
  }
  orc_phi0_weighted(p->ndim, p->dims, beta, n_src, src, w, prev);
  free(w);
  memcpy(phi, prev, sizeof(double) * N);
  if (terms) memcpy(terms, prev, sizeof(double) * N);
  for (int i = 1; i <= p->T; ++i) {
    for (int64_t x = 0; x < N; ++x) psi[x] = gamma_out[x] * prev[x];
    conv_apply(c, p->conv, psi, cur);
    double sgn = (i & 1) ? -1.0 : 1.0;
    for (int64_t x = 0; x < N; ++x) phi[x] += sgn * cur[x];
    if (terms) memcpy(terms + (int64_t)i * N, cur, sizeof(double) * N);
    double *t = prev;
    prev = cur;
    cur = t;
  }
  free(prev);
  free(cur);
  free(psi);
  if (info) {
    info[0] = ft;
    info[1] = beta;
    info[2] = lo;
    info[3] = hi;
    info[4] = c0;
    info[6] = (double)c->Np;
    info[7] = 0.0;
  }
  return 0;
}

int orc_solve(const orc_problem *p, const double *f, int32_t n_src,
              const int32_t *src, double *S, double *phi_out, double *terms,
              double *info) {
  if (check_problem(p, f, n_src, src) || !S) return -1;
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
  int64_t N = grid_size(p);
  double *phi = phi_out ? phi_out : (double *)malloc(sizeof(double) * N);
  double *gam = (double *)malloc(sizeof(double) * N);
  conv_plan c;
  memset(&c, 0, sizeof(c));
  int rc = forward(p, f, n_src, src, phi, terms, gam, &c, info);
  if (rc == 0) {
    int64_t bad = 0;
    for (int64_t x = 0; x < N; ++x) {
      if (phi[x] > 0 && isfinite(phi[x])) {
        S[x] = -p->hbar * log(phi[x]);
      } else {
        S[x] = INFINITY;
        ++bad;
      }
    }
    if (info) info[5] = (double)bad;
  }
  conv_plan_free(&c);
  free(gam);
  if (!phi_out) free(phi);
  return rc;
}

/* Reverse sweep of the recurrence with ftilde fixed:
 *   lambda = dL/dphi = -hbar dL/dS / phi
 *   a_T = (-1)^T lambda;  for i = T..1:  b_i = kappa (*) a_i  (kappa even),
 *   dL/dgamma += phi_{i-1} b_i,  a_{i-1} = (-1)^{i-1} lambda + gamma b_i
 *   dL/df = dL/dgamma * 2 f / ftilde^2                                     */
int orc_adjoint(const orc_problem *p, const double *f, int32_t n_src,
                const int32_t *src, const double *dLdS, double *dLdf,
                double *info) {
  if (check_problem(p, f, n_src, src) || !dLdS || !dLdf) return -1;
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
  int64_t N = grid_size(p);
  int T = p->T;
  double *terms = (double *)malloc(sizeof(double) * N * (size_t)(T + 1));
  double *phi = (double *)malloc(sizeof(double) * N);
  double *gam = (double *)malloc(sizeof(double) * N);
  double *lam = (double *)malloc(sizeof(double) * N);
  double *a = (double *)malloc(sizeof(double) * N);
  double *b = (double *)malloc(sizeof(double) * N);
  double *g = (double *)calloc((size_t)N, sizeof(double));
  double inf[8] = {0};
  conv_plan c;
  memset(&c, 0, sizeof(c));
  int rc = -2;
  if (terms && phi && gam && lam && a && b && g)
    rc = forward(p, f, n_src, src, phi, terms, gam, &c, inf);
  if (rc == 0) {
    double ft = inf[0];
    for (int64_t x = 0; x < N; ++x)
      lam[x] = (phi[x] > 0 && isfinite(phi[x])) ? -p->hbar * dLdS[x] / phi[x]
                                                 : 0.0;
    double sT = (T & 1) ? -1.0 : 1.0;
    for (int64_t x = 0; x < N; ++x) a[x] = sT * lam[x];
    for (int i = T; i >= 1; --i) {
      conv_apply(&c, p->conv, a, b);
      const double *prev = terms + (int64_t)(i - 1) * N;
      double s = ((i - 1) & 1) ? -1.0 : 1.0;
      for (int64_t x = 0; x < N; ++x) {
        g[x] += prev[x] * b[x];
        a[x] = s * lam[x] + gam[x] * b[x];
      }
    }
    for (int64_t x = 0; x < N; ++x) dLdf[x] = g[x] * 2.0 * f[x] / (ft * ft);
    if (info) memcpy(info, inf, sizeof(inf));
  }
  conv_plan_free(&c);
  free(terms);
  free(phi);
  free(gam);
  free(lam);
  free(a);
  free(b);
  free(g);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Log-domain direct path (reference forcing sup f).                         */
/* ------------------------------------------------------------------------ */
/* With ftilde = sup f every gamma = f^2/ftilde^2 - 1 is <= 0 while kappa > 0,
 * so t_i = (-1)^i phi_i = kappa (*) ((-gamma) t_{i-1}) is a sum of
 * non-negative products for every i (the monotone case of Section 5.1), and
 * phi = sum_i t_i.  Carried as logarithms, each sum is a log-sum-exp: every
 * value keeps full relative accuracy at any distance from the sources,
 * where exp(-S/hbar) underflows double precision and FFT rounding noise
 * swamps the value.  O(N^2) per term: tiny grids only. */

/* ln kappa at distance r (grid units) */
static double log_kappa_at(int ndim, double beta, double r) {
  if (r == 0.0) return log(orc_kappa0(ndim, beta));
  double x = beta * r;
  if (ndim == 2) {
    double lk0 = x <= 2.0 ? log(orc_bessel_k0(x)) : -x + log(k_integral_scaled(x, 0));
    return log(beta * beta / (2.0 * PI)) + lk0;
  }
  return log(beta * beta / (4.0 * PI * r)) - x;
}

/* ln(e^a + e^b) */
static double log_add(double a, double b) {
  if (a == -INFINITY) return b;
  if (b == -INFINITY) return a;
  double m = a > b ? a : b;
  return m + log1p(exp(-fabs(a - b)));
}

int orc_solve_logdirect(const orc_problem *p, const double *f, int32_t n_src,
                        const int32_t *src, double *S, double *logphi,
                        double *info) {
  if (check_problem(p, f, n_src, src) || !S || p->ft_mode != ORC_FT_FMAX) return -1;
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
  int64_t N = grid_size(p);
  double ft, lo, hi;
  int rc = reference_forcing(p, f, N, &ft, &lo, &hi);
  if (rc) return rc;
  double beta = ft * p->h / p->hbar;
  int64_t n0 = p->dims[0], n1 = p->dims[1], n2 = p->ndim == 3 ? p->dims[2] : 1;
  double *lk = (double *)malloc(sizeof(double) * N);   /* ln kappa, orthant */
  double *lg = (double *)malloc(sizeof(double) * N);   /* ln(-gamma) */
  double *prev = (double *)malloc(sizeof(double) * N); /* ln t_{i-1} */
  double *cur = (double *)malloc(sizeof(double) * N);
  double *lphi = logphi ? logphi : (double *)malloc(sizeof(double) * N);
  if (!lk || !lg || !prev || !cur || !lphi) {
    free(lk);
    free(lg);
    free(prev);
    free(cur);
    if (!logphi) free(lphi);
    return -2;
  }
  double c0 = 0.0;
  for (int64_t a = 0; a < n0; ++a)
    for (int64_t b = 0; b < n1; ++b)
      for (int64_t e = 0; e < n2; ++e) {
        int64_t i = (a * n1 + b) * n2 + e;
        lk[i] = log_kappa_at(p->ndim, beta, sqrt((double)(a * a + b * b + e * e)));
        double g = f[i] * f[i] / (ft * ft) - 1.0;  /* <= 0 */
        if (fabs(g) > c0) c0 = fabs(g);
        lg[i] = -g > 0.0 ? log(-g) : -INFINITY;
      }
  /* ln phi_0 = ln sum_k exp(-s_k/hbar - beta |x - y_k|) (eq. phi_0Solution) */
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < N; ++x) {
    int64_t xa = x / (n1 * n2), xb = (x / n2) % n1, xe = x % n2;
    double acc = -INFINITY;
    for (int k = 0; k < n_src; ++k) {
      double d0 = (double)(xa - src[k * p->ndim]);
      double d1 = (double)(xb - src[k * p->ndim + 1]);
      double d2 = p->ndim == 3 ? (double)(xe - src[k * p->ndim + 2]) : 0.0;
      double lw = p->src_s ? -p->src_s[k] / p->hbar : 0.0;
      acc = log_add(acc, lw - beta * sqrt(d0 * d0 + d1 * d1 + d2 * d2));
    }
    prev[x] = acc;
    lphi[x] = acc;
  }
  for (int i = 1; i <= p->T; ++i) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t x = 0; x < N; ++x) {
      int64_t xa = x / (n1 * n2), xb = (x / n2) % n1, xe = x % n2;
      /* ln t_i(x) = ln sum_y kappa(x-y) (-gamma(y)) t_{i-1}(y): the largest
         summand first, then the sum of the others relative to it */
      double m = -INFINITY;
      for (int64_t y = 0; y < N; ++y) {
        int64_t ya = y / (n1 * n2), yb = (y / n2) % n1, ye = y % n2;
        int64_t k = (llabs(xa - ya) * n1 + llabs(xb - yb)) * n2 + llabs(xe - ye);
        double v = lk[k] + lg[y] + prev[y];
        if (v > m) m = v;
      }
      double sum = 0.0;
      if (m > -INFINITY)
        for (int64_t y = 0; y < N; ++y) {
          int64_t ya = y / (n1 * n2), yb = (y / n2) % n1, ye = y % n2;
          int64_t k = (llabs(xa - ya) * n1 + llabs(xb - yb)) * n2 + llabs(xe - ye);
          sum += exp(lk[k] + lg[y] + prev[y] - m);
        }
      cur[x] = m > -INFINITY ? m + log(sum) : -INFINITY;
      lphi[x] = log_add(lphi[x], cur[x]);
    }
    double *t = prev;
    prev = cur;
    cur = t;
  }
  for (int64_t x = 0; x < N; ++x) S[x] = -p->hbar * lphi[x];
  if (info) {
    info[0] = ft;
    info[1] = beta;
    info[2] = lo;
    info[3] = hi;
    info[4] = c0;
    info[5] = 0.0;
    info[6] = 0.0;
    info[7] = 0.0;
  }
  free(lk);
  free(lg);
  free(prev);
  free(cur);
  if (!logphi) free(lphi);
  return 0;
}

/* ln kappa on the orthant of offsets (for tests of the log-domain path) */
int orc_log_kappa(int ndim, const int64_t *dims, double beta, double *out) {
  if ((ndim != 2 && ndim != 3) || !dims || !out || !(beta > 0)) return -1;
  int64_t n0 = dims[0], n1 = dims[1], n2 = ndim == 3 ? dims[2] : 1;
  for (int64_t a = 0; a < n0; ++a)
    for (int64_t b = 0; b < n1; ++b)
      for (int64_t c = 0; c < n2; ++c)
        out[(a * n1 + b) * n2 + c] =
            log_kappa_at(ndim, beta, sqrt((double)(a * a + b * b + c * c)));
  return 0;
}
