/*
 * oracle.h -- plain FP64 CPU oracle for the linearised eikonal solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code
 * with the GPU path (its own FFT, its own Bessel functions, its own kernel
 * table); the two meet only in the seeded input generators.
 *
 * What it computes (paper, Sections 3-5; algorithm of Table 1):
 *   ftilde  reference forcing: nu = sqrt((fmin^2 + fmax^2)/2)  (Section 5.1,
 *           eq. fTildeValue), or sup f (Section 5.1), or a given value
 *   beta    = ftilde*h/hbar,  gamma(x) = f(x)^2/ftilde^2 - 1
 *   kappa   normalised Green's kernel kappa(m) = ftilde^2 h^D G(h m)
 *           (eqs. GreensFunction2D/3D); kappa(0) is the average of
 *           ftilde^2 h^D G over the equal-volume ball around the origin
 *   phi_0   = sum_k exp(-beta |m - y_k|)           (eq. phi_0Solution, C = 1)
 *   phi_i   = kappa (*) (gamma phi_{i-1}), linear convolution over the grid
 *                                        (eqs. phiRecRelation, phi_i_Solution)
 *   phi     = sum_{i=0..T} (-1)^i phi_i               (eq. phiSolution)
 *   S       = -hbar ln phi   (+inf where phi <= 0 or not finite) (eq. SfromPhi)
 *
 * Arrays are C order (last index fastest), double precision, owned by the
 * caller.  Functions return 0 on success and a negative value on bad input.
 */
#ifndef EIKONAL_ORACLE_H
#define EIKONAL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FT_NU = 0, ORC_FT_FMAX = 1, ORC_FT_GIVEN = 2 };
enum { ORC_CONV_FFT = 0, ORC_CONV_DIRECT = 1 };

typedef struct {
  int32_t ndim;          /* 2 or 3 */
  int64_t dims[3];       /* grid points per axis */
  double h;              /* grid spacing */
  double hbar;
  int32_t T;             /* correction terms; phi has T+1 terms */
  int32_t ft_mode;       /* ORC_FT_* */
  double ftilde_given;   /* used when ft_mode == ORC_FT_GIVEN */
  int32_t conv;          /* ORC_CONV_FFT or ORC_CONV_DIRECT */
  int32_t nthreads;      /* OpenMP threads for FFT lines; <= 0: leave as is */
  const double *src_s;   /* nullable: S at the sources (default 0), n_src values */
} orc_problem;

/* info[0..7] = ftilde, beta, fmin, fmax, c0_bound = max|gamma|,
 *              count of phi <= 0, padded size of the FFT grid, 0 */

/* In-place complex FFT of length M (power of two), interleaved re/im.
 * inverse = 0: X[k] = sum_j x[j] exp(-2 pi i jk/M); inverse = 1: with the
 * opposite sign and a factor 1/M. */
int orc_fft(int64_t M, double *data, int inverse);

double orc_bessel_k0(double x);
double orc_bessel_k1(double x);

/* kappa(0) for the given dimension (cell average over the equal-volume ball) */
double orc_kappa0(int ndim, double beta);

/* kappa on the orthant: kappa[m0][m1][(m2)] for 0 <= m_d < dims[d]. */
int orc_kappa(int ndim, const int64_t *dims, double beta, double *kappa);

/* Real spectrum of the padded, evenly extended kernel on the unique orthant
 * [0..M0/2] x [0..M1/2] (x [0..M2/2]), M_d = next power of two >= 2 n_d - 1.
 * Returns the number of entries written or < 0. */
int64_t orc_ghat(int ndim, const int64_t *dims, double beta, double *ghat);

/* phi_0 on the grid. */
int orc_phi0(int ndim, const int64_t *dims, double beta, int32_t n_src,
             const int32_t *src, double *phi0);
/* phi_0 with a weight per source: sum_k w_k exp(-beta |m - y_k|); w_k =
 * exp(-s_k / hbar) gives sources with S(y_k) = s_k (w NULL: all 1). */
int orc_phi0_weighted(int ndim, const int64_t *dims, double beta, int32_t n_src,
                      const int32_t *src, const double *w, double *phi0);

/* out = kappa (*) in (linear convolution over the grid). */
int orc_conv(int ndim, const int64_t *dims, double beta, const double *in,
             double *out, int32_t method, int32_t nthreads);

/* Full solve.  S (N) required; phi (N) and terms ((T+1)*N) may be NULL. */
int orc_solve(const orc_problem *p, const double *f, int32_t n_src,
              const int32_t *src, double *S, double *phi, double *terms,
              double *info);

/* Adjoint of the solve with ftilde held fixed: given dL/dS (N) returns
 * dL/df (N).  Points with phi <= 0 contribute nothing. */
int orc_adjoint(const orc_problem *p, const double *f, int32_t n_src,
                const int32_t *src, const double *dLdS, double *dLdf,
                double *info);

/* Log-domain direct path: the same series for ftilde = sup f (ft_mode must
 * be ORC_FT_FMAX; every term is then non-negative), each term's O(N^2) sum
 * as a log-sum-exp: S = -hbar ln phi with full relative accuracy at any
 * distance.  logphi (N, nullable) receives ln phi.  info as orc_solve. */
int orc_solve_logdirect(const orc_problem *p, const double *f, int32_t n_src,
                        const int32_t *src, double *S, double *logphi,
                        double *info);
/* ln kappa on the orthant 0 <= m_d < n_d. */
int orc_log_kappa(int ndim, const int64_t *dims, double beta, double *out);

#ifdef __cplusplus
}
#endif
#endif
