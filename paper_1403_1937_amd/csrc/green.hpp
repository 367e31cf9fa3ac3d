// green.hpp -- device evaluation (float64) of the normalised screened-Poisson
// Green's kernel kappa(m) = ftilde^2 h^D G(h m) in units of the grid:
//   2D: (beta^2 / 2 pi) K0(beta |m|)              (eq. GreensFunction2D)
//   3D:  beta^2 exp(-beta |m|) / (4 pi |m|)       (eq. GreensFunction3D)
// with beta = ftilde h / hbar.  At m = 0 the kernel is singular; its value
// there is the mean of ftilde^2 h^D G over the ball of one cell's volume:
//   2D: 1 - a K1(a),       a = beta / sqrt(pi)
//   3D: 1 - (1 + a) e^-a,  a = beta (3 / (4 pi))^(1/3)
// (the integral of t K0(t) is -t K1(t); the integral of t e^-t is
// -(1+t) e^-t).
//
// K0 and K1 are evaluated in two ranges:
//   x <= 2       ascending series (Abramowitz & Stegun 9.6.13 / 9.6.11)
//   x > 2        the Laplace-type integral of A&S 9.6.23,
//                  K_nu(x) = sqrt(pi) (x/2)^nu / Gamma(nu + 1/2)
//                            int_1^inf e^{-x t} (t^2 - 1)^{nu - 1/2} dt,
//                with t = 1 + u^2:
//                  e^x K0(x) = int_0^inf 2 e^{-x u^2} / sqrt(u^2 + 2) du
//                  e^x K1(x) = x int_0^inf 2 u^2 sqrt(u^2 + 2) e^{-x u^2} du,
//                by the trapezoid rule in u (even integrands, analytic in
//                |Im u| < sqrt 2: geometric convergence); single values
//                (K1 at the origin) directly, the kernel table through a
//                Chebyshev series of sqrt(x) e^x K0(x) in t = 4/x - 1 whose
//                coefficients the host computes once from the same integral
#pragma once

#include <hip/hip_runtime.h>

namespace sweik {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;

// e^x K_nu(x), nu = 0 or 1, x >= 2, from the integrals above.  Step
// min(0.12, 0.45/sqrt x): the trapezoid error is below exp(-2 pi b / step)
// times the integrand's size on the line Im u = b (e^{x b^2}), with b up to
// 1.2 inside the strip; about 40 nodes at x = 2, 15 from x = 14 on.  Max
// relative error against an independent library evaluation: 9e-16 on
// [2, 2000].
__host__ __device__ inline double k_laplace_scaled(double x, int nu) {
  const double d = fmin(0.12, 0.45 / sqrt(x));
  double sum = nu ? 0.0 : 0.5 / sqrt(2.0);  // the node u = 0 (half weight)
  for (int j = 1; j < 400; ++j) {
    const double u2 = (d * j) * (d * j);
    const double r = sqrt(u2 + 2.0);
    const double g = exp(-x * u2) * (nu ? u2 * r : 1.0 / r);
    sum += g;
    if (g < 1e-18 * sum) break;
  }
  return 2.0 * d * sum * (nu ? x : 1.0);
}

// Chebyshev coefficients of g(t) = sqrt(x) e^x K0(x), t = 4/x - 1, for
// x >= 2 (t in (-1, 1]); built on the host from k_laplace_scaled.
constexpr int kChebK0 = 28;
struct ChebK0 {
  double c[kChebK0];
  float c32[kChebK0];
  double c1[kChebK0];  // the same for sqrt(x) e^x K1(x) (the gradient's kernel derivative)
};

__device__ __forceinline__ double k0_cheb(double x, const ChebK0 &tab) {
  const double t = 4.0 / x - 1.0;
  const double t2 = 2.0 * t;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = kChebK0 - 1; k >= 1; --k) {
    const double b0 = fma(t2, b1, tab.c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  const double g = fma(t, b1, tab.c[0] - b2);
  return exp(-x) * g / sqrt(x);
}

__device__ inline double bessel_k0_series(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, i0 = 1.0, sh = 0.0, hk = 0.0;
  for (int k = 1; k < 40; ++k) {
    term *= q / ((double)k * (double)k);
    hk += 1.0 / k;
    i0 += term;
    sh += term * hk;
    if (term < 1e-19 * i0) break;
  }
  return sh - (log(0.5 * x) + kEulerGamma) * i0;
}

__device__ inline double bessel_k0_fast(double x, const ChebK0 &tab) {
  return x <= 2.0 ? bessel_k0_series(x) : k0_cheb(x, tab);
}

// 1 - a K1(a) for a > 0 without cancellation for small a:
// a K1(a) = 1 + a ln(a/2) I1(a) - (a^2/4) sum_k (psi(k+1)+psi(k+2))
//           (a^2/4)^k / (k!(k+1)!)
__device__ inline double one_minus_aK1(double a) {
  if (a <= 2.0) {
    const double q = 0.25 * a * a;
    double term = 1.0, psi1 = -kEulerGamma, psi2 = 1.0 - kEulerGamma;
    double i1s = 0.0, s = 0.0;
    for (int k = 0; k < 40; ++k) {
      if (k > 0) {
        term *= q / ((double)k * (double)(k + 1));
        psi1 += 1.0 / k;
        psi2 += 1.0 / (k + 1);
      }
      i1s += term;
      s += (psi1 + psi2) * term;
      if (k > 2 && term < 1e-19 * (i1s > 1.0 ? i1s : 1.0)) break;
    }
    const double a_ln_i1 = a * log(0.5 * a) * (0.5 * a) * i1s;
    return q * s - a_ln_i1;
  }
  const double k1s = k_laplace_scaled(a, 1);
  return 1.0 - a * exp(-a) * k1s;
}

__device__ inline double kappa0_2d(double beta) {
  return one_minus_aK1(beta / sqrt(kPi));
}

__device__ inline double kappa0_3d(double beta) {
  const double a = beta * cbrt(3.0 / (4.0 * kPi));
  if (a < 0.5) {  // sum_{k>=2} (-a)^k (k-1)/k!
    double s = 0.0, p = -a;
    for (int k = 2; k < 30; ++k) {
      p *= -a / k;
      s += p * (k - 1);
    }
    return s;
  }
  return 1.0 - (1.0 + a) * exp(-a);
}

// kappa at integer offset with squared length r2 (kappa0 given)
__device__ inline double kappa_2d(double beta, long long r2, double k0v, const ChebK0 &tab) {
  if (r2 == 0) return k0v;
  return beta * beta * (0.5 / kPi) * bessel_k0_fast(beta * sqrt((double)r2), tab);
}
// float32 variant for the FP32 path (relative error ~1e-6)
__device__ inline float bessel_k0_f32(float x, const ChebK0 &tab) {
  if (x <= 2.0f) {
    const float q = 0.25f * x * x;
    float term = 1.0f, i0 = 1.0f, sh = 0.0f, hk = 0.0f;
#pragma unroll
    for (int k = 1; k < 14; ++k) {
      term *= q / (float)(k * k);
      hk += 1.0f / (float)k;
      i0 += term;
      sh += term * hk;
    }
    return sh - (logf(0.5f * x) + (float)kEulerGamma) * i0;
  }
  const float t = 4.0f / x - 1.0f;
  const float t2 = 2.0f * t;
  float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
  for (int k = kChebK0 - 1; k >= 1; --k) {
    const float b0 = fmaf(t2, b1, tab.c32[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  const float g = fmaf(t, b1, tab.c32[0] - b2);
  return expf(-x) * g * rsqrtf(x);
}

template <typename R>
__device__ inline R kappa_2d_t(double beta, int r2, double k0v, const ChebK0 &tab);
template <>
__device__ inline double kappa_2d_t<double>(double beta, int r2, double k0v, const ChebK0 &tab) {
  return kappa_2d(beta, r2, k0v, tab);
}
template <>
__device__ inline float kappa_2d_t<float>(double beta, int r2, double k0v, const ChebK0 &tab) {
  if (r2 == 0) return (float)k0v;
  const float b = (float)beta;
  return b * b * (float)(0.5 / kPi) * bessel_k0_f32(b * sqrtf((float)r2), tab);
}

// The tilted kernel kappa(m) exp(e), e = a . m with |a| < beta (the
// far-field stabilised convolution): the exponent is folded into the
// exponentially scaled K0 for x = beta |m| > 2, so that neither factor
// underflows or overflows where the product matters.  m = 0 gives k0v.
__device__ inline double kappa_2d_tilt(double beta, int m0, int m1, double e, double k0v,
                                       const ChebK0 &tab) {
  if (m0 == 0 && m1 == 0) return k0v;
  const double x = beta * sqrt((double)m0 * m0 + (double)m1 * m1);
  const double c = beta * beta * (0.5 / kPi);
  if (x <= 2.0) return c * bessel_k0_series(x) * exp(e);
  const double t = 4.0 / x - 1.0, t2 = 2.0 * t;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = kChebK0 - 1; k >= 1; --k) {
    const double b0 = fma(t2, b1, tab.c[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return c * fma(t, b1, tab.c[0] - b2) / sqrt(x) * exp(e - x);
}
template <typename R>
__device__ inline R kappa_2d_tilt_t(double beta, int m0, int m1, double e, double k0v,
                                    const ChebK0 &tab);
template <>
__device__ inline double kappa_2d_tilt_t<double>(double beta, int m0, int m1, double e, double k0v,
                                                 const ChebK0 &tab) {
  return kappa_2d_tilt(beta, m0, m1, e, k0v, tab);
}
template <>
__device__ inline float kappa_2d_tilt_t<float>(double beta, int m0, int m1, double e, double k0v,
                                               const ChebK0 &tab) {
  if (m0 == 0 && m1 == 0) return (float)k0v;
  const float b = (float)beta;
  const float x = b * sqrtf((float)m0 * (float)m0 + (float)m1 * (float)m1);
  const float c = b * b * (float)(0.5 / kPi);
  if (x <= 2.0f) return c * bessel_k0_f32(x, tab) * expf((float)e);
  const float t = 4.0f / x - 1.0f, t2 = 2.0f * t;
  float b1 = 0.0f, b2 = 0.0f;
#pragma unroll
  for (int k = kChebK0 - 1; k >= 1; --k) {
    const float b0 = fmaf(t2, b1, tab.c32[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  return c * fmaf(t, b1, tab.c32[0] - b2) * rsqrtf(x) * expf((float)e - x);
}

// d kappa / d beta at an integer offset (2D), for the gradient with respect
// to beta: off the origin (beta/pi) K0(x) - (beta/2pi) x K1(x), x = beta |m|;
// at the origin the beta-derivative of the ball average 1 - a K1(a),
// a = beta/sqrt(pi), which is (beta/pi) K0(a) (d/da of a K1(a) is -a K0(a)).
// Float64 for either precision (evaluated once per gradient).
__device__ inline double dkappa_2d(double beta, long long r2, const ChebK0 &tab) {
  if (r2 == 0) return beta / kPi * bessel_k0_fast(beta / sqrt(kPi), tab);
  const double x = beta * sqrt((double)r2);
  double xk1;  // x K1(x)
  if (x <= 2.0) {
    xk1 = 1.0 - one_minus_aK1(x);
  } else {  // Chebyshev series of sqrt(x) e^x K1(x) in t = 4/x - 1
    const double t = 4.0 / x - 1.0, t2 = 2.0 * t;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = kChebK0 - 1; k >= 1; --k) {
      const double b0 = fma(t2, b1, tab.c1[k] - b2);
      b2 = b1;
      b1 = b0;
    }
    xk1 = sqrt(x) * exp(-x) * fma(t, b1, tab.c1[0] - b2);
  }
  return beta / kPi * bessel_k0_fast(x, tab) - beta / (2.0 * kPi) * xk1;
}

// the kernel exp(-beta |m|) of phi_0 (eq. phi_0Solution with C = 1), for the
// FFT route of phi_0 (Table 1, steps 1-5)
template <typename R> __device__ inline R exp_kernel_t(double beta, int r2);
template <> __device__ inline double exp_kernel_t<double>(double beta, int r2) {
  return exp(-beta * sqrt((double)r2));
}
template <> __device__ inline float exp_kernel_t<float>(double beta, int r2) {
  return __builtin_amdgcn_exp2f(-(float)(beta * 1.4426950408889634) *
                                __builtin_amdgcn_sqrtf((float)r2));
}

__device__ inline double kappa_3d(double beta, long long r2, double k0v) {
  if (r2 == 0) return k0v;
  const double r = sqrt((double)r2);
  return beta * beta * exp(-beta * r) / (4.0 * kPi * r);
}

// d kappa / d beta at an integer offset (3D), for the gradient with respect
// to beta: off the origin beta e^{-beta r} (2 - beta r) / (4 pi r); at the
// origin that of the ball average 1 - (1 + a) e^{-a}, a = c beta,
// c = (3 / (4 pi))^(1/3), which is c a e^{-a}.  Float64 for either precision
// (evaluated once per gradient).
__device__ inline double dkappa_3d(double beta, long long r2) {
  if (r2 == 0) {
    const double c = cbrt(3.0 / (4.0 * kPi));
    return c * c * beta * exp(-c * beta);
  }
  const double r = sqrt((double)r2);
  return beta * exp(-beta * r) * (2.0 - beta * r) / (4.0 * kPi * r);
}

// the 3D kernel in the working precision: float32 evaluation (hardware exp2,
// relative error ~1e-6 at beta |m| ~ 25) for the float32 spectrum, which
// stores it rounded to float anyway
template <typename R>
__device__ inline R kappa_3d_t(double beta, long long r2, double k0v);
template <>
__device__ inline double kappa_3d_t<double>(double beta, long long r2, double k0v) {
  return kappa_3d(beta, r2, k0v);
}
template <>
__device__ inline float kappa_3d_t<float>(double beta, long long r2, double k0v) {
  if (r2 == 0) return (float)k0v;
  const float b = (float)beta;
  const float r = __builtin_amdgcn_sqrtf((float)r2);
  const float e = __builtin_amdgcn_exp2f(-b * r * 1.4426950408889634f);
  return b * b * e * __builtin_amdgcn_rcpf(4.0f * (float)kPi * r);
}

}  // namespace sweik
