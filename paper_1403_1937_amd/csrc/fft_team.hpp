// fft_team.hpp -- register/LDS Stockham FFT for gfx950 (wave64).
//
// A "team" of P = L/16 threads transforms one complex line of length L
// (power of two, 16 <= L <= 8192).  Thread t of the team always holds the
// 16 elements with indices t + P*j, j = 0..15, in registers: on entry these
// are the input samples, on exit the transform values at the same indices.
// Stages are Stockham autosort radix-16 steps (the last one radix 2, 4, 8 or
// 16); the data moves through LDS only between stages, so a line of length
// L costs ceil(log16 L) - 1 LDS round trips.  Because the first stage reads
// and the last stage writes the same index pattern, a forward transform, a
// pointwise spectral product and an inverse transform chain without any
// extra exchange.
//
// Twiddles come from a table tw[j] = exp(-2 pi i j / Lmax), j < Lmax, built
// once per solve in double precision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sweik {

template <typename R> struct cplx_t;
template <> struct cplx_t<float> { using type = float2; };
template <> struct cplx_t<double> { using type = double2; };
template <typename R> using cplx = typename cplx_t<R>::type;

template <typename C> __device__ __forceinline__ C cmake(decltype(C::x) a, decltype(C::x) b) {
  C c;
  c.x = a;
  c.y = b;
  return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmake<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmake<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return cmake<C>(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmake<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, decltype(C::x) s) { return cmake<C>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C cmul_mi(C a) {
  return INV ? cmake<C>(-a.y, a.x) : cmake<C>(a.y, -a.x);
}

// cos and sin of 2 pi m / 16, m = 0..15
__device__ constexpr double kCos16[16] = {
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173,
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
__device__ constexpr double kSin16[16] = {
    0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613,
    1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173,
    0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613,
    -1.0, -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};

// v *= exp(-+ 2 pi i m / R) with compile-time R, m  (sign: - forward, + inverse)
template <int R, int M, bool INV, typename C> __device__ __forceinline__ C twc(C v) {
  using T = decltype(C::x);
  constexpr int m16 = (M * (16 / R)) & 15;
  if constexpr (m16 == 0) {
    return v;
  } else if constexpr (m16 == 4) {
    return cmul_mi<INV>(v);
  } else if constexpr (m16 == 8) {
    return cmake<C>(-v.x, -v.y);
  } else if constexpr (m16 == 12) {
    return cmul_mi<!INV>(v);
  } else {
    const T c = (T)kCos16[m16];
    const T s = INV ? (T)kSin16[m16] : -(T)kSin16[m16];
    return cmake<C>(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// In-register DFT of length R in natural order: u[q] <- sum_r u[r] w^{rq}.
template <int R, bool INV, typename C> struct Dft;

template <bool INV, typename C> struct Dft<1, INV, C> {
  __device__ __forceinline__ static void run(C *) {}
};
template <bool INV, typename C> struct Dft<2, INV, C> {
  __device__ __forceinline__ static void run(C *u) {
    C a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  }
};
template <bool INV, typename C> struct Dft<4, INV, C> {
  __device__ __forceinline__ static void run(C *u) {
    C s02 = cadd(u[0], u[2]), d02 = csub(u[0], u[2]);
    C s13 = cadd(u[1], u[3]), d13 = cmul_mi<INV>(csub(u[1], u[3]));
    u[0] = cadd(s02, s13);
    u[2] = csub(s02, s13);
    u[1] = cadd(d02, d13);
    u[3] = csub(d02, d13);
  }
};

// R = 4 B: index n = B n1 + n2, frequency k = k1 + 4 k2.
template <int R, bool INV, typename C> struct Dft {
  static constexpr int B = R / 4;
  template <int N2, int K1> __device__ __forceinline__ static void tw(C (&y)[R]) {
    y[N2 * 4 + K1] = twc<R, N2 * K1, INV>(y[N2 * 4 + K1]);
    if constexpr (K1 + 1 < 4) tw<N2, K1 + 1>(y);
    else if constexpr (N2 + 1 < B) tw<N2 + 1, 0>(y);
  }
  __device__ __forceinline__ static void run(C *u) {
    C y[R];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      C t[4] = {u[n2], u[B + n2], u[2 * B + n2], u[3 * B + n2]};
      Dft<4, INV, C>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) y[n2 * 4 + k1] = t[k1];
    }
    tw<0, 0>(y);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      C s[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) s[n2] = y[n2 * 4 + k1];
      Dft<B, INV, C>::run(s);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) u[k1 + 4 * k2] = s[k2];
    }
  }
};

// LDS index with one pad slot every 16 elements (breaks the stride-16
// pattern of the first Stockham stage).
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_line_len(int L) { return L + (L >> 4) + 1; }

// One Stockham stage of radix R on a team line.  p = product of earlier
// radices; LAST: results stay in registers (index t + P j), else they go to
// LDS at the autosort position.
template <int R, bool INV, bool LAST, typename C>
__device__ __forceinline__ void stage(C (&v)[16], int t, int P, int p, int L,
                                      C *lds, const C *__restrict__ tw,
                                      int lmax_log) {
  constexpr int NB = 16 / R;  // butterflies per thread
  const int logpr = 31 - __clz(p * R);
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int i = t + P * b;
    const int k = i & (p - 1);
    C u[R];
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = v[b + q * NB];
    if (p > 1) {
      const int sh = lmax_log - logpr;
#pragma unroll
      for (int q = 1; q < R; ++q) {
        C w = tw[(q * k) << sh];
        u[q] = INV ? cmulc(u[q], w) : cmul(u[q], w);
      }
    }
    Dft<R, INV, C>::run(u);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[b + q * NB] = u[q];
    } else {
      const int base = (i - k) * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) lds[lpad(base + q * p)] = u[q];
    }
  }
}

// Complex FFT of length L (16 <= L, power of two) held by a team.
// lds: the team's private LDS line (lds_line_len(L) elements).
// Barriers are block-wide: every thread of the block must call this with the
// same L.  The caller guarantees that no thread still reads `lds` from
// earlier work (a leading barrier is taken when lead_sync is set).
template <bool INV, typename C>
__device__ void team_fft(C (&v)[16], int t, int P, int L, C *lds,
                         const C *__restrict__ tw, int lmax_log,
                         bool lead_sync = true) {
  if (lead_sync) __syncthreads();
  int p = 1;
  while (true) {
    const int r = (L / p) >= 16 ? 16 : (L / p);
    const bool last = (p * r == L);
    if (last) {
      switch (r) {
        case 16: stage<16, INV, true>(v, t, P, p, L, lds, tw, lmax_log); break;
        case 8: stage<8, INV, true>(v, t, P, p, L, lds, tw, lmax_log); break;
        case 4: stage<4, INV, true>(v, t, P, p, L, lds, tw, lmax_log); break;
        default: stage<2, INV, true>(v, t, P, p, L, lds, tw, lmax_log); break;
      }
      return;
    }
    // r == 16 here
    stage<16, INV, false>(v, t, P, p, L, lds, tw, lmax_log);
    p *= 16;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = lds[lpad(t + P * j)];
    __syncthreads();
  }
}

// ---- block reductions ----------------------------------------------------

template <typename T> __device__ __forceinline__ T wave_max(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = y > x ? y : x;
  }
  return x;
}
template <typename T> __device__ __forceinline__ T wave_min(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    T y = __shfl_xor(x, o, 64);
    x = y < x ? y : x;
  }
  return x;
}
template <typename T> __device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ int wave_or(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
  return x;
}

}  // namespace sweik
