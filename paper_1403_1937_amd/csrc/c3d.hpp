// c3d.hpp -- passes along axes 1 and 0 of the 3D solve.
//
// A work-group owns CPW neighbouring k2 columns of one plane; a team of
// P = M/16 threads transforms one column of length M (the padded length of
// the axis).  Threads are ordered column-fastest, so one wave reads or writes
// CPW contiguous spectrum entries of a row per access.
//   C3_YF  plane i0: FFT along axis 1 of the n1 rows of s1 -> M1 rows of s2
//   C3_Z   plane k1: FFT along axis 0 of the n0 rows of s2, product with the
//          kernel spectrum g[min(k1, M1-k1)][min(k0, M0-k0)][k2], inverse
//          FFT, first n0 rows back into s2
//   C3_YI  plane i0: inverse FFT along axis 1 of the M1 rows of s2 -> first
//          n1 rows of s1o (s1, or a second spectrum of the full gradient)
//   C3_GY  kernel spectrum, plane d0: even extension along axis 1 of the
//          kernel table's line transforms, FFT, real part of k1 <= H1 -> s2
//   C3_GZ  kernel spectrum, plane k1 <= H1: even extension along axis 0,
//          FFT, real part of k0 <= H0, pre-scaled -> g
// The first group of a C3_YF launch also reduces the x pass's partial
// maxima of term `term` (the exponent step of the next term).
#pragma once

#include "common3d.hpp"

namespace sweik {

// C3_Z: planes k1 and M1 - k1 read the same kernel spectrum columns, so they
// are visited one after the other (0, H1, 1, M1 - 1, 2, M1 - 2, ...): the
// second read of a column block then hits in L2 instead of fetching the
// kernel spectrum twice from memory.
__device__ __forceinline__ int z_plane(int p, int M1) {
  if (p < 2) return p * (M1 / 2);
  const int i = (p - 2) / 2 + 1;
  return (p & 1) ? M1 - i : i;
}

// FULL: the loaded axis is exactly half the padded length (no bounds checks).
template <typename R, int MODE, int M, bool FULL>
__device__ __forceinline__ void c3_pass(const Args3<R> &a, int term, unsigned char *smem_raw,
                                        const int g) {
  using C = cplx<R>;
  constexpr int P = M / 16, CPW = c3_cpw<R>(M), NT = c3_threads<R>(M), LL = lds_line_len(M);
  constexpr int HM = M / 2;
  C *twl = reinterpret_cast<C *>(smem_raw);  // stage twiddle tables
  C *lines = twl + stage_tw_len(M, 16);

  const int tid = threadIdx.x, c = tid % CPW, t = tid / CPW;
  const int ncb = a.H2 / CPW;  // H2 is a multiple of CPW
  const int pg = g / ncb, k2 = (g - pg * ncb) * CPW + c;
  const int plane = MODE == C3_Z ? z_plane(pg, a.M1) : pg;
  C *line = lines + c * LL;
  const size_t H2 = (size_t)a.H2;

  if (MODE == C3_YF && term >= 0 && g == 0) {
    double mx = 0.0;
    for (int i = tid; i < a.nbx; i += NT) mx = fmax(mx, a.mu[(size_t)term * a.nbx + i]);
    mx = block_max(mx);
    if (tid == 0) a.mu_red[term] = mx;
  }

  // ---- issue the global reads -------------------------------------------------
  constexpr int NSR = (stage_tw_len(M, 16) + NT - 1) / NT;
  C twr[NSR > 0 ? NSR : 1];
  stage_tw_issue<M, 16>(twr, a.tw, a.lmax_log, tid, NT);
  C v[16];
  R gv[16];
  if constexpr (MODE == C3_YF) {
    const C *in = a.s1 + (size_t)plane * a.n1 * H2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int p = t + P * j;
      v[j] = (j < 8 && (FULL || p < a.n1)) ? in[(size_t)p * H2] : cmake<C>((R)0, (R)0);
    }
  } else if constexpr (MODE == C3_Z) {
    C *io = a.s2 + (size_t)plane * H2 + k2;
    const size_t st = (size_t)a.ld2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int p = t + P * j;
      v[j] = (j < 8 && (FULL || p < a.n0)) ? io[(size_t)p * st] : cmake<C>((R)0, (R)0);
    }
    const int k1 = plane <= a.H1 ? plane : a.M1 - plane;
    const R *gc = a.g + (size_t)k1 * (HM + 1) * H2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k0 = t + P * j;
      gv[j] = gc[(size_t)(k0 <= HM ? k0 : M - k0) * H2];
    }
  } else if constexpr (MODE == C3_YI) {
    const C *in = a.s2 + (size_t)plane * a.ld2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = in[(size_t)(t + P * j) * H2];
  } else if constexpr (MODE == C3_GY) {
    const C *in = a.s1 + (size_t)plane * a.n1 * H2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int p = t + P * j, s = p <= HM ? p : M - p;
      v[j] = s < a.n1 ? in[(size_t)s * H2] : cmake<C>((R)0, (R)0);
    }
  } else {  // C3_GZ
    const C *in = a.s2 + (size_t)plane * H2 + k2;
    const size_t st = (size_t)a.ld2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int p = t + P * j, s = p <= HM ? p : M - p;
      v[j] = s < a.n0 ? in[(size_t)s * st] : cmake<C>((R)0, (R)0);
    }
  }
  stage_tw_store<M, 16>(twr, twl, tid, NT);
  __syncthreads();

  // ---- transforms and stores ----------------------------------------------------
  if constexpr (MODE == C3_YI) {
    team_fft<M, true>(v, t, line, twl, false);
  } else {
    team_fft<M, false>(v, t, line, twl, false);
  }
  if constexpr (MODE == C3_YF) {
    C *out = a.s2 + (size_t)plane * a.ld2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) out[(size_t)(t + P * j) * H2] = v[j];
  } else if constexpr (MODE == C3_Z) {
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = cscale(v[j], gv[j]);
    team_fft<M, true>(v, t, line, twl, true);
    C *io = a.s2 + (size_t)plane * H2 + k2;
    const size_t st = (size_t)a.ld2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = t + P * j;
      if (FULL || p < a.n0) io[(size_t)p * st] = v[j];
    }
  } else if constexpr (MODE == C3_YI) {
    C *out = a.s1o + (size_t)plane * a.n1 * H2 + k2;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int p = t + P * j;
      if (FULL || p < a.n1) out[(size_t)p * H2] = v[j];
    }
  } else if constexpr (MODE == C3_GY) {
    C *out = a.s2 + (size_t)plane * a.ld2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k = t + P * j;
      if (k <= HM) out[(size_t)k * H2] = cmake<C>(v[j].x, (R)0);
    }
  } else {  // C3_GZ
    // the axis-2 transform returns twice the DFT; the round trips of the
    // three axes contribute 2 M2, M1 and M0
    const double sc = 1.0 / (4.0 * (double)a.M0 * (double)a.M1 * (double)a.M2);
    R *out = a.g + (size_t)plane * (HM + 1) * H2 + k2;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k0 = t + P * j;
      if (k0 <= HM) out[(size_t)k0 * H2] = (R)((double)v[j].x * sc);
    }
  }
}

template <typename R, int MODE, int M>
__global__ void __launch_bounds__(512) k_c3(Args3<R> a, int term) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = xcd_tile(blockIdx.x, gridDim.x);
  const int n = (MODE == C3_Z || MODE == C3_GZ) ? a.n0 : a.n1;
  if (2 * n == M)
    c3_pass<R, MODE, M, true>(a, term, smem_raw, g);
  else
    c3_pass<R, MODE, M, false>(a, term, smem_raw, g);
}

}  // namespace sweik
