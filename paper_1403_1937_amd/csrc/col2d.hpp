// col2d.hpp -- column passes of the 2D solve.
//
// One team of P = M0/16 threads per spectral column k1, CPW columns per
// work-group.  Lanes interleave the teams in groups of RB so that one wave
// reads RB contiguous rows of CPW neighbouring columns from each block of
// the blocked spectrum; work-groups are mapped so that neighbouring columns
// run on the same XCD (they share cache lines).
//   COL_CONV  forward FFT of the zero-padded column, product with the real
//             kernel spectrum Ghat[k0][k1], inverse FFT, keep the first rows
//   COL_GHAT  even extension of the column of the kernel table's row
//             transforms, forward FFT, keep the real part: Ghat
#pragma once

#include "common2d.hpp"

namespace sweik {

template <typename R, int MODE, int M0>
__global__ void __launch_bounds__(kThreads) k_col2(Args2<R> a) {
  using C = cplx<R>;
  constexpr int P = M0 / 16, CPW = col_cpw(M0), RB = spec_rb<R>(), LL = lds_line_len(M0);
  constexpr int H0 = M0 / 2, TWLOG = ilog2c(M0);
  constexpr int NTW = (H0 + kThreads - 1) / kThreads;
  static_assert(P % RB == 0, "column team must cover whole row blocks");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  C *twl = reinterpret_cast<C *>(smem_raw);  // exp(-2 pi i k / M0), k < M0/2
  C *lines = twl + H0;

  const int tid = threadIdx.x;
  const int grp = tid / RB, rr = tid - grp * RB;
  const int team = grp % CPW;
  const int t = (grp / CPW) * RB + rr;
  const int k1 = xcd_tile(blockIdx.x, gridDim.x) * CPW + team;
  const bool active = k1 < a.ldk;
  C *line = lines + team * LL;
  const int spec_rows = a.nb * RB;
  const size_t cstride = (size_t)a.ldk * RB;  // elements between blocks
  C *col = a.spec + (size_t)(active ? k1 : 0) * RB;

  // ---- issue the global reads -----------------------------------------------
  C twr[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int k = tid + u * kThreads;
    if (k < H0) twr[u] = a.tw[k << (a.lmax_log - TWLOG)];
  }
  C v[16];
  R gv[16];
  if constexpr (MODE == COL_CONV) {
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int rho = t + P * j;
      C x = cmake<C>((R)0, (R)0);
      if (j < 8 && active && rho < spec_rows) {
        const int b = rho / RB;
        x = col[b * cstride + (rho - b * RB)];
      }
      v[j] = x;
    }
    const R *gcol = a.g + (size_t)(active ? k1 : 0) * a.ldg;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int k0 = t + P * j;
      gv[j] = gcol[k0 <= H0 ? k0 : M0 - k0];
    }
  } else {
    // even extension of the column: x[rho] = x[M0 - rho]
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const int rho = t + P * j;
      const int sr = rho <= H0 ? rho : M0 - rho;
      C x = cmake<C>((R)0, (R)0);
      if (active && sr < spec_rows) {
        const int b = sr / RB;
        x = col[b * cstride + (sr - b * RB)];
      }
      v[j] = x;
    }
  }
#pragma unroll
  for (int u = 0; u < NTW; ++u) {
    const int k = tid + u * kThreads;
    if (k < H0) twl[k] = twr[u];
  }
  __syncthreads();

  team_fft<M0, TWLOG, false>(v, t, line, twl, false);
  if constexpr (MODE == COL_CONV) {
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = cscale(v[j], gv[j]);
    team_fft<M0, TWLOG, true>(v, t, line, twl, true);
    if (active) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int rho = t + P * j;
        if (rho < spec_rows) {
          const int b = rho / RB;
          col[b * cstride + (rho - b * RB)] = v[j];
        }
      }
    }
  } else {
    if (active) {
      // the row step's split transform is twice the DFT; the column and row
      // round trips contribute M0 and 2 M1: store Ghat / (2 M0 M1)
      const double sc = 1.0 / (4.0 * (double)M0 * (double)(2 * a.H1));
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
