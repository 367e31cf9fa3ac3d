// col2d.hpp -- column passes of the 2D solve.
//
// One team of P = M0/E threads per spectral column k1 (E = 16 or 8 elements
// per thread; 4096/E threads per work-group), CPW = 4096/M0 columns per
// work-group; an 8192-point column takes a work-group of its own.  Lanes interleave the teams in groups of RB so that one wave
// reads RB contiguous rows of CPW neighbouring columns from each block of
// the blocked spectrum; work-groups are mapped so that neighbouring columns
// run on the same XCD (they share cache lines).
//   COL_CONV  forward FFT of the zero-padded column, product with the real
//             kernel spectrum Ghat[k0][k1], inverse FFT, keep the first rows
//   COL_GHAT  even extension of the column of the kernel table's row
//             transforms, forward FFT, keep the real part: Ghat
//   COL_GHATC the tilted kernel's column (rows m0 >= 0 and m0 < 0 from two
//             row-transform tables), forward FFT: its complex spectrum, all
//             M0 frequencies (the tilted kernel is not even)
//   COL_CONVC COL_CONV with that complex kernel spectrum
// Column k1 = 0 holds two real sequences, the DC (re) and Nyquist (im) bins
// of the rows.  Their transforms A, B are Hermitian, so the product with
// their own kernel columns is Y = (Ga + Gb)/2 F + (Ga - Gb)/2 conj F(-k)
// with F = A + iB; the partner value F(-k) comes through LDS.  In the GHAT
// mode A and B are real: Ghat[.][0] = Re F, Ghat[.][H1] = Im F.
#pragma once

#include "common2d.hpp"

namespace sweik {

// FULL: every column of the work-group exists and every loaded row lies in
// the spectrum, so no element needs a bounds check.
template <typename R, int MODE, int M0, int E, bool FULL>
__device__ __forceinline__ void col_pass(const Args2<R> &a, int tile, unsigned char *smem_raw) {
  using C = cplx<R>;
  constexpr int P = M0 / E, CPW = col_cpw(M0), RB = spec_rb<R>(), LL = col_line_len<R>(M0);
  constexpr int NT = col_threads(M0, E);
  constexpr int H0 = M0 / 2;
  constexpr bool CONV = MODE == COL_CONV || MODE == COL_CONVC;
  constexpr bool CPLX = MODE == COL_CONVC;  // complex (tilted) kernel spectrum
  static_assert(P % RB == 0, "column team must cover whole row blocks");
  C *twl = reinterpret_cast<C *>(smem_raw);  // stage twiddle tables
  C *lines = twl + col_stage_tw<R>(M0);

  const int tid = threadIdx.x;
  const int grp = tid / RB, rr = tid - grp * RB;
  const int team = grp % CPW;
  const int t = (grp / CPW) * RB + rr;
  const int k1 = tile * CPW + team;
  const bool packed_wg = tile == 0;  // holds column 0 (uniform per work-group)
  const bool active = FULL || k1 < a.ldk;
  C *line = lines + team * LL;
  const int spec_rows = a.nb * RB;
  const size_t cstride = (size_t)a.ldk * RB;  // elements between blocks
  C *col = a.spec + (size_t)(active ? k1 : 0) * RB;
  auto at = [&](const C *base, int rho) -> C {  // row rho of this column
    const int b = rho / RB;
    return base[b * cstride + (rho - b * RB)];
  };

  // ---- issue the global reads -----------------------------------------------
  constexpr int NSR = (stage_tw_len(M0, E) + NT - 1) / NT;
  C twr[NSR > 0 ? NSR : 1];
  stage_tw_issue<M0, E>(twr, a.tw, a.lmax_log, tid, NT);
  C v[E];
  R gv[CPLX ? 1 : E], gb[CPLX ? 1 : E];
  C gvc[CPLX ? E : 1], gbc[CPLX ? E : 1];
  if constexpr (CONV) {
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int rho = t + P * j;
      C x = cmake<C>((R)0, (R)0);
      if (j < E / 2 && (FULL || (active && rho < spec_rows))) x = at(col, rho);
      v[j] = x;
    }
    if constexpr (CPLX) {
      // the tilted kernel is not even: all M0 frequencies of the column
      const C *gcol = a.gc + (size_t)(active ? k1 : 0) * M0;
#pragma unroll
      for (int j = 0; j < E; ++j) gvc[j] = gcol[t + P * j];
      if (packed_wg && k1 == 0) {
        const C *gnyq = a.gc + (size_t)a.ldk * M0;  // kernel column of bin H1
#pragma unroll
        for (int j = 0; j < E; ++j) gbc[j] = gnyq[t + P * j];
      }
    } else {
      const R *gcol = a.g + (size_t)(active ? k1 : 0) * a.ldg;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k0 = t + P * j;
        gv[j] = gcol[k0 <= H0 ? k0 : M0 - k0];
      }
      if (packed_wg && k1 == 0) {
        const R *gnyq = a.g + (size_t)a.ldk * a.ldg;  // kernel column of bin H1
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int k0 = t + P * j;
          gb[j] = gnyq[k0 <= H0 ? k0 : M0 - k0];
        }
      }
    }
  } else if constexpr (MODE == COL_GHATC) {
    // the tilted kernel's column: rows m0 = rho >= 0 from the row transforms
    // of the table rows m0 >= 0, rows m0 = rho - M0 < 0 from those of the
    // rows m0 <= 0 (row -m0 of spec_neg), zero in between
    const C *cneg = a.spec_neg + (size_t)(active ? k1 : 0) * RB;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int rho = t + P * j;
      C x = cmake<C>((R)0, (R)0);
      if (active) {
        if (rho < a.n0) x = at(col, rho);
        else if (M0 - rho < a.n0) x = at(cneg, M0 - rho);
      }
      v[j] = x;
    }
  } else {
    // even extension of the column: x[rho] = x[M0 - rho]
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const int rho = t + P * j;
      const int sr = rho <= H0 ? rho : M0 - rho;
      C x = cmake<C>((R)0, (R)0);
      if (active && sr < spec_rows) x = at(col, sr);
      v[j] = x;
    }
  }
  stage_tw_store<M0, E>(twr, twl, tid, NT);
  __syncthreads();

  team_fft<M0, false>(v, t, line, twl, false);
  // Column 0 holds two real sequences, A (the rows' DC bins) and B (their
  // Nyquist bins): with F = A^ + i B^ their transforms are A^ = (F(k) +
  // conj F(-k)) / 2 and B^ = (F(k) - conj F(-k)) / 2i.  The partner values
  // F(-k) come through LDS (every team of the work-group takes part); the
  // partner array lives only in the work-group holding column 0, which keeps
  // the registers of the other work-groups' path at their minimum.
  auto partner = [&](C (&pv)[E]) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) line[lpad(t + P * j)] = v[j];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < E; ++j) pv[j] = line[lpad((M0 - (t + P * j)) & (M0 - 1))];
  };
  if constexpr (CONV) {
    if (packed_wg) {
      C pv[E];
      partner(pv);
      if (k1 == 0) {
        // Y = A^ Ga + i B^ Gb = F (Ga + Gb) / 2 + conj F(-k) (Ga - Gb) / 2
#pragma unroll
        for (int j = 0; j < E; ++j) {
          if constexpr (CPLX) {
            const C al = cscale(cadd(gvc[j], gbc[j]), (R)0.5), de = cscale(csub(gvc[j], gbc[j]), (R)0.5);
            v[j] = cadd(cmul(v[j], al), cmul(cconj(pv[j]), de));
          } else {
            const R al = (gv[j] + gb[j]) * (R)0.5, de = (gv[j] - gb[j]) * (R)0.5;
            v[j] = cadd(cscale(v[j], al), cscale(cconj(pv[j]), de));
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < E; ++j) {
          if constexpr (CPLX) v[j] = cmul(v[j], gvc[j]);
          else v[j] = cscale(v[j], gv[j]);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if constexpr (CPLX) v[j] = cmul(v[j], gvc[j]);
        else v[j] = cscale(v[j], gv[j]);
      }
    }
    team_fft<M0, true>(v, t, line, twl, true);
    if (active) {
#pragma unroll
      for (int j = 0; j < E / 2; ++j) {
        const int rho = t + P * j;
        if (FULL || rho < spec_rows) {
          const int b = rho / RB;
          col[b * cstride + (rho - b * RB)] = v[j];
        }
      }
    }
  } else if constexpr (MODE == COL_GHATC) {
    C pv[E];
    if (packed_wg) partner(pv);
    if (active) {
      // scaled as Ghat below; all M0 frequencies, complex
      const R sc = (R)(1.0 / (4.0 * (double)M0 * (double)(2 * a.H1)));
      C *gcol = a.gc + (size_t)k1 * M0;
      C *gnyq = a.gc + (size_t)a.ldk * M0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k0 = t + P * j;
        if (k1 == 0) {
          const C fa = cscale(cadd(v[j], cconj(pv[j])), (R)0.5);   // A^
          const C d = csub(v[j], cconj(pv[j]));
          const C fb = cmake<C>(d.y * (R)0.5, -d.x * (R)0.5);    // B^ = d / 2i
          gcol[k0] = cscale(fa, sc);
          gnyq[k0] = cscale(fb, sc);
        } else {
          gcol[k0] = cscale(v[j], sc);
        }
      }
    }
  } else {
    if (active) {
      // the row step's split transform is twice the DFT; the column and row
      // round trips contribute M0 and 2 M1: store Ghat / (2 M0 M1)
      const double sc = 1.0 / (4.0 * (double)M0 * (double)(2 * a.H1));
      R *gcol = a.g + (size_t)k1 * a.ldg;
      R *gnyq = a.g + (size_t)a.ldk * a.ldg;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int k0 = t + P * j;
        if (k0 <= H0) {
          gcol[k0] = (R)((double)v[j].x * sc);
          if (k1 == 0) gnyq[k0] = (R)((double)v[j].y * sc);
        }
      }
    }
  }
}

template <typename R, int MODE, int M0, int E>
__device__ __forceinline__ void col_block(const Args2<R> &a, int tile, unsigned char *smem_raw) {
  if ((tile + 1) * col_cpw(M0) <= a.ldk && a.nb * spec_rb<R>() >= M0 / 2)
    col_pass<R, MODE, M0, E, true>(a, tile, smem_raw);
  else
    col_pass<R, MODE, M0, E, false>(a, tile, smem_raw);
}

template <typename R, int MODE, int M0, int E>
__global__ void __launch_bounds__(col_threads(M0, E)) k_col2(Args2<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  col_block<R, MODE, M0, E>(a, xcd_tile(blockIdx.x, gridDim.x), smem_raw);
}

// Uneven batch: one launch over the column work-groups of every instance of
// a size class (neighbouring tiles of an instance share an XCD).
template <typename R, int MODE, int M0, int E>
__global__ void __launch_bounds__(col_threads(M0, E)) k_col2_batch(const BatchItem<R> *__restrict__ items,
                                                         int nitems) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int g = xcd_tile(blockIdx.x, gridDim.x);
  const int i = find_item(items, nitems, g);
  const Args2<R> a = item_args(items[i]);
  col_block<R, MODE, M0, E>(a, g - items[i].begin, smem_raw);
}

}  // namespace sweik
