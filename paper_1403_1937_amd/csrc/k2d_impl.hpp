// k2d_impl.hpp -- launchers of the 2D kernels: the run-time line lengths and
// the schedule (E elements per team thread) select compile-time
// instantiations.  Each instantiation unit includes this once and
// instantiates one family (row passes of one E, or column passes and the
// small kernels) for one precision.
#pragma once

#include <algorithm>

#include "col2d.hpp"
#include "launch2d.hpp"
#include "row2d.hpp"

namespace sweik {

template <typename K> static hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// H = M1/2 of a row pass and M0 of a column pass, as template dispatch
#define SWEIK_ROW_LENGTHS(F, ...)                                                   \
  switch (H) {                                                                      \
    case 32: return F<32>(__VA_ARGS__);                                              \
    case 64: return F<64>(__VA_ARGS__);                                              \
    case 128: return F<128>(__VA_ARGS__);                                            \
    case 256: return F<256>(__VA_ARGS__);                                            \
    case 512: return F<512>(__VA_ARGS__);                                            \
    case 1024: return F<1024>(__VA_ARGS__);                                          \
    case 2048: return F<2048>(__VA_ARGS__);                                          \
    case 4096: return F<4096>(__VA_ARGS__);                                          \
    case 8192: return F<8192>(__VA_ARGS__);                                          \
  }                                                                                 \
  return hipErrorInvalidValue;
#define SWEIK_COL_LENGTHS(F, ...)                                                   \
  switch (M0) {                                                                     \
    case 64: return F<64>(__VA_ARGS__);                                              \
    case 128: return F<128>(__VA_ARGS__);                                            \
    case 256: return F<256>(__VA_ARGS__);                                            \
    case 512: return F<512>(__VA_ARGS__);                                            \
    case 1024: return F<1024>(__VA_ARGS__);                                          \
    case 2048: return F<2048>(__VA_ARGS__);                                          \
    case 4096: return F<4096>(__VA_ARGS__);                                          \
    case 8192: return F<8192>(__VA_ARGS__);                                          \
  }                                                                                 \
  return hipErrorInvalidValue;

template <typename R, int E, int MODE> struct RowLaunch {
  template <int H> static hipError_t one(dim3 grid, hipStream_t st, const Args2<R> &a, int term) {
    constexpr size_t lds = row_lds_bytes<R>(H, MODE);
    if constexpr (!row_ok<R>(H, E, MODE)) {  // rejected by the planner
      return hipErrorInvalidValue;
    } else {
      static const hipError_t attr = set_lds(k_row2<R, MODE, H, E>, lds);
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL((k_row2<R, MODE, H, E>), grid, dim3(row_threads(H, E)), lds, st, a, term);
      return hipGetLastError();
    }
  }
  template <int H>
  static hipError_t batch(int nblocks, hipStream_t st, const BatchItem<R> *items, int nitems,
                          int term) {
    constexpr size_t lds = row_lds_bytes<R>(H, MODE);
    if constexpr (!row_ok<R>(H, E, MODE)) {
      return hipErrorInvalidValue;
    } else {
      static const hipError_t attr = set_lds(k_row2_batch<R, MODE, H, E>, lds);
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL((k_row2_batch<R, MODE, H, E>), dim3(nblocks), dim3(row_threads(H, E)),
                         lds, st, items, nitems, term);
      return hipGetLastError();
    }
  }
  static hipError_t run(int H, dim3 grid, hipStream_t st, const Args2<R> &a, int term) {
    SWEIK_ROW_LENGTHS(one, grid, st, a, term)
  }
  static hipError_t run_batch(int H, int nblocks, hipStream_t st, const BatchItem<R> *items,
                              int nitems, int term) {
    SWEIK_ROW_LENGTHS(batch, nblocks, st, items, nitems, term)
  }
};

template <typename R, int E> struct RowInitLaunch {
  template <int H>
  static hipError_t one(hipStream_t st, const Args2<R> &ag, const Args2<R> &ap, int nbr) {
    if constexpr (!row_init_pairs<R>(H) || H < E) {  // not planned
      return hipErrorInvalidValue;
    } else {
      constexpr size_t lds = row_init_lds_bytes<R>(H);
      static const hipError_t attr = set_lds(k_row2_init<R, H, E>, lds);
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL((k_row2_init<R, H, E>), dim3(2 * nbr), dim3(row_threads(H, E)), lds, st,
                         ag, ap, nbr);
      return hipGetLastError();
    }
  }
  static hipError_t run(int H, hipStream_t st, const Args2<R> &ag, const Args2<R> &ap, int nbr) {
    SWEIK_ROW_LENGTHS(one, st, ag, ap, nbr)
  }
};

template <typename R, int E>
hipError_t launch_row2_init_e(int H, int nbr, hipStream_t st, const Args2<R> &ag,
                              const Args2<R> &ap) {
  return RowInitLaunch<R, E>::run(H, st, ag, ap, nbr);
}

template <typename R, int E>
hipError_t launch_row2_e(int mode, int H, dim3 grid, hipStream_t st, const Args2<R> &a, int term) {
  switch (mode) {
    case ROW_GHAT: return RowLaunch<R, E, ROW_GHAT>::run(H, grid, st, a, term);
    case ROW_PHI0: return RowLaunch<R, E, ROW_PHI0>::run(H, grid, st, a, term);
    case ROW_TERM: return RowLaunch<R, E, ROW_TERM>::run(H, grid, st, a, term);
    case ROW_ADJ0: return RowLaunch<R, E, ROW_ADJ0>::run(H, grid, st, a, term);
    case ROW_ADJ: return RowLaunch<R, E, ROW_ADJ>::run(H, grid, st, a, term);
    case ROW_SEED: return RowLaunch<R, E, ROW_SEED>::run(H, grid, st, a, term);
    case ROW_LAST: return RowLaunch<R, E, ROW_LAST>::run(H, grid, st, a, term);
    case ROW_DGHAT: return RowLaunch<R, E, ROW_DGHAT>::run(H, grid, st, a, term);
    case ROW_ADJ0_B: return RowLaunch<R, E, ROW_ADJ0_B>::run(H, grid, st, a, term);
    case ROW_ADJ_B: return RowLaunch<R, E, ROW_ADJ_B>::run(H, grid, st, a, term);
    // the tilted solve's own passes run with radix-16 teams only
    case ROW_GHATT:
      if constexpr (E == 16) return RowLaunch<R, E, ROW_GHATT>::run(H, grid, st, a, term);
      break;
    case ROW_LASTT:
      if constexpr (E == 16) return RowLaunch<R, E, ROW_LASTT>::run(H, grid, st, a, term);
      break;
  }
  return hipErrorInvalidValue;
}

template <typename R, int E>
hipError_t launch_row2_batch_e(int mode, int H, int nblocks, hipStream_t st,
                               const BatchItem<R> *items, int nitems, int term) {
  switch (mode) {
    case ROW_GHAT: return RowLaunch<R, E, ROW_GHAT>::run_batch(H, nblocks, st, items, nitems, term);
    case ROW_PHI0: return RowLaunch<R, E, ROW_PHI0>::run_batch(H, nblocks, st, items, nitems, term);
    case ROW_TERM: return RowLaunch<R, E, ROW_TERM>::run_batch(H, nblocks, st, items, nitems, term);
    case ROW_LAST: return RowLaunch<R, E, ROW_LAST>::run_batch(H, nblocks, st, items, nitems, term);
    // the tilted solve's passes over all tilts (radix-16 teams only)
    case ROW_GHATT:
      if constexpr (E == 16)
        return RowLaunch<R, E, ROW_GHATT>::run_batch(H, nblocks, st, items, nitems, term);
      break;
    case ROW_LASTT:
      if constexpr (E == 16)
        return RowLaunch<R, E, ROW_LASTT>::run_batch(H, nblocks, st, items, nitems, term);
      break;
  }
  return hipErrorInvalidValue;
}

template <typename R, int E, int MODE> struct ColLaunch {
  template <int M0> static hipError_t one(dim3 grid, hipStream_t st, const Args2<R> &a) {
    constexpr size_t lds = col_lds_bytes<R>(M0);
    if constexpr (!col_ok<R>(M0, E)) {  // rejected by the planner
      return hipErrorInvalidValue;
    } else {
      static const hipError_t attr = set_lds(k_col2<R, MODE, M0, E>, lds);
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL((k_col2<R, MODE, M0, E>), grid, dim3(col_threads(M0, E)), lds, st, a);
      return hipGetLastError();
    }
  }
  template <int M0>
  static hipError_t batch(int nblocks, hipStream_t st, const BatchItem<R> *items, int nitems) {
    constexpr size_t lds = col_lds_bytes<R>(M0);
    if constexpr (!col_ok<R>(M0, E)) {
      return hipErrorInvalidValue;
    } else {
      static const hipError_t attr = set_lds(k_col2_batch<R, MODE, M0, E>, lds);
      if (attr != hipSuccess) return attr;
      hipLaunchKernelGGL((k_col2_batch<R, MODE, M0, E>), dim3(nblocks), dim3(col_threads(M0, E)),
                         lds, st, items, nitems);
      return hipGetLastError();
    }
  }
  static hipError_t run(int M0, dim3 grid, hipStream_t st, const Args2<R> &a) {
    SWEIK_COL_LENGTHS(one, grid, st, a)
  }
  static hipError_t run_batch(int M0, int nblocks, hipStream_t st, const BatchItem<R> *items,
                              int nitems) {
    SWEIK_COL_LENGTHS(batch, nblocks, st, items, nitems)
  }
};

template <typename R, int E>
hipError_t launch_col2_e(int mode, int M0, dim3 grid, hipStream_t st, const Args2<R> &a) {
  switch (mode) {
    case COL_GHAT: return ColLaunch<R, E, COL_GHAT>::run(M0, grid, st, a);
    case COL_CONV: return ColLaunch<R, E, COL_CONV>::run(M0, grid, st, a);
    // the tilted solve's column passes run with radix-16 teams only
    case COL_GHATC:
      if constexpr (E == 16) return ColLaunch<R, E, COL_GHATC>::run(M0, grid, st, a);
      break;
    case COL_CONVC:
      if constexpr (E == 16) return ColLaunch<R, E, COL_CONVC>::run(M0, grid, st, a);
      break;
  }
  return hipErrorInvalidValue;
}

template <typename R, int E>
hipError_t launch_col2_batch_e(int mode, int M0, int nblocks, hipStream_t st,
                               const BatchItem<R> *items, int nitems) {
  switch (mode) {
    case COL_GHAT: return ColLaunch<R, E, COL_GHAT>::run_batch(M0, nblocks, st, items, nitems);
    case COL_CONV: return ColLaunch<R, E, COL_CONV>::run_batch(M0, nblocks, st, items, nitems);
    case COL_GHATC:
      if constexpr (E == 16)
        return ColLaunch<R, E, COL_GHATC>::run_batch(M0, nblocks, st, items, nitems);
      break;
    case COL_CONVC:
      if constexpr (E == 16)
        return ColLaunch<R, E, COL_CONVC>::run_batch(M0, nblocks, st, items, nitems);
      break;
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_prep_batch(int nitems, hipStream_t st, const BatchItem<R> *items) {
  hipLaunchKernelGGL(k_prep_batch<R>, dim3(nitems * kRedBlocks), dim3(256), 0, st, items);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_prep(const R *f, long long N, double *red, cplx<R> *tw, int lmax,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_prep<R>, dim3(kRedBlocks), dim3(256), 0, st, f, N, red, tw, lmax);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_adj_prep(const R *dLdS, const double *phi, long long N, double hbar,
                           double *red, cplx<R> *tw, int lmax, hipStream_t st) {
  hipLaunchKernelGGL(k_adj_prep<R>, dim3(kRedBlocks), dim3(256), 0, st, dLdS, phi, N, hbar, red,
                     tw, lmax);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_seed_scatter(R *grid, const int *src, const R *src_s, int n_src, double hbar,
                               int n0, int n1, int n2, hipStream_t st) {
  const int nb = std::max(1, std::min((n_src + 255) / 256, 1024));
  hipLaunchKernelGGL(k_seed_scatter<R>, dim3(nb), dim3(256), 0, st, grid, src, src_s, n_src, hbar,
                     n0, n1, n2);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_adj_full_finish(const R *f, long long N, const Params *par, const double *gpart,
                                  int nbr, long long *ext, int ft_mode, double h, double hbar,
                                  R *dLdf, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_argext<R>, dim3(kRedBlocks), dim3(256), 0, st, f, N, par, ext);
  hipLaunchKernelGGL(k_adj_full_finish<R>, dim3(1), dim3(256), 0, st, gpart, nbr,
                     (const long long *)ext, (int)kRedBlocks, par, ft_mode, h, hbar, dLdf, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_source_lse(R *S, double *acc, long long N, double hbar, int first, int last,
                             sweik_info *info, hipStream_t st) {
  const long long nb = std::min<long long>((N + 255) / 256, 4096);
  hipLaunchKernelGGL(k_source_lse<R>, dim3((unsigned)std::max<long long>(nb, 1)), dim3(256), 0, st,
                     S, acc, N, hbar, first, last, info);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_tilt_items(const Args2<R> &base, const TiltTable &tt, int n_tilt,
                             unsigned char *slices, const TiltSlice &sl, BatchItem<R> *rows,
                             BatchItem<R> *negs, BatchItem<R> *cols, hipStream_t st) {
  hipLaunchKernelGGL(k_tilt_items<R>, dim3(1), dim3(64), 0, st, base, tt, n_tilt, slices, sl, rows,
                     negs, cols);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_tilt_select(R *S, const unsigned char *slices, const TiltSlice &sl, int n_tilt,
                              long long N, int count, sweik_info *info, hipStream_t st) {
  const long long nb = std::min<long long>((N + 255) / 256, 4096);
  hipLaunchKernelGGL(k_tilt_select<R>, dim3((unsigned)std::max<long long>(nb, 1)), dim3(256), 0,
                     st, S, slices, sl, n_tilt, N, count, info);
  return hipGetLastError();
}

template <typename R> hipError_t launch_fill(R *out, long long N, R v, hipStream_t st) {
  const long long nb = std::min<long long>((N + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill<R>, dim3((unsigned)std::max<long long>(nb, 1)), dim3(256), 0, st, out,
                     N, v);
  return hipGetLastError();
}

#define SWEIK_INSTANTIATE_2D_ROWS(R, E)                                                     \
  template hipError_t launch_row2_e<R, E>(int, int, dim3, hipStream_t, const Args2<R> &, int); \
  template hipError_t launch_row2_init_e<R, E>(int, int, hipStream_t, const Args2<R> &,      \
                                               const Args2<R> &);                            \
  template hipError_t launch_row2_batch_e<R, E>(int, int, int, hipStream_t,                 \
                                                const BatchItem<R> *, int, int);

#define SWEIK_INSTANTIATE_2D_COLS_E(R, E)                                                   \
  template hipError_t launch_col2_e<R, E>(int, int, dim3, hipStream_t, const Args2<R> &);   \
  template hipError_t launch_col2_batch_e<R, E>(int, int, int, hipStream_t,                 \
                                                const BatchItem<R> *, int);

#define SWEIK_INSTANTIATE_2D_COLS(R)                                                        \
  template hipError_t launch_col2_e<R, 16>(int, int, dim3, hipStream_t, const Args2<R> &);  \
  template hipError_t launch_col2_e<R, 8>(int, int, dim3, hipStream_t, const Args2<R> &);   \
  template hipError_t launch_col2_batch_e<R, 16>(int, int, int, hipStream_t,                \
                                                 const BatchItem<R> *, int);                \
  template hipError_t launch_col2_batch_e<R, 8>(int, int, int, hipStream_t,                 \
                                                const BatchItem<R> *, int);                 \
  template hipError_t launch_prep<R>(const R *, long long, double *, cplx<R> *, int,        \
                                     hipStream_t);                                          \
  template hipError_t launch_adj_prep<R>(const R *, const double *, long long, double,      \
                                         double *, cplx<R> *, int, hipStream_t);            \
  template hipError_t launch_fill<R>(R *, long long, R, hipStream_t);                       \
  template hipError_t launch_source_lse<R>(R *, double *, long long, double, int, int,      \
                                           sweik_info *, hipStream_t);                      \
  template hipError_t launch_tilt_items<R>(const Args2<R> &, const TiltTable &, int,        \
                                           unsigned char *, const TiltSlice &,              \
                                           BatchItem<R> *, BatchItem<R> *, BatchItem<R> *,  \
                                           hipStream_t);                                    \
  template hipError_t launch_tilt_select<R>(R *, const unsigned char *, const TiltSlice &,  \
                                            int, long long, int, sweik_info *, hipStream_t); \
  template hipError_t launch_adj_full_finish<R>(const R *, long long, const Params *,         \
                                                const double *, int, long long *, int, double, \
                                                double, R *, double *, hipStream_t);           \
  template hipError_t launch_seed_scatter<R>(R *, const int *, const R *, int, double, int, int, \
                                             int, hipStream_t);                                  \
  template hipError_t launch_prep_batch<R>(int, hipStream_t, const BatchItem<R> *);

}  // namespace sweik
