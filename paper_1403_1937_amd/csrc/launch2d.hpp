// launch2d.hpp -- host-side declarations of the 2D kernel launchers.  The
// row passes of each schedule E and precision are instantiated in
// k2d_row<E>_<prec>.hip, the column passes and small kernels in
// k2d_col_<prec>.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "common2d.hpp"

namespace sweik {

// Keeps a description of a failed launch for sweik_last_error (thread-local).
void note_launch_error(const char *family, int mode, int length, int E, hipError_t err);

template <typename R, int E>
hipError_t launch_row2_e(int mode, int H, dim3 grid, hipStream_t st, const Args2<R> &a, int term);
template <typename R, int E>
hipError_t launch_col2_e(int mode, int M0, dim3 grid, hipStream_t st, const Args2<R> &a);
template <typename R, int E>
hipError_t launch_row2_init_e(int H, int nbr, hipStream_t st, const Args2<R> &ag,
                              const Args2<R> &ap);
template <typename R, int E>
hipError_t launch_row2_batch_e(int mode, int H, int nblocks, hipStream_t st,
                               const BatchItem<R> *items, int nitems, int term);
template <typename R, int E>
hipError_t launch_col2_batch_e(int mode, int M0, int nblocks, hipStream_t st,
                               const BatchItem<R> *items, int nitems);
template <typename R>
hipError_t launch_prep(const R *f, long long N, double *red, cplx<R> *tw, int lmax,
                       hipStream_t st);
template <typename R>
hipError_t launch_adj_prep(const R *dLdS, const double *phi, long long N, double hbar,
                           double *red, cplx<R> *tw, int lmax, hipStream_t st);
template <typename R> hipError_t launch_fill(R *out, long long N, R v, hipStream_t st);
template <typename R>
hipError_t launch_source_lse(R *S, double *acc, long long N, double hbar, int first, int last,
                             sweik_info *info, hipStream_t st);
// the tilted solve: the tilts' work lists (k_tilt_items) and the per-point
// choice of tilt (k_tilt_select)
template <typename R>
hipError_t launch_tilt_items(const Args2<R> &base, const TiltTable &tt, int n_tilt,
                             unsigned char *slices, const TiltSlice &sl, BatchItem<R> *rows,
                             BatchItem<R> *negs, BatchItem<R> *cols, hipStream_t st);
template <typename R>
hipError_t launch_tilt_select(R *S, const unsigned char *slices, const TiltSlice &sl, int n_tilt,
                              long long N, int count, sweik_info *info, hipStream_t st);
// full gradient: argmin / argmax of f (kRedBlocks partials in ext, 2 x
// kRedBlocks long long) and the scalar derivatives (see k_adj_full_finish)
template <typename R>
hipError_t launch_adj_full_finish(const R *f, long long N, const Params *par, const double *gpart,
                                  int nbr, long long *ext, int ft_mode, double h, double hbar,
                                  R *dLdf, double *out, hipStream_t st);
template <typename R>
hipError_t launch_seed_scatter(R *grid, const int *src, const R *src_s, int n_src, double hbar,
                               int n0, int n1, int n2, hipStream_t st);  // 2D: n2 = 0
template <typename R>
hipError_t launch_prep_batch(int nitems, hipStream_t st, const BatchItem<R> *items);

// schedule dispatch: E = 16 (radix-16 stages, 256 threads per work-group),
// 8 (radix-8 stages, 512 threads) or, in float32 only, 4 (radix-4 stages,
// 1024 threads)
template <typename R> struct RadixFour {
  static hipError_t row(int, int, dim3, hipStream_t, const Args2<R> &, int) {
    return hipErrorInvalidValue;
  }
  static hipError_t col(int, int, dim3, hipStream_t, const Args2<R> &) {
    return hipErrorInvalidValue;
  }
  static hipError_t row_batch(int, int, int, hipStream_t, const BatchItem<R> *, int, int) {
    return hipErrorInvalidValue;
  }
  static hipError_t row_init(int, int, hipStream_t, const Args2<R> &, const Args2<R> &) {
    return hipErrorInvalidValue;
  }
  static hipError_t col_batch(int, int, int, hipStream_t, const BatchItem<R> *, int) {
    return hipErrorInvalidValue;
  }
};
template <> struct RadixFour<float> {
  static hipError_t row(int mode, int H, dim3 g, hipStream_t st, const Args2<float> &a, int term) {
    return launch_row2_e<float, 4>(mode, H, g, st, a, term);
  }
  static hipError_t col(int mode, int M0, dim3 g, hipStream_t st, const Args2<float> &a) {
    return launch_col2_e<float, 4>(mode, M0, g, st, a);
  }
  static hipError_t row_batch(int mode, int H, int nb, hipStream_t st,
                              const BatchItem<float> *items, int n, int term) {
    return launch_row2_batch_e<float, 4>(mode, H, nb, st, items, n, term);
  }
  static hipError_t row_init(int H, int nbr, hipStream_t st, const Args2<float> &ag,
                             const Args2<float> &ap) {
    return launch_row2_init_e<float, 4>(H, nbr, st, ag, ap);
  }
  static hipError_t col_batch(int mode, int M0, int nb, hipStream_t st,
                              const BatchItem<float> *items, int n) {
    return launch_col2_batch_e<float, 4>(mode, M0, nb, st, items, n);
  }
};

template <typename R>
inline hipError_t launch_row2(int mode, int H, int E, dim3 grid, hipStream_t st,
                              const Args2<R> &a, int term) {
  const hipError_t err = E == 16  ? launch_row2_e<R, 16>(mode, H, grid, st, a, term)
                         : E == 8 ? launch_row2_e<R, 8>(mode, H, grid, st, a, term)
                         : E == 4 ? RadixFour<R>::row(mode, H, grid, st, a, term)
                                  : hipErrorInvalidValue;
  if (err != hipSuccess) note_launch_error("row pass", mode, H, E, err);
  return err;
}
// the paired kernel-table + phi_0 row pass (2 nbr work-groups)
template <typename R>
inline hipError_t launch_row2_init(int H, int E, int nbr, hipStream_t st, const Args2<R> &ag,
                                   const Args2<R> &ap) {
  const hipError_t err = E == 16  ? launch_row2_init_e<R, 16>(H, nbr, st, ag, ap)
                         : E == 8 ? launch_row2_init_e<R, 8>(H, nbr, st, ag, ap)
                         : E == 4 ? RadixFour<R>::row_init(H, nbr, st, ag, ap)
                                  : hipErrorInvalidValue;
  if (err != hipSuccess) note_launch_error("paired kernel-table and phi_0 row pass", -1, H, E, err);
  return err;
}
template <typename R>
inline hipError_t launch_col2(int mode, int M0, int E, dim3 grid, hipStream_t st,
                              const Args2<R> &a) {
  const hipError_t err = E == 16  ? launch_col2_e<R, 16>(mode, M0, grid, st, a)
                         : E == 8 ? launch_col2_e<R, 8>(mode, M0, grid, st, a)
                         : E == 4 ? RadixFour<R>::col(mode, M0, grid, st, a)
                                  : hipErrorInvalidValue;
  if (err != hipSuccess) note_launch_error("column pass", mode, M0, E, err);
  return err;
}
template <typename R>
inline hipError_t launch_row2_batch(int mode, int H, int E, int nblocks, hipStream_t st,
                                    const BatchItem<R> *items, int nitems, int term) {
  const hipError_t err =
      E == 16  ? launch_row2_batch_e<R, 16>(mode, H, nblocks, st, items, nitems, term)
      : E == 8 ? launch_row2_batch_e<R, 8>(mode, H, nblocks, st, items, nitems, term)
      : E == 4 ? RadixFour<R>::row_batch(mode, H, nblocks, st, items, nitems, term)
               : hipErrorInvalidValue;
  if (err != hipSuccess) note_launch_error("batched row pass", mode, H, E, err);
  return err;
}
template <typename R>
inline hipError_t launch_col2_batch(int mode, int M0, int E, int nblocks, hipStream_t st,
                                    const BatchItem<R> *items, int nitems) {
  const hipError_t err = E == 16  ? launch_col2_batch_e<R, 16>(mode, M0, nblocks, st, items, nitems)
                         : E == 8 ? launch_col2_batch_e<R, 8>(mode, M0, nblocks, st, items, nitems)
                         : E == 4 ? RadixFour<R>::col_batch(mode, M0, nblocks, st, items, nitems)
                                  : hipErrorInvalidValue;
  if (err != hipSuccess) note_launch_error("batched column pass", mode, M0, E, err);
  return err;
}

}  // namespace sweik
