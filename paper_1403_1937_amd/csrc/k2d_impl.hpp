// k2d_impl.hpp -- launchers of the 2D kernels: the run-time line lengths
// select compile-time instantiations.  Included once per precision.
#pragma once

#include "col2d.hpp"
#include "launch2d.hpp"
#include "row2d.hpp"

namespace sweik {

template <typename K> static hipError_t set_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R, int MODE, int H>
static hipError_t row_one(dim3 grid, hipStream_t st, const Args2<R> &a, int term) {
  constexpr size_t lds = row_lds_bytes<R>(H, MODE);
  if constexpr (lds > kLdsDevice) {  // rejected by the planner
    return hipErrorInvalidValue;
  } else {
    static const hipError_t attr = set_lds(k_row2<R, MODE, H>, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_row2<R, MODE, H>), grid, dim3(kThreads), lds, st, a, term);
    return hipGetLastError();
  }
}

template <typename R, int MODE>
static hipError_t row_mode(int H, dim3 grid, hipStream_t st, const Args2<R> &a, int term) {
  switch (H) {
    case 32: return row_one<R, MODE, 32>(grid, st, a, term);
    case 64: return row_one<R, MODE, 64>(grid, st, a, term);
    case 128: return row_one<R, MODE, 128>(grid, st, a, term);
    case 256: return row_one<R, MODE, 256>(grid, st, a, term);
    case 512: return row_one<R, MODE, 512>(grid, st, a, term);
    case 1024: return row_one<R, MODE, 1024>(grid, st, a, term);
    case 2048: return row_one<R, MODE, 2048>(grid, st, a, term);
    case 4096: return row_one<R, MODE, 4096>(grid, st, a, term);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_row2(int mode, int H, dim3 grid, hipStream_t st, const Args2<R> &a, int term) {
  switch (mode) {
    case ROW_GHAT: return row_mode<R, ROW_GHAT>(H, grid, st, a, term);
    case ROW_PHI0: return row_mode<R, ROW_PHI0>(H, grid, st, a, term);
    case ROW_TERM: return row_mode<R, ROW_TERM>(H, grid, st, a, term);
    case ROW_ADJ0: return row_mode<R, ROW_ADJ0>(H, grid, st, a, term);
    case ROW_ADJ: return row_mode<R, ROW_ADJ>(H, grid, st, a, term);
  }
  return hipErrorInvalidValue;
}

template <typename R, int MODE, int M0>
static hipError_t col_one(dim3 grid, hipStream_t st, const Args2<R> &a) {
  constexpr size_t lds = col_lds_bytes<R>(M0);
  if constexpr (lds > kLdsDevice) {  // rejected by the planner
    return hipErrorInvalidValue;
  } else {
    static const hipError_t attr = set_lds(k_col2<R, MODE, M0>, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_col2<R, MODE, M0>), grid, dim3(kThreads), lds, st, a);
    return hipGetLastError();
  }
}

template <typename R, int MODE>
static hipError_t col_mode(int M0, dim3 grid, hipStream_t st, const Args2<R> &a) {
  switch (M0) {
    case 64: return col_one<R, MODE, 64>(grid, st, a);
    case 128: return col_one<R, MODE, 128>(grid, st, a);
    case 256: return col_one<R, MODE, 256>(grid, st, a);
    case 512: return col_one<R, MODE, 512>(grid, st, a);
    case 1024: return col_one<R, MODE, 1024>(grid, st, a);
    case 2048: return col_one<R, MODE, 2048>(grid, st, a);
    case 4096: return col_one<R, MODE, 4096>(grid, st, a);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_col2(int mode, int M0, dim3 grid, hipStream_t st, const Args2<R> &a) {
  return mode == COL_GHAT ? col_mode<R, COL_GHAT>(M0, grid, st, a)
                          : col_mode<R, COL_CONV>(M0, grid, st, a);
}

// ---- uneven batches -------------------------------------------------------
template <typename R, int MODE, int H>
static hipError_t row_batch_one(int nblocks, hipStream_t st, const BatchItem<R> *items,
                                int nitems, int term) {
  constexpr size_t lds = row_lds_bytes<R>(H, MODE);
  if constexpr (lds > kLdsDevice) {
    return hipErrorInvalidValue;
  } else {
    static const hipError_t attr = set_lds(k_row2_batch<R, MODE, H>, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_row2_batch<R, MODE, H>), dim3(nblocks), dim3(kThreads), lds, st, items,
                       nitems, term);
    return hipGetLastError();
  }
}

template <typename R, int MODE>
static hipError_t row_batch_mode(int H, int nblocks, hipStream_t st, const BatchItem<R> *items,
                                 int nitems, int term) {
  switch (H) {
    case 32: return row_batch_one<R, MODE, 32>(nblocks, st, items, nitems, term);
    case 64: return row_batch_one<R, MODE, 64>(nblocks, st, items, nitems, term);
    case 128: return row_batch_one<R, MODE, 128>(nblocks, st, items, nitems, term);
    case 256: return row_batch_one<R, MODE, 256>(nblocks, st, items, nitems, term);
    case 512: return row_batch_one<R, MODE, 512>(nblocks, st, items, nitems, term);
    case 1024: return row_batch_one<R, MODE, 1024>(nblocks, st, items, nitems, term);
    case 2048: return row_batch_one<R, MODE, 2048>(nblocks, st, items, nitems, term);
    case 4096: return row_batch_one<R, MODE, 4096>(nblocks, st, items, nitems, term);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_row2_batch(int mode, int H, int nblocks, hipStream_t st,
                             const BatchItem<R> *items, int nitems, int term) {
  switch (mode) {
    case ROW_GHAT: return row_batch_mode<R, ROW_GHAT>(H, nblocks, st, items, nitems, term);
    case ROW_PHI0: return row_batch_mode<R, ROW_PHI0>(H, nblocks, st, items, nitems, term);
    case ROW_TERM: return row_batch_mode<R, ROW_TERM>(H, nblocks, st, items, nitems, term);
  }
  return hipErrorInvalidValue;
}

template <typename R, int MODE, int M0>
static hipError_t col_batch_one(int nblocks, hipStream_t st, const BatchItem<R> *items,
                                int nitems) {
  constexpr size_t lds = col_lds_bytes<R>(M0);
  if constexpr (lds > kLdsDevice) {
    return hipErrorInvalidValue;
  } else {
    static const hipError_t attr = set_lds(k_col2_batch<R, MODE, M0>, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_col2_batch<R, MODE, M0>), dim3(nblocks), dim3(kThreads), lds, st,
                       items, nitems);
    return hipGetLastError();
  }
}

template <typename R, int MODE>
static hipError_t col_batch_mode(int M0, int nblocks, hipStream_t st, const BatchItem<R> *items,
                                 int nitems) {
  switch (M0) {
    case 64: return col_batch_one<R, MODE, 64>(nblocks, st, items, nitems);
    case 128: return col_batch_one<R, MODE, 128>(nblocks, st, items, nitems);
    case 256: return col_batch_one<R, MODE, 256>(nblocks, st, items, nitems);
    case 512: return col_batch_one<R, MODE, 512>(nblocks, st, items, nitems);
    case 1024: return col_batch_one<R, MODE, 1024>(nblocks, st, items, nitems);
    case 2048: return col_batch_one<R, MODE, 2048>(nblocks, st, items, nitems);
    case 4096: return col_batch_one<R, MODE, 4096>(nblocks, st, items, nitems);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_col2_batch(int mode, int M0, int nblocks, hipStream_t st,
                             const BatchItem<R> *items, int nitems) {
  return mode == COL_GHAT ? col_batch_mode<R, COL_GHAT>(M0, nblocks, st, items, nitems)
                          : col_batch_mode<R, COL_CONV>(M0, nblocks, st, items, nitems);
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

template <typename R> hipError_t launch_fill(R *out, long long N, R v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill<R>, dim3(kRedBlocks), dim3(256), 0, st, out, N, v);
  return hipGetLastError();
}

#define SWEIK_INSTANTIATE_2D(R)                                                              \
  template hipError_t launch_row2<R>(int, int, dim3, hipStream_t, const Args2<R> &, int);  \
  template hipError_t launch_col2<R>(int, int, dim3, hipStream_t, const Args2<R> &);       \
  template hipError_t launch_prep<R>(const R *, long long, double *, cplx<R> *, int,       \
                                     hipStream_t);                                         \
  template hipError_t launch_adj_prep<R>(const R *, const double *, long long, double,     \
                                         double *, cplx<R> *, int, hipStream_t);           \
  template hipError_t launch_fill<R>(R *, long long, R, hipStream_t);                      \
  template hipError_t launch_row2_batch<R>(int, int, int, hipStream_t, const BatchItem<R> *, \
                                           int, int);                                      \
  template hipError_t launch_col2_batch<R>(int, int, int, hipStream_t, const BatchItem<R> *, \
                                           int);                                           \
  template hipError_t launch_prep_batch<R>(int, hipStream_t, const BatchItem<R> *);

}  // namespace sweik
