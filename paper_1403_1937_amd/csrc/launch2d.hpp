// launch2d.hpp -- host-side declarations of the 2D kernel launchers (one
// instantiation per precision, in k2d_f32.hip and k2d_f64.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common2d.hpp"

namespace sweik {

template <typename R>
hipError_t launch_row2(int mode, int H, dim3 grid, hipStream_t st, const Args2<R> &a, int term);
template <typename R>
hipError_t launch_col2(int mode, int M0, dim3 grid, hipStream_t st, const Args2<R> &a);
template <typename R>
hipError_t launch_prep(const R *f, long long N, double *red, cplx<R> *tw, int lmax,
                       hipStream_t st);
template <typename R>
hipError_t launch_adj_prep(const R *dLdS, const double *phi, long long N, double hbar,
                           double *red, cplx<R> *tw, int lmax, hipStream_t st);
template <typename R> hipError_t launch_fill(R *out, long long N, R v, hipStream_t st);
template <typename R>
hipError_t launch_row2_batch(int mode, int H, int nblocks, hipStream_t st,
                             const BatchItem<R> *items, int nitems, int term);
template <typename R>
hipError_t launch_col2_batch(int mode, int M0, int nblocks, hipStream_t st,
                             const BatchItem<R> *items, int nitems);
template <typename R>
hipError_t launch_prep_batch(int nitems, hipStream_t st, const BatchItem<R> *items);

}  // namespace sweik
