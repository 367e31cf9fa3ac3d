// k3d_impl.hpp -- launchers of the 3D kernels: the run-time line lengths
// select compile-time instantiations.  Included once per precision.
#pragma once

#include "c3d.hpp"
#include "launch3d.hpp"
#include "x3d.hpp"

namespace sweik {

template <typename K> static hipError_t set_lds3(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename R, int MODE, int H>
static hipError_t x3_one(int nblocks, hipStream_t st, const Args3<R> &a, int term) {
  constexpr size_t lds = x_lds_bytes<R>(H);
  if constexpr (lds + x_lds_static<R>(MODE) > kLdsDevice) {  // rejected by the planner
    return hipErrorInvalidValue;
  } else {
    static const hipError_t attr = set_lds3(k_x3<R, MODE, H>, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_x3<R, MODE, H>), dim3(nblocks), dim3(kThreads), lds, st, a, term);
    return hipGetLastError();
  }
}

template <typename R, int MODE>
static hipError_t x3_mode(int H, int nblocks, hipStream_t st, const Args3<R> &a, int term) {
  switch (H) {
    case 32: return x3_one<R, MODE, 32>(nblocks, st, a, term);
    case 64: return x3_one<R, MODE, 64>(nblocks, st, a, term);
    case 128: return x3_one<R, MODE, 128>(nblocks, st, a, term);
    case 256: return x3_one<R, MODE, 256>(nblocks, st, a, term);
    case 512: return x3_one<R, MODE, 512>(nblocks, st, a, term);
    case 1024: return x3_one<R, MODE, 1024>(nblocks, st, a, term);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_x3(int mode, int H, int nblocks, hipStream_t st, const Args3<R> &a, int term) {
  switch (mode) {
    case X_GHAT: return x3_mode<R, X_GHAT>(H, nblocks, st, a, term);
    case X_PHI0: return x3_mode<R, X_PHI0>(H, nblocks, st, a, term);
    case X_TERM: return x3_mode<R, X_TERM>(H, nblocks, st, a, term);
    case X_LAST: return x3_mode<R, X_LAST>(H, nblocks, st, a, term);
    case X_ADJ0: return x3_mode<R, X_ADJ0>(H, nblocks, st, a, term);
    case X_ADJ: return x3_mode<R, X_ADJ>(H, nblocks, st, a, term);
    case X_DGHAT: return x3_mode<R, X_DGHAT>(H, nblocks, st, a, term);
    case X_ADJ0_B: return x3_mode<R, X_ADJ0_B>(H, nblocks, st, a, term);
    case X_ADJ_B: return x3_mode<R, X_ADJ_B>(H, nblocks, st, a, term);
    case X_PHI0F: return x3_mode<R, X_PHI0F>(H, nblocks, st, a, term);
    case X_ETAB: return x3_mode<R, X_ETAB>(H, nblocks, st, a, term);
    case X_SEED: return x3_mode<R, X_SEED>(H, nblocks, st, a, term);
  }
  return hipErrorInvalidValue;
}

template <typename R, int MODE, int M>
static hipError_t c3_one(int nblocks, hipStream_t st, const Args3<R> &a, int term) {
  constexpr size_t lds = c3_lds_bytes<R>(M);
  if constexpr (lds + kC3LdsStatic > kLdsDevice) {  // rejected by the planner
    return hipErrorInvalidValue;
  } else {
    static const hipError_t attr = set_lds3(k_c3<R, MODE, M>, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((k_c3<R, MODE, M>), dim3(nblocks), dim3(c3_threads<R>(M)), lds, st, a,
                       term);
    return hipGetLastError();
  }
}

template <typename R, int MODE>
static hipError_t c3_mode(int M, int nblocks, hipStream_t st, const Args3<R> &a, int term) {
  switch (M) {
    case 64: return c3_one<R, MODE, 64>(nblocks, st, a, term);
    case 128: return c3_one<R, MODE, 128>(nblocks, st, a, term);
    case 256: return c3_one<R, MODE, 256>(nblocks, st, a, term);
    case 512: return c3_one<R, MODE, 512>(nblocks, st, a, term);
    case 1024: return c3_one<R, MODE, 1024>(nblocks, st, a, term);
    case 2048: return c3_one<R, MODE, 2048>(nblocks, st, a, term);
  }
  return hipErrorInvalidValue;
}

template <typename R>
hipError_t launch_c3(int mode, int M, int nblocks, hipStream_t st, const Args3<R> &a, int term) {
  switch (mode) {
    case C3_YF: return c3_mode<R, C3_YF>(M, nblocks, st, a, term);
    case C3_Z: return c3_mode<R, C3_Z>(M, nblocks, st, a, term);
    case C3_YI: return c3_mode<R, C3_YI>(M, nblocks, st, a, term);
    case C3_GY: return c3_mode<R, C3_GY>(M, nblocks, st, a, term);
    case C3_GZ: return c3_mode<R, C3_GZ>(M, nblocks, st, a, term);
  }
  return hipErrorInvalidValue;
}

#define SWEIK_INSTANTIATE_3D(R)                                                           \
  template hipError_t launch_x3<R>(int, int, int, hipStream_t, const Args3<R> &, int);    \
  template hipError_t launch_c3<R>(int, int, int, hipStream_t, const Args3<R> &, int);

}  // namespace sweik
