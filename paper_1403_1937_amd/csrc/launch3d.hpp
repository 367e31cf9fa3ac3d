// launch3d.hpp -- host-side declarations of the 3D kernel launchers (one
// instantiation per precision, in k3d_f32.hip and k3d_f64.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common3d.hpp"

namespace sweik {

// x pass over all n0 n1 lines: mode XMode, line length H = H2
template <typename R>
hipError_t launch_x3(int mode, int H, int nblocks, hipStream_t st, const Args3<R> &a, int term);
// column pass: mode C3Mode, transform length M (M1 for the y modes, M0 for
// the z modes), nblocks = planes x H2 / c3_cpw<R>(M)
template <typename R>
hipError_t launch_c3(int mode, int M, int nblocks, hipStream_t st, const Args3<R> &a, int term);

}  // namespace sweik
