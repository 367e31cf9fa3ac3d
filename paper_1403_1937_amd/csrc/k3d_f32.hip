// k3d_f32.hip -- float instantiation of the 3D kernels.
#include "k3d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_3D(float)
}
