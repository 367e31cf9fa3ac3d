// k2d_f32.hip -- float32 instantiation of the 2D kernels.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D(float)
}
