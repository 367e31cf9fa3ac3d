// k2d_f64.hip -- float64 instantiation of the 2D kernels.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D(double)
}
