// k2d_row16_f64.hip -- double instantiation of the 2D row passes, 16 elements per thread.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D_ROWS(double, 16)
}
