// k2d_row8_f64.hip -- double instantiation of the 2D row passes, 8 elements per thread.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D_ROWS(double, 8)
}
