// k2d_row4_f32.hip -- float instantiation of the 2D row passes, 4 elements per thread.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D_ROWS(float, 4)
}
