// k2d_col4_f32.hip -- float instantiation of the 2D column passes, 4 elements per thread.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D_COLS_E(float, 4)
}
