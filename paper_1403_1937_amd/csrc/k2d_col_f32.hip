// k2d_col_f32.hip -- float instantiation of the 2D column passes and small kernels.
#include "k2d_impl.hpp"

namespace sweik {
SWEIK_INSTANTIATE_2D_COLS(float)
}
