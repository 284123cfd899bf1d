// Single-precision (complex64) instantiation of the 1D line kernels.
#include "setd_launch_impl.hpp"

namespace setd {
SETD_INSTANTIATE_LINES(float)
}
