// Single-precision (complex64) instantiation of the SETD passes.
#include "setd_launch_impl.hpp"

namespace setd {
SETD_INSTANTIATE(float)
}
