// Double-precision (complex128) instantiation of the SETD passes.
#include "setd_launch_impl.hpp"

namespace setd {
SETD_INSTANTIATE(double)
}
