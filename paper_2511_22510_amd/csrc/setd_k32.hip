// Single-precision (complex64) instantiation of the SETD passes.
#include "setd_launch_impl.hpp"

namespace setd {
SETD_INSTANTIATE(float)
// launches shared by lattice classes exist for complex64 states only
template hipError_t launch_multi2d<float>(const MultiClass (&)[4], int, int, hipStream_t);
}
