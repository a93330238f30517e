// Kernel instantiations for one equation (Euler1D), N = 1..4, FP64 and MP32.
#include "crkfr_launch.hpp"

namespace crkfr {
CRKFR_DEFINE_EQ(euler1d, Euler1D)
}  // namespace crkfr
