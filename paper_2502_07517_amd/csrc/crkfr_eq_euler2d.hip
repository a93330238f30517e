// Kernel instantiations for one equation (Euler2D), N = 1..4, FP64 and MP32.
#include "crkfr_launch.hpp"

namespace crkfr {
CRKFR_DEFINE_EQ(euler2d, Euler2D)
}  // namespace crkfr
