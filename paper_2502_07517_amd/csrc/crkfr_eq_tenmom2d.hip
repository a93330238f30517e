// Kernel instantiations for one equation (TenMom2D), N = 1..4, FP64 and MP32.
#include "crkfr_launch.hpp"

namespace crkfr {
CRKFR_DEFINE_EQ(tenmom2d, TenMom2D)
}  // namespace crkfr
