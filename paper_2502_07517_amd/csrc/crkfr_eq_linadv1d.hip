// Kernel instantiations for one equation (LinAdv1D), N = 1..4, FP64 and MP32.
#include "crkfr_launch.hpp"

namespace crkfr {
CRKFR_DEFINE_EQ(linadv1d, LinAdv1D)
}  // namespace crkfr
