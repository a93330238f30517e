// Kernel instantiations for one equation (Burgers1D), N = 1..4, FP64 and MP32.
#include "crkfr_launch.hpp"

namespace crkfr {
CRKFR_DEFINE_EQ(burgers1d, Burgers1D)
}  // namespace crkfr
