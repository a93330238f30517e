// Kernel instantiations for one equation (TenMom1D), N = 1..4, FP64 and MP32.
#include "crkfr_launch.hpp"

namespace crkfr {
CRKFR_DEFINE_EQ(tenmom1d, TenMom1D)
}  // namespace crkfr
