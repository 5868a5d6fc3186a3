// salec_cycle_f64.hip -- FP64 instantiations of the cycle kernel.
#include "salec_cycle.hpp"

namespace salec {
SALEC_CYCLE_TABLE(double, f64)
}  // namespace salec
