// salec_cycle_dm_f64.hip -- FP64 instantiations of the cycle kernel's damage family.
#include "salec_cycle.hpp"

namespace salec {
SALEC_CYCLE_DM_TABLE(double, f64)
}  // namespace salec
