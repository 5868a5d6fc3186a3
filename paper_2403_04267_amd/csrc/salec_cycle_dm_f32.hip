// salec_cycle_dm_f32.hip -- mixed-mode instantiations of the cycle kernel's damage family.
#include "salec_cycle.hpp"

namespace salec {
SALEC_CYCLE_DM_TABLE(float, f32)
}  // namespace salec
