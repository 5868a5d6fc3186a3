// salec_cycle_f32.hip -- mixed-mode instantiations of the cycle kernel (FP32
// bulk arithmetic; FP64 energy, mass and volume sums and Courant reduction).
#include "salec_cycle.hpp"

namespace salec {
SALEC_CYCLE_TABLE(float, f32)
}  // namespace salec
