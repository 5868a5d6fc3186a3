// salec_cycle.hip -- tile shapes of the cycle kernel and its launchers.
#include "salec_internal.hpp"

namespace salec {

// must match the order of SALEC_CYCLE_TABLE
static const int kShapes[][3] = {{64, 16, 512}, {64, 16, 1024}, {32, 32, 1024}, {32, 16, 256}};

int n_variants() { return (int)(sizeof(kShapes) / sizeof(kShapes[0])); }

void variant_shape(int v, int* tw, int* th, int* nt) {
  *tw = kShapes[v][0];
  *th = kShapes[v][1];
  *nt = kShapes[v][2];
}

hipError_t launch_cycle(int v, int prec, const Inst* insts, const TileRef* sched, int nsched, int grid,
                        hipStream_t st) {
  CycleFn f = prec == 0 ? cycle_kernel_f64(v) : cycle_kernel_f32(v);
  if (!f) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f, dim3(grid), dim3(kShapes[v][2]), 0, st, insts, sched, nsched);
  return hipGetLastError();
}

hipError_t launch_prime(const Inst& in, hipStream_t st) {
  return in.g.prec == 0 ? launch_prime_f64(in, st) : launch_prime_f32(in, st);
}

}  // namespace salec
