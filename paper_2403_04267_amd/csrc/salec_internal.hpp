// salec_internal.hpp -- launchers shared by the kernels and the host runtime
// of libsalec (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "salec_device.hpp"

namespace salec {

constexpr unsigned kDiagBlocks = 240;
constexpr int kDiagQ = 6;  // mass, ie, ke, mass_out, mass_pml, ie_out

using CycleFn = void (*)(const Inst*, const TileRef*, int);

// cycle kernel: tile-shape variants, one instantiation per bulk type
int n_variants();
void variant_shape(int v, int* tw, int* th, int* nt);
// the shape measured fastest on a filled device, per bulk type (0 FP64, 1 FP32)
int default_variant(int prec);
// (geo: the family that reads the geometry from the instances' tables, for
// stretched grids; nm: material slots, 2 or 3; pm: per-material closure;
// dm: damage and acoustic fluidization; null where the shape is not built
// for that family)
CycleFn cycle_kernel_f64(int v, bool geo, int nm, bool pm);
CycleFn cycle_kernel_f32(int v, bool geo, int nm, bool pm);
CycleFn cycle_kernel_dm_f64(int v, bool geo, int nm, bool pm);
CycleFn cycle_kernel_dm_f32(int v, bool geo, int nm, bool pm);
hipError_t launch_cycle(int v, int prec, bool geo, int nm, bool pm, bool dm, const Inst* insts,
                        const TileRef* sched, int nsched, int grid, hipStream_t st);
// end of a cycle: per-instance Courant minimum, clock, errors
hipError_t launch_finalize(const Inst* insts, int n_inst, hipStream_t st);
// workgroups of shape v that fit on the device at once (0 if unknown)
int resident_groups(int v, int prec, bool geo, int nm, bool pm, bool dm);
// whether shape v exists for this precision, family, material count, closure
// and damage
bool variant_available(int v, int prec, bool geo, int nm, bool pm, bool dm);

// EoS cache and Courant candidates of the current state (start of a run)
hipError_t launch_prime_f64(const Inst& in, hipStream_t st);
hipError_t launch_prime_f32(const Inst& in, hipStream_t st);
hipError_t launch_prime(const Inst& in, hipStream_t st);

// set-up, outputs and diagnostics of one instance
hipError_t launch_scene(const Inst& in, int surface_j, int layer_j, int layer2_j, int S, double R, double zc,
                        double v_imp, const double* rho_row, double* scratch, hipStream_t st);
hipError_t launch_start_run(const Inst& in, hipStream_t st);
hipError_t launch_finalize0(const Inst& in, hipStream_t st);
hipError_t launch_eos_out(const Inst& in, double* p, double* c2, hipStream_t st);
hipError_t launch_diag(const Inst& in, long long n_pml, double* red, double* out, hipStream_t st);

}  // namespace salec
