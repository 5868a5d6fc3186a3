// salec_internal.hpp -- launchers shared by the kernels and the host runtime
// of libsalec (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "salec_device.hpp"

namespace salec {

constexpr unsigned kDiagBlocks = 240;

void launch_cycle(const Geo& g, const State& S0, const State& S1, const Work& w, const Pml& pm, Scal* sc,
                  hipStream_t st);
void launch_cycle_fused(const Geo& g, const State& S0, const State& S1, const Work& w, const Pml& pm, Scal* sc,
                        hipStream_t st);
void fused_tiles(int NR, int NZ, int* tr, int* tz);
void launch_dt0(const Geo& g, const State& S0, const State& S1, Scal* sc, hipStream_t st);
void launch_scene(const Geo& g, const State& S0, const Work& w, int surface_j, int S, double R, double zc,
                  double v_imp, hipStream_t st);
void launch_eos_out(const Geo& g, const State& S0, const State& S1, const Scal* sc, double* p, double* c2,
                    hipStream_t st);
void launch_diag(const Geo& g, const State& S0, const State& S1, const Work& w, const Pml& pm, const Scal* sc,
                 long long n_pml, double* out, hipStream_t st);
void launch_start_run(const Geo& g, const State& S0, const Pml& pm, Scal* sc, hipStream_t st);

}  // namespace salec
