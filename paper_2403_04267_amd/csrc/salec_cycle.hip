// salec_cycle.hip -- tile shapes of the cycle kernel and its launchers.
#include "salec_internal.hpp"

namespace salec {

// Tile shapes (cells r x z, threads), in the order of SALEC_CYCLE_TABLE.
// 768-thread tiles run one workgroup per CU at three waves per SIMD (LDS
// holds one tile); 512-thread tiles are capped at 128 registers so that two
// workgroups (four waves per SIMD) share a CU where two tiles fit the LDS
// (the FP32 instantiation); 256-thread tiles run three to a CU. Shape 11 is
// built only for the per-material closure and three material slots, whose
// wider LDS records leave no 768-thread tile of the other sizes room. Shapes
// 12-14 are near-square 768-thread tiles that keep two cells of the widest
// halo per thread: less halo recomputed per owned cell (1.40 halo-inclusive
// cells for 35 x 31 against 1.56 for 64 x 14) and tile counts that fill whole
// rounds of one workgroup per CU (35 x 31: 1020 tiles on a 1050-cell square;
// 32 x 34: 256 tiles on the 512 x 532 stretched grid). Each is built where
// its LDS records fit: 35 x 31 for two slots and for three on uniform grids,
// 32 x 34 for two slots, 27 x 27 for the per-material closure with three.
static const int kShapes[][3] = {
    {64, 14, 768},
    {40, 16, 512},
    {32, 20, 512},
    {64, 15, 768},
    {64, 16, 768},
    {48, 20, 768},
    {40, 24, 768},
    {28, 18, 512},
    {64, 16, 1024},
    {32, 32, 1024},
    {20, 13, 256},
    {48, 14, 768},
    {35, 31, 768},
    {32, 34, 768},
    {27, 27, 768}};

int default_variant(int) { return 12; }

int n_variants() { return (int)(sizeof(kShapes) / sizeof(kShapes[0])); }

void variant_shape(int v, int* tw, int* th, int* nt) {
  *tw = kShapes[v][0];
  *th = kShapes[v][1];
  *nt = kShapes[v][2];
}

static CycleFn cycle_kernel(int v, int prec, bool geo, int nm, bool pm, bool dm) {
  if (v < 0 || v >= n_variants()) return nullptr;
  if (dm) return prec == 0 ? cycle_kernel_dm_f64(v, geo, nm, pm) : cycle_kernel_dm_f32(v, geo, nm, pm);
  return prec == 0 ? cycle_kernel_f64(v, geo, nm, pm) : cycle_kernel_f32(v, geo, nm, pm);
}

bool variant_available(int v, int prec, bool geo, int nm, bool pm, bool dm) {
  return cycle_kernel(v, prec, geo, nm, pm, dm) != nullptr;
}

hipError_t launch_cycle(int v, int prec, bool geo, int nm, bool pm, bool dm, const Inst* insts,
                        const TileRef* sched, int nsched, int grid, hipStream_t st) {
  CycleFn f = cycle_kernel(v, prec, geo, nm, pm, dm);
  if (!f) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f, dim3(grid), dim3(kShapes[v][2]), 0, st, insts, sched, nsched);
  return hipGetLastError();
}

// End of a cycle, one workgroup per instance: the Courant minimum over the
// instance's tiles, then time, cycle count, next step (growth cap, maximum,
// stop time) and sticky errors (Sec. 7). The clock is read while the tile
// minima load (eight per thread in flight at a time), so the kernel costs
// about two memory round trips.
constexpr int kFinalizeThreads = 256;

__global__ __launch_bounds__(kFinalizeThreads) void k_finalize(const Inst* __restrict__ insts) {
  using CInst = const __attribute__((address_space(4))) Inst;
  const Inst& in = *(const Inst*)((CInst*)insts + blockIdx.x);
  Scal* sc = in.sc;
  const int tid = threadIdx.x;
  double t0 = 0.0, dt0 = 0.0;
  unsigned fl = 0;
  int err = 0;
  if (tid == 0) {
    t0 = sc->t;
    dt0 = sc->dt;
    fl = sc->flags;
    err = sc->err;
  }
  // the tile minima in batches of eight loads in flight (from a clamped
  // index; the minimum takes them in the order of a plain strided loop)
  double m = __builtin_huge_val();
  for (int q0 = tid; q0 < in.ntiles; q0 += 8 * kFinalizeThreads) {
    double v[8];
#pragma unroll
    for (int r = 0; r < 8; r++) v[r] = in.dtpart[min(q0 + r * kFinalizeThreads, in.ntiles - 1)];
#pragma unroll
    for (int r = 0; r < 8; r++)
      if (q0 + r * kFinalizeThreads < in.ntiles) m = dmin(m, v[r]);
  }
  for (int off = 32; off > 0; off >>= 1) m = dmin(m, __shfl_down(m, off, 64));
  __shared__ double part[kFinalizeThreads / 64];
  if ((tid & 63) == 0) part[tid >> 6] = m;
  __syncthreads();
  if (tid != 0 || err) return;
  for (int q = 1; q < kFinalizeThreads / 64; q++) m = dmin(m, part[q]);
  m = dmin(m, part[0]);
  const Geo& g = in.g;
  double t = t0 + dt0;
  sc->t = t;
  sc->cycle = sc->cycle + 1;
  double dtn = dmin(dmin(m, g.dt_grow * dt0), g.dt_max);
  if (g.t_stop > 0) dtn = dmin(dtn, dmax(g.t_stop - t, 0.0));
  sc->dt_prev = dt0;
  sc->dt = dtn;
  int e = 0;
  if (fl & kFlagNonFinite) e = -4;
  else if (fl & kFlagNegMass) e = -5;
  bool stopped = g.t_stop > 0 && t >= g.t_stop;
  if (e == 0 && !stopped && dtn < g.dt_floor) e = -6;
  if (e) {
    sc->err = e;
    sc->err_cycle = (int)sc->cycle;
  }
}

hipError_t launch_finalize(const Inst* insts, int n_inst, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3(n_inst), dim3(kFinalizeThreads), 0, st, insts);
  return hipGetLastError();
}

int resident_groups(int v, int prec, bool geo, int nm, bool pm, bool dm) {
  CycleFn f = cycle_kernel(v, prec, geo, nm, pm, dm);
  int per_cu = 0, cus = 0, dev = 0;
  if (!f || hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)f, kShapes[v][2], 0) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_prime(const Inst& in, hipStream_t st) {
  return in.g.prec == 0 ? launch_prime_f64(in, st) : launch_prime_f32(in, st);
}

}  // namespace salec
