// salec_kernels.hip -- set-up, output and diagnostic kernels of one instance
// of the r-z SALE scheme with PML (Li et al., SALEc-2D): the impact scene of
// Sec. 4 (target half-space, spherical projectile), the start of a run, the
// EoS of the current state for output, and compensated conservation totals.
// The per-cycle grid update is the cycle kernel (salec_cycle.hpp).
#include "salec_device.hpp"
#include "salec_internal.hpp"

namespace salec {

namespace {

__device__ __forceinline__ bool cell_of(const Geo& g, int& i, int& j) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.NR * g.NZ) return false;
  j = (int)(t / g.NR);
  i = (int)(t - (long long)j * g.NR);
  return true;
}

__device__ __forceinline__ bool node_of(const Geo& g, int& i, int& j) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)(g.NR + 1) * (g.NZ + 1)) return false;
  j = (int)(t / (g.NR + 1));
  i = (int)(t - (long long)j * (g.NR + 1));
  return true;
}

inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

// ======================================================================
// scene set-up: target half-space, spherical projectile, momentum-exact
// node velocities (state level 0)
// ======================================================================
template <class T>
__global__ void k_scene_cells(Inst in, int surface_j, int layer_j, int layer2_j, int S, double R, double zc,
                              const double* rho_row, double* fproj) {
  const Geo& g = in.g;
  const State& S0 = in.S[0];
  int i, j;
  if (!cell_of(g, i, j)) return;
  long long c = cidx(g, i, j);
  double num = 0.0, den = 0.0;
  const Col<double> cg = col_of<double>(g, in.geo, i);
  const double zj = zn_of(g, in.geo, j), dzj = dz_of(g, in.geo, j);
  for (int l = 0; l < S; l++) {
    double zl = zj + (((double)l + 0.5) / (double)S) * dzj;
    for (int k = 0; k < S; k++) {
      double rk = cg.rw + (((double)k + 0.5) / (double)S) * cg.dr;
      double dzl = zl - zc;
      if (rk * rk + dzl * dzl <= R * R) num += rk;
      den += rk;
    }
  }
  double fp = R > 0.0 ? num / den : 0.0;
  int mp = g.nmat - 1;  // the projectile: the last material
  double f[kMaxMat] = {0.0, 0.0, 0.0};
  double rho;
  if (j < surface_j) {  // target row: the layer's material (the last one is the deepest)
    const int mt = g.nmat == 3 && j < layer2_j ? 2 : (g.nmat > 1 && j < layer_j ? 1 : 0);
    f[mt] = 1.0;
    rho = rho_row ? rho_row[j] : g.m[mt].rho0;
  } else {
    f[mp] = fp;
    rho = fp * g.m[mp].rho0;
  }
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) S0.f[m][c] = f[m];
  S0.rho[c] = rho;
  S0.I[c] = 0.0;
  if (g.closure) {  // per-material closure: each cell holds one material's mass
    const int own = j < surface_j ? (g.nmat == 3 && j < layer2_j ? 2 : (g.nmat > 1 && j < layer_j ? 1 : 0)) : mp;
    for (int m = 0; m < g.nmat; m++) {
      S0.mu[m][c] = m == own ? rho : 0.0;
      S0.Im[m][c] = 0.0;
    }
  }
  if (g.any_strength)
    for (int k = 0; k < 3; k++) ((T*)S0.s[k])[c] = T(0);
  fproj[c] = fp;
}

template <class T>
__global__ void k_scene_nodes(Inst in, const double* fproj, double v_imp) {
  const Geo& g = in.g;
  const State& S0 = in.S[0];
  int i, j;
  if (!node_of(g, i, j)) return;
  int mp = g.nmat - 1;  // the projectile: the last material
  double Mt = 0.0, Mp = 0.0;
  const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
  for (int q = 0; q < 4; q++) {
    if (qi[q] < 0 || qi[q] >= g.NR || qj[q] < 0 || qj[q] >= g.NZ) continue;
    long long c = cidx(g, qi[q], qj[q]);
    double V = col_of<double>(g, in.geo, qi[q]).az * dz_of(g, in.geo, qj[q]);
    Mt += S0.rho[c] * V;
    Mp += fproj[c] * g.m[mp].rho0 * V;
  }
  double vr = 0.0, vz = Mt > 0.0 ? -v_imp * (Mp / Mt) : 0.0;
  if (i == 0 || i == g.NR) vr = 0.0;
  if (j == 0) {
    vr = 0.0;
    vz = 0.0;
  }
  if (g.top_closed && j == g.NZ) vz = 0.0;
  long long n = nidx(g, i, j);
  ((T*)S0.v[0])[n] = (T)vr;
  ((T*)S0.v[1])[n] = (T)vz;
}

// start of a run (state in level 0, PML auxiliaries and budgets already
// cleared): PML reference density = current density, clock reset
__global__ void k_start_run(Inst in) {
  const Geo& g = in.g;
  Scal* sc = in.sc;
  const Pml& pm = in.pm;
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nb = (long long)g.pml_b * g.NR, nu = nb + (long long)g.n_z * g.pml_r;
  if (t == 0) {
    sc->t = 0.0;
    sc->dt = 0.0;
    sc->dt_prev = 0.0;
    sc->cycle = 0;
    sc->dtmin = 0x7FF0000000000000ull;
    sc->flags = 0;
    sc->pad = 0;
    sc->err = 0;
    sc->err_cycle = -1;
  }
  if (!g.pml_on || t >= nu) return;
  int i, j;
  if (t < nb) {
    j = (int)(t / g.NR);
    i = (int)(t - (long long)j * g.NR);
  } else {
    long long u = t - nb;
    j = g.pml_b + (int)(u / g.pml_r);
    i = g.n_r + (int)(u - (long long)(j - g.pml_b) * g.pml_r);
  }
  pm.rref[t] = in.S[0].rho[cidx(g, i, j)];
}

// first step of a run: the Courant minimum with no growth cap
__global__ void k_finalize0(Inst in) {
  const Geo& g = in.g;
  Scal* sc = in.sc;
  double dt = dmin(__longlong_as_double((long long)sc->dtmin), g.dt_max);
  if (g.t_stop > 0) dt = dmin(dt, g.t_stop);
  sc->dt = dt;
  sc->dt_prev = 0.0;
  sc->dtmin = 0x7FF0000000000000ull;
}

// EoS of the current state (outputs only)
template <class T>
__global__ void k_eos_out(Inst in, double* p, double* c2) {
  const Geo& g = in.g;
  int i, j;
  if (!cell_of(g, i, j)) return;
  const State& S = in.S[in.sc->cycle & 1];
  long long c = cidx(g, i, j);
  double f[kMaxMat];
  for (int m = 0; m < kMaxMat; m++) f[m] = m < g.nmat ? S.f[m][c] : 0.0;
  Mix<T> mx;
  if (g.closure) {
    double mu[kMaxMat], Im[kMaxMat];
    T pmv[kMaxMat];
    for (int m = 0; m < kMaxMat; m++) {
      mu[m] = m < g.nmat ? S.mu[m][c] : 0.0;
      Im[m] = m < g.nmat ? S.Im[m][c] : 0.0;
    }
    mx = mixture_pm<T>(g, S.rho[c], f, mu, Im, pmv);
  } else {
    mx = mixture<T>(g, S.rho[c], S.I[c], f);
  }
  p[c] = (double)mx.p;
  c2[c] = (double)mx.c2;
}

// ======================================================================
// diagnostics: compensated totals in a fixed reduction tree
// ======================================================================
struct KS {
  double s, c;
};
__device__ __forceinline__ void ks_add(KS& k, double v) {
  double t = k.s + v;
  if (fabs(k.s) >= fabs(v)) k.c += (k.s - t) + v;
  else k.c += (v - t) + k.s;
  k.s = t;
}
__device__ __forceinline__ KS ks_merge(KS a, KS b) {
  KS r = a;
  ks_add(r, b.s);
  r.c += b.c;
  return r;
}

template <class T>
__global__ void k_diag_partial(Inst in, long long n_pml, double* red) {
  const Geo& g = in.g;
  const State& S = in.S[in.sc->cycle & 1];
  const T* v0 = (const T*)S.v[0];
  const T* v1 = (const T*)S.v[1];
  KS acc[kDiagQ];
  for (int q = 0; q < kDiagQ; q++) acc[q] = {0.0, 0.0};
  long long ncell = (long long)g.NR * g.NZ, nnode = (long long)(g.NR + 1) * (g.NZ + 1);
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += stride) {
    int j = (int)(t / g.NR), i = (int)(t - (long long)j * g.NR);
    long long c = cidx(g, i, j);
    double M = S.rho[c] * (col_of<double>(g, in.geo, i).az * dz_of(g, in.geo, j));
    ks_add(acc[0], M);
    ks_add(acc[1], M * S.I[c]);
  }
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nnode; t += stride) {
    int j = (int)(t / (g.NR + 1)), i = (int)(t - (long long)j * (g.NR + 1));
    double Mq[4] = {0, 0, 0, 0};
    const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
    for (int q = 0; q < 4; q++) {
      if (qi[q] < 0 || qi[q] >= g.NR || qj[q] < 0 || qj[q] >= g.NZ) continue;
      Mq[q] = S.rho[cidx(g, qi[q], qj[q])] * (col_of<double>(g, in.geo, qi[q]).az * dz_of(g, in.geo, qj[q]));
    }
    double M = 0.25 * ((Mq[0] + Mq[1]) + (Mq[2] + Mq[3]));
    long long n = nidx(g, i, j);
    double a = (double)v0[n], b = (double)v1[n];
    ks_add(acc[2], 0.5 * M * (a * a + b * b));
  }
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < g.NR; t += stride) {
    ks_add(acc[3], in.mout[t]);
    ks_add(acc[5], in.eout[t]);
  }
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n_pml; t += stride)
    ks_add(acc[4], in.pm.msink[t]);
  __shared__ double sh[256 * 2];
  for (int q = 0; q < kDiagQ; q++) {
    sh[2 * threadIdx.x] = acc[q].s;
    sh[2 * threadIdx.x + 1] = acc[q].c;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        KS a{sh[2 * threadIdx.x], sh[2 * threadIdx.x + 1]};
        KS b{sh[2 * (threadIdx.x + off)], sh[2 * (threadIdx.x + off) + 1]};
        KS r = ks_merge(a, b);
        sh[2 * threadIdx.x] = r.s;
        sh[2 * threadIdx.x + 1] = r.c;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      red[(blockIdx.x * kDiagQ + q) * 2] = sh[0];
      red[(blockIdx.x * kDiagQ + q) * 2 + 1] = sh[1];
    }
    __syncthreads();
  }
}

__global__ void k_diag_final(const double* red, int nblocks, double* out) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < kDiagQ; q++) {
    KS a{0.0, 0.0};
    for (int b = 0; b < nblocks; b++) a = ks_merge(a, KS{red[(b * kDiagQ + q) * 2], red[(b * kDiagQ + q) * 2 + 1]});
    out[q] = a.s + a.c;
  }
}

// ======================================================================
// launchers
// ======================================================================
hipError_t launch_scene(const Inst& in, int surface_j, int layer_j, int layer2_j, int S, double R, double zc,
                        double v_imp, const double* rho_row, double* scratch, hipStream_t st) {
  const int bs = 256;
  long long nc = (long long)in.g.NR * in.g.NZ, nn = (long long)(in.g.NR + 1) * (in.g.NZ + 1);
  if (in.g.prec == 0) {
    hipLaunchKernelGGL(k_scene_cells<double>, dim3(nblk(nc, bs)), dim3(bs), 0, st, in, surface_j, layer_j, layer2_j, S, R, zc,
                       rho_row, scratch);
    hipLaunchKernelGGL(k_scene_nodes<double>, dim3(nblk(nn, bs)), dim3(bs), 0, st, in, scratch, v_imp);
  } else {
    hipLaunchKernelGGL(k_scene_cells<float>, dim3(nblk(nc, bs)), dim3(bs), 0, st, in, surface_j, layer_j, layer2_j, S, R, zc,
                       rho_row, scratch);
    hipLaunchKernelGGL(k_scene_nodes<float>, dim3(nblk(nn, bs)), dim3(bs), 0, st, in, scratch, v_imp);
  }
  return hipGetLastError();
}

hipError_t launch_start_run(const Inst& in, hipStream_t st) {
  long long nu = (long long)in.g.pml_b * in.g.NR + (long long)in.g.n_z * in.g.pml_r;
  if (nu < 1) nu = 1;
  hipLaunchKernelGGL(k_start_run, dim3(nblk(nu, 256)), dim3(256), 0, st, in);
  return hipGetLastError();
}

hipError_t launch_finalize0(const Inst& in, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize0, dim3(1), dim3(1), 0, st, in);
  return hipGetLastError();
}

hipError_t launch_eos_out(const Inst& in, double* p, double* c2, hipStream_t st) {
  const int bs = 256;
  long long nc = (long long)in.g.NR * in.g.NZ;
  if (in.g.prec == 0)
    hipLaunchKernelGGL(k_eos_out<double>, dim3(nblk(nc, bs)), dim3(bs), 0, st, in, p, c2);
  else
    hipLaunchKernelGGL(k_eos_out<float>, dim3(nblk(nc, bs)), dim3(bs), 0, st, in, p, c2);
  return hipGetLastError();
}

hipError_t launch_diag(const Inst& in, long long n_pml, double* red, double* out, hipStream_t st) {
  if (in.g.prec == 0)
    hipLaunchKernelGGL(k_diag_partial<double>, dim3(kDiagBlocks), dim3(256), 0, st, in, n_pml, red);
  else
    hipLaunchKernelGGL(k_diag_partial<float>, dim3(kDiagBlocks), dim3(256), 0, st, in, n_pml, red);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, red, (int)kDiagBlocks, out);
  return hipGetLastError();
}

}  // namespace salec
