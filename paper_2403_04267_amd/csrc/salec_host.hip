// salec_host.hip -- host runtime of libsalec: validation, layout of the
// caller's device buffer, scene set-up, HIP-graph capture and replay of the
// cycle, field I/O, checkpoints and diagnostics. Implements include/salec.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/salec.h"
#include "salec_internal.hpp"

using namespace salec;

namespace {

constexpr size_t kAlign = 256;
constexpr int kGraphCycles = 16;  // cycles per captured graph
constexpr uint64_t kStateMagic = 0x53414c4543535431ull;  // "SALECST1"

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's buffer (or a dry run for sizing).
struct Carver {
  uint8_t* base;
  size_t off = 0;
  explicit Carver(void* b) : base((uint8_t*)b) {}
  double* d(size_t n) {
    size_t o = off;
    off = align_up(off + n * sizeof(double));
    return base ? (double*)(base + o) : nullptr;
  }
  template <class T>
  T* obj() {
    size_t o = off;
    off = align_up(off + sizeof(T));
    return base ? (T*)(base + o) : nullptr;
  }
};

struct Layout {
  Scal* sc = nullptr;
  State S[2];
  Pml pm{};
  Work w{};
  double* diag_out = nullptr;
  size_t aux_off = 0;        // [aux_off, persist_bytes): PML auxiliaries and budgets
  size_t persist_bytes = 0;  // [0, persist_bytes): checkpointed region
  size_t total = 0;
  long long n_pml = 0;
};

void carve(const Geo& g, void* base, Layout& L) {
  Carver cv(base);
  long long nc = (long long)g.NZ * g.pc, nn = (long long)(g.NZ + 1) * g.pn;
  // persistent region: scalars, both state copies, PML auxiliaries, budgets
  L.sc = cv.obj<Scal>();
  for (int b = 0; b < 2; b++) {
    State& S = L.S[b];
    S.rho = cv.d(nc);
    S.I = cv.d(nc);
    for (int m = 0; m < kMaxMat; m++) S.f[m] = m < g.nmat ? cv.d(nc) : nullptr;
    for (int k = 0; k < 3; k++) S.s[k] = g.any_strength ? cv.d(nc) : nullptr;
    S.v[0] = cv.d(nn);
    S.v[1] = cv.d(nn);
  }
  L.aux_off = cv.off;
  long long nbc = (long long)g.pml_b * g.NR, nrc = (long long)g.NZ * g.pml_r;
  long long nbn = (long long)g.pml_b * (g.NR + 1), nrn = (long long)(g.NZ + 1) * g.pml_r;
  long long nu = nbc + (long long)g.n_z * g.pml_r;
  L.n_pml = g.pml_on ? nu : 0;
  Pml& pm = L.pm;
  auto opt = [&](long long n) { return (g.pml_on && n > 0) ? cv.d((size_t)n) : nullptr; };
  pm.rref = opt(nu);
  pm.msink = opt(nu);
  for (int lv = 0; lv < 2; lv++) {
    PmlAux& a = pm.a[lv];
    a.b_phi1 = opt(nbc);
    a.b_phi3 = opt(nbc);
    a.b_psi2 = opt(nbc);
    a.r_phi1 = opt(nrc);
    a.r_phi3 = opt(nrc);
    a.r_psi2 = opt(nrc);
    a.b_phi2r = opt(nbn);
    a.b_phi2z = opt(nbn);
    a.b_psi1r = opt(nbn);
    a.b_psi1z = opt(nbn);
    a.r_phi2r = opt(nrn);
    a.r_phi2z = opt(nrn);
    a.r_psi1r = opt(nrn);
    a.r_psi1z = opt(nrn);
  }
  L.w.mout = cv.d(g.pc);
  L.w.eout = cv.d(g.pc);
  L.persist_bytes = cv.off;
  // constants
  pm.dcz = cv.d(g.NZ);
  pm.dnz = cv.d(g.NZ + 1);
  pm.dcr = cv.d(g.NR);
  pm.dnr = cv.d(g.NR + 1);
  // per-cycle scratch
  Work& w = L.w;
  for (int k = 0; k < 4; k++) w.sg[k] = cv.d(nc);
  w.p = cv.d(nc);
  w.Q = cv.d(nc);
  w.G = cv.d(nc);
  w.Y = cv.d(nc);
  w.rmat = cv.d(nc);
  w.phi = cv.d(nc);
  w.sx = cv.d(nc);
  w.vL[0] = cv.d(nn);
  w.vL[1] = cv.d(nn);
  w.J = cv.d(nc);
  w.IL = cv.d(nc);
  for (int k = 0; k < 3; k++) w.sL[k] = cv.d(nc);
  for (int m = 0; m < kMaxMat; m++) w.fL[m] = m < g.nmat ? cv.d(nc) : nullptr;
  w.lam = cv.d(nc);
  w.outv = cv.d(nc);
  w.Fr = cv.d((size_t)g.NZ * g.pn);
  w.Fz = cv.d((size_t)(g.NZ + 1) * g.pc);
  w.heat = cv.d(nn);
  w.red = cv.d((size_t)kDiagBlocks * 12);
  w.dtpart = cv.d((size_t)g.nblocks_fused + 1);
  L.diag_out = cv.d(8);
  L.total = cv.off;
}

int validate(const salec_grid* g, const salec_material* mats, const salec_pml* pml, std::string& why) {
  if (!g || !mats || !pml) return why = "null argument", SALEC_E_INVALID;
  if (g->n_r < 1 || g->n_z < 1 || g->pml_r < 0 || g->pml_b < 0) return why = "grid sizes", SALEC_E_INVALID;
  if ((long long)(g->n_r + g->pml_r + 1) * (g->n_z + g->pml_b + 1) > (1ll << 31))
    return why = "grid too large for one context", SALEC_E_INVALID;
  if (g->nmat < 1 || g->nmat > SALEC_MAX_MAT) return why = "nmat must be 1 or 2", SALEC_E_INVALID;
  if (g->precision != SALEC_FP64) return why = "only SALEC_FP64 is implemented", SALEC_E_INVALID;
  if (!(g->dr > 0) || !(g->dz > 0)) return why = "cell size must be > 0", SALEC_E_INVALID;
  if (!(g->cfl > 0) || g->cfl > 1.0) return why = "cfl must be in (0, 1]", SALEC_E_INVALID;
  if (!(g->dt_grow >= 1.0) || !(g->dt_max > 0) || g->dt_floor < 0 || g->q_lin < 0 || g->q_quad < 0)
    return why = "time-step or viscosity parameters", SALEC_E_INVALID;
  for (int m = 0; m < g->nmat; m++) {
    const salec_material& M = mats[m];
    if (!(M.rho0 > 0) || !(M.E0 > 0) || !(M.Ecv > M.Eiv) || M.A < 0 || M.B < 0 || M.c_floor_frac < 0)
      return why = "Tillotson parameters of material " + std::to_string(m), SALEC_E_INVALID;
    if (M.strength && (!(M.Ylim > M.Y0) || M.Y0 < 0 || M.mu_f < 0 || !(M.poisson > -1.0 && M.poisson < 0.5)))
      return why = "strength parameters of material " + std::to_string(m), SALEC_E_INVALID;
  }
  if (pml->enabled && !(pml->R > 0 && pml->R < 1)) return why = "PML reflection coefficient", SALEC_E_INVALID;
  return SALEC_OK;
}

Geo make_geo(const salec_grid* gr, const salec_material* mats, const salec_pml* pml) {
  Geo g{};
  std::memset(&g, 0, sizeof(g));
  g.n_r = gr->n_r;
  g.n_z = gr->n_z;
  g.pml_r = gr->pml_r;
  g.pml_b = gr->pml_b;
  g.NR = gr->n_r + gr->pml_r;
  g.NZ = gr->n_z + gr->pml_b;
  g.nmat = gr->nmat;
  g.top_closed = gr->top_closed;
  g.pc = (int)((g.NR + 31) / 32 * 32);
  g.pn = (int)((g.NR + 1 + 31) / 32 * 32);
  g.pml_on = pml->enabled ? 1 : 0;
  {
    int tr, tz;
    fused_tiles(g.NR, g.NZ, &tr, &tz);
    g.nblocks_fused = tr * tz;
  }
  g.dr = gr->dr;
  g.dz = gr->dz;
  g.cfl = gr->cfl;
  g.dt_grow = gr->dt_grow;
  g.dt_max = gr->dt_max;
  g.dt_floor = gr->dt_floor;
  g.t_stop = gr->t_stop;
  g.q_lin = gr->q_lin;
  g.q_quad = gr->q_quad;
  g.rho_ref = 0.0;
  for (int m = 0; m < gr->nmat; m++) {
    const salec_material& M = mats[m];
    MatC& c = g.m[m];
    c.rho0 = M.rho0;
    c.A = M.A;
    c.B = M.B;
    c.E0 = M.E0;
    c.a = M.a;
    c.b = M.b;
    c.alpha = M.alpha;
    c.beta = M.beta;
    c.Eiv = M.Eiv;
    c.Ecv = M.Ecv;
    c.p_min = M.p_min;
    c.cf2 = M.c_floor_frac * M.A / M.rho0;
    c.strength = M.strength ? 1 : 0;
    c.gfac = M.strength ? 3.0 * (1.0 - 2.0 * M.poisson) / (2.0 * (1.0 + M.poisson)) : 0.0;
    c.Y0 = M.Y0;
    c.mu_f = M.mu_f;
    c.Ylim = M.Ylim;
    c.pcav = kPcavFrac * M.A;
    if (M.strength) g.any_strength = 1;
    if (M.rho0 > g.rho_ref) g.rho_ref = M.rho0;
  }
  g.same_mat = 1;
  for (int m = 1; m < gr->nmat; m++)
    if (std::memcmp(&g.m[m], &g.m[0], sizeof(MatC)) != 0) g.same_mat = 0;
  return g;
}

// damping profile d(y) = (3c / 2 delta) (y / delta)^2 log(1/R)  (Sec. 3)
double pml_d(double c, double delta, double y, double R) { return 1.5 * c / delta * (y / delta) * (y / delta) * std::log(1.0 / R); }

void pml_profiles(const Geo& g, const salec_material* mats, const salec_pml* pml, std::vector<double>& dcz,
                  std::vector<double>& dnz, std::vector<double>& dcr, std::vector<double>& dnr) {
  dcz.assign(g.NZ, 0.0);
  dnz.assign(g.NZ + 1, 0.0);
  dcr.assign(g.NR, 0.0);
  dnr.assign(g.NR + 1, 0.0);
  if (!pml->enabled) return;
  double c = pml->c_ref;
  if (!(c > 0)) {
    const salec_material& m0 = mats[0];
    double G0 = m0.strength ? 3.0 * m0.A * (1.0 - 2.0 * m0.poisson) / (2.0 * (1.0 + m0.poisson)) : 0.0;
    c = std::sqrt((m0.A + (4.0 / 3.0) * G0) / m0.rho0);
  }
  if (g.pml_b > 0) {
    double delta = g.pml_b * g.dz;
    for (int j = 0; j < g.pml_b; j++) dcz[j] = pml_d(c, delta, ((double)(g.pml_b - j) - 0.5) * g.dz, pml->R);
    for (int j = 0; j < g.pml_b; j++) dnz[j] = pml_d(c, delta, (double)(g.pml_b - j) * g.dz, pml->R);
  }
  if (g.pml_r > 0) {
    double delta = g.pml_r * g.dr;
    for (int i = g.n_r; i < g.NR; i++) dcr[i] = pml_d(c, delta, ((double)(i - g.n_r) + 0.5) * g.dr, pml->R);
    for (int i = g.n_r + 1; i <= g.NR; i++) dnr[i] = pml_d(c, delta, (double)(i - g.n_r) * g.dr, pml->R);
  }
}

}  // namespace

struct salec_ctx {
  Geo g{};
  Layout L;
  void* buf = nullptr;
  hipStream_t st = nullptr;
  bool own_stream = false;
  hipGraphExec_t gx1 = nullptr, gxN = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  bool phased = false;  // one kernel per phase instead of the fused cycle
  std::string err;
};

namespace {

int hip_fail(salec_ctx* x, hipError_t e, const char* where) {
  if (x) x->err = std::string(where) + ": " + hipGetErrorString(e);
  return SALEC_E_HIP;
}
#define HIPCHK(x, call)                                      \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail((x), e_, #call); \
  } while (0)

// Clears PML auxiliaries and budgets, sets the PML reference density and the
// clock, and computes the first time step; the state is in copy 0.
int start_run(salec_ctx* x) {
  Layout& L = x->L;
  uint8_t* base = (uint8_t*)L.sc;
  if (L.persist_bytes > L.aux_off)
    HIPCHK(x, hipMemsetAsync(base + L.aux_off, 0, L.persist_bytes - L.aux_off, x->st));
  launch_start_run(x->g, L.S[0], L.pm, L.sc, x->st);
  launch_dt0(x->g, L.S[0], L.S[1], L.sc, x->st);
  HIPCHK(x, hipGetLastError());
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int capture(salec_ctx* x, int ncyc, hipGraphExec_t* out) {
  hipGraph_t gr = nullptr;
  HIPCHK(x, hipStreamBeginCapture(x->st, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < ncyc; k++) {
    if (x->phased)
      launch_cycle(x->g, x->L.S[0], x->L.S[1], x->L.w, x->L.pm, x->L.sc, x->st);
    else
      launch_cycle_fused(x->g, x->L.S[0], x->L.S[1], x->L.w, x->L.pm, x->L.sc, x->st);
  }
  hipError_t e = hipStreamEndCapture(x->st, &gr);
  if (e != hipSuccess) return hip_fail(x, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return hip_fail(x, e, "hipGraphInstantiate");
  return SALEC_OK;
}

Scal read_scal(salec_ctx* x) {
  Scal s{};
  (void)hipMemcpyAsync(&s, x->L.sc, sizeof(Scal), hipMemcpyDeviceToHost, x->st);
  (void)hipStreamSynchronize(x->st);
  return s;
}

const State& current(salec_ctx* x, const Scal& s) { return (s.cycle & 1) ? x->L.S[1] : x->L.S[0]; }

int copy_cells_out(salec_ctx* x, double* host, const double* dev) {
  const Geo& g = x->g;
  HIPCHK(x, hipMemcpy2DAsync(host, g.NR * sizeof(double), dev, g.pc * sizeof(double), g.NR * sizeof(double), g.NZ,
                             hipMemcpyDeviceToHost, x->st));
  return SALEC_OK;
}
int copy_nodes_out(salec_ctx* x, double* host, const double* dev) {
  const Geo& g = x->g;
  HIPCHK(x, hipMemcpy2DAsync(host, (g.NR + 1) * sizeof(double), dev, g.pn * sizeof(double),
                             (g.NR + 1) * sizeof(double), g.NZ + 1, hipMemcpyDeviceToHost, x->st));
  return SALEC_OK;
}
int copy_cells_in(salec_ctx* x, double* dev, const double* host) {
  const Geo& g = x->g;
  HIPCHK(x, hipMemcpy2DAsync(dev, g.pc * sizeof(double), host, g.NR * sizeof(double), g.NR * sizeof(double), g.NZ,
                             hipMemcpyHostToDevice, x->st));
  return SALEC_OK;
}
int copy_nodes_in(salec_ctx* x, double* dev, const double* host) {
  const Geo& g = x->g;
  HIPCHK(x, hipMemcpy2DAsync(dev, g.pn * sizeof(double), host, (g.NR + 1) * sizeof(double),
                             (g.NR + 1) * sizeof(double), g.NZ + 1, hipMemcpyHostToDevice, x->st));
  return SALEC_OK;
}

}  // namespace

extern "C" {

size_t salec_plan(const salec_grid* grid, const salec_material* mats, const salec_pml* pml) {
  std::string why;
  if (validate(grid, mats, pml, why) != SALEC_OK) return 0;
  Geo g = make_geo(grid, mats, pml);
  Layout L;
  carve(g, nullptr, L);
  return L.total;
}

int salec_init(const salec_grid* grid, const salec_material* mats, const salec_pml* pml, const salec_scene* scene,
               void* dev_buf, size_t dev_bytes, void* stream, salec_ctx** out) {
  if (!out) return SALEC_E_INVALID;
  *out = nullptr;
  salec_ctx* x = new salec_ctx();
  int rc = validate(grid, mats, pml, x->err);
  if (rc == SALEC_OK && scene && (scene->subsample < 1 || !(scene->radius > 0))) {
    x->err = "scene parameters";
    rc = SALEC_E_INVALID;
  }
  if (rc != SALEC_OK) {
    *out = x;  // keep the message reachable through salec_last_error
    return rc;
  }
  x->g = make_geo(grid, mats, pml);
  Layout probe;
  carve(x->g, nullptr, probe);
  if (!dev_buf || dev_bytes < probe.total || ((uintptr_t)dev_buf % kAlign) != 0) {
    x->err = "device buffer smaller than salec_plan() or not 256-byte aligned";
    *out = x;
    return SALEC_E_BUFFER;
  }
  x->buf = dev_buf;
  carve(x->g, dev_buf, x->L);
  {
    const char* pe = std::getenv("SALEC_PIPELINE");
    x->phased = pe && std::strcmp(pe, "phased") == 0;
  }
  if (stream) {
    x->st = (hipStream_t)stream;
  } else {
    hipError_t e = hipStreamCreate(&x->st);
    if (e != hipSuccess) {
      *out = x;
      return hip_fail(x, e, "hipStreamCreate");
    }
    x->own_stream = true;
  }
  *out = x;
  HIPCHK(x, hipEventCreate(&x->ev0));
  HIPCHK(x, hipEventCreate(&x->ev1));
  HIPCHK(x, hipMemsetAsync(dev_buf, 0, x->L.total, x->st));
  std::vector<double> dcz, dnz, dcr, dnr;
  pml_profiles(x->g, mats, pml, dcz, dnz, dcr, dnr);
  HIPCHK(x, hipMemcpyAsync((void*)x->L.pm.dcz, dcz.data(), dcz.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipMemcpyAsync((void*)x->L.pm.dnz, dnz.data(), dnz.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipMemcpyAsync((void*)x->L.pm.dcr, dcr.data(), dcr.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipMemcpyAsync((void*)x->L.pm.dnr, dnr.data(), dnr.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
  if (scene) {
    double zc = (double)scene->surface_j * x->g.dz + scene->radius;
    launch_scene(x->g, x->L.S[0], x->L.w, scene->surface_j, scene->subsample, scene->radius, zc, scene->v_imp, x->st);
    HIPCHK(x, hipGetLastError());
  }
  HIPCHK(x, hipStreamSynchronize(x->st));  // host vectors above go out of scope
  rc = start_run(x);
  if (rc) return rc;
  rc = capture(x, 1, &x->gx1);
  if (rc) return rc;
  rc = capture(x, kGraphCycles, &x->gxN);
  if (rc) return rc;
  return SALEC_OK;
}

int salec_enqueue(salec_ctx* x, int32_t n) {
  if (!x || n < 0 || !x->gx1) return SALEC_E_INVALID;
  int32_t big = n / kGraphCycles, rem = n % kGraphCycles;
  for (int32_t k = 0; k < big; k++) HIPCHK(x, hipGraphLaunch(x->gxN, x->st));
  for (int32_t k = 0; k < rem; k++) HIPCHK(x, hipGraphLaunch(x->gx1, x->st));
  return SALEC_OK;
}

int salec_step(salec_ctx* x, int32_t n) {
  if (!x || n < 0 || !x->gx1) return SALEC_E_INVALID;
  HIPCHK(x, hipEventRecord(x->ev0, x->st));
  int rc = salec_enqueue(x, n);
  if (rc) return rc;
  HIPCHK(x, hipEventRecord(x->ev1, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  float ms = 0.0f;
  HIPCHK(x, hipEventElapsedTime(&ms, x->ev0, x->ev1));
  x->last_ms = ms;
  Scal s = read_scal(x);
  if (s.err) {
    x->err = "device error " + std::to_string(s.err) + " at cycle " + std::to_string(s.err_cycle);
    return s.err;
  }
  return SALEC_OK;
}

int salec_last_step_ms(salec_ctx* x, double* ms) {
  if (!x || !ms) return SALEC_E_INVALID;
  *ms = x->last_ms;
  return SALEC_OK;
}

int salec_get_fields(salec_ctx* x, const salec_fields* o) {
  if (!x || !o || !x->gx1) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  Scal s = read_scal(x);
  const State& S = current(x, s);
  const Geo& g = x->g;
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1);
  int rc = SALEC_OK;
  if (o->rho && (rc = copy_cells_out(x, o->rho, S.rho))) return rc;
  if (o->I && (rc = copy_cells_out(x, o->I, S.I))) return rc;
  if (o->f)
    for (int m = 0; m < g.nmat; m++)
      if ((rc = copy_cells_out(x, o->f + m * NC, S.f[m]))) return rc;
  if (o->s) {
    if (g.any_strength) {
      for (int k = 0; k < 3; k++)
        if ((rc = copy_cells_out(x, o->s + k * NC, S.s[k]))) return rc;
    } else {
      std::memset(o->s, 0, 3 * NC * sizeof(double));
    }
  }
  if (o->v) {
    if ((rc = copy_nodes_out(x, o->v, S.v[0]))) return rc;
    if ((rc = copy_nodes_out(x, o->v + NN, S.v[1]))) return rc;
  }
  if (o->p || o->c2) {
    launch_eos_out(g, x->L.S[0], x->L.S[1], x->L.sc, x->L.w.sg[0], x->L.w.sg[1], x->st);
    HIPCHK(x, hipGetLastError());
    if (o->p && (rc = copy_cells_out(x, o->p, x->L.w.sg[0]))) return rc;
    if (o->c2 && (rc = copy_cells_out(x, o->c2, x->L.w.sg[1]))) return rc;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int salec_set_fields(salec_ctx* x, const salec_fields* in) {
  if (!x || !in || !in->rho || !in->I || !in->f || !in->v || !x->gx1) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  const Geo& g = x->g;
  const State& S = x->L.S[0];
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1);
  int rc;
  if ((rc = copy_cells_in(x, S.rho, in->rho))) return rc;
  if ((rc = copy_cells_in(x, S.I, in->I))) return rc;
  for (int m = 0; m < g.nmat; m++)
    if ((rc = copy_cells_in(x, S.f[m], in->f + m * NC))) return rc;
  if (g.any_strength) {
    for (int k = 0; k < 3; k++) {
      if (in->s) {
        if ((rc = copy_cells_in(x, S.s[k], in->s + k * NC))) return rc;
      } else {
        HIPCHK(x, hipMemsetAsync(S.s[k], 0, (size_t)g.NZ * g.pc * sizeof(double), x->st));
      }
    }
  }
  if ((rc = copy_nodes_in(x, S.v[0], in->v))) return rc;
  if ((rc = copy_nodes_in(x, S.v[1], in->v + NN))) return rc;
  return start_run(x);
}

int salec_get_pml(salec_ctx* x, double* ca, double* na) {
  if (!x || !x->gx1) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  const Geo& g = x->g;
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1);
  const Pml& pm = x->L.pm;
  Scal sc_now = read_scal(x);
  const PmlAux& au = pm.a[sc_now.cycle & 1];
  auto fetch = [&](const double* dev, size_t n, std::vector<double>& h) -> int {
    h.assign(n, 0.0);
    if (dev && n) HIPCHK(x, hipMemcpy(h.data(), dev, n * sizeof(double), hipMemcpyDeviceToHost));
    return SALEC_OK;
  };
  size_t nbc = (size_t)g.pml_b * g.NR, nrc = (size_t)g.NZ * g.pml_r, nu = nbc + (size_t)g.n_z * g.pml_r;
  size_t nbn = (size_t)g.pml_b * (g.NR + 1), nrn = (size_t)(g.NZ + 1) * g.pml_r;
  if (ca) {
    std::memset(ca, 0, 8 * NC * sizeof(double));
    if (g.pml_on) {
      std::vector<double> h[8];
      const double* b[3] = {au.b_phi1, au.b_phi3, au.b_psi2};
      const double* r[3] = {au.r_phi1, au.r_phi3, au.r_psi2};
      for (int k = 0; k < 3; k++) {
        if (fetch(b[k], nbc, h[k]) || fetch(r[k], nrc, h[3 + k])) return SALEC_E_HIP;
      }
      if (fetch(pm.rref, nu, h[6]) || fetch(pm.msink, nu, h[7])) return SALEC_E_HIP;
      for (int j = 0; j < g.NZ; j++)
        for (int i = 0; i < g.NR; i++) {
          size_t c = (size_t)j * g.NR + i;
          if (j < g.pml_b)
            for (int k = 0; k < 3; k++) ca[k * NC + c] = h[k][(size_t)j * g.NR + i];
          if (i >= g.n_r)
            for (int k = 0; k < 3; k++) ca[(3 + k) * NC + c] = h[3 + k][(size_t)j * g.pml_r + (i - g.n_r)];
          long long u = -1;
          if (j < g.pml_b) u = (long long)j * g.NR + i;
          else if (i >= g.n_r) u = (long long)nbc + (long long)(j - g.pml_b) * g.pml_r + (i - g.n_r);
          if (u >= 0) {
            ca[6 * NC + c] = h[6][u];
            ca[7 * NC + c] = h[7][u];
          }
        }
    }
  }
  if (na) {
    std::memset(na, 0, 8 * NN * sizeof(double));
    if (g.pml_on) {
      std::vector<double> h[8];
      const double* b[4] = {au.b_phi2r, au.b_phi2z, au.b_psi1r, au.b_psi1z};
      const double* r[4] = {au.r_phi2r, au.r_phi2z, au.r_psi1r, au.r_psi1z};
      for (int k = 0; k < 4; k++)
        if (fetch(b[k], nbn, h[k]) || fetch(r[k], nrn, h[4 + k])) return SALEC_E_HIP;
      for (int j = 0; j <= g.NZ; j++)
        for (int i = 0; i <= g.NR; i++) {
          size_t n = (size_t)j * (g.NR + 1) + i;
          if (j < g.pml_b)
            for (int k = 0; k < 4; k++) na[k * NN + n] = h[k][(size_t)j * (g.NR + 1) + i];
          if (i > g.n_r)
            for (int k = 0; k < 4; k++) na[(4 + k) * NN + n] = h[4 + k][(size_t)j * g.pml_r + (i - g.n_r - 1)];
        }
    }
  }
  return SALEC_OK;
}

size_t salec_state_bytes(const salec_ctx* x) {
  if (!x || !x->gx1) return 0;
  return 16 + x->L.persist_bytes;
}

int salec_get_state(salec_ctx* x, void* blob, size_t bytes) {
  if (!x || !blob || !x->gx1) return SALEC_E_INVALID;
  if (bytes < salec_state_bytes(x)) return SALEC_E_BUFFER;
  HIPCHK(x, hipStreamSynchronize(x->st));
  uint64_t head[2] = {kStateMagic, (uint64_t)x->L.persist_bytes};
  std::memcpy(blob, head, 16);
  HIPCHK(x, hipMemcpy((uint8_t*)blob + 16, x->L.sc, x->L.persist_bytes, hipMemcpyDeviceToHost));
  return SALEC_OK;
}

int salec_set_state(salec_ctx* x, const void* blob, size_t bytes) {
  if (!x || !blob || !x->gx1) return SALEC_E_INVALID;
  if (bytes < salec_state_bytes(x)) return SALEC_E_BUFFER;
  uint64_t head[2];
  std::memcpy(head, blob, 16);
  if (head[0] != kStateMagic || head[1] != x->L.persist_bytes) {
    x->err = "state blob does not match this context";
    return SALEC_E_INVALID;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  HIPCHK(x, hipMemcpy(x->L.sc, (const uint8_t*)blob + 16, x->L.persist_bytes, hipMemcpyHostToDevice));
  return SALEC_OK;
}

int salec_diag(salec_ctx* x, salec_diag_t* out) {
  if (!x || !out || !x->gx1) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  launch_diag(x->g, x->L.S[0], x->L.S[1], x->L.w, x->L.pm, x->L.sc, x->L.n_pml, x->L.diag_out, x->st);
  HIPCHK(x, hipGetLastError());
  double q[6];
  HIPCHK(x, hipMemcpyAsync(q, x->L.diag_out, sizeof(q), hipMemcpyDeviceToHost, x->st));
  Scal s = read_scal(x);
  out->t = s.t;
  out->dt = s.dt;
  out->dt_prev = s.dt_prev;
  out->cycle = s.cycle;
  out->mass = q[0];
  out->ie = q[1];
  out->ke = q[2];
  out->mass_out = q[3];
  out->mass_pml = q[4];
  out->ie_out = q[5];
  out->err = s.err;
  out->err_cycle = s.err_cycle;
  return SALEC_OK;
}

const char* salec_last_error(const salec_ctx* x) { return x ? x->err.c_str() : "null context"; }

void salec_destroy(salec_ctx* x) {
  if (!x) return;
  if (x->st) (void)hipStreamSynchronize(x->st);
  if (x->gx1) (void)hipGraphExecDestroy(x->gx1);
  if (x->gxN) (void)hipGraphExecDestroy(x->gxN);
  if (x->ev0) (void)hipEventDestroy(x->ev0);
  if (x->ev1) (void)hipEventDestroy(x->ev1);
  if (x->own_stream && x->st) (void)hipStreamDestroy(x->st);
  delete x;
}

}  // extern "C"
