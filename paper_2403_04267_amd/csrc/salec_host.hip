// salec_host.hip -- host runtime of libsalec: validation, layout of the
// caller's device buffer for one impact or an ensemble, scene set-up, launch
// schedules and their tuner, HIP-graph capture and replay of the cycle, field
// I/O, checkpoints and diagnostics. Implements include/salec.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/salec.h"
#include "salec_internal.hpp"

using namespace salec;

namespace {

constexpr size_t kAlign = 256;
constexpr int kGraphCycles = 16;                         // cycles per captured graph
constexpr uint64_t kStateMagic = 0x53414c4543535432ull;  // "SALECST2"
constexpr int kXcds = 8;                                 // L2 domains the schedule groups tiles by

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator over the caller's buffer (or a dry run for sizing).
struct Carver {
  uint8_t* base;
  size_t off = 0;
  explicit Carver(void* b) : base((uint8_t*)b) {}
  void* bytes(size_t n) {
    size_t o = off;
    off = align_up(off + n);
    return base ? (void*)(base + o) : nullptr;
  }
  double* d(size_t n) { return (double*)bytes(n * sizeof(double)); }
  template <class T>
  T* obj(size_t n = 1) {
    return (T*)bytes(n * sizeof(T));
  }
};

// Host view of one member: its constants, its device descriptor and the
// byte range of its persistent (checkpointed) state.
struct Member {
  Geo g{};
  Inst d{};
  long long n_pml = 0;
  size_t aux_off = 0, aux_end = 0;  // PML auxiliaries and budgets (cleared at a run start)
  std::vector<double> dcz, dnz, dcr, dnr;
  std::vector<double> p0;  // initial pressure per cell row (host copy)
  // geometry: node / centre radii, widths, half-column areas, area per unit
  // height; node / centre heights, row heights
  std::vector<double> rn, rcn, drc, awc, aec, azc, zn, zcn, dzr;
  salec_scene scene{};
  bool has_scene = false;
};

// Grid geometry of a member: uniform from dr, dz, or the running sums of a
// stretched grid's widths and heights with centres halfway.
void build_geometry(Member& mb, const salec_grid* gr) {
  const int NR = mb.g.NR, NZ = mb.g.NZ;
  mb.rn.assign(NR + 1, 0.0);
  mb.rcn.assign(NR, 0.0);
  mb.drc.assign(NR, 0.0);
  mb.awc.assign(NR, 0.0);
  mb.aec.assign(NR, 0.0);
  mb.azc.assign(NR, 0.0);
  mb.zn.assign(NZ + 1, 0.0);
  mb.zcn.assign(NZ, 0.0);
  mb.dzr.assign(NZ, 0.0);
  for (int i = 0; i < NR; i++) {
    double rw, re, rc, dr;
    if (gr->dr_col) {
      dr = gr->dr_col[i];
      rw = mb.rn[i];
      re = rw + dr;
      rc = rw + 0.5 * dr;
    } else {
      dr = gr->dr;
      rw = (double)i * dr;
      re = (double)(i + 1) * dr;
      rc = ((double)i + 0.5) * dr;
    }
    mb.rn[i] = rw;
    mb.rn[i + 1] = re;
    mb.rcn[i] = rc;
    mb.drc[i] = dr;
    mb.awc[i] = 0.5 * (rc * rc - rw * rw);
    mb.aec[i] = 0.5 * (re * re - rc * rc);
    mb.azc[i] = rc * dr;
  }
  for (int j = 0; j < NZ; j++) {
    if (gr->dz_row) {
      mb.dzr[j] = gr->dz_row[j];
      mb.zn[j + 1] = mb.zn[j] + mb.dzr[j];
      mb.zcn[j] = mb.zn[j] + 0.5 * mb.dzr[j];
    } else {
      mb.dzr[j] = gr->dz;
      mb.zn[j] = (double)j * gr->dz;
      mb.zn[j + 1] = (double)(j + 1) * gr->dz;
      mb.zcn[j] = ((double)j + 0.5) * gr->dz;
    }
  }
}

// The device copy of the geometry: six column fields of NR + 1 entries, then
// the row heights and the node heights (NZ + 1 entries each).
std::vector<double> geometry_table(const Member& mb) {
  const int NR = mb.g.NR, NZ = mb.g.NZ, s = NR + 1;
  std::vector<double> t((size_t)6 * s + 2 * (size_t)(NZ + 1), 0.0);
  for (int i = 0; i <= NR; i++) t[i] = mb.rn[i];
  for (int i = 0; i < NR; i++) {
    t[s + i] = mb.rcn[i];
    t[2 * s + i] = mb.drc[i];
    t[3 * s + i] = mb.awc[i];
    t[4 * s + i] = mb.aec[i];
    t[5 * s + i] = mb.azc[i];
  }
  for (int j = 0; j < NZ; j++) t[6 * s + j] = mb.dzr[j];
  for (int j = 0; j <= NZ; j++) t[6 * s + (NZ + 1) + j] = mb.zn[j];
  return t;
}

// Lithostatic target column (Sec. 3: the initial pressure p0 with
// -grad p0 + rho g = 0), rows below surface_j: cell-centre pressures from
// p = 0 at the surface over the piecewise-constant density (top row
// g rho dz / 2, then g (rho_{j+1} dz_{j+1} / 2 + rho_j dz_j / 2) per row),
// each row's density the cold (E = 0)
// compressed Tillotson state of its pressure, mu = 2p / (A + sqrt(A^2 + 4Bp)),
// iterated with the pressure to a fixed point (at most 50 passes). p0 is then
// the cold pressure A mu + B mu^2 of the final density, evaluated as the
// cycle kernel evaluates the equation of state at E = 0, so that a target at
// rest is in exact discrete equilibrium (p - p0 = 0 in every cell).
void lithostatic_column(const Member& mb, int surface_j, int layer_j, int layer2_j, double grav,
                        std::vector<double>& rho_row, std::vector<double>& p0) {
  const Geo& g = mb.g;
  for (int j = surface_j - 1; j >= 0; j--) {
    const MatC& m = g.m[g.nmat == 3 && j < layer2_j ? 2 : (g.nmat > 1 && j < layer_j ? 1 : 0)];
    const bool top = j == surface_j - 1;
    const double p_up = top ? 0.0 : p0[j + 1];
    const double w_up = top ? 0.0 : grav * (0.5 * mb.dzr[j + 1]) * rho_row[j + 1];
    const double hj = grav * (0.5 * mb.dzr[j]);
    double r = m.rho0;
    for (int it = 0; it < 50; it++) {
      double p = p_up + (w_up + hj * r);
      double mu = 2.0 * p / (m.A + std::sqrt(m.A * m.A + 4.0 * m.B * p));
      double rn = m.rho0 * (1.0 + mu);
      if (rn == r) break;
      r = rn;
    }
    const double mu = r / m.rho0 - 1.0;
    rho_row[j] = r;
    p0[j] = m.A * mu + m.B * mu * mu;
  }
}

int tiles_of(const Geo& g, int v, int* tr, int* tz) {
  int tw, th, nt;
  variant_shape(v, &tw, &th, &nt);
  *tr = (g.NR + tw - 1) / tw;
  *tz = (g.NZ + th - 1) / th;
  return *tr * *tz;
}

// Persistent state of one member: scalars, both state levels (with their
// EoS caches), PML auxiliaries of both levels, reference density, sink and
// outflow budgets.
void carve_persistent(Member& mb, Carver& cv) {
  const Geo& g = mb.g;
  size_t es = g.prec ? sizeof(float) : sizeof(double);
  long long nc = (long long)g.NZ * g.pc, nn = (long long)(g.NZ + 1) * g.pn;
  Inst& d = mb.d;
  d.sc = cv.obj<Scal>();
  for (int b = 0; b < 2; b++) {
    State& S = d.S[b];
    S.rho = cv.d(nc);
    S.I = cv.d(nc);
    for (int m = 0; m < kMaxMat; m++) S.f[m] = m < g.nmat ? cv.d(nc) : nullptr;
    for (int k = 0; k < 3; k++) S.s[k] = g.any_strength ? cv.bytes(nc * es) : nullptr;
    S.v[0] = cv.bytes(nn * es);
    S.v[1] = cv.bytes(nn * es);
    for (int k = 0; k < kEos; k++) S.eos[k] = cv.bytes(nc * es);
    for (int m = 0; m < kMaxMat; m++) {
      const bool on = g.closure && m < g.nmat;
      S.mu[m] = on ? cv.d(nc) : nullptr;
      S.Im[m] = on ? cv.d(nc) : nullptr;
      S.pmat[m] = on ? cv.bytes(nc * es) : nullptr;
    }
    S.dmg = g.dmg ? cv.d(nc) : nullptr;
    S.vib = g.dmg ? cv.d(nc) : nullptr;
  }
  mb.aux_off = cv.off;
  long long nbc = (long long)g.pml_b * g.NR, nrc = (long long)g.NZ * g.pml_r;
  long long nbn = (long long)g.pml_b * (g.NR + 1), nrn = (long long)(g.NZ + 1) * g.pml_r;
  long long nu = nbc + (long long)g.n_z * g.pml_r;
  mb.n_pml = g.pml_on ? nu : 0;
  Pml& pm = d.pm;
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
  d.mout = cv.d(g.pc);
  d.eout = cv.d(g.pc);
  mb.aux_end = cv.off;
}

// Constants and per-cycle scratch of one member.
void carve_constants(Member& mb, Carver& cv) {
  const Geo& g = mb.g;
  Pml& pm = mb.d.pm;
  pm.dcz = cv.d(g.NZ);
  pm.dnz = cv.d(g.NZ + 1);
  pm.dcr = cv.d(g.NR);
  pm.dnr = cv.d(g.NR + 1);
  int most = 0;
  for (int v = 0; v < n_variants(); v++) {
    int tr, tz;
    most = std::max(most, tiles_of(g, v, &tr, &tz));
  }
  mb.d.dtpart = cv.d((size_t)most);
  mb.d.p0 = cv.d((size_t)g.NZ);
  mb.d.geo = cv.d((size_t)6 * (g.NR + 1) + 2 * (size_t)(g.NZ + 1));
}

// Entries of the largest schedule over all tile shapes.
size_t schedule_capacity(const std::vector<Member>& ms) {
  size_t cap = 0;
  for (int v = 0; v < n_variants(); v++) {
    size_t t = 0;
    for (const Member& mb : ms) {
      int tr, tz;
      t += (size_t)tiles_of(mb.g, v, &tr, &tz);
    }
    cap = std::max(cap, (t + kXcds - 1) / kXcds * kXcds);
  }
  return cap;
}

struct Layout {
  size_t persist_bytes = 0, total = 0;
  Inst* d_inst = nullptr;
  TileRef* d_sched = nullptr;
  size_t sched_cap = 0;
  double *scratch = nullptr, *red = nullptr, *diag_out = nullptr;
};

// Buffer layout: every member's persistent state first (one contiguous,
// checkpointable block), then descriptors, the schedule, constants and the
// shared scratch.
void carve_all(std::vector<Member>& ms, void* base, Layout& L) {
  Carver cv(base);
  for (Member& mb : ms) carve_persistent(mb, cv);
  L.persist_bytes = cv.off;
  L.d_inst = cv.obj<Inst>(ms.size());
  L.sched_cap = schedule_capacity(ms);
  L.d_sched = cv.obj<TileRef>(L.sched_cap);
  size_t most = 0;
  for (Member& mb : ms) {
    carve_constants(mb, cv);
    most = std::max(most, (size_t)mb.g.NZ * mb.g.pc);
  }
  L.scratch = cv.d(2 * most);
  L.red = cv.d((size_t)kDiagBlocks * kDiagQ * 2);
  L.diag_out = cv.d(8);
  L.total = cv.off;
}

int validate(const salec_grid* g, const salec_material* mats, const salec_pml* pml, std::string& why) {
  if (!g || !mats || !pml) return why = "null argument", SALEC_E_INVALID;
  if (g->n_r < 1 || g->n_z < 1 || g->pml_r < 0 || g->pml_b < 0) return why = "grid sizes", SALEC_E_INVALID;
  if ((long long)(g->n_r + g->pml_r + 1) * (g->n_z + g->pml_b + 1) > (1ll << 31))
    return why = "grid too large for one instance", SALEC_E_INVALID;
  if (g->nmat < 1 || g->nmat > SALEC_MAX_MAT) return why = "nmat must be 1, 2 or 3", SALEC_E_INVALID;
  if (g->precision != SALEC_FP64 && g->precision != SALEC_MIXED) return why = "precision", SALEC_E_INVALID;
  if (g->closure != SALEC_CLOSURE_SHARED && g->closure != SALEC_CLOSURE_PER_MATERIAL)
    return why = "closure must be 0 or 1", SALEC_E_INVALID;
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
    if (M.damage != 0 && M.damage != 1) return why = "damage must be 0 or 1", SALEC_E_INVALID;
    if (M.damage && (!M.strength || !(M.Yd0 >= 0) || !(M.Ydm >= M.Yd0) || !(M.mu_d >= 0) || !(M.eps_fb > 0) ||
                     !(M.B_dmg >= 0) || !std::isfinite(M.p_bd) || !(M.gamma_eta >= 0) || !(M.gamma_T >= 0) ||
                     !(M.c_vib >= 0) || ((M.gamma_eta > 0 || M.gamma_T > 0) && !(M.af_h > 0))))
      return why = "damage parameters of material " + std::to_string(m) +
                   " (damage needs strength; block size > 0 with gamma_eta or gamma_T)",
             SALEC_E_INVALID;
  }
  if (pml->enabled && !(pml->R > 0 && pml->R < 1)) return why = "PML reflection coefficient", SALEC_E_INVALID;
  if (pml->damp_stress != 0 && pml->damp_stress != 1) return why = "PML damp_stress must be 0 or 1", SALEC_E_INVALID;
  if (pml->placement != 0 && pml->placement != 1) return why = "PML placement must be 0 or 1", SALEC_E_INVALID;
  if (pml->reserved != 0) return why = "PML reserved field must be 0", SALEC_E_INVALID;
  return SALEC_OK;
}

template <class T>
void fill_mat(MatT<T>& c, const salec_material& M) {
  c.rho0 = (T)M.rho0;
  c.A = (T)M.A;
  c.B = (T)M.B;
  c.E0 = (T)M.E0;
  c.a = (T)M.a;
  c.b = (T)M.b;
  c.alpha = (T)M.alpha;
  c.beta = (T)M.beta;
  c.Eiv = (T)M.Eiv;
  c.Ecv = (T)M.Ecv;
  c.p_min = (T)M.p_min;
  c.cf2 = (T)(M.c_floor_frac * M.A / M.rho0);
  c.strength = M.strength ? 1 : 0;
  c.gfac = (T)(M.strength ? 3.0 * (1.0 - 2.0 * M.poisson) / (2.0 * (1.0 + M.poisson)) : 0.0);
  c.Y0 = (T)M.Y0;
  c.mu_f = (T)M.mu_f;
  c.Ylim = (T)M.Ylim;
  c.pcav = (T)(kPcavFrac * M.A);
  // reciprocals for the FP32 arithmetic (the FP64 arithmetic divides)
  c.irho0 = (T)(1.0 / M.rho0);
  c.Ar = (T)(M.A / M.rho0);
  c.idE = (T)(1.0 / (M.Ecv - M.Eiv));
  c.iYd = (T)(M.strength && M.Ylim != M.Y0 ? 1.0 / (M.Ylim - M.Y0) : 0.0);
  // damage and the block model: the longitudinal speed at rest
  // sqrt((A + 4G/3) / rho0), the kinematic viscosity gamma_eta cL0 h and the
  // decay time gamma_T h / cL0 (formed in FP64)
  c.damage = M.damage ? 1 : 0;
  double cL0 = 0.0, nub = 0.0, Tvib = 0.0;
  if (M.damage) {
    double G = 3.0 * M.A * (1.0 - 2.0 * M.poisson) / (2.0 * (1.0 + M.poisson));
    cL0 = std::sqrt((M.A + (4.0 / 3.0) * G) / M.rho0);
    nub = M.gamma_eta * cL0 * M.af_h;
    Tvib = M.gamma_T * M.af_h / cL0;
  }
  c.Yd0 = (T)(M.damage ? M.Yd0 : 0.0);
  c.mu_d = (T)(M.damage ? M.mu_d : 0.0);
  c.Ydm = (T)(M.damage ? M.Ydm : 0.0);
  c.eps_fb = (T)(M.damage ? M.eps_fb : 0.0);
  c.B_dmg = (T)(M.damage ? M.B_dmg : 0.0);
  c.p_bd = (T)(M.damage ? M.p_bd : 0.0);
  c.c_vib = (T)(M.damage ? M.c_vib : 0.0);
  c.cL0 = (T)cL0;
  c.nub = (T)nub;
  c.Tvib = (T)Tvib;
}

Geo make_geo(const salec_grid* gr, const salec_material* mats, const salec_pml* pml) {
  Geo g;
  std::memset(&g, 0, sizeof(g));
  g.n_r = gr->n_r;
  g.n_z = gr->n_z;
  g.pml_r = gr->pml_r;
  g.pml_b = gr->pml_b;
  g.NR = gr->n_r + gr->pml_r;
  g.NZ = gr->n_z + gr->pml_b;
  g.nmat = gr->nmat;
  g.top_closed = gr->top_closed;
  g.closure = gr->closure;
  g.prec = gr->precision == SALEC_MIXED ? 1 : 0;
  // row pitch: 64 elements for FP32 rows, 32 for FP64 (256 bytes either way)
  int q = g.prec ? 64 : 32;
  g.pc = (g.NR + q - 1) / q * q;
  g.pn = (g.NR + 1 + q - 1) / q * q;
  g.pml_on = pml->enabled ? 1 : 0;
  g.damp_stress = pml->enabled && pml->damp_stress ? 1 : 0;
  g.pml_place = pml->enabled && pml->placement ? 1 : 0;
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
    fill_mat(g.m[m], mats[m]);
    fill_mat(g.mf[m], mats[m]);
    if (mats[m].strength) g.any_strength = 1;
    if (mats[m].damage) g.dmg = 1;
    if (mats[m].rho0 > g.rho_ref) g.rho_ref = mats[m].rho0;
  }
  g.stretched = (gr->dr_col || gr->dz_row) ? 1 : 0;
  g.drf = (float)g.dr;
  g.dzf = (float)g.dz;
  g.q_linf = (float)g.q_lin;
  g.q_quadf = (float)g.q_quad;
  g.rho_reff = (float)g.rho_ref;
  g.same_mat = 1;
  for (int m = 1; m < gr->nmat; m++)
    if (std::memcmp(&g.m[m], &g.m[0], sizeof(MatC)) != 0) g.same_mat = 0;
  return g;
}

// damping profile d(y) = (3c / 2 delta) (y / delta)^2 log(1/R)  (Sec. 3)
double pml_d(double c, double delta, double y, double R) { return 1.5 * c / delta * (y / delta) * (y / delta) * std::log(1.0 / R); }

void pml_profiles(Member& mb, const salec_material* mats, const salec_pml* pml) {
  const Geo& g = mb.g;
  mb.dcz.assign(g.NZ, 0.0);
  mb.dnz.assign(g.NZ + 1, 0.0);
  mb.dcr.assign(g.NR, 0.0);
  mb.dnr.assign(g.NR + 1, 0.0);
  if (!pml->enabled) return;
  // c: the largest acoustic speed (Sec. 3); by default the largest
  // longitudinal speed at rest over the materials
  double c = pml->c_ref;
  if (!(c > 0)) {
    c = 0.0;
    for (int m = 0; m < g.nmat; m++) {
      const salec_material& M = mats[m];
      double G = M.strength ? 3.0 * M.A * (1.0 - 2.0 * M.poisson) / (2.0 * (1.0 + M.poisson)) : 0.0;
      c = std::max(c, std::sqrt((M.A + (4.0 / 3.0) * G) / M.rho0));
    }
  }
  // y from the inner face of each layer, at cell centres and at nodes
  if (g.pml_b > 0) {
    double zf = mb.zn[g.pml_b], delta = zf - mb.zn[0];
    for (int j = 0; j < g.pml_b; j++) mb.dcz[j] = pml_d(c, delta, zf - mb.zcn[j], pml->R);
    for (int j = 0; j < g.pml_b; j++) mb.dnz[j] = pml_d(c, delta, zf - mb.zn[j], pml->R);
  }
  if (g.pml_r > 0) {
    double rf = mb.rn[g.n_r], delta = mb.rn[g.NR] - rf;
    for (int i = g.n_r; i < g.NR; i++) mb.dcr[i] = pml_d(c, delta, mb.rcn[i] - rf, pml->R);
    for (int i = g.n_r + 1; i <= g.NR; i++) mb.dnr[i] = pml_d(c, delta, mb.rn[i] - rf, pml->R);
  }
}

int check_members(const salec_instance* inst, int32_t n, std::vector<Member>& ms, std::string& why) {
  if (!inst || n < 1) return why = "no instances", SALEC_E_INVALID;
  ms.assign((size_t)n, Member{});
  for (int32_t k = 0; k < n; k++) {
    const salec_instance& I = inst[k];
    int rc = validate(&I.grid, I.mats, &I.pml, why);
    if (rc) return why = "instance " + std::to_string(k) + ": " + why, rc;
    if (I.grid.precision != inst[0].grid.precision)
      return why = "every instance of a context must use the same precision", SALEC_E_INVALID;
    if (I.grid.closure != inst[0].grid.closure)
      return why = "every instance of a context must use the same closure", SALEC_E_INVALID;
    const salec_scene& sc = I.scene;
    if (I.has_scene && (sc.subsample < 1 || !(sc.radius >= 0) || !(sc.gravity >= 0) || sc.surface_j < 0 ||
                        sc.surface_j > I.grid.n_z + I.grid.pml_b || sc.layer_j < 0 || sc.layer_j > sc.surface_j ||
                        sc.layer2_j < 0 || sc.layer2_j > sc.layer_j || (I.grid.nmat < 3 && sc.layer2_j != 0)))
      return why = "instance " + std::to_string(k) + ": scene parameters", SALEC_E_INVALID;
    const int NR = I.grid.n_r + I.grid.pml_r, NZ = I.grid.n_z + I.grid.pml_b;
    for (int i = 0; I.grid.dr_col && i < NR; i++)
      if (!(I.grid.dr_col[i] > 0) || !std::isfinite(I.grid.dr_col[i]))
        return why = "instance " + std::to_string(k) + ": column widths", SALEC_E_INVALID;
    for (int j = 0; I.grid.dz_row && j < NZ; j++)
      if (!(I.grid.dz_row[j] > 0) || !std::isfinite(I.grid.dz_row[j]))
        return why = "instance " + std::to_string(k) + ": row heights", SALEC_E_INVALID;
    ms[k].g = make_geo(&I.grid, I.mats, &I.pml);
    build_geometry(ms[k], &I.grid);
    ms[k].d.g = ms[k].g;
    ms[k].has_scene = I.has_scene != 0;
    ms[k].scene = I.scene;
  }
  // one cycle-kernel family per context: when some member accumulates
  // damage, every member carries the damage state (zero where no material
  // of that member is damaging, which the damage arithmetic leaves at zero)
  int any_dmg = 0;
  for (const Member& mb : ms) any_dmg |= mb.g.dmg;
  for (Member& mb : ms) {
    mb.g.dmg = any_dmg;
    mb.d.g = mb.g;
  }
  return SALEC_OK;
}

}  // namespace

struct salec_ctx {
  std::vector<Member> ms;
  Layout L;
  int prec = 0;
  bool geo = false;  // some member is stretched: the cycle kernel reads geometry tables
  int nm = 2;        // material slots of the cycle kernel: 3 when some member has three materials
  bool pm = false;   // per-material closure (every member shares the closure)
  bool dm = false;   // damage and acoustic fluidization (some member's material)
  void* buf = nullptr;
  hipStream_t st = nullptr;
  bool own_stream = false;
  hipGraphExec_t gx1 = nullptr, gxN = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = 0.0;
  int variant = 0, grid = 0, nsched = 0;
  double tuned_ms = 0.0;
  bool ready = false;
  double* diag_scratch = nullptr;  // this device's copy of `scratch` (salec_diag_totals)
  std::string err;
};

// Scratch of salec_diag_totals: the compensated partial sums (sum and
// compensation) of the kDiagQ totals of every block of the fixed reduction
// tree. Its size does not depend on the instance: every grid reduces into
// these kDiagBlocks blocks. Each GPU the library runs on holds its own copy
// until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device (kept per device below).
constexpr size_t kDiagScratch = (size_t)kDiagBlocks * kDiagQ * 2;
static __device__ __align__(256) double scratch[kDiagScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
hipError_t scratch_address(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

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

// Clears member k's PML auxiliaries and budgets, sets its PML reference
// density and clock, and computes the EoS cache and first time step of its
// state (level 0).
int start_run(salec_ctx* x, int k) {
  Member& mb = x->ms[k];
  uint8_t* base = (uint8_t*)x->buf;
  if (mb.aux_end > mb.aux_off) HIPCHK(x, hipMemsetAsync(base + mb.aux_off, 0, mb.aux_end - mb.aux_off, x->st));
  HIPCHK(x, launch_start_run(mb.d, x->st));
  HIPCHK(x, launch_prime(mb.d, x->st));
  HIPCHK(x, launch_finalize0(mb.d, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

// Tile list of every member for tile shape v, grouped into kXcds contiguous
// chunks: entry e is position e / kXcds of chunk e % kXcds, so the
// workgroups one L2 domain runs work on neighbouring tiles. Tiles that reach
// into a PML strip cost about a fifth more than the others (the layers'
// auxiliaries); a workgroup drawing several of them would finish last, so
// they are spread where each workgroup takes only a few tiles: first evenly
// over the chunks (a strip tile of a chunk holding too many changes places
// with another chunk's plain tile), then to the first positions of each
// chunk, which the grid-stride order hands to different workgroups.
int build_schedule(salec_ctx* x, int v) {
  std::vector<TileRef> list;
  std::vector<char> strip;
  int tw, th, nthr;
  variant_shape(v, &tw, &th, &nthr);
  for (size_t k = 0; k < x->ms.size(); k++) {
    Member& mb = x->ms[k];
    int tr, tz;
    int nt = tiles_of(mb.g, v, &tr, &tz);
    mb.d.tiles_r = tr;
    mb.d.tiles_z = tz;
    mb.d.ntiles = nt;
    for (int t = 0; t < nt; t++) {
      const int i1 = std::min((t % tr + 1) * tw, mb.g.NR), j0 = (t / tr) * th;
      list.push_back(TileRef{(int)k, t});
      strip.push_back(mb.g.pml_on && (i1 > mb.g.n_r || j0 < mb.g.pml_b));
    }
  }
  size_t T = list.size(), per = (T + kXcds - 1) / kXcds;
  std::vector<std::vector<size_t>> chunk(kXcds);
  for (size_t i = 0; i < T; i++) chunk[i / per].push_back(i);
  // only where each workgroup takes a few tiles (with many, the mix averages out)
  if (x->grid > 0 && T <= 16 * (size_t)x->grid) {
    std::vector<size_t> n(kXcds, 0), ps(kXcds), pp(kXcds);
    size_t total = 0;
    for (int c = 0; c < kXcds; c++) {
      for (size_t i : chunk[c]) n[c] += strip[i];
      total += n[c];
      ps[c] = pp[c] = chunk[c].size();  // scan positions for strip / plain tiles, from the end
    }
    const size_t want = (total + kXcds - 1) / kXcds;
    for (int a = 0; a < kXcds; a++)
      for (int b = 0; b < kXcds && n[a] > want; b++)
        while (n[a] > want && n[b] < want) {
          while (ps[a] > 0 && !strip[chunk[a][ps[a] - 1]]) ps[a]--;
          while (pp[b] > 0 && strip[chunk[b][pp[b] - 1]]) pp[b]--;
          if (ps[a] == 0 || pp[b] == 0) break;
          std::swap(chunk[a][ps[a] - 1], chunk[b][pp[b] - 1]);
          n[a]--, n[b]++;
        }
    for (int c = 0; c < kXcds; c++)
      std::stable_partition(chunk[c].begin(), chunk[c].end(), [&](size_t i) { return strip[i] != 0; });
  }
  std::vector<TileRef> sched(per * kXcds);
  for (size_t e = 0; e < sched.size(); e++) {
    const std::vector<size_t>& ch = chunk[e % kXcds];
    size_t q = e / kXcds;
    sched[e] = q < ch.size() ? list[ch[q]] : TileRef{-1, 0};
  }
  if (sched.size() > x->L.sched_cap) {
    x->err = "schedule larger than its reserved space";
    return SALEC_E_INVALID;
  }
  std::vector<Inst> di(x->ms.size());
  for (size_t k = 0; k < x->ms.size(); k++) di[k] = x->ms[k].d;
  HIPCHK(x, hipMemcpyAsync(x->L.d_inst, di.data(), di.size() * sizeof(Inst), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipMemcpyAsync(x->L.d_sched, sched.data(), sched.size() * sizeof(TileRef), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  x->nsched = (int)sched.size();
  return SALEC_OK;
}

int capture(salec_ctx* x, int ncyc, hipGraphExec_t* out) {
  hipGraph_t gr = nullptr;
  int grid = x->grid > 0 ? std::min(x->grid, x->nsched) : x->nsched;
  HIPCHK(x, hipStreamBeginCapture(x->st, hipStreamCaptureModeThreadLocal));
  hipError_t le = hipSuccess;
  for (int k = 0; k < ncyc && le == hipSuccess; k++) {
    le = launch_cycle(x->variant, x->prec, x->geo, x->nm, x->pm, x->dm, x->L.d_inst, x->L.d_sched, x->nsched, grid, x->st);
    if (le == hipSuccess) le = launch_finalize(x->L.d_inst, (int)x->ms.size(), x->st);
  }
  hipError_t e = hipStreamEndCapture(x->st, &gr);
  if (le != hipSuccess) {
    if (gr) (void)hipGraphDestroy(gr);
    return hip_fail(x, le, "launch_cycle");
  }
  if (e != hipSuccess) return hip_fail(x, e, "hipStreamEndCapture");
  e = hipGraphInstantiate(out, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return hip_fail(x, e, "hipGraphInstantiate");
  return SALEC_OK;
}

// Selects a schedule: uploads descriptors and tile list, recaptures graphs.
// whether (v, grid) names a schedule this context can run; nothing changes
int check_schedule(salec_ctx* x, int v, int grid) {
  if (v < 0 || v >= n_variants() || grid < 0) {
    x->err = "schedule out of range";
    return SALEC_E_INVALID;
  }
  if (!variant_available(v, x->prec, x->geo, x->nm, x->pm, x->dm)) {
    x->err = "tile shape not built for this material count, closure and damage (its tile does not fit the LDS)";
    return SALEC_E_INVALID;
  }
  return SALEC_OK;
}

int use_schedule(salec_ctx* x, int v, int grid) {
  int rc0 = check_schedule(x, v, grid);
  if (rc0) return rc0;
  HIPCHK(x, hipStreamSynchronize(x->st));
  if (x->gx1) (void)hipGraphExecDestroy(x->gx1);
  if (x->gxN) (void)hipGraphExecDestroy(x->gxN);
  x->gx1 = x->gxN = nullptr;
  x->variant = v;
  x->grid = grid > 0 ? (grid + kXcds - 1) / kXcds * kXcds : 0;
  int rc = build_schedule(x, v);
  if (rc) return rc;
  rc = capture(x, 1, &x->gx1);
  if (rc) return rc;
  return capture(x, kGraphCycles, &x->gxN);
}

Scal read_scal(salec_ctx* x, int k) {
  Scal s{};
  (void)hipMemcpyAsync(&s, x->ms[k].d.sc, sizeof(Scal), hipMemcpyDeviceToHost, x->st);
  (void)hipStreamSynchronize(x->st);
  return s;
}

size_t elem_size(const salec_ctx* x) { return x->prec ? sizeof(float) : sizeof(double); }

// 2D copies between packed host FP64 arrays and pitched device arrays of
// element size es (FP32 device arrays are converted on the host).
int copy_out(salec_ctx* x, double* host, const void* dev, int w, int h, int pitch, size_t es) {
  if (es == sizeof(double)) {
    HIPCHK(x, hipMemcpy2DAsync(host, w * sizeof(double), dev, pitch * es, w * es, h, hipMemcpyDeviceToHost, x->st));
    return SALEC_OK;
  }
  std::vector<float> tmp((size_t)w * h);
  HIPCHK(x, hipMemcpy2DAsync(tmp.data(), w * es, dev, pitch * es, w * es, h, hipMemcpyDeviceToHost, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  for (size_t t = 0; t < tmp.size(); t++) host[t] = (double)tmp[t];
  return SALEC_OK;
}
int copy_in(salec_ctx* x, void* dev, const double* host, int w, int h, int pitch, size_t es) {
  if (es == sizeof(double)) {
    HIPCHK(x, hipMemcpy2DAsync(dev, pitch * es, host, w * sizeof(double), w * es, h, hipMemcpyHostToDevice, x->st));
    HIPCHK(x, hipStreamSynchronize(x->st));
    return SALEC_OK;
  }
  std::vector<float> tmp((size_t)w * h);
  for (size_t t = 0; t < tmp.size(); t++) tmp[t] = (float)host[t];
  HIPCHK(x, hipMemcpy2DAsync(dev, pitch * es, tmp.data(), w * es, w * es, h, hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int init_common(salec_ctx* x, void* dev_buf, size_t dev_bytes, void* stream) {
  Layout probe;
  carve_all(x->ms, nullptr, probe);
  if (!dev_buf || dev_bytes < probe.total || ((uintptr_t)dev_buf % kAlign) != 0) {
    x->err = "device buffer smaller than the plan or not 256-byte aligned";
    return SALEC_E_BUFFER;
  }
  x->buf = dev_buf;
  x->prec = x->ms[0].g.prec;
  x->pm = x->ms[0].g.closure == SALEC_CLOSURE_PER_MATERIAL;
  x->dm = x->ms[0].g.dmg != 0;
  for (const Member& mb : x->ms) {
    if (mb.g.stretched) x->geo = true;
    if (mb.g.nmat > 2) x->nm = 3;
  }
  carve_all(x->ms, dev_buf, x->L);
  if (stream) {
    x->st = (hipStream_t)stream;
  } else {
    HIPCHK(x, hipStreamCreate(&x->st));
    x->own_stream = true;
  }
  HIPCHK(x, hipEventCreate(&x->ev0));
  HIPCHK(x, hipEventCreate(&x->ev1));
  HIPCHK(x, scratch_address(&x->diag_scratch));
  HIPCHK(x, hipMemsetAsync(dev_buf, 0, x->L.total, x->st));
  for (size_t k = 0; k < x->ms.size(); k++) {
    Member& mb = x->ms[k];
    mb.d.g = mb.g;
    HIPCHK(x, hipMemcpyAsync((void*)mb.d.pm.dcz, mb.dcz.data(), mb.dcz.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
    HIPCHK(x, hipMemcpyAsync((void*)mb.d.pm.dnz, mb.dnz.data(), mb.dnz.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
    HIPCHK(x, hipMemcpyAsync((void*)mb.d.pm.dcr, mb.dcr.data(), mb.dcr.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
    HIPCHK(x, hipMemcpyAsync((void*)mb.d.pm.dnr, mb.dnr.data(), mb.dnr.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
    const std::vector<double> geo = geometry_table(mb);
    HIPCHK(x, hipMemcpyAsync((void*)mb.d.geo, geo.data(), geo.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
    mb.p0.assign((size_t)mb.g.NZ, 0.0);
    std::vector<double> rho_row;
    if (mb.has_scene && mb.scene.gravity > 0) {
      rho_row.assign((size_t)mb.g.NZ, 0.0);
      lithostatic_column(mb, mb.scene.surface_j, mb.scene.layer_j, mb.scene.layer2_j, mb.scene.gravity, rho_row,
                         mb.p0);
    }
    HIPCHK(x, hipMemcpyAsync((void*)mb.d.p0, mb.p0.data(), mb.p0.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
    mb.g.has_p0 = 0;
    for (double v : mb.p0)
      if (v != 0.0) mb.g.has_p0 = 1;
    mb.d.g = mb.g;
    if (mb.has_scene) {
      const salec_scene& sc = mb.scene;
      double zc = mb.zn[sc.surface_j] + sc.radius;
      // per-row densities of a lithostatic target go after the projectile fractions
      double* rr = nullptr;
      if (!rho_row.empty()) {
        rr = x->L.scratch + (size_t)mb.g.NZ * mb.g.pc;
        HIPCHK(x, hipMemcpyAsync(rr, rho_row.data(), rho_row.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
      }
      HIPCHK(x, launch_scene(mb.d, sc.surface_j, sc.layer_j, sc.layer2_j, sc.subsample, sc.radius, zc, sc.v_imp,
                             rr, x->L.scratch, x->st));
    }
    HIPCHK(x, hipStreamSynchronize(x->st));  // the profile vectors are reused below
    int rc = start_run(x, (int)k);
    if (rc) return rc;
  }
  // the default shape; a persistent grid when it has fewer workgroups than tiles
  int v0 = default_variant(x->prec);
  // fall back along the shapes every family has when the default is not built
  for (int alt : {0, 14, 1, 7, 10})
    if (!variant_available(v0, x->prec, x->geo, x->nm, x->pm, x->dm)) v0 = alt;
  int rc = use_schedule(x, v0, 0);
  if (rc) return rc;
  const int g0 = resident_groups(v0, x->prec, x->geo, x->nm, x->pm, x->dm);
  if (g0 > 0 && g0 < x->nsched && (rc = use_schedule(x, v0, g0))) return rc;
  x->ready = true;
  return SALEC_OK;
}

bool member_ok(const salec_ctx* x, int32_t k) { return x && x->ready && k >= 0 && (size_t)k < x->ms.size(); }

}  // namespace

extern "C" {

size_t salec_plan_batch(const salec_instance* inst, int32_t n) {
  std::vector<Member> ms;
  std::string why;
  if (check_members(inst, n, ms, why) != SALEC_OK) return 0;
  Layout L;
  carve_all(ms, nullptr, L);
  return L.total;
}

size_t salec_plan(const salec_grid* grid, const salec_material* mats, const salec_pml* pml) {
  if (!grid || !mats || !pml) return 0;
  salec_instance I;
  std::memset(&I, 0, sizeof(I));
  I.grid = *grid;
  for (int m = 0; m < grid->nmat && m < SALEC_MAX_MAT; m++) I.mats[m] = mats[m];
  I.pml = *pml;
  return salec_plan_batch(&I, 1);
}

int salec_init_batch(const salec_instance* inst, int32_t n, void* dev_buf, size_t dev_bytes, void* stream,
                     salec_ctx** out) {
  if (!out) return SALEC_E_INVALID;
  salec_ctx* x = new salec_ctx();
  *out = x;  // returned even on failure, so salec_last_error() can explain it
  int rc = check_members(inst, n, x->ms, x->err);
  if (rc) return rc;
  for (int32_t k = 0; k < n; k++) pml_profiles(x->ms[k], inst[k].mats, &inst[k].pml);
  return init_common(x, dev_buf, dev_bytes, stream);
}

int salec_init(const salec_grid* grid, const salec_material* mats, const salec_pml* pml, const salec_scene* scene,
               void* dev_buf, size_t dev_bytes, void* stream, salec_ctx** out) {
  if (!out) return SALEC_E_INVALID;
  if (!grid || !mats || !pml) {
    salec_ctx* x = new salec_ctx();
    x->err = "null argument";
    *out = x;
    return SALEC_E_INVALID;
  }
  salec_instance I;
  std::memset(&I, 0, sizeof(I));
  I.grid = *grid;
  for (int m = 0; m < grid->nmat && m < SALEC_MAX_MAT; m++) I.mats[m] = mats[m];
  I.pml = *pml;
  if (scene) {
    I.scene = *scene;
    I.has_scene = 1;
  }
  return salec_init_batch(&I, 1, dev_buf, dev_bytes, stream, out);
}

int32_t salec_num_instances(const salec_ctx* x) { return x ? (int32_t)x->ms.size() : 0; }

int salec_enqueue(salec_ctx* x, int32_t n) {
  if (!x || n < 0 || !x->ready) return SALEC_E_INVALID;
  int32_t big = n / kGraphCycles, rem = n % kGraphCycles;
  for (int32_t k = 0; k < big; k++) HIPCHK(x, hipGraphLaunch(x->gxN, x->st));
  for (int32_t k = 0; k < rem; k++) HIPCHK(x, hipGraphLaunch(x->gx1, x->st));
  return SALEC_OK;
}

int salec_step(salec_ctx* x, int32_t n) {
  if (!x || n < 0 || !x->ready) return SALEC_E_INVALID;
  HIPCHK(x, hipEventRecord(x->ev0, x->st));
  int rc = salec_enqueue(x, n);
  if (rc) return rc;
  HIPCHK(x, hipEventRecord(x->ev1, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  float ms = 0.0f;
  HIPCHK(x, hipEventElapsedTime(&ms, x->ev0, x->ev1));
  x->last_ms = ms;
  for (size_t k = 0; k < x->ms.size(); k++) {
    Scal s = read_scal(x, (int)k);
    if (s.err) {
      x->err = "instance " + std::to_string(k) + ": device error " + std::to_string(s.err) + " at cycle " +
               std::to_string(s.err_cycle);
      return s.err;
    }
  }
  return SALEC_OK;
}

int salec_set_p0(salec_ctx* x, int32_t k, const double* p0) {
  if (!member_ok(x, k) || !p0) return SALEC_E_INVALID;
  Member& mb = x->ms[k];
  for (int j = 0; j < mb.g.NZ; j++)
    if (!std::isfinite(p0[j])) {
      x->err = "initial pressure not finite";
      return SALEC_E_INVALID;
    }
  HIPCHK(x, hipStreamSynchronize(x->st));
  mb.p0.assign(p0, p0 + mb.g.NZ);
  HIPCHK(x, hipMemcpyAsync((void*)mb.d.p0, mb.p0.data(), mb.p0.size() * sizeof(double), hipMemcpyHostToDevice, x->st));
  mb.g.has_p0 = 0;
  for (double v : mb.p0)
    if (v != 0.0) mb.g.has_p0 = 1;
  mb.d.g.has_p0 = mb.g.has_p0;
  // the descriptor carries the flag: upload it again (graphs read it at run time)
  HIPCHK(x, hipMemcpyAsync(x->L.d_inst + k, &mb.d, sizeof(Inst), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int salec_get_p0(salec_ctx* x, int32_t k, double* p0) {
  if (!member_ok(x, k) || !p0) return SALEC_E_INVALID;
  std::copy(x->ms[k].p0.begin(), x->ms[k].p0.end(), p0);
  return SALEC_OK;
}

int salec_time_kernels(salec_ctx* x, int32_t n, double* cycle_ms, double* finalize_ms) {
  if (!x || n < 1 || n > 100000 || !x->ready || !cycle_ms || !finalize_ms) return SALEC_E_INVALID;
  // one event before the first cycle, then one after each kernel; the host
  // queues every cycle before waiting, so the kernels run back to back
  std::vector<hipEvent_t> ev(2 * (size_t)n + 1, nullptr);
  int rc = SALEC_OK;
  for (auto& e : ev)
    if (hipEventCreate(&e) != hipSuccess) {
      rc = hip_fail(x, hipErrorOutOfMemory, "hipEventCreate");
      break;
    }
  const int grid = x->grid > 0 ? std::min(x->grid, x->nsched) : x->nsched;
  hipError_t e = rc ? hipErrorOutOfMemory : hipEventRecord(ev[0], x->st);
  for (int c = 0; c < n && e == hipSuccess; c++) {
    e = launch_cycle(x->variant, x->prec, x->geo, x->nm, x->pm, x->dm, x->L.d_inst, x->L.d_sched, x->nsched, grid, x->st);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * c + 1], x->st);
    if (e == hipSuccess) e = launch_finalize(x->L.d_inst, (int)x->ms.size(), x->st);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * c + 2], x->st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(x->st);
  double a = 0.0, b = 0.0;
  for (int c = 0; c < n && e == hipSuccess; c++) {
    float m1 = 0.0f, m2 = 0.0f;
    e = hipEventElapsedTime(&m1, ev[2 * c], ev[2 * c + 1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&m2, ev[2 * c + 1], ev[2 * c + 2]);
    a += m1;
    b += m2;
  }
  for (auto& q : ev)
    if (q) (void)hipEventDestroy(q);
  if (rc) return rc;
  if (e != hipSuccess) return hip_fail(x, e, "salec_time_kernels");
  *cycle_ms = a / n;
  *finalize_ms = b / n;
  for (size_t k = 0; k < x->ms.size(); k++) {
    Scal s = read_scal(x, (int)k);
    if (s.err) {
      x->err = "instance " + std::to_string(k) + ": device error " + std::to_string(s.err) + " at cycle " +
               std::to_string(s.err_cycle);
      return s.err;
    }
  }
  return SALEC_OK;
}

int salec_last_step_ms(salec_ctx* x, double* ms) {
  if (!x || !ms) return SALEC_E_INVALID;
  *ms = x->last_ms;
  return SALEC_OK;
}

int salec_get_fields(salec_ctx* x, int32_t k, const salec_fields* o) {
  if (!member_ok(x, k) || !o) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  Member& mb = x->ms[k];
  Scal s = read_scal(x, k);
  const State& S = mb.d.S[s.cycle & 1];
  const Geo& g = mb.g;
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1), es = elem_size(x);
  int rc = SALEC_OK;
  if (o->rho && (rc = copy_out(x, o->rho, S.rho, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if (o->I && (rc = copy_out(x, o->I, S.I, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if (o->f)
    for (int m = 0; m < g.nmat; m++)
      if ((rc = copy_out(x, o->f + m * NC, S.f[m], g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if (o->s) {
    if (g.any_strength) {
      for (int q = 0; q < 3; q++)
        if ((rc = copy_out(x, o->s + q * NC, S.s[q], g.NR, g.NZ, g.pc, es))) return rc;
    } else {
      std::memset(o->s, 0, 3 * NC * sizeof(double));
    }
  }
  if (o->v) {
    if ((rc = copy_out(x, o->v, S.v[0], g.NR + 1, g.NZ + 1, g.pn, es))) return rc;
    if ((rc = copy_out(x, o->v + NN, S.v[1], g.NR + 1, g.NZ + 1, g.pn, es))) return rc;
  }
  if (o->p || o->c2) {
    double* p = x->L.scratch;
    double* c2 = x->L.scratch + (size_t)g.NZ * g.pc;
    HIPCHK(x, launch_eos_out(mb.d, p, c2, x->st));
    if (o->p && (rc = copy_out(x, o->p, p, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
    if (o->c2 && (rc = copy_out(x, o->c2, c2, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int salec_set_fields(salec_ctx* x, int32_t k, const salec_fields* in) {
  if (!member_ok(x, k) || !in || !in->rho || !in->I || !in->f || !in->v) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  const State& S = mb.d.S[0];
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1), es = elem_size(x);
  int rc;
  if ((rc = copy_in(x, S.rho, in->rho, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if ((rc = copy_in(x, S.I, in->I, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  for (int m = 0; m < g.nmat; m++)
    if ((rc = copy_in(x, S.f[m], in->f + m * NC, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if (g.any_strength) {
    for (int q = 0; q < 3; q++) {
      if (in->s) {
        if ((rc = copy_in(x, S.s[q], in->s + q * NC, g.NR, g.NZ, g.pc, es))) return rc;
      } else {
        HIPCHK(x, hipMemsetAsync(S.s[q], 0, (size_t)g.NZ * g.pc * es, x->st));
      }
    }
  }
  if ((rc = copy_in(x, S.v[0], in->v, g.NR + 1, g.NZ + 1, g.pn, es))) return rc;
  if ((rc = copy_in(x, S.v[1], in->v + NN, g.NR + 1, g.NZ + 1, g.pn, es))) return rc;
  // intact, quiet rock (salec_set_damage sets other damage)
  if (g.dmg) {
    HIPCHK(x, hipMemsetAsync(S.dmg, 0, (size_t)g.NZ * g.pc * sizeof(double), x->st));
    HIPCHK(x, hipMemsetAsync(S.vib, 0, (size_t)g.NZ * g.pc * sizeof(double), x->st));
  }
  if (g.closure) {
    // every material of a cell at the cell's matter density and energy
    std::vector<double> mu(g.nmat * NC), Im(g.nmat * NC);
    for (size_t c = 0; c < NC; c++) {
      double phi = 0.0;
      for (int m = 0; m < g.nmat; m++) phi += in->f[m * NC + c];
      const double den = phi > kPhiEps ? phi : kPhiEps;
      for (int m = 0; m < g.nmat; m++) {
        mu[m * NC + c] = in->rho[c] * (in->f[m * NC + c] / den);
        Im[m * NC + c] = in->I[c];
      }
    }
    for (int m = 0; m < g.nmat; m++) {
      if ((rc = copy_in(x, S.mu[m], mu.data() + m * NC, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
      if ((rc = copy_in(x, S.Im[m], Im.data() + m * NC, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
    }
  }
  return start_run(x, k);
}

}  // extern "C"

namespace {
// A new run starts from level 0: copies member k's state there when the
// current cycle left it in level 1 (the EoS cache is recomputed by the run
// start).
int state_to_level0(salec_ctx* x, int k) {
  if (!(read_scal(x, k).cycle & 1)) return SALEC_OK;
  const Member& mb = x->ms[k];
  const Geo& g = mb.g;
  const State &A = mb.d.S[1], &B = mb.d.S[0];
  const size_t cb = (size_t)g.NZ * g.pc * sizeof(double), ce = (size_t)g.NZ * g.pc * elem_size(x);
  const size_t nb = (size_t)(g.NZ + 1) * g.pn * elem_size(x);
  auto cp = [&](void* d, const void* s_, size_t n) {
    return s_ ? hipMemcpyAsync(d, s_, n, hipMemcpyDeviceToDevice, x->st) : hipSuccess;
  };
  HIPCHK(x, cp(B.rho, A.rho, cb));
  HIPCHK(x, cp(B.I, A.I, cb));
  for (int m = 0; m < g.nmat; m++) HIPCHK(x, cp(B.f[m], A.f[m], cb));
  for (int q = 0; q < 3; q++) HIPCHK(x, cp(B.s[q], A.s[q], ce));
  for (int q = 0; q < 2; q++) HIPCHK(x, cp(B.v[q], A.v[q], nb));
  for (int m = 0; m < g.nmat; m++) {
    HIPCHK(x, cp(B.mu[m], A.mu[m], cb));
    HIPCHK(x, cp(B.Im[m], A.Im[m], cb));
  }
  HIPCHK(x, cp(B.dmg, A.dmg, cb));
  HIPCHK(x, cp(B.vib, A.vib, cb));
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}
}  // namespace

extern "C" {

int salec_set_damage(salec_ctx* x, int32_t k, const double* D, const double* vib) {
  if (!member_ok(x, k)) return SALEC_E_INVALID;
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  if (!g.dmg) {
    x->err = "damage state needs a material with damage";
    return SALEC_E_INVALID;
  }
  const size_t NC = (size_t)g.NR * g.NZ;
  for (size_t c = 0; c < NC; c++)
    if ((D && !(D[c] >= 0.0 && D[c] <= 1.0)) || (vib && !(vib[c] >= 0.0 && std::isfinite(vib[c])))) {
      x->err = "damage must lie in [0, 1] and the vibration speed be finite and >= 0";
      return SALEC_E_INVALID;
    }
  HIPCHK(x, hipStreamSynchronize(x->st));
  int rc = state_to_level0(x, k);
  if (rc) return rc;
  const State& S = mb.d.S[0];
  if (D && (rc = copy_in(x, S.dmg, D, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if (vib && (rc = copy_in(x, S.vib, vib, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  return start_run(x, k);
}

int salec_get_damage(salec_ctx* x, int32_t k, double* D, double* vib) {
  if (!member_ok(x, k)) return SALEC_E_INVALID;
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  if (!g.dmg) {
    x->err = "damage state needs a material with damage";
    return SALEC_E_INVALID;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  const State& S = mb.d.S[read_scal(x, k).cycle & 1];
  int rc;
  if (D && (rc = copy_out(x, D, S.dmg, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if (vib && (rc = copy_out(x, vib, S.vib, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int salec_set_materials(salec_ctx* x, int32_t k, const double* mu, const double* Im) {
  if (!member_ok(x, k) || !mu || !Im) return SALEC_E_INVALID;
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  if (!g.closure) {
    x->err = "per-material state needs the per-material closure";
    return SALEC_E_INVALID;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  int rc0 = state_to_level0(x, k);
  if (rc0) return rc0;
  const State& S = mb.d.S[0];
  size_t NC = (size_t)g.NR * g.NZ;
  std::vector<double> rho(NC, 0.0), I(NC, 0.0);
  for (size_t c = 0; c < NC; c++) {
    double r = 0.0, e = 0.0;
    for (int m = 0; m < g.nmat; m++) r += mu[m * NC + c];
    for (int m = 0; m < g.nmat; m++) e += mu[m * NC + c] * Im[m * NC + c];
    if (!std::isfinite(r) || !std::isfinite(e)) {
      x->err = "non-finite per-material state";
      return SALEC_E_INVALID;
    }
    rho[c] = r;
    I[c] = r > 0.0 ? e / r : 0.0;
  }
  int rc;
  for (int m = 0; m < g.nmat; m++) {
    if ((rc = copy_in(x, S.mu[m], mu + m * NC, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
    if ((rc = copy_in(x, S.Im[m], Im + m * NC, g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  }
  if ((rc = copy_in(x, S.rho, rho.data(), g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  if ((rc = copy_in(x, S.I, I.data(), g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  return start_run(x, k);
}

int salec_get_materials(salec_ctx* x, int32_t k, double* mu, double* Im) {
  if (!member_ok(x, k)) return SALEC_E_INVALID;
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  if (!g.closure) {
    x->err = "per-material state needs the per-material closure";
    return SALEC_E_INVALID;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  const State& S = mb.d.S[read_scal(x, k).cycle & 1];
  size_t NC = (size_t)g.NR * g.NZ;
  int rc;
  for (int m = 0; m < g.nmat; m++) {
    if (mu && (rc = copy_out(x, mu + m * NC, S.mu[m], g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
    if (Im && (rc = copy_out(x, Im + m * NC, S.Im[m], g.NR, g.NZ, g.pc, sizeof(double)))) return rc;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

int salec_get_pml(salec_ctx* x, int32_t k, double* ca, double* na) {
  if (!member_ok(x, k)) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1);
  const Pml& pm = mb.d.pm;
  Scal sc_now = read_scal(x, k);
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
      for (int q = 0; q < 3; q++)
        if (fetch(b[q], nbc, h[q]) || fetch(r[q], nrc, h[3 + q])) return SALEC_E_HIP;
      if (fetch(pm.rref, nu, h[6]) || fetch(pm.msink, nu, h[7])) return SALEC_E_HIP;
      for (int j = 0; j < g.NZ; j++)
        for (int i = 0; i < g.NR; i++) {
          size_t c = (size_t)j * g.NR + i;
          if (j < g.pml_b)
            for (int q = 0; q < 3; q++) ca[q * NC + c] = h[q][(size_t)j * g.NR + i];
          if (i >= g.n_r)
            for (int q = 0; q < 3; q++) ca[(3 + q) * NC + c] = h[3 + q][(size_t)j * g.pml_r + (i - g.n_r)];
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
      for (int q = 0; q < 4; q++)
        if (fetch(b[q], nbn, h[q]) || fetch(r[q], nrn, h[4 + q])) return SALEC_E_HIP;
      for (int j = 0; j <= g.NZ; j++)
        for (int i = 0; i <= g.NR; i++) {
          size_t n = (size_t)j * (g.NR + 1) + i;
          if (j < g.pml_b)
            for (int q = 0; q < 4; q++) na[q * NN + n] = h[q][(size_t)j * (g.NR + 1) + i];
          if (i > g.n_r)
            for (int q = 0; q < 4; q++) na[(4 + q) * NN + n] = h[4 + q][(size_t)j * g.pml_r + (i - g.n_r - 1)];
        }
    }
  }
  return SALEC_OK;
}

int salec_set_pml(salec_ctx* x, int32_t k, const double* ca, const double* na) {
  if (!member_ok(x, k)) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  Member& mb = x->ms[k];
  const Geo& g = mb.g;
  if (!g.pml_on) return SALEC_OK;
  size_t NC = (size_t)g.NR * g.NZ, NN = (size_t)(g.NR + 1) * (g.NZ + 1);
  const Pml& pm = mb.d.pm;
  const PmlAux& au = pm.a[read_scal(x, k).cycle & 1];
  size_t nbc = (size_t)g.pml_b * g.NR, nrc = (size_t)g.NZ * g.pml_r, nu = nbc + (size_t)g.n_z * g.pml_r;
  size_t nbn = (size_t)g.pml_b * (g.NR + 1), nrn = (size_t)(g.NZ + 1) * g.pml_r;
  // the layouts of salec_get_pml gathered back into the strips; everything
  // is checked before anything is written
  std::vector<double> hc[8], hn[8];
  if (ca) {
    for (int q = 0; q < 3; q++) {
      hc[q].assign(nbc, 0.0);
      hc[3 + q].assign(nrc, 0.0);
    }
    hc[6].assign(nu, 0.0);
    hc[7].assign(nu, 0.0);
    for (int j = 0; j < g.NZ; j++)
      for (int i = 0; i < g.NR; i++) {
        size_t c = (size_t)j * g.NR + i;
        if (j < g.pml_b)
          for (int q = 0; q < 3; q++) hc[q][(size_t)j * g.NR + i] = ca[q * NC + c];
        if (i >= g.n_r)
          for (int q = 0; q < 3; q++) hc[3 + q][(size_t)j * g.pml_r + (i - g.n_r)] = ca[(3 + q) * NC + c];
        long long u = -1;
        if (j < g.pml_b) u = (long long)j * g.NR + i;
        else if (i >= g.n_r) u = (long long)nbc + (long long)(j - g.pml_b) * g.pml_r + (i - g.n_r);
        if (u >= 0) {
          hc[6][u] = ca[6 * NC + c];
          hc[7][u] = ca[7 * NC + c];
        }
      }
  }
  if (na) {
    for (int q = 0; q < 4; q++) {
      hn[q].assign(nbn, 0.0);
      hn[4 + q].assign(nrn, 0.0);
    }
    for (int j = 0; j <= g.NZ; j++)
      for (int i = 0; i <= g.NR; i++) {
        size_t n = (size_t)j * (g.NR + 1) + i;
        if (j < g.pml_b)
          for (int q = 0; q < 4; q++) hn[q][(size_t)j * (g.NR + 1) + i] = na[q * NN + n];
        if (i > g.n_r)
          for (int q = 0; q < 4; q++) hn[4 + q][(size_t)j * g.pml_r + (i - g.n_r - 1)] = na[(4 + q) * NN + n];
      }
  }
  for (int t = 0; t < 8; t++)
    for (const std::vector<double>* h : {&hc[t], &hn[t]})
      for (double v : *h)
        if (!std::isfinite(v)) {
          x->err = "PML auxiliaries not finite";
          return SALEC_E_INVALID;
        }
  auto put = [&](double* dev, const std::vector<double>& h) -> int {
    if (dev && !h.empty()) HIPCHK(x, hipMemcpy(dev, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
    return SALEC_OK;
  };
  if (ca) {
    double* b[3] = {au.b_phi1, au.b_phi3, au.b_psi2};
    double* r[3] = {au.r_phi1, au.r_phi3, au.r_psi2};
    for (int q = 0; q < 3; q++)
      if (put(b[q], hc[q]) || put(r[q], hc[3 + q])) return SALEC_E_HIP;
    if (put(pm.rref, hc[6]) || put(pm.msink, hc[7])) return SALEC_E_HIP;
  }
  if (na) {
    double* b[4] = {au.b_phi2r, au.b_phi2z, au.b_psi1r, au.b_psi1z};
    double* r[4] = {au.r_phi2r, au.r_phi2z, au.r_psi1r, au.r_psi1z};
    for (int q = 0; q < 4; q++)
      if (put(b[q], hn[q]) || put(r[q], hn[4 + q])) return SALEC_E_HIP;
  }
  return SALEC_OK;
}

int salec_set_clock(salec_ctx* x, int32_t k, double t, double dt) {
  if (!member_ok(x, k)) return SALEC_E_INVALID;
  const Geo& g = x->ms[k].g;
  if (!std::isfinite(t) || t < 0.0 || !std::isfinite(dt) || !(dt > 0.0) || dt > g.dt_max) {
    x->err = "clock needs t >= 0 and 0 < dt <= dt_max";
    return SALEC_E_INVALID;
  }
  if (g.t_stop > 0 && dt > g.t_stop - t) {
    x->err = "time step passes the stop time";
    return SALEC_E_INVALID;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  Scal s = read_scal(x, k);
  s.t = t;
  s.dt = dt;
  HIPCHK(x, hipMemcpyAsync(x->ms[k].d.sc, &s, sizeof(Scal), hipMemcpyHostToDevice, x->st));
  HIPCHK(x, hipStreamSynchronize(x->st));
  return SALEC_OK;
}

size_t salec_state_bytes(const salec_ctx* x) {
  if (!x || !x->ready) return 0;
  return 32 + x->L.persist_bytes;
}

int salec_get_state(salec_ctx* x, void* blob, size_t bytes) {
  if (!x || !blob || !x->ready) return SALEC_E_INVALID;
  if (bytes < salec_state_bytes(x)) return SALEC_E_BUFFER;
  HIPCHK(x, hipStreamSynchronize(x->st));
  uint64_t head[4] = {kStateMagic, (uint64_t)x->L.persist_bytes, (uint64_t)x->ms.size(), (uint64_t)x->prec};
  std::memcpy(blob, head, 32);
  HIPCHK(x, hipMemcpy((uint8_t*)blob + 32, x->buf, x->L.persist_bytes, hipMemcpyDeviceToHost));
  return SALEC_OK;
}

int salec_set_state(salec_ctx* x, const void* blob, size_t bytes) {
  if (!x || !blob || !x->ready) return SALEC_E_INVALID;
  if (bytes < salec_state_bytes(x)) return SALEC_E_BUFFER;
  uint64_t head[4];
  std::memcpy(head, blob, 32);
  if (head[0] != kStateMagic || head[1] != x->L.persist_bytes || head[2] != x->ms.size() ||
      head[3] != (uint64_t)x->prec) {
    x->err = "state blob does not match this context";
    return SALEC_E_INVALID;
  }
  HIPCHK(x, hipStreamSynchronize(x->st));
  HIPCHK(x, hipMemcpy(x->buf, (const uint8_t*)blob + 32, x->L.persist_bytes, hipMemcpyHostToDevice));
  return SALEC_OK;
}

int salec_diag(salec_ctx* x, int32_t k, salec_diag_t* out) {
  if (!member_ok(x, k) || !out) return SALEC_E_INVALID;
  HIPCHK(x, hipStreamSynchronize(x->st));
  Member& mb = x->ms[k];
  HIPCHK(x, launch_diag(mb.d, mb.n_pml, x->L.red, x->L.diag_out, x->st));
  double q[kDiagQ];
  HIPCHK(x, hipMemcpyAsync(q, x->L.diag_out, sizeof(q), hipMemcpyDeviceToHost, x->st));
  Scal s = read_scal(x, k);
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

int salec_diag_totals(salec_ctx* x, int32_t k, double* dev_totals) {
  if (!member_ok(x, k) || !dev_totals) return SALEC_E_INVALID;
  if (!x->diag_scratch) {
    x->err = "salec_diag_totals: no device scratch for this context";
    return SALEC_E_HIP;
  }
  // every block overwrites all its partials, so nothing needs clearing
  Member& mb = x->ms[k];
  HIPCHK(x, launch_diag(mb.d, mb.n_pml, x->diag_scratch, dev_totals, x->st));
  return SALEC_OK;
}

int32_t salec_num_variants(void) { return n_variants(); }

int salec_get_schedule(const salec_ctx* x, salec_schedule* out) {
  if (!x || !out || !x->ready) return SALEC_E_INVALID;
  std::memset(out, 0, sizeof(*out));
  out->variant = x->variant;
  variant_shape(x->variant, &out->tile_r, &out->tile_z, &out->threads);
  out->grid = x->grid;
  out->ms_per_cycle = x->tuned_ms;
  return SALEC_OK;
}

int salec_set_schedule(salec_ctx* x, int32_t variant, int32_t grid) {
  if (!x || !x->ready) return SALEC_E_INVALID;
  // a schedule the context cannot run is refused without touching it
  int rc = check_schedule(x, variant, grid);
  if (rc) return rc;
  x->tuned_ms = 0.0;
  rc = use_schedule(x, variant, grid);
  if (rc) x->ready = false;
  return rc;
}

int salec_tune(salec_ctx* x, int32_t cycles, salec_schedule* out) {
  if (!x || !x->ready || cycles < 1) return SALEC_E_INVALID;
  int best_v = x->variant, best_g = x->grid;
  double best = 1e300;
  for (int v = 0; v < n_variants(); v++) {
    if (!variant_available(v, x->prec, x->geo, x->nm, x->pm, x->dm)) continue;
    // one workgroup per tile, and as many workgroups as fit at once walking
    // the tiles (when that is fewer than the tiles)
    int grids[2] = {0, resident_groups(v, x->prec, x->geo, x->nm, x->pm, x->dm)};
    for (int gi = 0; gi < 2; gi++) {
      if (gi == 1 && (grids[1] <= 0 || grids[1] >= x->nsched)) continue;
      int rc = use_schedule(x, v, grids[gi]);
      if (rc) {
        x->ready = false;
        return rc;
      }
      if ((rc = salec_step(x, 1))) return rc;
      if ((rc = salec_step(x, cycles))) return rc;
      double ms = x->last_ms / cycles;
      if (ms < best) {
        best = ms;
        best_v = v;
        best_g = grids[gi];
      }
    }
  }
  int rc = use_schedule(x, best_v, best_g);
  if (rc) {
    x->ready = false;
    return rc;
  }
  x->tuned_ms = best;
  if (out) return salec_get_schedule(x, out);
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
