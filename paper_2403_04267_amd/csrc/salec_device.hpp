// salec_device.hpp -- device-side data layout and per-cell physics of the
// r-z SALE cycle with PML (internal to libsalec).
//
// Method: Li et al., SALEc-2D. Sec. 2 eqs. (1)-(5) (Lagrangian + Eulerian
// split), Sec. 3 (PML), Sec. 4 (boundary conditions), Table 1 (strength),
// Sec. 7 (Courant step). The discrete readings of points the paper leaves
// open (staggered grid, Tillotson EoS, viscosity, mixed cells, remap) are
// the ones documented with the library; every expression below keeps the
// evaluation order of that discrete algorithm so FP64 results reproduce it
// to rounding.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace salec {

constexpr int kMaxMat = 3;
constexpr double kPhiEps = 1e-12;       // volume fraction treated as void
constexpr double kRhoEosFloor = 1e-6;   // EoS density floor (x rho0)
constexpr double kRhoDenFloor = 1e-6;   // energy-update density floor (x rho_ref)
constexpr double kPmlRhoFloor = 1e-3;   // PML density floor (x rho_ref)
constexpr double kMAccEps = 1e-3;       // acceleration mass floor (x rho_ref V_dual)
constexpr double kMRemapFloor = 1e-9;   // remap denominator floor (x rho_ref V)
constexpr double kWLo = 1e-3, kWHi = 1e-2;  // CFL void-weight ramp
constexpr double kNegMassTol = 1e-9;    // density below -tol rho_ref is an error
constexpr double kPcavFrac = 1e-4;      // cavitation pressure ramp (x A)
constexpr double kFPmEps = 1e-6;        // per-material closure: below this volume
                                        // fraction a material takes the cell's matter density
constexpr double kVibOn = 1e-3;         // block model: vibration speed (m/s) above which
                                        // its viscosity acts fully (linear ramp below)

// error flags raised by kernels, turned into codes by the finalize kernel
constexpr unsigned kFlagNonFinite = 1u, kFlagNegMass = 2u;

// Material constants in the bulk arithmetic type (double; float copies for
// the mixed mode).
template <class T>
struct MatT {
  T rho0, A, B, E0, a, b, alpha, beta, Eiv, Ecv;
  T p_min, cf2;   // pressure floor, c^2 floor
  T gfac;         // shear / bulk modulus ratio (0: no strength)
  T Y0, mu_f, Ylim;
  T pcav;         // cavitation pressure ramp
  // 1/rho0, A/rho0, 1/(Ecv - Eiv), 1/(Ylim - Y0), formed once on the host in
  // FP64; only the FP32 arithmetic uses them (FP64 divides as the method does)
  T irho0, Ar, idE, iYd;
  // damage and the block model of acoustic fluidization (Table 1's damaged
  // cohesion, friction and limit; gamma_eta, gamma_T, c_vib): the damaged
  // curve, the failure strain max(eps_fb, B_dmg (p - p_bd)), the
  // longitudinal speed at rest cL0, the kinematic viscosity gamma_eta cL0 h
  // and the vibration decay time gamma_T h / cL0 (h: block size)
  T Yd0, mu_d, Ydm, eps_fb, B_dmg, p_bd, cL0, nub, Tvib, c_vib;
  int strength, damage;
};
using MatC = MatT<double>;
using MatF = MatT<float>;

struct Geo {
  int NR, NZ, n_r, n_z, pml_r, pml_b, nmat, top_closed;
  int pc, pn;          // row pitch (elements) of cell and node arrays
  int any_strength, pml_on;
  int same_mat;        // all materials share every constant: evaluate the laws once
  int prec;            // 0: FP64 throughout; 1: FP32 bulk with FP64 energy, mass and volume sums
  int has_p0;          // nonzero initial (lithostatic) pressure profile
  int stretched;       // per-column widths / per-row heights from the geometry table
  int closure;         // 0: shared material density and energy; 1: per material
  int damp_stress;     // the PML layers also relax the deviatoric stress (extension)
  int pml_place;       // 1: phi in the Lagrangian and psi in the Eulerian step
  int dmg;             // some material accumulates damage (state D, v_vib)
  double dr, dz, cfl, dt_grow, dt_max, dt_floor, t_stop, q_lin, q_quad;
  double rho_ref;
  float drf, dzf, q_linf, q_quadf, rho_reff, pad_f;
  MatC m[kMaxMat];
  MatF mf[kMaxMat];
};

template <class T> struct GeoT;
template <> struct GeoT<double> {
  static __device__ __forceinline__ const MatC& mat(const Geo& g, int m) { return g.m[m]; }
  static __device__ __forceinline__ double dr(const Geo& g) { return g.dr; }
  static __device__ __forceinline__ double dz(const Geo& g) { return g.dz; }
  static __device__ __forceinline__ double q_lin(const Geo& g) { return g.q_lin; }
  static __device__ __forceinline__ double q_quad(const Geo& g) { return g.q_quad; }
  static __device__ __forceinline__ double rho_ref(const Geo& g) { return g.rho_ref; }
};
template <> struct GeoT<float> {
  static __device__ __forceinline__ const MatF& mat(const Geo& g, int m) { return g.mf[m]; }
  static __device__ __forceinline__ float dr(const Geo& g) { return g.drf; }
  static __device__ __forceinline__ float dz(const Geo& g) { return g.dzf; }
  static __device__ __forceinline__ float q_lin(const Geo& g) { return g.q_linf; }
  static __device__ __forceinline__ float q_quad(const Geo& g) { return g.q_quadf; }
  static __device__ __forceinline__ float rho_ref(const Geo& g) { return g.rho_reff; }
};

// EoS results of a state level, written with the state that produced them
// and read by the next cycle (p, c^2, G, Y, cavitation weight).
constexpr int kEos = 5;

// One copy of the evolving state (two copies ping-pong by cycle parity).
// rho, I and f are FP64 in every precision; stress, velocity and the EoS
// cache hold the bulk type (double, or float in the mixed mode). With the
// per-material closure, mu (partial densities: mass of each material per
// cell volume) and Im (its specific energies) are the FP64 state, rho and I
// their sum and mass-weighted energy, and pmat caches each material's
// pressure with the EoS.
struct State {
  double *rho, *I, *f[kMaxMat];
  void *s[3], *v[2], *eos[kEos];
  double *mu[kMaxMat], *Im[kMaxMat];
  void* pmat[kMaxMat];
  // damage and block-model vibration speed (FP64 in every precision;
  // allocated when some material accumulates damage)
  double *dmg, *vib;
};

// Scalars living in device memory so that captured graphs can be replayed.
struct Scal {
  double t, dt, dt_prev;
  long long cycle;
  unsigned long long dtmin;  // bit pattern of the running minimum (dt > 0)
  unsigned flags;
  unsigned pad;
  int err, err_cycle;
};

// PML auxiliaries of one time level; two levels ping-pong by cycle parity so
// that halo reads of neighbouring tiles always see the old values.
struct PmlAux {
  double *b_phi1, *b_phi3, *b_psi2;               // bottom strip cells  [pml_b][NR]
  double *r_phi1, *r_phi3, *r_psi2;               // right strip cells   [NZ][pml_r]
  double *b_phi2r, *b_phi2z, *b_psi1r, *b_psi1z;  // bottom strip nodes  [pml_b][NR+1]
  double *r_phi2r, *r_phi2z, *r_psi1r, *r_psi1z;  // right strip nodes   [NZ+1][pml_r]
};

struct Pml {
  const double *dcz, *dnz, *dcr, *dnr;  // damping profiles
  double *rref, *msink;                 // union of strip cells (single level)
  PmlAux a[2];
};

// One simulation instance as the cycle kernel sees it (device resident).
struct Inst {
  Geo g;
  State S[2];
  Pml pm;
  Scal* sc;
  double* dtpart;         // per-tile Courant minima
  double *mout, *eout;    // per-column outflow budgets (mass, internal energy)
  const double* p0;       // initial pressure per cell row (read when g.has_p0)
  // geometry table of a stretched grid (read when g.stretched): six column
  // fields of NR + 1 entries (node radius, centre radius, width, west / east
  // half areas, area per unit height), then the row heights and the node
  // heights (NZ + 1 entries each)
  const double* geo;
  int tiles_r, tiles_z;   // tile grid of this instance
  int ntiles, pad;
};

// One entry of the launch schedule: a tile of an instance.
struct TileRef {
  int inst, tile;
};

__device__ __forceinline__ double dmax(double a, double b) { return a > b ? a : b; }
__device__ __forceinline__ double dmin(double a, double b) { return a < b ? a : b; }

__device__ __forceinline__ long long cidx(const Geo& g, int i, int j) { return (long long)j * g.pc + i; }
__device__ __forceinline__ long long nidx(const Geo& g, int i, int j) { return (long long)j * g.pn + i; }
__device__ __forceinline__ long long fridx(const Geo& g, int i, int j) { return (long long)j * g.pn + i; }
__device__ __forceinline__ long long fzidx(const Geo& g, int i, int j) { return (long long)j * g.pc + i; }

// PML storage: union index of a layer cell (bottom block first, then the
// part of the right strip above it), and per-strip indices.
__device__ __forceinline__ long long pml_cell_union(const Geo& g, int i, int j) {
  if (j < g.pml_b) return (long long)j * g.NR + i;
  return (long long)g.pml_b * g.NR + (long long)(j - g.pml_b) * g.pml_r + (i - g.n_r);
}
__device__ __forceinline__ long long pml_bc(const Geo& g, int i, int j) { return (long long)j * g.NR + i; }
__device__ __forceinline__ long long pml_rc(const Geo& g, int i, int j) { return (long long)j * g.pml_r + (i - g.n_r); }
__device__ __forceinline__ long long pml_bn(const Geo& g, int i, int j) { return (long long)j * (g.NR + 1) + i; }
__device__ __forceinline__ long long pml_rn(const Geo& g, int i, int j) { return (long long)j * g.pml_r + (i - g.n_r - 1); }

// ------------------------------------------------------------------ exp
// e^x by Cody & Waite reduction (x = k ln2 + r, ln2 as a 32-bit head plus a
// tail) and the degree-13 Taylor polynomial of e^r in Horner form, scaled by
// 2^k built from its exponent bits. Below e^-700 the result is 0, above
// e^709 +inf. A fixed published method, so every IEEE-754 implementation of
// it rounds identically (no contraction: built with -ffp-contract=off).
__device__ inline double exp_cw(double x) {
  if (x != x) return x;
  if (x < -700.0) return 0.0;
  if (x > 709.0) return __builtin_huge_val();
  const double inv_ln2 = 0x1.71547652b82fep+0;
  const double ln2_hi = 0x1.62e42fee00000p-1;
  const double ln2_lo = 0x1.a39ef35793c76p-33;
  double kd = floor(x * inv_ln2 + 0.5);
  double r = (x - kd * ln2_hi) - kd * ln2_lo;
  double q = 1.0 / 6227020800.0;
  q = q * r + 1.0 / 479001600.0;
  q = q * r + 1.0 / 39916800.0;
  q = q * r + 1.0 / 3628800.0;
  q = q * r + 1.0 / 362880.0;
  q = q * r + 1.0 / 40320.0;
  q = q * r + 1.0 / 5040.0;
  q = q * r + 1.0 / 720.0;
  q = q * r + 1.0 / 120.0;
  q = q * r + 1.0 / 24.0;
  q = q * r + 1.0 / 6.0;
  q = q * r + 0.5;
  q = q * r + 1.0;
  q = q * r + 1.0;
  long long k = (long long)kd;
  return q * __longlong_as_double((k + 1023) << 52);
}

// Elementary operations of the bulk type. FP64 keeps IEEE division, square
// root and the fixed exponential above (reproducible to the bit); the mixed
// mode's FP32 uses the hardware reciprocal, square root and exponential.
// divk(a, b, ib) and qk(a, b, q) divide by a material constant b: FP64 forms
// the quotient a / b, FP32 multiplies by the reciprocal ib (or takes the
// quotient q) the host formed once.
template <class T> struct Num;
template <> struct Num<double> {
  static __device__ __forceinline__ double div(double a, double b) { return a / b; }
  static __device__ __forceinline__ double divk(double a, double b, double) { return a / b; }
  static __device__ __forceinline__ double qk(double a, double b, double) { return a / b; }
  static __device__ __forceinline__ double sqr(double a) { return sqrt(a); }
  static __device__ __forceinline__ double ex(double a) { return exp_cw(a); }
  static __device__ __forceinline__ double inf() { return __builtin_huge_val(); }
};
template <> struct Num<float> {
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  static __device__ __forceinline__ float divk(float a, float, float ib) { return a * ib; }
  static __device__ __forceinline__ float qk(float, float, float q) { return q; }
  static __device__ __forceinline__ float sqr(float a) { return __builtin_sqrtf(a); }
  static __device__ __forceinline__ float ex(float a) { return __expf(a); }
  static __device__ __forceinline__ float inf() { return __builtin_huge_valf(); }
};
template <class T> __device__ __forceinline__ T tmax(T a, T b) { return a > b ? a : b; }
template <class T> __device__ __forceinline__ T tmin(T a, T b) { return a < b ? a : b; }

// ------------------------------------------------------------------ EoS
// Density terms of the Tillotson law at material density rho (floored at
// 1e-6 rho0): r, eta = r / rho0, mu = eta - 1, z = 1 / eta - 1. FP32 forms
// them in FP64 from the FP64 density and rounds once, since mu and z cancel
// most of their digits in weak waves.
template <class T>
struct Dens {
  T r, eta, mu, z;
};
__device__ __forceinline__ Dens<double> dens_terms(const MatC& m, double rho, double*) {
  Dens<double> d;
  double rf = m.rho0 * kRhoEosFloor;
  d.r = rho > rf ? rho : rf;
  d.eta = d.r / m.rho0;
  d.mu = d.eta - 1.0;
  d.z = 1.0 / d.eta - 1.0;
  return d;
}
__device__ __forceinline__ Dens<float> dens_terms(const MatC& m, double rho, float*) {
  // mu from the FP64 density (one FP64 multiply); eta = 1 + mu and
  // z = 1/eta - 1 = -mu/eta then lose nothing in FP32
  Dens<float> d;
  double rf = m.rho0 * kRhoEosFloor;
  double r = rho > rf ? rho : rf;
  d.r = (float)r;
  d.mu = (float)((r - m.rho0) * m.irho0);
  d.eta = 1.0f + d.mu;
  d.z = -Num<float>::div(d.mu, d.eta);
  return d;
}

// Four-region Tillotson pressure and squared sound speed at the density
// terms d and specific internal energy e (the EoS sees max(e, 0)).
template <class T>
__device__ inline void tillotson(const MatT<T>& m, const Dens<T>& d, T e, T& p_out, T& c2_out) {
  using N = Num<T>;
  const T r = d.r, eta = d.eta, mu = d.mu;
  T E = e > T(0) ? e : T(0);
  T w = N::div(E, m.E0 * eta * eta) + T(1);
  T bw = N::div(m.b, w);
  T pc = (m.a + bw) * r * E + m.A * mu + m.B * mu * mu;
  T pc_E = r * (m.a + bw - N::div(m.b * (w - T(1)), w * w));
  T pc_r = (m.a + bw) * E + N::div(T(2) * m.b * E * (w - T(1)), w * w) +
           N::divk(m.A + T(2) * m.B * mu, m.rho0, m.irho0);
  T p, dpdE, dpdr;
  if (r >= m.rho0 || E <= m.Eiv) {
    p = pc;
    dpdE = pc_E;
    dpdr = pc_r;
  } else {
    T z = d.z;
    T ea = N::ex(-m.alpha * z * z);
    T eb = N::ex(-m.beta * z);
    T rr = r * r;
    T brw = N::div(m.b * r * E, w);
    T pe = m.a * r * E + (brw + m.A * mu * eb) * ea;
    T pe_E = m.a * r + ea * m.b * r * (N::div(T(1), w) - N::div(w - T(1), w * w));
    T pe_r = m.a * E +
             ea * (N::div(m.b * E, w) + N::div(T(2) * m.b * E * (w - T(1)), w * w) + N::qk(m.A, m.rho0, m.Ar) * eb +
                   N::div(m.A * mu * m.beta * eb * m.rho0, rr)) +
             N::div((brw + m.A * mu * eb) * ea * T(2) * m.alpha * z * m.rho0, rr);
    if (E >= m.Ecv) {
      p = pe;
      dpdE = pe_E;
      dpdr = pe_r;
    } else {
      T x = N::divk(E - m.Eiv, m.Ecv - m.Eiv, m.idE);
      p = x * pe + (T(1) - x) * pc;
      dpdE = x * pe_E + (T(1) - x) * pc_E + N::divk(pe - pc, m.Ecv - m.Eiv, m.idE);
      dpdr = x * pe_r + (T(1) - x) * pc_r;
    }
  }
  p_out = p;
  c2_out = dpdr + N::div(p, r * r) * dpdE;
}

// intact-rock yield curve (Table 1 parameters)
template <class T>
__device__ inline T yield_strength(const MatT<T>& m, T p) {
  if (!m.strength) return T(0);
  if (p >= T(0)) {
    T mp = m.mu_f * p;
    return m.Y0 + Num<T>::div(mp, T(1) + Num<T>::divk(mp, m.Ylim - m.Y0, m.iYd));
  }
  return tmax(T(0), m.Y0 + m.mu_f * p);
}

// Strength of a material with damage D (Table 1's damaged cohesion Y_d0,
// friction mu_d and limit Y_dm): the damaged curve min(Y_d0 + mu_d q, Y_dm)
// at the effective pressure q = max(p - pv, 0), pv the block model's
// vibration pressure, for p >= 0, max(0, Y_d0 + mu_d p) in tension, never
// above the intact curve; the two blend linearly in D.
template <class T>
__device__ inline T yield_damaged(const MatT<T>& m, T p, T D, T pv) {
  T Yi = yield_strength(m, p);
  if (!m.strength || !m.damage) return Yi;
  T Yd;
  if (p >= T(0))
    Yd = tmin(m.Yd0 + m.mu_d * tmax(p - pv, T(0)), m.Ydm);
  else
    Yd = tmax(T(0), m.Yd0 + m.mu_d * p);
  Yd = tmin(Yd, Yi);
  return (T(1) - D) * Yi + D * Yd;
}

// strength fades linearly between incipient and complete vaporisation
template <class T>
__device__ inline T softening(const MatT<T>& m, T e) {
  T E = e > T(0) ? e : T(0);
  return tmin(tmax(Num<T>::divk(m.Ecv - E, m.Ecv - m.Eiv, m.idE), T(0)), T(1));
}

template <class T>
struct Mix {
  T p, c2, G, Y, rmat, phi, sx;
};

// volume fraction of matter, its floored value den (the weights of the
// materials are f_m / den) and the shared material density of a mixed cell
template <class T>
__device__ __forceinline__ void matter(const Geo& g, T rho, const T* f, T& phi, T& den, T& rm) {
  phi = T(0);
#pragma unroll
  for (int m = 0; m < kMaxMat; m++)
    if (m < g.nmat) phi += f[m];
  den = phi > T(kPhiEps) ? phi : T(kPhiEps);
  rm = Num<T>::div(rho, den);
}

// Mixed-cell state from the FP64 cell state (rho, I, f): all materials
// share rho_mat = rho / phi and I; p, c^2, G, Y are volume-fraction
// weighted; sx is the expansion weight of the cavitation rule (1 above the
// tension floor + ramp). Arithmetic in T (the density terms as above).
// DM: the yield is the damaged strength at the cell's damage Dc and the
// vibration pressure rho_mat cL0 vibc of each material.
template <class T, bool DM = false>
__device__ inline Mix<T> mixture(const Geo& g, double rho, double I, const double* fd, double Dc = 0.0,
                                 double vibc = 0.0) {
  using N = Num<T>;
  Mix<T> o;
  T f[kMaxMat];
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) f[m] = m < g.nmat ? (T)fd[m] : T(0);
  T phi, den, rm;
  matter(g, (T)rho, f, phi, den, rm);
  // material density for the density terms, in FP64
  double phid = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxMat; m++)
    if (m < g.nmat) phid += fd[m];
  double rmd = rho / (phid > kPhiEps ? phid : kPhiEps);
  T Ie = (T)I;
  T p = T(0), c2 = T(0), G = T(0);
  T wm[kMaxMat], pmv[kMaxMat], c2v[kMaxMat], sov[kMaxMat];
  // A material absent from the cell (f = 0) would add exactly +0 to every
  // sum below (its laws give finite values times a zero weight), so it is
  // not evaluated at all; sums that skip it are bit-identical.
  bool have0 = false;
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) {
    if (m >= g.nmat) break;
    const MatT<T>& M = GeoT<T>::mat(g, m);
    wm[m] = N::div(f[m], den);
    pmv[m] = c2v[m] = sov[m] = T(0);
    if (fd[m] == 0.0) continue;
    if (m > 0 && g.same_mat && have0) {
      // identical constants and inputs give identical results
      pmv[m] = pmv[0];
      c2v[m] = c2v[0];
      sov[m] = sov[0];
    } else {
      T pm, c2m;
      Dens<T> dn = dens_terms(g.m[m], rmd, (T*)nullptr);
      tillotson(M, dn, Ie, pm, c2m);
      pmv[m] = tmax(pm, M.p_min);
      c2v[m] = tmax(c2m, M.cf2);
      sov[m] = softening(M, Ie);
      if (m == 0) have0 = true;
    }
    p += wm[m] * pmv[m];
    c2 += wm[m] * c2v[m];
    G += wm[m] * (sov[m] * (M.gfac * (rm * c2v[m])));
  }
  T Y = T(0), pmin = T(0), ps = T(0), y0 = T(0);
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) {
    if (m >= g.nmat) break;
    if (fd[m] == 0.0) continue;
    const MatT<T>& M = GeoT<T>::mat(g, m);
    T ym;
    if (m > 0 && g.same_mat && have0)
      ym = y0;
    else if constexpr (DM)
      ym = yield_damaged(M, p, (T)Dc, rm * M.cL0 * (T)vibc);
    else
      ym = yield_strength(M, p);
    if (m == 0) y0 = ym;
    Y += wm[m] * (sov[m] * ym);
    pmin += wm[m] * M.p_min;
    ps += wm[m] * M.pcav;
  }
  T d = p - pmin;
  o.sx = d >= ps ? T(1) : (ps > T(0) ? N::div(tmax(d, T(0)), ps) : T(0));
  o.p = p;
  o.c2 = c2;
  o.G = G;
  o.Y = Y;
  o.rmat = rm;
  o.phi = phi;
  return o;
}

// Per-material closure: the same volume-fraction average, every material at
// its own density rho_m = mu_m / f_m (below a volume fraction of kFPmEps, or
// without mass, at the cell's matter density) and its own specific energy
// Im_m. pmv receives each material's pressure after its floor (0 for a
// material absent from the cell, which adds nothing anywhere).
template <class T, bool DM = false>
__device__ inline Mix<T> mixture_pm(const Geo& g, double rho, const double* fd, const double* mud,
                                    const double* Imd, T* pmv, double Dc = 0.0, double vibc = 0.0) {
  using N = Num<T>;
  Mix<T> o;
  T f[kMaxMat];
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) f[m] = m < g.nmat ? (T)fd[m] : T(0);
  T phi, den, rm;
  matter(g, (T)rho, f, phi, den, rm);
  double phid = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxMat; m++)
    if (m < g.nmat) phid += fd[m];
  double rmd = rho / (phid > kPhiEps ? phid : kPhiEps);
  T p = T(0), c2 = T(0), G = T(0);
  T wm[kMaxMat], sov[kMaxMat], rmv[kMaxMat];
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) {
    pmv[m] = T(0);
    rmv[m] = T(0);
    if (m >= g.nmat) break;
    const MatT<T>& M = GeoT<T>::mat(g, m);
    wm[m] = N::div(f[m], den);
    sov[m] = T(0);
    if (fd[m] == 0.0) continue;
    double rmm = fd[m] > kFPmEps && mud[m] > 0.0 ? mud[m] / fd[m] : rmd;
    rmv[m] = (T)rmm;
    T pm, c2m;
    Dens<T> dn = dens_terms(g.m[m], rmm, (T*)nullptr);
    T Ie = (T)Imd[m];
    tillotson(M, dn, Ie, pm, c2m);
    pmv[m] = tmax(pm, M.p_min);
    T c2v = tmax(c2m, M.cf2);
    sov[m] = softening(M, Ie);
    p += wm[m] * pmv[m];
    c2 += wm[m] * c2v;
    G += wm[m] * (sov[m] * (M.gfac * ((T)rmm * c2v)));
  }
  T Y = T(0), pmin = T(0), ps = T(0);
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) {
    if (m >= g.nmat) break;
    if (fd[m] == 0.0) continue;
    const MatT<T>& M = GeoT<T>::mat(g, m);
    T ym;
    if constexpr (DM)
      ym = yield_damaged(M, p, (T)Dc, rmv[m] * M.cL0 * (T)vibc);
    else
      ym = yield_strength(M, p);
    Y += wm[m] * (sov[m] * ym);
    pmin += wm[m] * M.p_min;
    ps += wm[m] * M.pcav;
  }
  T d = p - pmin;
  o.sx = d >= ps ? T(1) : (ps > T(0) ? N::div(tmax(d, T(0)), ps) : T(0));
  o.p = p;
  o.c2 = c2;
  o.G = G;
  o.Y = Y;
  o.rmat = rm;
  o.phi = phi;
  return o;
}

// material volume ratio (void closes first; expansion gated by cavitation)
template <class T>
__device__ __forceinline__ T material_ratio(T J, T phi, T sx) {
  if (J < T(1)) return tmin(T(1), Num<T>::div(J, tmax(phi, T(kPhiEps))));
  return T(1) + (J - T(1)) * sx;
}

// Volume-change terms of a cell whose volume ratio over the step is
// J = 1 + dD (dD = dt * div v). FP64 forms them from J exactly as the
// discrete algorithm is written; FP32 forms them from dD, because J - 1 and
// 1 - ratio would cancel away most of the digits of dD in single precision.
template <class T> struct Vol;
template <> struct Vol<double> {
  static __device__ __forceinline__ double jm1(double J, double) { return J - 1.0; }
  static __device__ __forceinline__ double ratio(double J, double, double phi, double sx) {
    return material_ratio(J, phi, sx);
  }
  // 1 - ratio, for J < 1
  static __device__ __forceinline__ double closing(double J, double, double phi, double sx) {
    return 1.0 - material_ratio(J, phi, sx);
  }
};
template <> struct Vol<float> {
  static __device__ __forceinline__ float jm1(float, float dD) { return dD; }
  static __device__ __forceinline__ float ratio(float J, float dD, float phi, float sx) {
    if (J < 1.0f) return tmin(1.0f, Num<float>::div(J, tmax(phi, (float)kPhiEps)));
    return 1.0f + dD * sx;
  }
  static __device__ __forceinline__ float closing(float, float dD, float phi, float) {
    float ph = tmax(phi, (float)kPhiEps);
    return tmax(0.0f, Num<float>::div((ph - 1.0f) - dD, ph));
  }
};

// Geometry of one cell column (per radian): node radii rw, re, centre radius
// rc, width dr, the r-weighted areas of its west and east halves
// aw = 0.5 (rc^2 - rw^2), ae = 0.5 (re^2 - rc^2), and its area per unit
// height az = rc dr. The west and east halves of node i are aw(i) and
// ae(i - 1).
template <class T>
struct Col {
  T rw, re, rc, dr, aw, ae, az;
};

// Column i of a uniform grid. FP64 evaluates the half areas as written; FP32
// uses the exact factored forms dr^2 (2i + 1/2) / 4 and dr^2 (2i + 3/2) / 4,
// since the difference of squares cancels at large radius.
template <class T> __device__ Col<T> col_uniform(const Geo& g, int i);
template <>
__device__ __forceinline__ Col<double> col_uniform<double>(const Geo& g, int i) {
  Col<double> c;
  c.rw = (double)i * g.dr;
  c.re = (double)(i + 1) * g.dr;
  c.rc = ((double)i + 0.5) * g.dr;
  c.dr = g.dr;
  c.aw = 0.5 * (c.rc * c.rc - c.rw * c.rw);
  c.ae = 0.5 * (c.re * c.re - c.rc * c.rc);
  c.az = c.rc * g.dr;
  return c;
}
template <>
__device__ __forceinline__ Col<float> col_uniform<float>(const Geo& g, int i) {
  Col<float> c;
  c.rw = (float)i * g.drf;
  c.re = (float)(i + 1) * g.drf;
  c.rc = ((float)i + 0.5f) * g.drf;
  c.dr = g.drf;
  c.aw = (0.25f * g.drf * g.drf) * (2.0f * (float)i + 0.5f);
  c.ae = (0.25f * g.drf * g.drf) * (2.0f * (float)i + 1.5f);
  c.az = c.rc * g.drf;
  return c;
}

// Column i from six FP64 fields with the given stride (0 <= i <= NR; at
// i = NR only the node radius is meaningful).
template <class T>
__device__ __forceinline__ Col<T> col_fields(const double* t, int stride, int i) {
  Col<T> c;
  c.rw = (T)t[i];
  c.re = (T)t[i + 1];
  c.rc = (T)t[stride + i];
  c.dr = (T)t[2 * stride + i];
  c.aw = (T)t[3 * stride + i];
  c.ae = (T)t[4 * stride + i];
  c.az = (T)t[5 * stride + i];
  return c;
}

// Column geometry, row height and node height of an instance, from its
// table when the grid is stretched (kernels outside the cycle kernel).
template <class T>
__device__ __forceinline__ Col<T> col_of(const Geo& g, const double* geo, int i) {
  return g.stretched ? col_fields<T>(geo, g.NR + 1, i) : col_uniform<T>(g, i);
}
__device__ __forceinline__ double dz_of(const Geo& g, const double* geo, int j) {
  return g.stretched ? geo[6 * (g.NR + 1) + j] : g.dz;
}
__device__ __forceinline__ double zn_of(const Geo& g, const double* geo, int j) {
  return g.stretched ? geo[6 * (g.NR + 1) + (g.NZ + 1) + j] : (double)j * g.dz;
}

// ------------------------------------------------------------------ kinematics
template <class T>
struct Kin {
  T D, Dr, Dz, err, ezz, ett, erz, om, dvr_dz, dvz_dr;
};

// Face-mean velocities and rates of a cell of column c and height dz from
// the corner velocities (SW, SE, NW, NE). Axial faces weight their nodes by
// the r-weighted areas of the node dual cells, so the node force is the exact
// volume gradient.
template <class T>
__device__ inline Kin<T> kinematics(const Col<T>& c, T dz, const T vr[4], const T vz[4]) {
  using N = Num<T>;
  Kin<T> k;
  T Arw = c.rw * dz, Are = c.re * dz, V = c.az * dz;
  T aw = c.aw, ae = c.ae;
  T ur_w = T(0.5) * (vr[0] + vr[2]);
  T ur_e = T(0.5) * (vr[1] + vr[3]);
  T Ur_w = Arw * ur_w;
  T Ur_e = Are * ur_e;
  T Uz_s = aw * vz[0] + ae * vz[1];
  T Uz_n = aw * vz[2] + ae * vz[3];
  k.Dr = N::div(Ur_e - Ur_w, V);
  k.Dz = N::div(Uz_n - Uz_s, V);
  k.D = N::div((Ur_e - Ur_w) + (Uz_n - Uz_s), V);
  k.err = N::div(ur_e - ur_w, c.dr);
  k.ezz = k.Dz;
  k.ett = N::div(T(0.5) * (ur_w + ur_e), c.rc);
  k.dvr_dz = N::div((aw * vr[2] + ae * vr[3]) - (aw * vr[0] + ae * vr[1]), V);
  k.dvz_dr = N::div(T(0.5) * (vz[1] + vz[3]) - T(0.5) * (vz[0] + vz[2]), c.dr);
  k.erz = T(0.5) * (k.dvr_dz + k.dvz_dr);
  k.om = T(0.5) * (k.dvr_dz - k.dvz_dr);
  return k;
}

}  // namespace salec
