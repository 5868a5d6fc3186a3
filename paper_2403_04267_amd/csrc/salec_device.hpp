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

constexpr int kMaxMat = 2;
constexpr double kPhiEps = 1e-12;       // volume fraction treated as void
constexpr double kRhoEosFloor = 1e-6;   // EoS density floor (x rho0)
constexpr double kRhoDenFloor = 1e-6;   // energy-update density floor (x rho_ref)
constexpr double kPmlRhoFloor = 1e-3;   // PML density floor (x rho_ref)
constexpr double kMAccEps = 1e-3;       // acceleration mass floor (x rho_ref V_dual)
constexpr double kMRemapFloor = 1e-9;   // remap denominator floor (x rho_ref V)
constexpr double kWLo = 1e-3, kWHi = 1e-2;  // CFL void-weight ramp
constexpr double kNegMassTol = 1e-9;    // density below -tol rho_ref is an error
constexpr double kPcavFrac = 1e-4;      // cavitation pressure ramp (x A)

// error flags raised by kernels, turned into codes by the finalize kernel
constexpr unsigned kFlagNonFinite = 1u, kFlagNegMass = 2u;

struct MatC {
  double rho0, A, B, E0, a, b, alpha, beta, Eiv, Ecv;
  double p_min, cf2;   // pressure floor, c^2 floor
  double gfac;         // shear / bulk modulus ratio (0: no strength)
  double Y0, mu_f, Ylim;
  double pcav;         // cavitation pressure ramp
  int strength, pad;
};

struct Geo {
  int NR, NZ, n_r, n_z, pml_r, pml_b, nmat, top_closed;
  int pc, pn;          // row pitch (elements) of cell and node arrays
  int any_strength, pml_on;
  int nblocks_fused;   // workgroups of the fused cycle kernel
  int same_mat;        // all materials share every constant: evaluate the laws once
  double dr, dz, cfl, dt_grow, dt_max, dt_floor, t_stop, q_lin, q_quad;
  double rho_ref;
  MatC m[kMaxMat];
};

// One copy of the evolving state (two copies ping-pong by cycle parity).
struct State {
  double *rho, *I, *f[kMaxMat], *s[3], *v[2];
};

// Scalars living in device memory so that captured graphs can be replayed.
struct Scal {
  double t, dt, dt_prev;
  long long cycle;
  unsigned long long dtmin;  // bit pattern of the running minimum (dt > 0)
  unsigned flags;
  unsigned done;             // blocks of the current cycle that have finished
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

struct Work {
  double *sg[4];                          // phi-scaled total stress rr, zz, tt, rz
  double *p, *Q, *G, *Y, *rmat, *phi, *sx;
  double *vL[2];                          // Lagrangian node velocity
  double *J, *IL, *sL[3], *fL[kMaxMat];  // Lagrangian cell state
  double *lam, *outv;                     // donor outflow limiter
  double *Fr, *Fz;                        // face mass fluxes (radial: NZ x (NR+1), axial: (NZ+1) x NR)
  double *heat;                           // node specific heat of the remap
  double *mout, *eout;                    // per-column outflow budgets
  double *red;                            // reduction partials
  double *dtpart;                         // per-block Courant minima of the fused cycle
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

// ------------------------------------------------------------------ EoS
// Four-region Tillotson pressure and squared sound speed at material density
// rho and specific internal energy e (the EoS sees max(e, 0) and a density
// floor of 1e-6 rho0).
__device__ inline void tillotson(const MatC& m, double rho, double e, double& p_out, double& c2_out) {
  double rf = m.rho0 * kRhoEosFloor;
  double r = rho > rf ? rho : rf;
  double E = e > 0.0 ? e : 0.0;
  double eta = r / m.rho0;
  double mu = eta - 1.0;
  double w = E / (m.E0 * eta * eta) + 1.0;
  double pc = (m.a + m.b / w) * r * E + m.A * mu + m.B * mu * mu;
  double pc_E = r * (m.a + m.b / w - m.b * (w - 1.0) / (w * w));
  double pc_r = (m.a + m.b / w) * E + 2.0 * m.b * E * (w - 1.0) / (w * w) + (m.A + 2.0 * m.B * mu) / m.rho0;
  double p, dpdE, dpdr;
  if (r >= m.rho0 || E <= m.Eiv) {
    p = pc;
    dpdE = pc_E;
    dpdr = pc_r;
  } else {
    double z = 1.0 / eta - 1.0;
    double ea = exp_cw(-m.alpha * z * z);
    double eb = exp_cw(-m.beta * z);
    double pe = m.a * r * E + (m.b * r * E / w + m.A * mu * eb) * ea;
    double pe_E = m.a * r + ea * m.b * r * (1.0 / w - (w - 1.0) / (w * w));
    double pe_r = m.a * E +
                  ea * (m.b * E / w + 2.0 * m.b * E * (w - 1.0) / (w * w) + (m.A / m.rho0) * eb +
                        m.A * mu * m.beta * eb * m.rho0 / (r * r)) +
                  (m.b * r * E / w + m.A * mu * eb) * ea * 2.0 * m.alpha * z * m.rho0 / (r * r);
    if (E >= m.Ecv) {
      p = pe;
      dpdE = pe_E;
      dpdr = pe_r;
    } else {
      double x = (E - m.Eiv) / (m.Ecv - m.Eiv);
      p = x * pe + (1.0 - x) * pc;
      dpdE = x * pe_E + (1.0 - x) * pc_E + (pe - pc) / (m.Ecv - m.Eiv);
      dpdr = x * pe_r + (1.0 - x) * pc_r;
    }
  }
  p_out = p;
  c2_out = dpdr + p / (r * r) * dpdE;
}

// intact-rock yield curve (Table 1 parameters)
__device__ inline double yield_strength(const MatC& m, double p) {
  if (!m.strength) return 0.0;
  if (p >= 0.0) {
    double mp = m.mu_f * p;
    return m.Y0 + mp / (1.0 + mp / (m.Ylim - m.Y0));
  }
  return dmax(0.0, m.Y0 + m.mu_f * p);
}

// strength fades linearly between incipient and complete vaporisation
__device__ inline double softening(const MatC& m, double e) {
  double E = e > 0.0 ? e : 0.0;
  return dmin(dmax((m.Ecv - E) / (m.Ecv - m.Eiv), 0.0), 1.0);
}

struct Mix {
  double p, c2, G, Y, rmat, phi, sx;
};

// Mixed-cell state: all materials share rho_mat = rho / phi and I; p, c^2,
// G, Y are volume-fraction weighted; sx is the expansion weight of the
// cavitation rule (1 above the tension floor + ramp).
__device__ inline Mix mixture(const Geo& g, double rho, double I, const double* f) {
  Mix o;
  double phi = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxMat; m++)
    if (m < g.nmat) phi += f[m];
  double den = phi > kPhiEps ? phi : kPhiEps;
  double rm = rho / den;
  double p = 0.0, c2 = 0.0, G = 0.0;
  double wm[kMaxMat], pmv[kMaxMat], c2v[kMaxMat], sov[kMaxMat];
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) {
    if (m >= g.nmat) break;
    const MatC& M = g.m[m];
    wm[m] = f[m] / den;
    if (m > 0 && g.same_mat) {
      // identical constants and inputs give identical results
      pmv[m] = pmv[0];
      c2v[m] = c2v[0];
      sov[m] = sov[0];
    } else {
      double pm, c2m;
      tillotson(M, rm, I, pm, c2m);
      pmv[m] = dmax(pm, M.p_min);
      c2v[m] = dmax(c2m, M.cf2);
      sov[m] = softening(M, I);
    }
    p += wm[m] * pmv[m];
    c2 += wm[m] * c2v[m];
    G += wm[m] * (sov[m] * (M.gfac * (rm * c2v[m])));
  }
  double Y = 0.0, pmin = 0.0, ps = 0.0, y0 = 0.0;
#pragma unroll
  for (int m = 0; m < kMaxMat; m++) {
    if (m >= g.nmat) break;
    const MatC& M = g.m[m];
    double ym = (m > 0 && g.same_mat) ? y0 : yield_strength(M, p);
    if (m == 0) y0 = ym;
    Y += wm[m] * (sov[m] * ym);
    pmin += wm[m] * M.p_min;
    ps += wm[m] * M.pcav;
  }
  double d = p - pmin;
  o.sx = d >= ps ? 1.0 : (ps > 0.0 ? dmax(d, 0.0) / ps : 0.0);
  o.p = p;
  o.c2 = c2;
  o.G = G;
  o.Y = Y;
  o.rmat = rm;
  o.phi = phi;
  return o;
}

// material volume ratio (void closes first; expansion gated by cavitation)
__device__ __forceinline__ double material_ratio(double J, double phi, double sx) {
  if (J < 1.0) return dmin(1.0, J / dmax(phi, kPhiEps));
  return 1.0 + (J - 1.0) * sx;
}

// ------------------------------------------------------------------ kinematics
struct Kin {
  double ur_w, ur_e, Ur_w, Ur_e, Uz_s, Uz_n;
  double D, Dr, Dz, err, ezz, ett, erz, om, dvr_dz, dvz_dr;
};

// Face-mean velocities and rates of cell column i from the corner velocities
// (SW, SE, NW, NE). Axial faces weight their nodes by the r-weighted areas of
// the node dual cells, so the node force is the exact volume gradient.
__device__ inline Kin kinematics(const Geo& g, int i, const double vr[4], const double vz[4]) {
  Kin k;
  double rw = (double)i * g.dr, re = (double)(i + 1) * g.dr;
  double rc = ((double)i + 0.5) * g.dr;
  double Arw = rw * g.dz, Are = re * g.dz, Az = rc * g.dr, V = Az * g.dz;
  double aw = 0.5 * (rc * rc - rw * rw), ae = 0.5 * (re * re - rc * rc);
  k.ur_w = 0.5 * (vr[0] + vr[2]);
  k.ur_e = 0.5 * (vr[1] + vr[3]);
  k.Ur_w = Arw * k.ur_w;
  k.Ur_e = Are * k.ur_e;
  k.Uz_s = aw * vz[0] + ae * vz[1];
  k.Uz_n = aw * vz[2] + ae * vz[3];
  k.Dr = (k.Ur_e - k.Ur_w) / V;
  k.Dz = (k.Uz_n - k.Uz_s) / V;
  k.D = ((k.Ur_e - k.Ur_w) + (k.Uz_n - k.Uz_s)) / V;
  k.err = (k.ur_e - k.ur_w) / g.dr;
  k.ezz = (k.Uz_n - k.Uz_s) / V;
  k.ett = (0.5 * (k.ur_w + k.ur_e)) / rc;
  k.dvr_dz = ((aw * vr[2] + ae * vr[3]) - (aw * vr[0] + ae * vr[1])) / V;
  k.dvz_dr = (0.5 * (vz[1] + vz[3]) - 0.5 * (vz[0] + vz[2])) / g.dr;
  k.erz = 0.5 * (k.dvr_dz + k.dvz_dr);
  k.om = 0.5 * (k.dvr_dz - k.dvz_dr);
  return k;
}

__device__ __forceinline__ double cell_volume(const Geo& g, int i) {
  return (((double)i + 0.5) * g.dr * g.dr) * g.dz;
}

}  // namespace salec
