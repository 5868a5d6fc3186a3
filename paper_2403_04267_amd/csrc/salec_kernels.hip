// salec_kernels.hip -- gfx950 kernels of one explicit cycle of the r-z SALE
// scheme with PML (Li et al., SALEc-2D: Sec. 2 eqs. (1)-(5), Sec. 3, Sec. 4,
// Sec. 7), plus scene set-up, the Courant reduction and diagnostics.
//
// Pipeline of one cycle (all on one stream, captured into a HIP graph):
//   k_stress    cells : EoS, artificial viscosity, phi-scaled total stress
//   k_force     nodes : control-volume force, acceleration, PML psi1 -> v^L
//   k_lagrange  cells : strain rates, stress update, internal energy, PML psi2
//   k_limiter   cells : outflow volume and donor limiter
//   k_remap     cells : donor-cell fluxes and remap, PML phi1 / phi3, budgets
//   k_mremap    nodes : dual-cell momentum remap, KE-loss heat, PML phi2
//   k_final     cells : heat, checks, EoS of the new state, dt candidates
//   k_finalize  1 lane: dt, t, cycle, errors
// The state ping-pongs between two copies selected by the cycle parity read
// from device memory, so one captured cycle can be replayed any number of
// times.
#include "salec_device.hpp"
#include "salec_internal.hpp"

namespace salec {

__device__ __forceinline__ void pick(const Scal* sc, const State& S0, const State& S1, State& src, State& dst) {
  if (sc->cycle & 1) {
    src = S1;
    dst = S0;
  } else {
    src = S0;
    dst = S1;
  }
}

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

__device__ __forceinline__ void load_f(const Geo& g, const State& S, long long c, double* f) {
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) f[m] = S.f[m][c];
}

__device__ __forceinline__ void apply_bc(const Geo& g, int i, int j, double& vr, double& vz) {
  if (i == 0 || i == g.NR) vr = 0.0;
  if (j == 0) {
    vr = 0.0;
    vz = 0.0;
  }
  if (g.top_closed && j == g.NZ) vz = 0.0;
}

// ======================================================================
// (a) EoS, viscosity, stress
// ======================================================================
__global__ void k_stress(Geo g, State S0, State S1, Work w, const Scal* sc) {
  if (sc->err) return;
  int i, j;
  if (!cell_of(g, i, j)) return;
  State S, D;
  pick(sc, S0, S1, S, D);
  double dt = sc->dt;
  long long c = cidx(g, i, j);
  double f[kMaxMat];
  load_f(g, S, c, f);
  Mix mx = mixture(g, S.rho[c], S.I[c], f);
  double vr4[4] = {S.v[0][nidx(g, i, j)], S.v[0][nidx(g, i + 1, j)], S.v[0][nidx(g, i, j + 1)], S.v[0][nidx(g, i + 1, j + 1)]};
  double vz4[4] = {S.v[1][nidx(g, i, j)], S.v[1][nidx(g, i + 1, j)], S.v[1][nidx(g, i, j + 1)], S.v[1][nidx(g, i + 1, j + 1)]};
  Kin k = kinematics(g, i, vr4, vz4);
  double L = dmin(g.dr, g.dz);
  double Jn = 1.0 + dt * k.D;
  double Dm = Jn < 1.0 ? (1.0 - material_ratio(Jn, mx.phi, mx.sx)) / dt : 0.0;
  double Ld = L * Dm;
  double Q = mx.rmat * (g.q_quad * Ld * Ld + g.q_lin * sqrt(mx.c2) * Ld);
  double P = mx.p + Q;
  double srr = 0.0, szz = 0.0, srz = 0.0;
  if (g.any_strength) {
    srr = S.s[0][c];
    szz = S.s[1][c];
    srz = S.s[2][c];
  }
  double stt = -(srr + szz);
  w.p[c] = mx.p;
  w.G[c] = mx.G;
  w.Y[c] = mx.Y;
  w.rmat[c] = mx.rmat;
  w.phi[c] = mx.phi;
  w.sx[c] = mx.sx;
  w.Q[c] = Q;
  w.sg[0][c] = mx.phi * (srr - P);
  w.sg[1][c] = mx.phi * (szz - P);
  w.sg[2][c] = mx.phi * (stt - P);
  w.sg[3][c] = mx.phi * srz;
}

// ======================================================================
// (b) node force, acceleration, PML psi1, boundary conditions
// ======================================================================
__global__ void k_force(Geo g, State S0, State S1, Work w, Pml pm, const Scal* sc) {
  if (sc->err) return;
  int i, j;
  if (!node_of(g, i, j)) return;
  State S, D;
  pick(sc, S0, S1, S, D);
  const PmlAux& po = pm.a[sc->cycle & 1];
  const PmlAux& pn = pm.a[(sc->cycle & 1) ^ 1];
  double dt = sc->dt, hdz = 0.5 * g.dz;
  // quadrants NE = (i, j), NW = (i-1, j), SE = (i, j-1), SW = (i-1, j-1)
  double srr[4] = {0, 0, 0, 0}, szz[4] = {0, 0, 0, 0}, stt[4] = {0, 0, 0, 0}, srz[4] = {0, 0, 0, 0},
         rh[4] = {0, 0, 0, 0};
  const int qi[4] = {i, i - 1, i, i - 1}, qj[4] = {j, j, j - 1, j - 1};
  for (int q = 0; q < 4; q++) {
    if (qi[q] < 0 || qi[q] >= g.NR || qj[q] < 0 || qj[q] >= g.NZ) continue;
    long long c = cidx(g, qi[q], qj[q]);
    srr[q] = w.sg[0][c];
    szz[q] = w.sg[1][c];
    stt[q] = w.sg[2][c];
    srz[q] = w.sg[3][c];
    rh[q] = S.rho[c];
  }
  double rN = (double)i * g.dr;
  double rE = ((double)i + 0.5) * g.dr;
  double rW = ((double)i - 0.5) * g.dr;
  double aE = i < g.NR ? 0.5 * (rE * rE - rN * rN) : 0.0;
  double aW = i > 0 ? 0.5 * (rN * rN - rW * rW) : 0.0;
  double Frr = hdz * ((rE * (srr[0] - stt[0]) + rN * stt[0]) + (rE * (srr[2] - stt[2]) + rN * stt[2])) -
               hdz * ((rW * (srr[1] - stt[1]) + rN * stt[1]) + (rW * (srr[3] - stt[3]) + rN * stt[3]));
  double Frz = (aW * srz[1] + aE * srz[0]) - (aW * srz[3] + aE * srz[2]);
  double Fzr = hdz * (rE * (srz[0] + srz[2]) - rW * (srz[1] + srz[3]));
  double Fzz = (aW * szz[1] + aE * szz[0]) - (aW * szz[3] + aE * szz[2]);
  double Fr = Frr + Frz, Fz = Fzr + Fzz;
  double VcE = aE * hdz, VcW = aW * hdz;
  double macc = VcE * (rh[0] + rh[2]) + VcW * (rh[1] + rh[3]);
  double nzh = (double)((j < g.NZ) + (j > 0));
  double Vd = (VcE + VcW) * nzh;
  double mt = dmax(macc, kMAccEps * g.rho_ref * Vd);
  long long n = nidx(g, i, j);
  double psr = 0.0, psz = 0.0, db = 0.0, drr = 0.0;
  long long kb = -1, kr = -1;
  if (g.pml_on) {
    db = pm.dnz[j];
    drr = pm.dnr[i];
    if (j < g.pml_b) kb = pml_bn(g, i, j);
    if (i > g.n_r) kr = pml_rn(g, i, j);
    double br = kb >= 0 ? po.b_psi1r[kb] : 0.0, bz = kb >= 0 ? po.b_psi1z[kb] : 0.0;
    double rr = kr >= 0 ? po.r_psi1r[kr] : 0.0, rz = kr >= 0 ? po.r_psi1z[kr] : 0.0;
    psr = br + rr;
    psz = bz + rz;
  }
  double Fer = Fr - Vd * psr, Fez = Fz - Vd * psz;
  double vLr = S.v[0][n] + dt * (Fer / mt);
  double vLz = S.v[1][n] + dt * (Fez / mt);
  if (db > 0.0) {
    pn.b_psi1r[kb] = po.b_psi1r[kb] - dt * db * (Frr / Vd);
    pn.b_psi1z[kb] = po.b_psi1z[kb] - dt * db * (Fzr / Vd);
  }
  if (drr > 0.0) {
    pn.r_psi1r[kr] = po.r_psi1r[kr] - dt * drr * (Frz / Vd);
    pn.r_psi1z[kr] = po.r_psi1z[kr] - dt * drr * (Fzz / Vd);
  }
  apply_bc(g, i, j, vLr, vLz);
  w.vL[0][n] = vLr;
  w.vL[1][n] = vLz;
}

// ======================================================================
// (c) Lagrangian cell update
// ======================================================================
__global__ void k_lagrange(Geo g, State S0, State S1, Work w, Pml pm, const Scal* sc) {
  if (sc->err) return;
  int i, j;
  if (!cell_of(g, i, j)) return;
  State S, D;
  pick(sc, S0, S1, S, D);
  const PmlAux& po = pm.a[sc->cycle & 1];
  const PmlAux& pn = pm.a[(sc->cycle & 1) ^ 1];
  double dt = sc->dt;
  long long c = cidx(g, i, j);
  const long long nd[4] = {nidx(g, i, j), nidx(g, i + 1, j), nidx(g, i, j + 1), nidx(g, i + 1, j + 1)};
  double vr4[4], vz4[4];
  for (int q = 0; q < 4; q++) {
    vr4[q] = w.vL[0][nd[q]];
    vz4[q] = w.vL[1][nd[q]];
  }
  Kin k = kinematics(g, i, vr4, vz4);
  double s0rr = 0.0, s0zz = 0.0, s0rz = 0.0;
  if (g.any_strength) {
    s0rr = S.s[0][c];
    s0zz = S.s[1][c];
    s0rz = S.s[2][c];
  }
  double srr = s0rr, szz = s0zz, srz = s0rz;
  if (g.any_strength) {
    // Jaumann rate and radial return onto the yield surface
    double G = w.G[c], Y = w.Y[c];
    double tr3 = ((k.err + k.ezz) + k.ett) / 3.0;
    double om = k.om;
    double dsrr = 2.0 * G * (k.err - tr3) + 2.0 * om * srz;
    double dszz = 2.0 * G * (k.ezz - tr3) - 2.0 * om * srz;
    double dsrz = 2.0 * G * k.erz + om * (szz - srr);
    srr = srr + dt * dsrr;
    szz = szz + dt * dszz;
    srz = srz + dt * dsrz;
    double J2 = srr * srr + szz * szz + srr * szz + srz * srz;
    double seq = sqrt(3.0 * J2);
    if (seq > Y) {
      double fac = Y / seq;
      srr = srr * fac;
      szz = szz * fac;
      srz = srz * fac;
    }
  }
  double stt = -(s0rr + s0zz);
  double P = w.p[c] + w.Q[c];
  double sde = ((s0rr * k.err + s0zz * k.ezz) + stt * k.ett) + 2.0 * s0rz * k.erz;
  double J = 1.0 + dt * k.D;
  double phi = w.phi[c];
  double Jm = material_ratio(J, phi, w.sx[c]);
  double Wdt = dt * sde - P * (J - 1.0);
  double rden = dmax(w.rmat[c], g.rho_ref * kRhoDenFloor);
  double rho = S.rho[c];
  double rt = dmax(rho, g.rho_ref * kPmlRhoFloor);
  // symplectic-step defect returned as heat, each corner mass to its cell
  double kd[4];
  for (int q = 0; q < 4; q++) {
    double dvr = w.vL[0][nd[q]] - S.v[0][nd[q]], dvz = w.vL[1][nd[q]] - S.v[1][nd[q]];
    kd[q] = 0.5 * (dvr * dvr + dvz * dvz);
  }
  double rN0 = (double)i * g.dr, rC = ((double)i + 0.5) * g.dr, rN1 = (double)(i + 1) * g.dr;
  double V = cell_volume(g, i), hdz = 0.5 * g.dz;
  double wW = (0.5 * (rC * rC - rN0 * rN0) * hdz) / V;
  double wE = (0.5 * (rN1 * rN1 - rC * rC) * hdz) / V;
  double hL = wW * (kd[0] + kd[2]) + wE * (kd[1] + kd[3]);
  double psi2 = 0.0, db = 0.0, drr = 0.0;
  long long kb = -1, kr = -1;
  if (g.pml_on) {
    db = pm.dcz[j];
    drr = pm.dcr[i];
    if (j < g.pml_b) kb = pml_bc(g, i, j);
    if (i >= g.n_r) kr = pml_rc(g, i, j);
    double b = kb >= 0 ? po.b_psi2[kb] : 0.0, r = kr >= 0 ? po.r_psi2[kr] : 0.0;
    psi2 = b + r;
  }
  double IL = ((S.I[c] + Wdt / rden) + hL) - dt * (psi2 / rt);
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) w.fL[m][c] = S.f[m][c] * (Jm / J);
  if (db > 0.0) {
    double Wr = ((s0rr * k.err + stt * k.ett) + s0rz * k.dvz_dr) - P * k.Dr;
    pn.b_psi2[kb] = po.b_psi2[kb] - dt * db * (phi * Wr);
  }
  if (drr > 0.0) {
    double Wz = (s0zz * k.ezz + s0rz * k.dvr_dz) - P * k.Dz;
    pn.r_psi2[kr] = po.r_psi2[kr] - dt * drr * (phi * Wz);
  }
  w.IL[c] = IL;
  w.sL[0][c] = srr;
  w.sL[1][c] = szz;
  w.sL[2][c] = srz;
  w.J[c] = J;
}

// face volumes swept during the step (radial face at r_i of row j; axial face
// at z_j of column i, nodes weighted by their dual areas)
__device__ __forceinline__ double dv_radial(const Geo& g, const Work& w, double dt, int i, int j) {
  double u = 0.5 * (w.vL[0][nidx(g, i, j)] + w.vL[0][nidx(g, i, j + 1)]);
  return dt * ((((double)i * g.dr) * g.dz) * u);
}
__device__ __forceinline__ double dv_axial(const Geo& g, const Work& w, double dt, int i, int j) {
  double rw = (double)i * g.dr, rc = ((double)i + 0.5) * g.dr;
  double re = (double)(i + 1) * g.dr;
  double aw = 0.5 * (rc * rc - rw * rw), ae = 0.5 * (re * re - rc * rc);
  return dt * (aw * w.vL[1][nidx(g, i, j)] + ae * w.vL[1][nidx(g, i + 1, j)]);
}

// ======================================================================
// (d) outflow volume and donor limiter
// ======================================================================
__global__ void k_limiter(Geo g, State S0, State S1, Work w, const Scal* sc) {
  if (sc->err) return;
  int i, j;
  if (!cell_of(g, i, j)) return;
  double dt = sc->dt;
  long long c = cidx(g, i, j);
  double dW = dv_radial(g, w, dt, i, j), dE = dv_radial(g, w, dt, i + 1, j);
  double dS = dv_axial(g, w, dt, i, j), dN = dv_axial(g, w, dt, i, j + 1);
  double O = ((dmax(-dW, 0.0) + dmax(dE, 0.0)) + dmax(-dS, 0.0)) + dmax(dN, 0.0);
  double VL = cell_volume(g, i) * w.J[c];
  w.outv[c] = O;
  w.lam[c] = O > VL ? dmax(VL, 0.0) / O : 1.0;
}

struct Donor {
  bool ok;
  long long c;
};

// effective volume and mass flux of a face given its swept volume and donor
__device__ __forceinline__ void face_flux(const Geo& g, const State& S, const Work& w, double dV, int ia, int ja,
                                          int ib, int jb, double& e, double& F) {
  // a = cell on the negative side, b = cell on the positive side
  e = 0.0;
  F = 0.0;
  int di, dj;
  if (dV > 0.0) {
    di = ia;
    dj = ja;
  } else if (dV < 0.0) {
    di = ib;
    dj = jb;
  } else {
    return;
  }
  double lam = 1.0, rhoL = 0.0;
  if (di >= 0 && di < g.NR && dj >= 0 && dj < g.NZ) {
    long long d = cidx(g, di, dj);
    lam = w.lam[d];
    rhoL = S.rho[d] / w.J[d];
  }
  e = dV * lam;
  F = e * rhoL;
}

// ======================================================================
// (e) donor-cell remap of mass, energy, stress, volume fractions; PML
// ======================================================================
__global__ void k_remap(Geo g, State S0, State S1, Work w, Pml pm, const Scal* sc) {
  if (sc->err) return;
  int i, j;
  if (!cell_of(g, i, j)) return;
  State S, D;
  pick(sc, S0, S1, S, D);
  const PmlAux& po = pm.a[sc->cycle & 1];
  const PmlAux& pn = pm.a[(sc->cycle & 1) ^ 1];
  double dt = sc->dt;
  long long c = cidx(g, i, j);
  double V = cell_volume(g, i);
  double dV[4] = {dv_radial(g, w, dt, i, j), dv_radial(g, w, dt, i + 1, j), dv_axial(g, w, dt, i, j),
                  dv_axial(g, w, dt, i, j + 1)};
  double dVe[4], F[4];
  face_flux(g, S, w, dV[0], i - 1, j, i, j, dVe[0], F[0]);
  face_flux(g, S, w, dV[1], i, j, i + 1, j, dVe[1], F[1]);
  face_flux(g, S, w, dV[2], i, j - 1, i, j, dVe[2], F[2]);
  face_flux(g, S, w, dV[3], i, j, i, j + 1, dVe[3], F[3]);
  const int di[4] = {i - 1, i + 1, i, i}, dj[4] = {j, j, j - 1, j + 1};
  const bool in[4] = {dV[0] > 0.0, dV[1] < 0.0, dV[2] > 0.0, dV[3] < 0.0};
  double netin = ((F[0] - F[1]) + F[2]) - F[3];
  double rho1 = S.rho[c] + netin / V;
  double M1 = rho1 * V;
  double min_ = 0.0, nI = 0.0, nsrr = 0.0, nszz = 0.0, nsrz = 0.0, vcut = 0.0;
  double nf[kMaxMat] = {0.0, 0.0};
  double IL = w.IL[c];
  double sLc[3] = {w.sL[0][c], w.sL[1][c], w.sL[2][c]};
  double fLc[kMaxMat];
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) fLc[m] = w.fL[m][c];
  double ed[4];
  for (int q = 0; q < 4; q++) {
    bool ok = di[q] >= 0 && di[q] < g.NR && dj[q] >= 0 && dj[q] < g.NZ;
    long long dc = ok ? cidx(g, di[q], dj[q]) : 0;
    if (in[q]) {
      double aF = fabs(F[q]), adV = fabs(dVe[q]);
      vcut += fabs(dV[q]) - adV;
      double Id = ok ? w.IL[dc] : 0.0;
      min_ += aF;
      nI += aF * (Id - IL);
      nsrr += aF * ((ok ? w.sL[0][dc] : 0.0) - sLc[0]);
      nszz += aF * ((ok ? w.sL[1][dc] : 0.0) - sLc[1]);
      nsrz += aF * ((ok ? w.sL[2][dc] : 0.0) - sLc[2]);
      _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) nf[m] += adV * ((ok ? w.fL[m][dc] : 0.0) - fLc[m]);
      ed[q] = F[q] * Id;
    } else {
      ed[q] = F[q] * IL;
    }
  }
  double den = dmax(dmax(M1, min_), kMRemapFloor * g.rho_ref * V);
  double I1 = IL + nI / den;
  if (g.any_strength) {
    D.s[0][c] = sLc[0] + nsrr / den;
    D.s[1][c] = sLc[1] + nszz / den;
    D.s[2][c] = sLc[2] + nsrz / den;
  }
  double ex = (1.0 - w.lam[c]) * w.outv[c] - vcut;
  double fs = 0.0;
  double f1[kMaxMat];
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) {
    f1[m] = dmax(fLc[m] + (nf[m] + fLc[m] * ex) / V, 0.0);
    fs += f1[m];
  }
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) D.f[m][c] = f1[m] / dmax(fs, 1.0);
  if (g.pml_on) {
    double db = pm.dcz[j], drr = pm.dcr[i];
    if (db > 0.0 || drr > 0.0) {
      long long kb = j < g.pml_b ? pml_bc(g, i, j) : -1;
      long long kr = i >= g.n_r ? pml_rc(g, i, j) : -1;
      long long ku = pml_cell_union(g, i, j);
      double dsum = db + drr;
      double p1b = kb >= 0 ? po.b_phi1[kb] : 0.0, p1r = kr >= 0 ? po.r_phi1[kr] : 0.0;
      double p3b = kb >= 0 ? po.b_phi3[kb] : 0.0, p3r = kr >= 0 ? po.r_phi3[kr] : 0.0;
      double rho2 = dmax(rho1 - dt * (dsum * (rho1 - pm.rref[ku]) + (p1b + p1r)), 0.0);
      double rt = dmax(rho1, g.rho_ref * kPmlRhoFloor);
      double I2 = I1 - dt * (dsum * I1 + (p3b + p3r) / rt);
      pm.msink[ku] = pm.msink[ku] + V * (rho1 - rho2);
      if (db > 0.0) {
        pn.b_phi1[kb] = p1b + db * ((F[1] - F[0]) / V);
        pn.b_phi3[kb] = p3b + db * ((ed[1] - ed[0]) / V);
      }
      if (drr > 0.0) {
        pn.r_phi1[kr] = p1r + drr * ((F[3] - F[2]) / V);
        pn.r_phi3[kr] = p3r + drr * ((ed[3] - ed[2]) / V);
      }
      rho1 = rho2;
      I1 = I2;
    }
  }
  D.rho[c] = rho1;
  D.I[c] = I1;
  // face mass fluxes for the momentum remap: each cell stores its west and
  // south faces; the last column / row also store the east / north faces
  w.Fr[fridx(g, i, j)] = F[0];
  if (i == g.NR - 1) w.Fr[fridx(g, i + 1, j)] = F[1];
  w.Fz[fzidx(g, i, j)] = F[2];
  if (j == g.NZ - 1) {
    w.Fz[fzidx(g, i, j + 1)] = F[3];
    w.mout[i] += F[3];
    w.eout[i] += ed[3];
  }
}

__device__ __forceinline__ double Fr_at(const Geo& g, const Work& w, int i, int j) {
  if (i < 0 || i > g.NR || j < 0 || j >= g.NZ) return 0.0;
  return w.Fr[fridx(g, i, j)];
}
__device__ __forceinline__ double Fz_at(const Geo& g, const Work& w, int i, int j) {
  if (i < 0 || i >= g.NR || j < 0 || j > g.NZ) return 0.0;
  return w.Fz[fzidx(g, i, j)];
}

// ======================================================================
// (f) momentum remap over the dual cells; KE-loss heat; PML phi2
// ======================================================================
__global__ void k_mremap(Geo g, State S0, State S1, Work w, Pml pm, const Scal* sc) {
  if (sc->err) return;
  int i, j;
  if (!node_of(g, i, j)) return;
  State S, D;
  pick(sc, S0, S1, S, D);
  const PmlAux& po = pm.a[sc->cycle & 1];
  const PmlAux& pn = pm.a[(sc->cycle & 1) ^ 1];
  double dt = sc->dt, hdz = 0.5 * g.dz;
  long long n = nidx(g, i, j);
  double M[4] = {0, 0, 0, 0};
  const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};  // SW SE NW NE
  bool qok[4];
  for (int q = 0; q < 4; q++) {
    qok[q] = !(qi[q] < 0 || qi[q] >= g.NR || qj[q] < 0 || qj[q] >= g.NZ);
    if (qok[q]) M[q] = S.rho[cidx(g, qi[q], qj[q])] * cell_volume(g, qi[q]);
  }
  double mL = 0.25 * ((M[0] + M[1]) + (M[2] + M[3]));
  double FD[4];
  FD[0] = 0.25 * ((Fr_at(g, w, i - 1, j - 1) + Fr_at(g, w, i, j - 1)) + (Fr_at(g, w, i - 1, j) + Fr_at(g, w, i, j)));
  FD[1] = 0.25 * ((Fr_at(g, w, i, j - 1) + Fr_at(g, w, i + 1, j - 1)) + (Fr_at(g, w, i, j) + Fr_at(g, w, i + 1, j)));
  FD[2] = 0.25 * ((Fz_at(g, w, i - 1, j - 1) + Fz_at(g, w, i, j - 1)) + (Fz_at(g, w, i - 1, j) + Fz_at(g, w, i, j)));
  FD[3] = 0.25 * ((Fz_at(g, w, i - 1, j) + Fz_at(g, w, i, j)) + (Fz_at(g, w, i - 1, j + 1) + Fz_at(g, w, i, j + 1)));
  if (i == 0) FD[0] = 0.0;
  if (i == g.NR) FD[1] = 0.0;
  if (j == 0) FD[2] = 0.0;
  const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
  const bool in[4] = {FD[0] > 0.0, FD[1] < 0.0, FD[2] > 0.0, FD[3] < 0.0};
  double m1 = mL + (((FD[0] - FD[1]) + FD[2]) - FD[3]);
  double vLr = w.vL[0][n], vLz = w.vL[1][n];
  double min_ = 0.0, nr = 0.0, nz = 0.0, kin = 0.0;
  double upr[4], upz[4];
  for (int q = 0; q < 4; q++) {
    bool ok = ni[q] >= 0 && ni[q] <= g.NR && nj[q] >= 0 && nj[q] <= g.NZ;
    if (in[q] && ok) {
      long long d = nidx(g, ni[q], nj[q]);
      double aF = fabs(FD[q]);
      double ur = w.vL[0][d], uz = w.vL[1][d];
      min_ += aF;
      nr += aF * (ur - vLr);
      nz += aF * (uz - vLz);
      upr[q] = ur;
      upz[q] = uz;
    } else {
      upr[q] = vLr;
      upz[q] = vLz;
    }
  }
  double rN = (double)i * g.dr;
  double rE = ((double)i + 0.5) * g.dr;
  double rW = ((double)i - 0.5) * g.dr;
  double aE = i < g.NR ? 0.5 * (rE * rE - rN * rN) : 0.0;
  double aW = i > 0 ? 0.5 * (rN * rN - rW * rW) : 0.0;
  double nzh = (double)((j < g.NZ) + (j > 0));
  double Vd = (aE * hdz + aW * hdz) * nzh;
  double den = dmax(dmax(m1, min_), kMRemapFloor * g.rho_ref * Vd);
  double v1r = vLr + nr / den;
  double v1z = vLz + nz / den;
  for (int q = 0; q < 4; q++) {
    bool ok = ni[q] >= 0 && ni[q] <= g.NR && nj[q] >= 0 && nj[q] <= g.NZ;
    if (in[q] && ok) {
      double ar = upr[q] - vLr, az = upz[q] - vLz;
      kin += fabs(FD[q]) * (ar * ar + az * az);
    }
  }
  double dKE = 0.5 * (kin - (nr * nr + nz * nz) / den);
  double Mn = 0.0;
  for (int q = 0; q < 4; q++)
    if (qok[q]) Mn += D.rho[cidx(g, qi[q], qj[q])] * cell_volume(g, qi[q]);
  w.heat[n] = Mn > kMRemapFloor * g.rho_ref * Vd ? dmax(dKE, 0.0) / Mn : 0.0;
  if (g.pml_on) {
    double db = pm.dnz[j], drr = pm.dnr[i];
    if (db > 0.0 || drr > 0.0) {
      long long kb = j < g.pml_b ? pml_bn(g, i, j) : -1;
      long long kr = i > g.n_r ? pml_rn(g, i, j) : -1;
      double dsum = db + drr;
      double mt = dmax(m1, kMAccEps * g.rho_ref * Vd);
      double bpr = kb >= 0 ? po.b_phi2r[kb] : 0.0, bpz = kb >= 0 ? po.b_phi2z[kb] : 0.0;
      double rpr = kr >= 0 ? po.r_phi2r[kr] : 0.0, rpz = kr >= 0 ? po.r_phi2z[kr] : 0.0;
      double pr = bpr + rpr, pz = bpz + rpz;
      double v2r = v1r - dt * (dsum * v1r + (pr * Vd) / mt);
      double v2z = v1z - dt * (dsum * v1z + (pz * Vd) / mt);
      if (db > 0.0) {
        pn.b_phi2r[kb] = bpr + db * ((FD[1] * upr[1] - FD[0] * upr[0]) / Vd);
        pn.b_phi2z[kb] = bpz + db * ((FD[1] * upz[1] - FD[0] * upz[0]) / Vd);
      }
      if (drr > 0.0) {
        pn.r_phi2r[kr] = rpr + drr * ((FD[3] * upr[3] - FD[2] * upr[2]) / Vd);
        pn.r_phi2z[kr] = rpz + drr * ((FD[3] * upz[3] - FD[2] * upz[2]) / Vd);
      }
      v1r = v2r;
      v1z = v2z;
    }
  }
  apply_bc(g, i, j, v1r, v1z);
  D.v[0][n] = v1r;
  D.v[1][n] = v1z;
}

// ======================================================================
// Courant candidate of one cell of a state (Sec. 7), shared by the cycle's
// last kernel and the initial step
// ======================================================================
__device__ inline double dt_candidate(const Geo& g, const State& S, int i, int j, double Ic) {
  long long c = cidx(g, i, j);
  double f[kMaxMat];
  load_f(g, S, c, f);
  Mix mx = mixture(g, S.rho[c], Ic, f);
  double cl2 = mx.c2 + (4.0 / 3.0) * mx.G / dmax(mx.rmat, g.rho_ref * kRhoDenFloor);
  double cl = sqrt(cl2);
  const long long nd[4] = {nidx(g, i, j), nidx(g, i + 1, j), nidx(g, i, j + 1), nidx(g, i + 1, j + 1)};
  double u = 0.0;
  for (int q = 0; q < 4; q++) {
    double a = S.v[0][nd[q]], b = S.v[1][nd[q]];
    double s = sqrt(a * a + b * b);
    u = dmax(u, s);
  }
  double wgt = dmin(dmax((mx.phi - kWLo) / (kWHi - kWLo), 0.0), 1.0);
  if (wgt > 0.0) return g.cfl * dmin(g.dr, g.dz) / ((cl + u) * wgt);
  return __builtin_huge_val();
}

__device__ __forceinline__ void block_min_to(unsigned long long* dst, double v) {
  // wavefront (64 lanes) shuffle reduction, then LDS across waves, then one
  // atomic min on the bit pattern (valid: all candidates are positive)
  for (int off = 32; off > 0; off >>= 1) v = dmin(v, __shfl_down(v, off, 64));
  __shared__ double part[16];
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    int nw = (blockDim.x + 63) >> 6;
    for (int k = 1; k < nw; k++) m = dmin(m, part[k]);
    atomicMin(dst, (unsigned long long)__double_as_longlong(m));
  }
}

__device__ __forceinline__ bool finite_d(double x) { return (x - x) == 0.0; }

// ======================================================================
// (g) heat, state checks, Courant candidates of the new state
// ======================================================================
__global__ void k_final(Geo g, State S0, State S1, Work w, Scal* sc) {
  if (sc->err) return;
  int i, j;
  bool live = cell_of(g, i, j);
  double cand = __builtin_huge_val();
  unsigned flags = 0;
  if (live) {
    State S, D;
    pick(sc, S0, S1, S, D);
    long long c = cidx(g, i, j);
    double h = (w.heat[nidx(g, i, j)] + w.heat[nidx(g, i + 1, j)]) + (w.heat[nidx(g, i, j + 1)] + w.heat[nidx(g, i + 1, j + 1)]);
    double I1 = D.I[c] + h;
    D.I[c] = I1;
    double s = D.rho[c] + I1;
    if (g.any_strength) s += D.s[0][c] + D.s[1][c] + D.s[2][c];
    _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) s += D.f[m][c];
    if (!finite_d(s)) flags |= kFlagNonFinite;
    if (D.rho[c] < -kNegMassTol * g.rho_ref) flags |= kFlagNegMass;
    if (!finite_d(D.v[0][nidx(g, i, j)] + D.v[1][nidx(g, i, j)])) flags |= kFlagNonFinite;
    if (i == g.NR - 1 && !finite_d(D.v[0][nidx(g, i + 1, j)] + D.v[1][nidx(g, i + 1, j)])) flags |= kFlagNonFinite;
    if (j == g.NZ - 1 && !finite_d(D.v[0][nidx(g, i, j + 1)] + D.v[1][nidx(g, i, j + 1)])) flags |= kFlagNonFinite;
    if (i == g.NR - 1 && j == g.NZ - 1 && !finite_d(D.v[0][nidx(g, i + 1, j + 1)] + D.v[1][nidx(g, i + 1, j + 1)]))
      flags |= kFlagNonFinite;
    cand = dt_candidate(g, D, i, j, I1);
  }
  if (flags) atomicOr(&sc->flags, flags);
  block_min_to(&sc->dtmin, cand);
}

// Courant candidates of the current state (initial step)
__global__ void k_dt0(Geo g, State S0, State S1, Scal* sc) {
  int i, j;
  bool live = cell_of(g, i, j);
  double cand = __builtin_huge_val();
  if (live) {
    State S, D;
    pick(sc, S0, S1, S, D);
    cand = dt_candidate(g, S, i, j, S.I[cidx(g, i, j)]);
  }
  block_min_to(&sc->dtmin, cand);
}

__device__ __forceinline__ double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }
constexpr unsigned long long kInfBits = 0x7FF0000000000000ull;

// first step of a run: no growth cap
__global__ void k_finalize0(Geo g, Scal* sc) {
  double dt = dmin(from_bits(sc->dtmin), g.dt_max);
  if (g.t_stop > 0) dt = dmin(dt, g.t_stop);
  sc->dt = dt;
  sc->dt_prev = 0.0;
  sc->dtmin = kInfBits;
}

// end of a cycle: advance time, next step (Courant, growth cap, maximum,
// stop time), sticky errors
__global__ void k_finalize(Geo g, Scal* sc) {
  if (sc->err) return;
  double t = sc->t + sc->dt;
  sc->t = t;
  sc->cycle = sc->cycle + 1;
  double dt = dmin(dmin(from_bits(sc->dtmin), g.dt_grow * sc->dt), g.dt_max);
  if (g.t_stop > 0) dt = dmin(dt, dmax(g.t_stop - t, 0.0));
  sc->dt_prev = sc->dt;
  sc->dt = dt;
  sc->dtmin = kInfBits;
  int e = 0;
  if (sc->flags & kFlagNonFinite) e = -4;
  else if (sc->flags & kFlagNegMass) e = -5;
  bool stopped = g.t_stop > 0 && t >= g.t_stop;
  if (e == 0 && !stopped && dt < g.dt_floor) e = -6;
  if (e) {
    sc->err = e;
    sc->err_cycle = (int)sc->cycle;
  }
}

// ======================================================================
// scene set-up: target half-space, spherical projectile, momentum-exact
// node velocities
// ======================================================================
__global__ void k_scene_cells(Geo g, State S0, Work w, int surface_j, int S, double R, double zc) {
  int i, j;
  if (!cell_of(g, i, j)) return;
  long long c = cidx(g, i, j);
  double num = 0.0, den = 0.0;
  for (int l = 0; l < S; l++) {
    double zl = ((double)j + ((double)l + 0.5) / (double)S) * g.dz;
    for (int k = 0; k < S; k++) {
      double rk = ((double)i + ((double)k + 0.5) / (double)S) * g.dr;
      double dzl = zl - zc;
      if (rk * rk + dzl * dzl <= R * R) num += rk;
      den += rk;
    }
  }
  double fp = num / den;
  int mp = g.nmat > 1 ? 1 : 0;
  double f[kMaxMat] = {0.0, 0.0};
  f[0] = j < surface_j ? 1.0 : 0.0;
  f[mp] = f[mp] + fp;
  double rho = 0.0;
  _Pragma("unroll") for (int m = 0; m < kMaxMat; m++) if (m < g.nmat) {
    S0.f[m][c] = f[m];
    rho += f[m] * g.m[m].rho0;
  }
  S0.rho[c] = rho;
  S0.I[c] = 0.0;
  if (g.any_strength) {
    S0.s[0][c] = 0.0;
    S0.s[1][c] = 0.0;
    S0.s[2][c] = 0.0;
  }
  w.p[c] = fp;  // scratch: projectile fraction for the node pass
}

__global__ void k_scene_nodes(Geo g, State S0, Work w, double v_imp) {
  int i, j;
  if (!node_of(g, i, j)) return;
  int mp = g.nmat > 1 ? 1 : 0;
  double Mt = 0.0, Mp = 0.0;
  const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
  for (int q = 0; q < 4; q++) {
    if (qi[q] < 0 || qi[q] >= g.NR || qj[q] < 0 || qj[q] >= g.NZ) continue;
    long long c = cidx(g, qi[q], qj[q]);
    double V = cell_volume(g, qi[q]);
    Mt += S0.rho[c] * V;
    Mp += w.p[c] * g.m[mp].rho0 * V;
  }
  double vr = 0.0, vz = Mt > 0.0 ? -v_imp * (Mp / Mt) : 0.0;
  apply_bc(g, i, j, vr, vz);
  long long n = nidx(g, i, j);
  S0.v[0][n] = vr;
  S0.v[1][n] = vz;
}

// start of a run (state in copy 0, PML auxiliaries and budgets already
// cleared): PML reference density = current density, clock reset
__global__ void k_start_run(Geo g, State S0, Pml pm, Scal* sc) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long nb = (long long)g.pml_b * g.NR, nu = nb + (long long)g.n_z * g.pml_r;
  if (t == 0) {
    sc->t = 0.0;
    sc->dt = 0.0;
    sc->dt_prev = 0.0;
    sc->cycle = 0;
    sc->dtmin = 0x7FF0000000000000ull;
    sc->flags = 0;
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
  pm.rref[t] = S0.rho[cidx(g, i, j)];
}

// EoS of the current state (outputs only)
__global__ void k_eos_out(Geo g, State S0, State S1, const Scal* sc, double* p, double* c2) {
  int i, j;
  if (!cell_of(g, i, j)) return;
  State S, D;
  pick(sc, S0, S1, S, D);
  long long c = cidx(g, i, j);
  double f[kMaxMat];
  load_f(g, S, c, f);
  Mix mx = mixture(g, S.rho[c], S.I[c], f);
  p[c] = mx.p;
  c2[c] = mx.c2;
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

constexpr int kDiagQ = 6;  // mass, ie, ke, mass_out, mass_pml, ie_out

__global__ void k_diag_partial(Geo g, State S0, State S1, Work w, Pml pm, const Scal* sc, long long n_pml) {
  State S, D;
  pick(sc, S0, S1, S, D);
  KS acc[kDiagQ];
  for (int q = 0; q < kDiagQ; q++) acc[q] = {0.0, 0.0};
  long long ncell = (long long)g.NR * g.NZ, nnode = (long long)(g.NR + 1) * (g.NZ + 1);
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < ncell; t += stride) {
    int j = (int)(t / g.NR), i = (int)(t - (long long)j * g.NR);
    long long c = cidx(g, i, j);
    double M = S.rho[c] * cell_volume(g, i);
    ks_add(acc[0], M);
    ks_add(acc[1], M * S.I[c]);
  }
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nnode; t += stride) {
    int j = (int)(t / (g.NR + 1)), i = (int)(t - (long long)j * (g.NR + 1));
    double Mq[4] = {0, 0, 0, 0};
    const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
    for (int q = 0; q < 4; q++) {
      if (qi[q] < 0 || qi[q] >= g.NR || qj[q] < 0 || qj[q] >= g.NZ) continue;
      Mq[q] = S.rho[cidx(g, qi[q], qj[q])] * cell_volume(g, qi[q]);
    }
    double M = 0.25 * ((Mq[0] + Mq[1]) + (Mq[2] + Mq[3]));
    long long n = nidx(g, i, j);
    double a = S.v[0][n], b = S.v[1][n];
    ks_add(acc[2], 0.5 * M * (a * a + b * b));
  }
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < g.NR; t += stride) {
    ks_add(acc[3], w.mout[t]);
    ks_add(acc[5], w.eout[t]);
  }
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < n_pml; t += stride) ks_add(acc[4], pm.msink[t]);
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
      w.red[(blockIdx.x * kDiagQ + q) * 2] = sh[0];
      w.red[(blockIdx.x * kDiagQ + q) * 2 + 1] = sh[1];
    }
    __syncthreads();
  }
}

__global__ void k_diag_final(Work w, int nblocks, double* out) {
  if (threadIdx.x != 0) return;
  for (int q = 0; q < kDiagQ; q++) {
    KS a{0.0, 0.0};
    for (int b = 0; b < nblocks; b++) a = ks_merge(a, KS{w.red[(b * kDiagQ + q) * 2], w.red[(b * kDiagQ + q) * 2 + 1]});
    out[q] = a.s + a.c;
  }
}

// ======================================================================
// launchers
// ======================================================================
static inline unsigned nblk(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_cycle(const Geo& g, const State& S0, const State& S1, const Work& w, const Pml& pm, Scal* sc,
                  hipStream_t st) {
  const int bs = 256;
  long long nc = (long long)g.NR * g.NZ, nn = (long long)(g.NR + 1) * (g.NZ + 1);
  hipLaunchKernelGGL(k_stress, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, w, sc);
  hipLaunchKernelGGL(k_force, dim3(nblk(nn, bs)), dim3(bs), 0, st, g, S0, S1, w, pm, sc);
  hipLaunchKernelGGL(k_lagrange, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, w, pm, sc);
  hipLaunchKernelGGL(k_limiter, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, w, sc);
  hipLaunchKernelGGL(k_remap, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, w, pm, sc);
  hipLaunchKernelGGL(k_mremap, dim3(nblk(nn, bs)), dim3(bs), 0, st, g, S0, S1, w, pm, sc);
  hipLaunchKernelGGL(k_final, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, w, sc);
  hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1), 0, st, g, sc);
}

void launch_dt0(const Geo& g, const State& S0, const State& S1, Scal* sc, hipStream_t st) {
  const int bs = 256;
  long long nc = (long long)g.NR * g.NZ;
  hipLaunchKernelGGL(k_dt0, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, sc);
  hipLaunchKernelGGL(k_finalize0, dim3(1), dim3(1), 0, st, g, sc);
}

void launch_scene(const Geo& g, const State& S0, const Work& w, int surface_j, int S, double R, double zc,
                  double v_imp, hipStream_t st) {
  const int bs = 256;
  long long nc = (long long)g.NR * g.NZ, nn = (long long)(g.NR + 1) * (g.NZ + 1);
  hipLaunchKernelGGL(k_scene_cells, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, w, surface_j, S, R, zc);
  hipLaunchKernelGGL(k_scene_nodes, dim3(nblk(nn, bs)), dim3(bs), 0, st, g, S0, w, v_imp);
}

void launch_start_run(const Geo& g, const State& S0, const Pml& pm, Scal* sc, hipStream_t st) {
  long long nu = (long long)g.pml_b * g.NR + (long long)g.n_z * g.pml_r;
  if (nu < 1) nu = 1;
  hipLaunchKernelGGL(k_start_run, dim3(nblk(nu, 256)), dim3(256), 0, st, g, S0, pm, sc);
}

void launch_eos_out(const Geo& g, const State& S0, const State& S1, const Scal* sc, double* p, double* c2,
                    hipStream_t st) {
  const int bs = 256;
  long long nc = (long long)g.NR * g.NZ;
  hipLaunchKernelGGL(k_eos_out, dim3(nblk(nc, bs)), dim3(bs), 0, st, g, S0, S1, sc, p, c2);
}

void launch_diag(const Geo& g, const State& S0, const State& S1, const Work& w, const Pml& pm, const Scal* sc,
                 long long n_pml, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_diag_partial, dim3(kDiagBlocks), dim3(256), 0, st, g, S0, S1, w, pm, sc, n_pml);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64), 0, st, w, (int)kDiagBlocks, out);
}

}  // namespace salec
