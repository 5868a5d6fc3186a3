// salec_fused.hip -- the whole explicit cycle of the r-z SALE scheme with PML
// (Li et al., SALEc-2D: Sec. 2 eqs. (1)-(5), Sec. 3, Sec. 4, Sec. 7) as ONE
// gfx950 kernel per cycle.
//
// Each workgroup owns a TW x TH tile of cells (and the nodes at their lower-
// left corners) and recomputes every phase over the halo it needs, keeping
// intermediates in LDS:
//   A  cells [i0-3, i0+TW+3)  EoS, viscosity, phi-scaled stress      -> LDS
//   B  nodes [i0-2, i0+TW+2]  control-volume force, PML psi1 -> v^L   -> LDS
//   C  cells [i0-2, i0+TW+1]  Lagrangian update, PML psi2, limiter     -> LDS
//   E1 faces of the cells below: volume and donor mass fluxes          -> LDS
//   E2 cells [i0-1, i0+TW]    donor-cell remap, PML phi1/phi3          -> LDS
//   F  nodes [i0, i0+TW]      momentum remap, KE-loss heat, PML phi2   -> LDS
//   G  cells of the tile      heat, checks, EoS of the new state, dt
// (the same ranges in z). Halo values are recomputed with bit-identical
// arithmetic; only the owner of a cell or node writes it. The state and the
// PML auxiliaries ping-pong by cycle parity, so all halo reads see level n.
// The Courant minimum is reduced per block (wave shuffles, then LDS) and the
// last block to finish (done counter) finalises t, dt and the cycle count.
#include "salec_device.hpp"
#include "salec_internal.hpp"

namespace salec {

template <int TW, int TH>
struct Regions {
  static constexpr int AW = TW + 6, AH = TH + 6, NA = AW * AH;  // cells, origin (i0-3, j0-3)
  static constexpr int BW = TW + 5, BH = TH + 5, NB = BW * BH;  // nodes, origin (i0-2, j0-2)
  static constexpr int CW = TW + 4, CH = TH + 4, NC = CW * CH;  // cells, origin (i0-2, j0-2)
  static constexpr int EW = TW + 2, EH = TH + 2, NE = EW * EH;  // cells, origin (i0-1, j0-1)
  static constexpr int FW = TW + 1, FH = TH + 1, NF = FW * FH;  // nodes, origin (i0, j0)
  static constexpr int RW = TW + 3, RH = TH + 2, NRF = RW * RH;  // radial faces, origin (i0-1, j0-1)
  static constexpr int ZW = TW + 2, ZH = TH + 3, NZF = ZW * ZH;  // axial faces, origin (i0-1, j0-1)
};

__device__ __forceinline__ bool in_cells(const Geo& g, int i, int j) {
  return i >= 0 && i < g.NR && j >= 0 && j < g.NZ;
}

template <int TW, int TH, int NT>
__global__ __launch_bounds__(NT) void k_cycle(Geo g, State S0, State S1, Pml pm, Work w, Scal* sc) {
  using R = Regions<TW, TH>;
  constexpr int UA = (R::NA + NT - 1) / NT;
  constexpr int UE = (R::NE + NT - 1) / NT;
  constexpr int NCOUT = 8;  // rhoL, lambda, IL, sL x3, fL x2
  static_assert(NCOUT * R::NC >= 4 * R::NA, "stress buffer must fit in the Lagrangian-state buffer");
  static_assert(NCOUT * R::NC >= 2 * R::NF, "heat/speed buffer must fit in the Lagrangian-state buffer");

  __shared__ double s_rho[R::NA];            // rho^n over A (0 outside the grid)
  __shared__ double s_big[NCOUT * R::NC];    // A: sigma[4][NA]; C..E2: Lagrangian state; F..G: heat, speed
  __shared__ double s_vL[2 * R::NB];         // v^L over B
  __shared__ double s_Fr[R::NRF], s_Fz[R::NZF];  // face mass fluxes (0 where no face)
  __shared__ double s_rho1[R::NE];           // rho^{n+1} over E (0 outside the grid)
  __shared__ double s_min[NT / 64];

  if (sc->err) return;
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * TW, j0 = blockIdx.y * TH;
  const int i1 = min(i0 + TW, g.NR), j1 = min(j0 + TH, g.NZ);  // owned cells [i0, i1) x [j0, j1)
  const int par = (int)(sc->cycle & 1);
  const State& S = par ? S1 : S0;
  const State& D = par ? S0 : S1;
  const PmlAux& po = pm.a[par];
  const PmlAux& pn = pm.a[par ^ 1];
  const double dt = sc->dt;
  const double hdz = 0.5 * g.dz;
  auto owns_cell = [&](int i, int j) { return i >= i0 && i < i1 && j >= j0 && j < j1; };
  auto owns_node = [&](int i, int j) {
    bool oi = (i >= i0 && i < i1) || (i == g.NR && i1 == g.NR);
    bool oj = (j >= j0 && j < j1) || (j == g.NZ && j1 == g.NZ);
    return oi && oj;
  };
  auto kA = [&](int i, int j) { return (i - (i0 - 3)) + (j - (j0 - 3)) * R::AW; };
  auto kB = [&](int i, int j) { return (i - (i0 - 2)) + (j - (j0 - 2)) * R::BW; };
  auto kC = [&](int i, int j) { return (i - (i0 - 2)) + (j - (j0 - 2)) * R::CW; };
  auto kE = [&](int i, int j) { return (i - (i0 - 1)) + (j - (j0 - 1)) * R::EW; };
  auto kF = [&](int i, int j) { return (i - i0) + (j - j0) * R::FW; };
  auto kR = [&](int i, int j) { return (i - (i0 - 1)) + (j - (j0 - 1)) * R::RW; };
  auto kZ = [&](int i, int j) { return (i - (i0 - 1)) + (j - (j0 - 1)) * R::ZW; };
  double* sig = s_big;  // [4][NA] during A..B
  double* cout = s_big; // [8][NC] during C..E2

  // ------------------------------------------------------------------ A
  double rP[UA], rG[UA], rY[UA], rRm[UA], rPhi[UA], rSx[UA];
#pragma unroll
  for (int u = 0; u < UA; u++) {
    int k = tid + u * NT;
    rP[u] = rG[u] = rY[u] = rRm[u] = rPhi[u] = rSx[u] = 0.0;
    if (k >= R::NA) continue;
    int i = i0 - 3 + k % R::AW, j = j0 - 3 + k / R::AW;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0, rh = 0.0;
    if (in_cells(g, i, j)) {
      long long c = cidx(g, i, j);
      double f[kMaxMat];
#pragma unroll
      for (int m = 0; m < kMaxMat; m++) f[m] = m < g.nmat ? S.f[m][c] : 0.0;
      rh = S.rho[c];
      Mix mx = mixture(g, rh, S.I[c], f);
      double vr4[4] = {S.v[0][nidx(g, i, j)], S.v[0][nidx(g, i + 1, j)], S.v[0][nidx(g, i, j + 1)],
                       S.v[0][nidx(g, i + 1, j + 1)]};
      double vz4[4] = {S.v[1][nidx(g, i, j)], S.v[1][nidx(g, i + 1, j)], S.v[1][nidx(g, i, j + 1)],
                       S.v[1][nidx(g, i + 1, j + 1)]};
      Kin kn = kinematics(g, i, vr4, vz4);
      double L = dmin(g.dr, g.dz);
      double Jn = 1.0 + dt * kn.D;
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
      s0 = mx.phi * (srr - P);
      s1 = mx.phi * (szz - P);
      s2 = mx.phi * (stt - P);
      s3 = mx.phi * srz;
      rP[u] = P;
      rG[u] = mx.G;
      rY[u] = mx.Y;
      rRm[u] = mx.rmat;
      rPhi[u] = mx.phi;
      rSx[u] = mx.sx;
    }
    sig[0 * R::NA + k] = s0;
    sig[1 * R::NA + k] = s1;
    sig[2 * R::NA + k] = s2;
    sig[3 * R::NA + k] = s3;
    s_rho[k] = rh;
  }
  __syncthreads();

  // ------------------------------------------------------------------ B
  for (int k = tid; k < R::NB; k += NT) {
    int i = i0 - 2 + k % R::BW, j = j0 - 2 + k / R::BW;
    double vLr = 0.0, vLz = 0.0;
    if (i >= 0 && i <= g.NR && j >= 0 && j <= g.NZ) {
      // quadrants NE = (i, j), NW = (i-1, j), SE = (i, j-1), SW = (i-1, j-1)
      const int qa[4] = {kA(i, j), kA(i - 1, j), kA(i, j - 1), kA(i - 1, j - 1)};
      double srr[4], szz[4], stt[4], srz[4], rh[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        srr[q] = sig[0 * R::NA + qa[q]];
        szz[q] = sig[1 * R::NA + qa[q]];
        stt[q] = sig[2 * R::NA + qa[q]];
        srz[q] = sig[3 * R::NA + qa[q]];
        rh[q] = s_rho[qa[q]];
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
      vLr = S.v[0][n] + dt * (Fer / mt);
      vLz = S.v[1][n] + dt * (Fez / mt);
      if (owns_node(i, j)) {
        if (db > 0.0) {
          pn.b_psi1r[kb] = po.b_psi1r[kb] - dt * db * (Frr / Vd);
          pn.b_psi1z[kb] = po.b_psi1z[kb] - dt * db * (Fzr / Vd);
        }
        if (drr > 0.0) {
          pn.r_psi1r[kr] = po.r_psi1r[kr] - dt * drr * (Frz / Vd);
          pn.r_psi1z[kr] = po.r_psi1z[kr] - dt * drr * (Fzz / Vd);
        }
      }
      if (i == 0 || i == g.NR) vLr = 0.0;
      if (j == 0) {
        vLr = 0.0;
        vLz = 0.0;
      }
      if (g.top_closed && j == g.NZ) vLz = 0.0;
    }
    s_vL[k] = vLr;
    s_vL[R::NB + k] = vLz;
  }
  __syncthreads();

  // face volumes from v^L (radial face at r_i of row j; axial face at z_j of
  // column i with dual-area node weights)
  auto dv_r = [&](int i, int j) {
    double u = 0.5 * (s_vL[kB(i, j)] + s_vL[kB(i, j + 1)]);
    return dt * ((((double)i * g.dr) * g.dz) * u);
  };
  auto dv_z = [&](int i, int j) {
    double rw = (double)i * g.dr, rc = ((double)i + 0.5) * g.dr;
    double re = (double)(i + 1) * g.dr;
    double aw = 0.5 * (rc * rc - rw * rw), ae = 0.5 * (re * re - rc * rc);
    return dt * (aw * s_vL[R::NB + kB(i, j)] + ae * s_vL[R::NB + kB(i + 1, j)]);
  };

  // ------------------------------------------------------------------ C
  // (same cell-to-thread map as A, so A's per-cell results stay in registers;
  // the stress buffer is dead after B, so results go straight into it)
#pragma unroll
  for (int u = 0; u < UA; u++) {
    int k = tid + u * NT;
    int i = i0 - 3 + k % R::AW, j = j0 - 3 + k / R::AW;
    bool inC = k < R::NA && i >= i0 - 2 && i < i0 + TW + 2 && j >= j0 - 2 && j < j0 + TH + 2;
    if (!inC) continue;
    // outside the grid: a void donor (rho^L = 0, lambda = 1, zero state)
    double oRhoL = 0.0, oLam = 1.0, oIL = 0.0, os0 = 0.0, os1 = 0.0, os2 = 0.0, of0 = 0.0, of1 = 0.0;
    if (in_cells(g, i, j)) {
      long long c = cidx(g, i, j);
      const long long nd[4] = {nidx(g, i, j), nidx(g, i + 1, j), nidx(g, i, j + 1), nidx(g, i + 1, j + 1)};
      const int nb[4] = {kB(i, j), kB(i + 1, j), kB(i, j + 1), kB(i + 1, j + 1)};
      double vr4[4], vz4[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        vr4[q] = s_vL[nb[q]];
        vz4[q] = s_vL[R::NB + nb[q]];
      }
      Kin kn = kinematics(g, i, vr4, vz4);
      double s0rr = 0.0, s0zz = 0.0, s0rz = 0.0;
      if (g.any_strength) {
        s0rr = S.s[0][c];
        s0zz = S.s[1][c];
        s0rz = S.s[2][c];
      }
      double srr = s0rr, szz = s0zz, srz = s0rz;
      if (g.any_strength) {
        double G = rG[u], Y = rY[u];
        double tr3 = ((kn.err + kn.ezz) + kn.ett) / 3.0;
        double om = kn.om;
        double dsrr = 2.0 * G * (kn.err - tr3) + 2.0 * om * srz;
        double dszz = 2.0 * G * (kn.ezz - tr3) - 2.0 * om * srz;
        double dsrz = 2.0 * G * kn.erz + om * (szz - srr);
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
      double P = rP[u];
      double sde = ((s0rr * kn.err + s0zz * kn.ezz) + stt * kn.ett) + 2.0 * s0rz * kn.erz;
      double J = 1.0 + dt * kn.D;
      double phi = rPhi[u];
      double Jm = material_ratio(J, phi, rSx[u]);
      double Wdt = dt * sde - P * (J - 1.0);
      double rden = dmax(rRm[u], g.rho_ref * kRhoDenFloor);
      double rho = S.rho[c];
      double rt = dmax(rho, g.rho_ref * kPmlRhoFloor);
      double kd[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        double dvr = vr4[q] - S.v[0][nd[q]], dvz = vz4[q] - S.v[1][nd[q]];
        kd[q] = 0.5 * (dvr * dvr + dvz * dvz);
      }
      double rN0 = (double)i * g.dr, rC = ((double)i + 0.5) * g.dr, rN1 = (double)(i + 1) * g.dr;
      double V = cell_volume(g, i);
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
      double f0 = S.f[0][c] * (Jm / J);
      double f1 = g.nmat > 1 ? S.f[1][c] * (Jm / J) : 0.0;
      if (owns_cell(i, j)) {
        if (db > 0.0) {
          double Wr = ((s0rr * kn.err + stt * kn.ett) + s0rz * kn.dvz_dr) - P * kn.Dr;
          pn.b_psi2[kb] = po.b_psi2[kb] - dt * db * (phi * Wr);
        }
        if (drr > 0.0) {
          double Wz = (s0zz * kn.ezz + s0rz * kn.dvr_dz) - P * kn.Dz;
          pn.r_psi2[kr] = po.r_psi2[kr] - dt * drr * (phi * Wz);
        }
      }
      // donor outflow limiter: volume leaving through the four faces vs V^L
      double dW = dv_r(i, j), dE = dv_r(i + 1, j), dS = dv_z(i, j), dN = dv_z(i, j + 1);
      double O = ((dmax(-dW, 0.0) + dmax(dE, 0.0)) + dmax(-dS, 0.0)) + dmax(dN, 0.0);
      double VL = V * J;
      oRhoL = rho / J;
      oIL = IL;
      os0 = srr;
      os1 = szz;
      os2 = srz;
      of0 = f0;
      of1 = f1;
      oLam = O > VL ? dmax(VL, 0.0) / O : 1.0;
    }
    int kc = kC(i, j);
    cout[0 * R::NC + kc] = oRhoL;
    cout[1 * R::NC + kc] = oLam;
    cout[2 * R::NC + kc] = oIL;
    cout[3 * R::NC + kc] = os0;
    cout[4 * R::NC + kc] = os1;
    cout[5 * R::NC + kc] = os2;
    cout[6 * R::NC + kc] = of0;
    cout[7 * R::NC + kc] = of1;
  }
  __syncthreads();

  // ------------------------------------------------------------------ E1
  // mass flux of every face the remap and the momentum remap touch; 0 where
  // there is no face
  for (int k = tid; k < R::NRF; k += NT) {
    int i = i0 - 1 + k % R::RW, j = j0 - 1 + k / R::RW;
    double F = 0.0;
    if (i >= 0 && i <= g.NR && j >= 0 && j < g.NZ) {
      double dV = dv_r(i, j);
      int d = dV > 0.0 ? kC(i - 1, j) : kC(i, j);
      if (dV > 0.0 || dV < 0.0) F = (dV * cout[1 * R::NC + d]) * cout[0 * R::NC + d];
    }
    s_Fr[k] = F;
  }
  for (int k = tid; k < R::NZF; k += NT) {
    int i = i0 - 1 + k % R::ZW, j = j0 - 1 + k / R::ZW;
    double F = 0.0;
    if (i >= 0 && i < g.NR && j >= 0 && j <= g.NZ) {
      double dV = dv_z(i, j);
      int d = dV > 0.0 ? kC(i, j - 1) : kC(i, j);
      if (dV > 0.0 || dV < 0.0) F = (dV * cout[1 * R::NC + d]) * cout[0 * R::NC + d];
    }
    s_Fz[k] = F;
  }
  __syncthreads();

  // ------------------------------------------------------------------ E2
  double eRho[UE], eI[UE], eF0[UE], eF1[UE], eS0[UE], eS1[UE], eS2[UE];
#pragma unroll
  for (int u = 0; u < UE; u++) {
    int k = tid + u * NT;
    eRho[u] = eI[u] = eF0[u] = eF1[u] = eS0[u] = eS1[u] = eS2[u] = 0.0;
    if (k >= R::NE) continue;
    int i = i0 - 1 + k % R::EW, j = j0 - 1 + k / R::EW;
    double rho1 = 0.0;
    if (in_cells(g, i, j)) {
      bool own = owns_cell(i, j);
      double V = cell_volume(g, i);
      double dV[4] = {dv_r(i, j), dv_r(i + 1, j), dv_z(i, j), dv_z(i, j + 1)};
      double F[4] = {s_Fr[kR(i, j)], s_Fr[kR(i + 1, j)], s_Fz[kZ(i, j)], s_Fz[kZ(i, j + 1)]};
      const int dk[4] = {kC(i - 1, j), kC(i + 1, j), kC(i, j - 1), kC(i, j + 1)};
      const bool in[4] = {dV[0] > 0.0, dV[1] < 0.0, dV[2] > 0.0, dV[3] < 0.0};
      int kc = kC(i, j);
      double netin = ((F[0] - F[1]) + F[2]) - F[3];
      rho1 = s_rho[kA(i, j)] + netin / V;
      double M1 = rho1 * V;
      double min_ = 0.0, nI = 0.0, nsrr = 0.0, nszz = 0.0, nsrz = 0.0, vcut = 0.0;
      double nf0 = 0.0, nf1 = 0.0;
      double IL = cout[2 * R::NC + kc];
      double sL0 = cout[3 * R::NC + kc], sL1 = cout[4 * R::NC + kc], sL2 = cout[5 * R::NC + kc];
      double fL0 = cout[6 * R::NC + kc], fL1 = cout[7 * R::NC + kc];
      double ed[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // e = dV * lambda of the donor (the own cell on outflow faces)
        int d = in[q] ? dk[q] : kc;
        if (in[q]) {
          double adV = fabs(dV[q] * cout[1 * R::NC + d]);
          double aF = fabs(F[q]);
          vcut += fabs(dV[q]) - adV;
          double Id = cout[2 * R::NC + d];
          min_ += aF;
          nI += aF * (Id - IL);
          nsrr += aF * (cout[3 * R::NC + d] - sL0);
          nszz += aF * (cout[4 * R::NC + d] - sL1);
          nsrz += aF * (cout[5 * R::NC + d] - sL2);
          nf0 += adV * (cout[6 * R::NC + d] - fL0);
          if (g.nmat > 1) nf1 += adV * (cout[7 * R::NC + d] - fL1);
          ed[q] = F[q] * Id;
        } else {
          ed[q] = F[q] * IL;
        }
      }
      double lam = cout[1 * R::NC + kc];
      double O = ((dmax(-dV[0], 0.0) + dmax(dV[1], 0.0)) + dmax(-dV[2], 0.0)) + dmax(dV[3], 0.0);
      double den = dmax(dmax(M1, min_), kMRemapFloor * g.rho_ref * V);
      double I1 = IL + nI / den;
      double ex = (1.0 - lam) * O - vcut;
      double f1a = dmax(fL0 + (nf0 + fL0 * ex) / V, 0.0);
      double f1b = g.nmat > 1 ? dmax(fL1 + (nf1 + fL1 * ex) / V, 0.0) : 0.0;
      double fs = g.nmat > 1 ? f1a + f1b : f1a;
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
          if (own) {
            pm.msink[ku] = pm.msink[ku] + V * (rho1 - rho2);
            if (db > 0.0) {
              pn.b_phi1[kb] = p1b + db * ((F[1] - F[0]) / V);
              pn.b_phi3[kb] = p3b + db * ((ed[1] - ed[0]) / V);
            }
            if (drr > 0.0) {
              pn.r_phi1[kr] = p1r + drr * ((F[3] - F[2]) / V);
              pn.r_phi3[kr] = p3r + drr * ((ed[3] - ed[2]) / V);
            }
          }
          rho1 = rho2;
          I1 = I2;
        }
      }
      if (own) {
        long long c = cidx(g, i, j);
        D.rho[c] = rho1;
        double fa = f1a / dmax(fs, 1.0);
        double fb = f1b / dmax(fs, 1.0);
        D.f[0][c] = fa;
        if (g.nmat > 1) D.f[1][c] = fb;
        double s0n = sL0 + nsrr / den, s1n = sL1 + nszz / den, s2n = sL2 + nsrz / den;
        if (g.any_strength) {
          D.s[0][c] = s0n;
          D.s[1][c] = s1n;
          D.s[2][c] = s2n;
        }
        if (j == g.NZ - 1) {
          w.mout[i] += F[3];
          w.eout[i] += ed[3];
        }
        eRho[u] = rho1;
        eI[u] = I1;
        eF0[u] = fa;
        eF1[u] = fb;
        eS0[u] = s0n;
        eS1[u] = s1n;
        eS2[u] = s2n;
      }
    }
    s_rho1[k] = rho1;
  }
  __syncthreads();

  // ------------------------------------------------------------------ F
  double* heat = s_big;           // [NF]
  double* speed = s_big + R::NF;  // [NF]
  for (int k = tid; k < R::NF; k += NT) {
    int i = i0 + k % R::FW, j = j0 + k / R::FW;
    if (i > g.NR || j > g.NZ) continue;
    // node mass: a quarter of the four cell masses (SW, SE, NW, NE)
    const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
    double M[4] = {0, 0, 0, 0};
    bool qok[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      qok[q] = in_cells(g, qi[q], qj[q]);
      if (qok[q]) M[q] = s_rho[kA(qi[q], qj[q])] * cell_volume(g, qi[q]);
    }
    double mL = 0.25 * ((M[0] + M[1]) + (M[2] + M[3]));
    double FD[4];
    FD[0] = 0.25 * ((s_Fr[kR(i - 1, j - 1)] + s_Fr[kR(i, j - 1)]) + (s_Fr[kR(i - 1, j)] + s_Fr[kR(i, j)]));
    FD[1] = 0.25 * ((s_Fr[kR(i, j - 1)] + s_Fr[kR(i + 1, j - 1)]) + (s_Fr[kR(i, j)] + s_Fr[kR(i + 1, j)]));
    FD[2] = 0.25 * ((s_Fz[kZ(i - 1, j - 1)] + s_Fz[kZ(i, j - 1)]) + (s_Fz[kZ(i - 1, j)] + s_Fz[kZ(i, j)]));
    FD[3] = 0.25 * ((s_Fz[kZ(i - 1, j)] + s_Fz[kZ(i, j)]) + (s_Fz[kZ(i - 1, j + 1)] + s_Fz[kZ(i, j + 1)]));
    if (i == 0) FD[0] = 0.0;
    if (i == g.NR) FD[1] = 0.0;
    if (j == 0) FD[2] = 0.0;
    const int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
    const bool in[4] = {FD[0] > 0.0, FD[1] < 0.0, FD[2] > 0.0, FD[3] < 0.0};
    double m1 = mL + (((FD[0] - FD[1]) + FD[2]) - FD[3]);
    int kb0 = kB(i, j);
    double vLr = s_vL[kb0], vLz = s_vL[R::NB + kb0];
    double min_ = 0.0, nr = 0.0, nz = 0.0, kin = 0.0;
    double upr[4], upz[4];
    bool ok[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      ok[q] = ni[q] >= 0 && ni[q] <= g.NR && nj[q] >= 0 && nj[q] <= g.NZ;
      if (in[q] && ok[q]) {
        int d = kB(ni[q], nj[q]);
        double aF = fabs(FD[q]);
        double ur = s_vL[d], uz = s_vL[R::NB + d];
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
#pragma unroll
    for (int q = 0; q < 4; q++) {
      if (in[q] && ok[q]) {
        double ar = upr[q] - vLr, az = upz[q] - vLz;
        kin += fabs(FD[q]) * (ar * ar + az * az);
      }
    }
    double dKE = 0.5 * (kin - (nr * nr + nz * nz) / den);
    double Mn = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++)
      if (qok[q]) Mn += s_rho1[kE(qi[q], qj[q])] * cell_volume(g, qi[q]);
    double h = Mn > kMRemapFloor * g.rho_ref * Vd ? dmax(dKE, 0.0) / Mn : 0.0;
    bool own = owns_node(i, j);
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
        if (own) {
          if (db > 0.0) {
            pn.b_phi2r[kb] = bpr + db * ((FD[1] * upr[1] - FD[0] * upr[0]) / Vd);
            pn.b_phi2z[kb] = bpz + db * ((FD[1] * upz[1] - FD[0] * upz[0]) / Vd);
          }
          if (drr > 0.0) {
            pn.r_phi2r[kr] = rpr + drr * ((FD[3] * upr[3] - FD[2] * upr[2]) / Vd);
            pn.r_phi2z[kr] = rpz + drr * ((FD[3] * upz[3] - FD[2] * upz[2]) / Vd);
          }
        }
        v1r = v2r;
        v1z = v2z;
      }
    }
    if (i == 0 || i == g.NR) v1r = 0.0;
    if (j == 0) {
      v1r = 0.0;
      v1z = 0.0;
    }
    if (g.top_closed && j == g.NZ) v1z = 0.0;
    if (own) {
      long long n = nidx(g, i, j);
      D.v[0][n] = v1r;
      D.v[1][n] = v1z;
    }
    heat[k] = h;
    speed[k] = sqrt(v1r * v1r + v1z * v1z);
    // a non-finite velocity makes the speed non-finite and is caught in G
  }
  __syncthreads();

  // ------------------------------------------------------------------ G
  double cand = __builtin_huge_val();
  unsigned flags = 0;
#pragma unroll
  for (int u = 0; u < UE; u++) {
    int k = tid + u * NT;
    if (k >= R::NE) continue;
    int i = i0 - 1 + k % R::EW, j = j0 - 1 + k / R::EW;
    if (!owns_cell(i, j)) continue;
    long long c = cidx(g, i, j);
    const int nf[4] = {kF(i, j), kF(i + 1, j), kF(i, j + 1), kF(i + 1, j + 1)};
    double h = (heat[nf[0]] + heat[nf[1]]) + (heat[nf[2]] + heat[nf[3]]);
    double I1 = eI[u] + h;
    D.I[c] = I1;
    double s = eRho[u] + I1;
    if (g.any_strength) s += eS0[u] + eS1[u] + eS2[u];
    s += eF0[u];
    if (g.nmat > 1) s += eF1[u];
    if (!((s - s) == 0.0)) flags |= kFlagNonFinite;
    if (eRho[u] < -kNegMassTol * g.rho_ref) flags |= kFlagNegMass;
    double u4 = 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      double sp = speed[nf[q]];
      if (!((sp - sp) == 0.0)) flags |= kFlagNonFinite;
      u4 = dmax(u4, sp);
    }
    double f[kMaxMat] = {eF0[u], eF1[u]};
    Mix mx = mixture(g, eRho[u], I1, f);
    double cl2 = mx.c2 + (4.0 / 3.0) * mx.G / dmax(mx.rmat, g.rho_ref * kRhoDenFloor);
    double cl = sqrt(cl2);
    double wgt = dmin(dmax((mx.phi - kWLo) / (kWHi - kWLo), 0.0), 1.0);
    if (wgt > 0.0) cand = dmin(cand, g.cfl * dmin(g.dr, g.dz) / ((cl + u4) * wgt));
  }
  if (flags) atomicOr(&sc->flags, flags);
  for (int off = 32; off > 0; off >>= 1) cand = dmin(cand, __shfl_down(cand, off, 64));
  if ((tid & 63) == 0) s_min[tid >> 6] = cand;
  __syncthreads();
  __shared__ bool s_last;
  if (tid == 0) {
    double m = s_min[0];
    for (int q = 1; q < NT / 64; q++) m = dmin(m, s_min[q]);
    int nblk = gridDim.x * gridDim.y;
    w.dtpart[blockIdx.x + blockIdx.y * gridDim.x] = m;
    __threadfence();
    unsigned prev = atomicAdd(&sc->done, 1u);
    s_last = (prev == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!s_last) return;
  // ------------------------------------------------------------ finalize
  __threadfence();
  int nblk = gridDim.x * gridDim.y;
  double m = __builtin_huge_val();
  for (int q = tid; q < nblk; q += NT) m = dmin(m, __hip_atomic_load(&w.dtpart[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  for (int off = 32; off > 0; off >>= 1) m = dmin(m, __shfl_down(m, off, 64));
  if ((tid & 63) == 0) s_min[tid >> 6] = m;
  __syncthreads();
  if (tid == 0) {
    double mm = s_min[0];
    for (int q = 1; q < NT / 64; q++) mm = dmin(mm, s_min[q]);
    double t = sc->t + sc->dt;
    sc->t = t;
    sc->cycle = sc->cycle + 1;
    double dtn = dmin(dmin(mm, g.dt_grow * sc->dt), g.dt_max);
    if (g.t_stop > 0) dtn = dmin(dtn, dmax(g.t_stop - t, 0.0));
    sc->dt_prev = sc->dt;
    sc->dt = dtn;
    sc->done = 0u;
    unsigned fl = __hip_atomic_load(&sc->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
}

constexpr int kTW = 64, kTH = 16, kNT = 512;

void fused_tiles(int NR, int NZ, int* tr, int* tz) {
  *tr = (NR + kTW - 1) / kTW;
  *tz = (NZ + kTH - 1) / kTH;
}

void launch_cycle_fused(const Geo& g, const State& S0, const State& S1, const Work& w, const Pml& pm, Scal* sc,
                        hipStream_t st) {
  int tr, tz;
  fused_tiles(g.NR, g.NZ, &tr, &tz);
  hipLaunchKernelGGL((k_cycle<kTW, kTH, kNT>), dim3(tr, tz), dim3(kNT), 0, st, g, S0, S1, pm, w, sc);
}

}  // namespace salec
