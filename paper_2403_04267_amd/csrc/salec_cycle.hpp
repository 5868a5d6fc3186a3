// salec_cycle.hpp -- the whole explicit cycle of the r-z SALE scheme with PML
// (Li et al., SALEc-2D: Sec. 2 eqs. (1)-(5), Sec. 3, Sec. 4, Sec. 7) as ONE
// gfx950 kernel launch per cycle, for one instance or a batch of instances.
//
// A launch walks a schedule of (instance, tile) entries. Each workgroup takes
// entries in a grid-stride loop; for a TW x TH tile of cells (and the nodes
// at their lower-left corners) it recomputes every phase over the halo it
// needs, keeping intermediates in LDS:
//   A  cells [i0-3, i0+TW+3)  viscosity, phi-scaled stress less p0 (EoS from cache) -> LDS
//   B  nodes [i0-2, i0+TW+2]  control-volume force, PML psi1 -> v^L         -> LDS
//   C  cells [i0-2, i0+TW+1]  Lagrangian update, PML psi2, limiter           -> LDS
//   E2 cells [i0-1, i0+TW]    face volume and donor mass fluxes, donor-cell
//                             remap, PML phi1/phi3                           -> LDS
//   F  nodes [i0, i0+TW]      momentum remap, KE-loss heat, PML phi2         -> LDS
//   G  cells of the tile      heat, checks, EoS of the new state (cached), dt
// (the same ranges in z). Halo values are recomputed with bit-identical
// arithmetic; only the owner of a cell or node writes it. The state, its EoS
// cache and the PML auxiliaries ping-pong by cycle parity, so every halo read
// sees level n. The Courant minimum of a tile is reduced with wave shuffles
// and LDS and stored per tile; the finalize kernel that follows in the same
// graph reduces each instance's tile minima and advances that instance's t,
// dt and cycle count, so instances keep their own dt.
//
// T is the bulk arithmetic and storage type of stress, velocity and the EoS
// cache (double, or float in the mixed mode). Density, volume fractions,
// internal energy, every mass / volume / energy flux and its sums, and the
// Courant reduction are FP64 in both modes.
#pragma once
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

// LDS copy of a stretched tile's geometry: six column fields over columns
// [i0-3, i0+TW+5), then the row heights over rows [j0-3, j0+TH+5)
template <int TW, int TH>
struct GeoLds {
  static constexpr int GC = TW + 8, GR = TH + 8, N = 6 * GC + GR;
};

template <int TW, int TH, class T, int NM, bool PM, bool DM = false>
struct Smem {
  using R = Regions<TW, TH>;
  // FP64 fields of C's results: rhoL, IL, f[NM]; per-material closure:
  // muL[NM], IL[NM], f[NM]; with damage also D^L and v_vib
  static constexpr int kNCd = (PM ? 3 * NM : 2 + NM) + (DM ? 2 : 0);
  static constexpr int kBigA = 4 * R::NA * (int)sizeof(T);                 // sigma[4][NA]
  static constexpr int kBigC = R::NC * (kNCd * 8 + 4 * (int)sizeof(T));    // C's FP64 fields | lambda, sL x3
  static constexpr int kBigF = R::NF * (8 + (int)sizeof(T));          // heat | speed
  static constexpr int kBig = kBigA > kBigC ? (kBigA > kBigF ? kBigA : kBigF) : (kBigC > kBigF ? kBigC : kBigF);
  static constexpr int kBigD = (kBig + 7) / 8;
  // the damping profiles are staged in LDS where the workgroup's LDS still
  // fits with them (else the phases read them from memory); kRest: every
  // other LDS array of the cycle kernel but s_min and s_geo
  static constexpr int kDamp = R::CW + R::CH + R::BW + R::BH;
  static constexpr int kRest = 8 * (R::NA + kBigD + R::NRF + R::NZF + R::NE) + 2 * R::NB * (int)sizeof(T);
};

// Sum of four per-face (or per-corner) terms ordered W, E, S, N (or SW, SE,
// NW, NE): the r pair plus the z pair, as the divergence of Sec. 2 is an r
// part plus a z part; a reflection in z then maps every sum onto itself
// exactly.
__device__ __forceinline__ double face_sum(const double t[4]) { return (t[0] + t[1]) + (t[2] + t[3]); }

// The same sum fed one term at a time in the order W, E, S, N (q = 0..3, a
// compile-time index in unrolled loops), so that only the pending pair is
// live: (t0 + t1) + (t2 + t3) bit for bit.
struct FaceAcc {
  double h = 0.0, r = 0.0;
  __device__ __forceinline__ void put(int q, double t) {
    if (q == 0 || q == 2)
      h = t;
    else if (q == 1)
      r = h + t;
    else
      h = h + t;
  }
  __device__ __forceinline__ double sum() const { return r + h; }
};

// Quotients of the FP64 sums by one shared denominator b. The FP64 kernel
// forms each quotient a / b as the discrete algorithm does; the mixed kernel,
// whose results are not meant to repeat the FP64 algorithm bit for bit,
// multiplies by the reciprocal formed once.
template <class T> struct Over;
template <> struct Over<double> {
  double b;
  __device__ __forceinline__ explicit Over(double b_) : b(b_) {}
  __device__ __forceinline__ double operator()(double a) const { return a / b; }
};
template <> struct Over<float> {
  double r;
  __device__ __forceinline__ explicit Over(double b_) : r(1.0 / b_) {}
  __device__ __forceinline__ double operator()(double a) const { return a * r; }
};

__device__ __forceinline__ bool in_cells(const Geo& g, int i, int j) {
  return i >= 0 && i < g.NR && j >= 0 && j < g.NZ;
}

// Courant candidate of one cell of a new state, and its EoS (cached for the
// next cycle). u4 is the largest corner speed, L = min(dr, dz) of the cell.
template <class T>
__device__ __forceinline__ double cell_dt(const Geo& g, const Mix<T>& mx, T u4, double L) {
  using N = Num<T>;
  T cl2 = mx.c2 + N::div(T(4.0 / 3.0) * mx.G, tmax(mx.rmat, GeoT<T>::rho_ref(g) * T(kRhoDenFloor)));
  T cl = N::sqr(cl2);
  T wgt = tmin(tmax(N::div(mx.phi - T(kWLo), T(kWHi - kWLo)), T(0)), T(1));
  if (wgt > T(0)) return g.cfl * L / (((double)cl + (double)u4) * (double)wgt);
  return __builtin_huge_val();
}

template <class T>
__device__ __forceinline__ void store_eos(const State& D, long long c, const Mix<T>& mx) {
  ((T*)D.eos[0])[c] = mx.p;
  ((T*)D.eos[1])[c] = mx.c2;
  ((T*)D.eos[2])[c] = mx.G;
  ((T*)D.eos[3])[c] = mx.Y;
  ((T*)D.eos[4])[c] = mx.sx;
}

// Reduces `cand` over the workgroup into s_min[0] (all threads call it).
template <int NT>
__device__ __forceinline__ double block_min(double cand, double* s_min) {
  for (int off = 32; off > 0; off >>= 1) cand = dmin(cand, __shfl_down(cand, off, 64));
  if ((threadIdx.x & 63) == 0) s_min[threadIdx.x >> 6] = cand;
  __syncthreads();
  double m = s_min[0];
  for (int q = 1; q < NT / 64; q++) m = dmin(m, s_min[q]);
  return m;
}

// register-array element by a run-time index without dynamic indexing
template <int N, class T>
__device__ __forceinline__ T reg_get(const T (&a)[N], int u) {
  T r = a[0];
#pragma unroll
  for (int q = 1; q < N; q++) r = (u == q) ? a[q] : r;
  return r;
}
template <int N, class T>
__device__ __forceinline__ void reg_put(T (&a)[N], int u, T v) {
#pragma unroll
  for (int q = 0; q < N; q++) a[q] = (u == q) ? v : a[q];
}

template <int TW, int TH, int NT, int WPE, class T, bool GEO, int NM, bool PM, bool DM, bool DL>
__device__ __forceinline__ void tile_cycle(const Inst& in, int tile, double* s_rho, double* s_bigd, T* s_vL,
                                           double* s_Fr, double* s_Fz, double* s_rho1, double* s_min,
                                           double* s_geo, double* s_damp) {
  using R = Regions<TW, TH>;
  using N = Num<T>;
  using GT = GeoT<T>;
  constexpr int UA = (R::NA + NT - 1) / NT;

  const Geo& g = in.g;
  Scal* sc = in.sc;
  // the instance's clock: written only by the finalize kernel between
  // launches, so read through the constant address space (scalar loads, one
  // batch) rather than as vector loads behind the error test
  using CScal = const __attribute__((address_space(4))) Scal;
  const CScal* csc = (const CScal*)sc;
  const int err = csc->err;
  const long long cyc = csc->cycle;
  const double dt = csc->dt;
  if (err) return;
  const int tid = threadIdx.x;
  const int ti = tile % in.tiles_r, tj = tile / in.tiles_r;
  const int i0 = ti * TW, j0 = tj * TH;
  const int i1 = min(i0 + TW, g.NR), j1 = min(j0 + TH, g.NZ);  // owned cells [i0, i1) x [j0, j1)
  const int par = (int)(cyc & 1);
  const State& S = in.S[par];
  const State& D = in.S[par ^ 1];
  const Pml& pm = in.pm;
  const PmlAux& po = pm.a[par];
  const PmlAux& pn = pm.a[par ^ 1];
  const T* Sv0 = (const T*)S.v[0];
  const T* Sv1 = (const T*)S.v[1];
  const T* Ss0 = (const T*)S.s[0];
  const T* Ss1 = (const T*)S.s[1];
  const T* Ss2 = (const T*)S.s[2];
  const T dtT = (T)dt;
  // Grid geometry: the uniform-grid kernel evaluates it from i and j; the
  // table kernel (GEO, launched when any instance is stretched) reads each
  // tile's columns and rows from the instance's table, staged in LDS first.
  using GL = GeoLds<TW, TH>;
  constexpr bool st = GEO;
  if constexpr (st) {
    const int gs = g.NR + 1;
    const double* grow = in.geo + 6 * gs;
    for (int k = tid; k < GL::N; k += NT) {
      double v = 0.0;
      if (k < 6 * GL::GC) {
        int f = k / GL::GC, i = i0 - 3 + (k - f * GL::GC);
        if (i >= 0 && i <= g.NR) v = in.geo[f * gs + i];
      } else {
        int j = j0 - 3 + (k - 6 * GL::GC);
        if (j >= 0 && j < g.NZ) v = grow[j];
      }
      s_geo[k] = v;
    }
    __syncthreads();
  }
  auto colT = [&](int i) -> Col<T> {
    return st ? col_fields<T>(s_geo, GL::GC, i - (i0 - 3)) : col_uniform<T>(g, i);
  };
  auto colD = [&](int i) -> Col<double> {
    return st ? col_fields<double>(s_geo, GL::GC, i - (i0 - 3)) : col_uniform<double>(g, i);
  };
  auto dzD = [&](int j) -> double { return st ? s_geo[6 * GL::GC + (j - (j0 - 3))] : g.dz; };
  auto dzT = [&](int j) -> T { return st ? (T)s_geo[6 * GL::GC + (j - (j0 - 3))] : GT::dz(g); };
  auto volD = [&](int i, int j) { return colD(i).az * dzD(j); };
  auto volT = [&](int i, int j) { return colT(i).az * dzT(j); };
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
  // Thread maps of the cell loops, row-major with the rows reordered. A and
  // C share one (A's results stay in registers for C): C's rows first, then
  // the row below and the row above them that only A covers, so C's loop
  // over the first AW (AH - 2) entries leaves whole waves idle instead of
  // masking lanes. E2 and G share another: the tile's rows first, then E2's
  // rows below and above it.
  auto a_cell = [&](int k, int& i, int& j) {
    int q = k / R::AW;
    i = i0 - 3 + (k - q * R::AW);
    j = q < R::AH - 2 ? j0 - 2 + q : (q == R::AH - 2 ? j0 - 3 : j0 + TH + 2);
  };
  auto e_cell = [&](int k, int& i, int& j) {
    int q = k / R::EW;
    i = i0 - 1 + (k - q * R::EW);
    j = q < TH ? j0 + q : (q == TH ? j0 - 1 : j0 + TH);
  };
  // C's FP64 fields during C..E2: rhoL, IL, f[NM], or with the per-material
  // closure muL[NM] (mu_m / J), IL[NM], f[NM]; then, with damage, D^L, v_vib
  constexpr int kNCd = Smem<TW, TH, T, NM, PM, DM>::kNCd;
  constexpr int kFo = PM ? 2 * NM : 2;  // first volume-fraction field
  constexpr int kDo = kFo + NM;         // damage field (then the vibration speed)
  T* sig = (T*)s_bigd;                // [4][NA] during A..B
  double* cd = s_bigd;                // [kNCd][NC] during C..E2
  T* ct = (T*)(s_bigd + kNCd * R::NC);  // [4][NC] lambda, sL x3 during C..E2
  double* heat = s_bigd;              // [NF] during F..G
  T* speed = (T*)(s_bigd + R::NF);    // [NF] during F..G
  T* s_kd = (T*)s_Fr;                 // [NB] during B..C: 1/2 |v^L - v^n|^2 per node
  static_assert(R::NB * (int)sizeof(T) <= (R::NRF + R::NZF) * 8, "node buffer must fit in the flux buffers");

  // The damping profiles of the tile's cell columns and rows (C's region)
  // and node columns and rows (B's region), staged in LDS during A for B, C,
  // E2 and F: the loads join A's batch (from a clamped index, or the density
  // array's first entry when there are no layers), the stores follow A's loop.
  constexpr int kDamp = R::CW + R::CH + R::BW + R::BH;
  double* s_dcr = s_damp;
  double* s_dcz = s_dcr + R::CW;
  double* s_dnr = s_dcz + R::CH;
  double* s_dnz = s_dnr + R::BW;
  bool damp_ok;
  double damp_v;
  {
    const int k = tid < kDamp ? tid : 0;
    const double* a;
    int idx, lim;
    if (k < R::CW) {
      a = pm.dcr, idx = i0 - 2 + k, lim = g.NR;
    } else if (k < R::CW + R::CH) {
      a = pm.dcz, idx = j0 - 2 + (k - R::CW), lim = g.NZ;
    } else if (k < R::CW + R::CH + R::BW) {
      a = pm.dnr, idx = i0 - 2 + (k - R::CW - R::CH), lim = g.NR + 1;
    } else {
      a = pm.dnz, idx = j0 - 2 + (k - R::CW - R::CH - R::BW), lim = g.NZ + 1;
    }
    damp_ok = g.pml_on && tid < kDamp && idx >= 0 && idx < lim;
    damp_v = (g.pml_on ? a : S.rho)[g.pml_on ? min(max(idx, 0), lim - 1) : 0];
  }

  // ------------------------------------------------------------------ A
  // 1024-thread workgroups keep the per-cell loops of A and C rolled: four
  // waves per SIMD leave no registers for two cells in flight at once
  constexpr int kUnroll = WPE >= 4 ? 1 : UA;
  T rP[UA];
  // level-n values A loads that C needs again, kept in registers for C
  // (FP64 tiles capped at 128 registers reload them instead)
  constexpr bool kKeepA = !(WPE >= 4 && sizeof(T) == 8);
  double rF[NM][UA];
  T rS0[UA], rS1[UA], rS2[UA], rSx[UA], rQ[PM ? UA : 1];
#pragma unroll
  for (int u = 0; u < (PM ? UA : 1); u++) rQ[u] = T(0);
#pragma unroll
  for (int u = 0; u < UA; u++) {
    rP[u] = rS0[u] = rS1[u] = rS2[u] = rSx[u] = T(0);
#pragma unroll
    for (int m = 0; m < NM; m++) rF[m][u] = 0.0;
  }
#pragma unroll kUnroll
  for (int u = 0; u < UA; u++) {
    int k = tid + u * NT;
    if (k >= R::NA) continue;
    int i, j;
    a_cell(k, i, j);
    T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
    double rh = 0.0;
    // v^n of the node at the cell's lower-left corner; B's nodes are these
    // corners of A's cells from (i0-2, j0-2) on, so A hands them to B in LDS
    // (read from a clamped node, and used only where the node exists)
    const bool node_ok = i >= 0 && i <= g.NR && j >= 0 && j <= g.NZ;
    const long long n0 = nidx(g, min(max(i, 0), g.NR), min(max(j, 0), g.NZ));
    const T v0r = Sv0[n0], v0z = Sv1[n0];
    if (in_cells(g, i, j)) {
      long long c = cidx(g, i, j);
      // every load of the cell first, with no branch among them (arrays a
      // material or the strength model lacks are replaced by one that exists,
      // read and unused), so that they are in flight together
      double fd[NM];
      T f[kMaxMat];
#pragma unroll
      for (int m = 0; m < kMaxMat; m++) {
        if (m < NM) {
          const double x = S.f[m < g.nmat ? m : 0][c];
          fd[m] = m < g.nmat ? x : 0.0;
        }
        f[m] = m < NM ? (T)fd[m] : T(0);
      }
      const T* St0 = g.any_strength ? Ss0 : (const T*)S.eos[0];
      const T* St1 = g.any_strength ? Ss1 : (const T*)S.eos[0];
      const T* St2 = g.any_strength ? Ss2 : (const T*)S.eos[0];
      const T l0 = St0[c], l1 = St1[c], l2 = St2[c];
      const T p0j = (T)(g.has_p0 ? in.p0 : S.rho)[j];
      rh = S.rho[c];
      T phi, den, rm;
      matter(g, (T)rh, f, phi, den, rm);
      T p = ((const T*)S.eos[0])[c], c2 = ((const T*)S.eos[1])[c], sx = ((const T*)S.eos[4])[c];
      T vr4[4] = {v0r, Sv0[nidx(g, i + 1, j)], Sv0[nidx(g, i, j + 1)], Sv0[nidx(g, i + 1, j + 1)]};
      T vz4[4] = {v0z, Sv1[nidx(g, i + 1, j)], Sv1[nidx(g, i, j + 1)], Sv1[nidx(g, i + 1, j + 1)]};
      const Col<T> cg = colT(i);
      const T dzj = dzT(j);
      Kin<T> kn = kinematics(cg, dzj, vr4, vz4);
      T L = tmin(cg.dr, dzj);
      T dDn = dtT * kn.D;
      T Jn = T(1) + dDn;
      T Dm = Jn < T(1) ? N::div(Vol<T>::closing(Jn, dDn, phi, sx), dtT) : T(0);
      T Ld = L * Dm;
      T Q = rm * (GT::q_quad(g) * Ld * Ld + GT::q_lin(g) * N::sqr(c2) * Ld);
      T P = p + Q;
      // the momentum balance (and so psi1) sees p - p0; C's energy terms keep P
      const T Pf = g.has_p0 ? P - p0j : P;
      const T srr = g.any_strength ? l0 : T(0), szz = g.any_strength ? l1 : T(0), srz = g.any_strength ? l2 : T(0);
      T stt = -(srr + szz);
      s0 = phi * (srr - Pf);
      s1 = phi * (szz - Pf);
      s2 = phi * (stt - Pf);
      s3 = phi * srz;
      reg_put(rP, u, P);
      if constexpr (PM) reg_put(rQ, u, Q);  // each material's p dV work uses p_m + Q
#pragma unroll
      for (int m = 0; m < NM; m++) reg_put(rF[m], u, fd[m]);
      reg_put(rS0, u, srr);
      reg_put(rS1, u, szz);
      reg_put(rS2, u, srz);
      reg_put(rSx, u, sx);
    }
    if (node_ok && i >= i0 - 2 && j >= j0 - 2) {
      s_vL[kB(i, j)] = v0r;
      s_vL[R::NB + kB(i, j)] = v0z;
    }
    const int ka = kA(i, j);
    sig[0 * R::NA + ka] = s0;
    sig[1 * R::NA + ka] = s1;
    sig[2 * R::NA + ka] = s2;
    sig[3 * R::NA + ka] = s3;
    s_rho[ka] = rh;
  }
  if (DL && tid < kDamp) s_damp[tid] = damp_ok ? damp_v : 0.0;
  __syncthreads();

  // ------------------------------------------------------------------ B
  for (int k = tid; k < R::NB; k += NT) {
    int i = i0 - 2 + k % R::BW, j = j0 - 2 + k / R::BW;
    T vLr = T(0), vLz = T(0), kdn = T(0);
    if (i >= 0 && i <= g.NR && j >= 0 && j <= g.NZ) {
      // the node's damping rates (staged in LDS by A where they fit; else
      // read here, ahead of the forces, from an array that always exists)
      const double dbl = DL ? s_dnz[j - (j0 - 2)] : (g.pml_on ? pm.dnz : S.rho)[g.pml_on ? j : 0];
      const double drl = DL ? s_dnr[i - (i0 - 2)] : (g.pml_on ? pm.dnr : S.rho)[g.pml_on ? i : 0];
      const T vnr = s_vL[k], vnz = s_vL[R::NB + k];  // v^n, from A
      // quadrants NE = (i, j), NW = (i-1, j), SE = (i, j-1), SW = (i-1, j-1)
      const int qa[4] = {kA(i, j), kA(i - 1, j), kA(i, j - 1), kA(i - 1, j - 1)};
      T srr[4], szz[4], stt[4], srz[4], rh[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        srr[q] = sig[0 * R::NA + qa[q]];
        szz[q] = sig[1 * R::NA + qa[q]];
        stt[q] = sig[2 * R::NA + qa[q]];
        srz[q] = sig[3 * R::NA + qa[q]];
        rh[q] = (T)s_rho[qa[q]];
      }
      // dual cell: from the west cell's centre rW to the east cell's centre
      // rE, half the row above (hN) and half the row below (hS)
      const Col<T> ce = colT(i), cw = colT(i - 1);
      T rN = ce.rw;
      T rE = i < g.NR ? ce.rc : T(0);
      T rW = i > 0 ? cw.rc : T(0);
      T aE = i < g.NR ? ce.aw : T(0);
      T aW = i > 0 ? cw.ae : T(0);
      T hN = j < g.NZ ? T(0.5) * dzT(j) : T(0);
      T hS = j > 0 ? T(0.5) * dzT(j - 1) : T(0);
      T Frr = (hN * (rE * (srr[0] - stt[0]) + rN * stt[0]) + hS * (rE * (srr[2] - stt[2]) + rN * stt[2])) -
              (hN * (rW * (srr[1] - stt[1]) + rN * stt[1]) + hS * (rW * (srr[3] - stt[3]) + rN * stt[3]));
      T Frz = (aW * srz[1] + aE * srz[0]) - (aW * srz[3] + aE * srz[2]);
      T Fzr = rE * (hN * srz[0] + hS * srz[2]) - rW * (hN * srz[1] + hS * srz[3]);
      T Fzz = (aW * szz[1] + aE * szz[0]) - (aW * szz[3] + aE * szz[2]);
      T Fr = Frr + Frz, Fz = Fzr + Fzz;
      T macc = (aE * hN * rh[0] + aW * hN * rh[1]) + (aE * hS * rh[2] + aW * hS * rh[3]);
      T Vd = (aE + aW) * (hN + hS);
      T mt = tmax(macc, T(kMAccEps) * GT::rho_ref(g) * Vd);
      T psr = T(0), psz = T(0);
      double db = 0.0, drr = 0.0;
      long long kb = -1, kr = -1;
      if (g.pml_on) {
        db = dbl;
        drr = drl;
        if (j < g.pml_b) kb = pml_bn(g, i, j);
        if (i > g.n_r) kr = pml_rn(g, i, j);
        // the auxiliary this step applies: psi1, or phi2 when the layers
        // follow Sec. 3's sentence as printed
        const double* ar_b = g.pml_place ? po.b_phi2r : po.b_psi1r;
        const double* az_b = g.pml_place ? po.b_phi2z : po.b_psi1z;
        const double* ar_r = g.pml_place ? po.r_phi2r : po.r_psi1r;
        const double* az_r = g.pml_place ? po.r_phi2z : po.r_psi1z;
        double br = kb >= 0 ? ar_b[kb] : 0.0, bz = kb >= 0 ? az_b[kb] : 0.0;
        double rr = kr >= 0 ? ar_r[kr] : 0.0, rz = kr >= 0 ? az_r[kr] : 0.0;
        psr = (T)(br + rr);
        psz = (T)(bz + rz);
      }
      T Fer = Fr - Vd * psr, Fez = Fz - Vd * psz;
      vLr = vnr + dtT * N::div(Fer, mt);
      vLz = vnz + dtT * N::div(Fez, mt);
      if (owns_node(i, j) && (db > 0.0 || drr > 0.0)) {
        if (db > 0.0) {
          pn.b_psi1r[kb] = po.b_psi1r[kb] - dt * db * (double)N::div(Frr, Vd);
          pn.b_psi1z[kb] = po.b_psi1z[kb] - dt * db * (double)N::div(Fzr, Vd);
        }
        if (drr > 0.0) {
          pn.r_psi1r[kr] = po.r_psi1r[kr] - dt * drr * (double)N::div(Frz, Vd);
          pn.r_psi1z[kr] = po.r_psi1z[kr] - dt * drr * (double)N::div(Fzz, Vd);
        }
      }
      if (i == 0 || i == g.NR) vLr = T(0);
      if (j == 0) {
        vLr = T(0);
        vLz = T(0);
      }
      if (g.top_closed && j == g.NZ) vLz = T(0);
      T dvr = vLr - vnr, dvz = vLz - vnz;
      kdn = T(0.5) * (dvr * dvr + dvz * dvz);
    }
    s_vL[k] = vLr;
    s_vL[R::NB + k] = vLz;
    s_kd[k] = kdn;
  }
  __syncthreads();

  // face volumes from v^L (radial face at r_i of row j; axial face at z_j of
  // column i with dual-area node weights)
  auto dv_r = [&](int i, int j) {
    T u = T(0.5) * (s_vL[kB(i, j)] + s_vL[kB(i, j + 1)]);
    return dtT * ((colT(i).rw * dzT(j)) * u);
  };
  auto dv_z = [&](int i, int j) {
    const Col<T> c = colT(i);
    return dtT * (c.aw * s_vL[R::NB + kB(i, j)] + c.ae * s_vL[R::NB + kB(i + 1, j)]);
  };

  // ------------------------------------------------------------------ C
  // (same cell-to-thread map as A, so A's per-cell results stay in registers;
  // the stress buffer is dead after B, so results go straight into it)
#pragma unroll kUnroll
  for (int u = 0; u < UA; u++) {
    int k = tid + u * NT;
    if (k >= (R::AH - 2) * R::AW) continue;
    int i, j;
    a_cell(k, i, j);
    if (i < i0 - 2 || i >= i0 + TW + 2) continue;
    // outside the grid: a void donor (rho^L = 0, lambda = 1, zero state)
    double oRhoL = 0.0, oIL = 0.0, of[NM], oMuL[NM], oILm[NM];
#pragma unroll
    for (int m = 0; m < NM; m++) of[m] = oMuL[m] = oILm[m] = 0.0;
    T oLam = T(1), os0 = T(0), os1 = T(0), os2 = T(0);
    double oDL = 0.0, oVib = 0.0;  // damage and vibration speed (void donor: 0)
    if (in_cells(g, i, j)) {
      long long c = cidx(g, i, j);
      // the cell's loads first, with no branch among them (as in A)
      const T Gl = ((const T*)S.eos[2])[c], Yl = ((const T*)S.eos[3])[c];
      double Il = 0.0;
      if constexpr (!PM) Il = S.I[c];
      const double dbl = DL ? s_dcz[j - (j0 - 2)] : (g.pml_on ? pm.dcz : S.rho)[g.pml_on ? j : 0];
      const double drl = DL ? s_dcr[i - (i0 - 2)] : (g.pml_on ? pm.dcr : S.rho)[g.pml_on ? i : 0];
      const int nb[4] = {kB(i, j), kB(i + 1, j), kB(i, j + 1), kB(i + 1, j + 1)};
      T vr4[4], vz4[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        vr4[q] = s_vL[nb[q]];
        vz4[q] = s_vL[R::NB + nb[q]];
      }
      const Col<T> cg = colT(i);
      const T dzj = dzT(j);
      Kin<T> kn = kinematics(cg, dzj, vr4, vz4);
      T s0rr = T(0), s0zz = T(0), s0rz = T(0);
      if (kKeepA) {
        s0rr = reg_get(rS0, u);
        s0zz = reg_get(rS1, u);
        s0rz = reg_get(rS2, u);
      } else if (g.any_strength) {
        s0rr = Ss0[c];
        s0zz = Ss1[c];
        s0rz = Ss2[c];
      }
      T srr = s0rr, szz = s0zz, srz = s0rz;
      if (g.any_strength) {
        T G = Gl, Y = Yl;
        T tr3 = N::div((kn.err + kn.ezz) + kn.ett, T(3));
        // damage: the volume-fraction weights of the level-n cell
        T dw[kMaxMat];
        if constexpr (DM) {
          oDL = S.dmg[c];
          oVib = S.vib[c];
          T fw[kMaxMat];
#pragma unroll
          for (int m = 0; m < kMaxMat; m++)
            fw[m] = m < NM && m < g.nmat ? (T)(kKeepA ? reg_get(rF[m], u) : S.f[m][c]) : T(0);
          T phw, dnw, rmw;
          matter(g, (T)s_rho[kA(i, j)], fw, phw, dnw, rmw);
          // block model: dynamic viscosity rho gamma_eta c h of the damaged
          // rock (weight D) while it vibrates (full above kVibOn); the flow
          // stress exceeds Y by 3 eta times the equivalent strain rate
          // sqrt(2/3 e':e') of the step (a Bingham material)
          T nu = T(0);
#pragma unroll
          for (int m = 0; m < kMaxMat; m++) {
            dw[m] = N::div(fw[m], dnw);
            if (m < NM && m < g.nmat && GT::mat(g, m).damage) nu += dw[m] * GT::mat(g, m).nub;
          }
          T eta = ((T)oDL * tmin(N::div((T)oVib, T(kVibOn)), T(1))) * (rmw * nu);
          T er = kn.err - tr3, ez = kn.ezz - tr3, et = kn.ett - tr3;
          T e2 = ((er * er + ez * ez) + et * et) + T(2) * (kn.erz * kn.erz);
          Y = Y + T(3) * eta * N::sqr(T(2.0 / 3.0) * e2);
        }
        T om = kn.om;
        T dsrr = T(2) * G * (kn.err - tr3) + T(2) * om * srz;
        T dszz = T(2) * G * (kn.ezz - tr3) - T(2) * om * srz;
        T dsrz = T(2) * G * kn.erz + om * (szz - srr);
        srr = srr + dtT * dsrr;
        szz = szz + dtT * dszz;
        srz = srz + dtT * dsrz;
        T J2 = srr * srr + szz * szz + srr * szz + srz * srz;
        T seq = N::sqr(T(3) * J2);
        if (seq > Y) {
          T fac = N::div(Y, seq);
          srr = srr * fac;
          szz = szz * fac;
          srz = srz * fac;
        }
        if constexpr (DM) {
          // damage grows by the equivalent plastic strain of the return,
          // (trial - yield) / 3G, over each damaging material's failure
          // strain max(eps_fb, B (p - p_bd)) at the cell's pressure
          // (volume-fraction weighted rate), capped at 1
          T dep = G > T(0) ? N::div(tmax(seq - Y, T(0)), T(3) * G) : T(0);
          T pc = ((const T*)S.eos[0])[c];
          T rate = T(0);
#pragma unroll
          for (int m = 0; m < kMaxMat; m++) {
            if (!(m < NM && m < g.nmat)) continue;
            const MatT<T>& M = GT::mat(g, m);
            if (M.damage) rate += N::div(dw[m], tmax(M.eps_fb, M.B_dmg * (pc - M.p_bd)));
          }
          oDL = dmin(oDL + (double)(dep * rate), 1.0);
        }
      }
      T stt = -(s0rr + s0zz);
      T P = reg_get(rP, u);
      T sde = ((s0rr * kn.err + s0zz * kn.ezz) + stt * kn.ett) + T(2) * s0rz * kn.erz;
      T dD = dtT * kn.D;
      T J = T(1) + dD;
      double rho = s_rho[kA(i, j)];
      double fn[NM];
      T fq[kMaxMat];
#pragma unroll
      for (int m = 0; m < kMaxMat; m++) {
        if (m < NM) fn[m] = kKeepA ? reg_get(rF[m], u) : (m < g.nmat ? S.f[m][c] : 0.0);
        fq[m] = m < NM ? (T)fn[m] : T(0);
      }
      T phi, den, rm;
      matter(g, (T)rho, fq, phi, den, rm);
      T Jm = Vol<T>::ratio(J, dD, phi, kKeepA ? reg_get(rSx, u) : ((const T*)S.eos[4])[c]);
      T Wdt = dtT * sde - P * Vol<T>::jm1(J, dD);
      T rden = tmax(rm, GT::rho_ref(g) * T(kRhoDenFloor));
      double rt = dmax(rho, g.rho_ref * kPmlRhoFloor);
      T kd[4];
#pragma unroll
      for (int q = 0; q < 4; q++) kd[q] = s_kd[nb[q]];
      T V = cg.az * dzj;
      T hdz = T(0.5) * dzj;
      T wW = N::div(cg.aw * hdz, V);
      T wE = N::div(cg.ae * hdz, V);
      T hL = wW * (kd[0] + kd[2]) + wE * (kd[1] + kd[3]);
      double psi2 = 0.0, db = 0.0, drr = 0.0;
      long long kb = -1, kr = -1;
      if (g.pml_on) {
        db = dbl;
        drr = drl;
        if (j < g.pml_b) kb = pml_bc(g, i, j);
        if (i >= g.n_r) kr = pml_rc(g, i, j);
        // the auxiliary this step applies to the energy: psi2, or phi3 as
        // printed (which then also applies phi1 to the mass below)
        const double* a_b = g.pml_place ? po.b_phi3 : po.b_psi2;
        const double* a_r = g.pml_place ? po.r_phi3 : po.r_psi2;
        double b = kb >= 0 ? a_b[kb] : 0.0, r = kr >= 0 ? a_r[kr] : 0.0;
        psi2 = b + r;
      }
      // the mass the Eulerian step starts from: with the printed placement
      // phi1 leaves the layer cell here (never below zero mass)
      double rhoE = rho;
      if (g.pml_place && (db > 0.0 || drr > 0.0)) {
        double b = kb >= 0 ? po.b_phi1[kb] : 0.0, r = kr >= 0 ? po.r_phi1[kr] : 0.0;
        rhoE = dmax(rho - dt * (b + r), 0.0);
      }
      double IL = 0.0;
      if constexpr (!PM) {
        IL = (Il + (double)N::div(Wdt, rden)) + (double)hL;
        // outside the strips psi2 is +0 and so is its term: x - (+0) = x
        if (kb >= 0 || kr >= 0) IL = IL - dt * (psi2 / rt);
      } else {
        // each material: deviatoric work and its own p dV work on the cell's
        // volume change, per unit of its own mass (density mu_m / f_m; below
        // kFPmEps or without mass the cell's matter density)
        double phid = 0.0;
#pragma unroll
        for (int m = 0; m < NM; m++)
          if (m < g.nmat) phid += fn[m];
        const double rmd = rho / (phid > kPhiEps ? phid : kPhiEps);
        const T Q = reg_get(rQ, u);
        const T jm1 = Vol<T>::jm1(J, dD);
        const double iJ = (double)J;
#pragma unroll
        for (int m = 0; m < NM; m++) {
          if (m >= g.nmat) continue;
          const double mud = S.mu[m][c];
          const double rmm = fn[m] > kFPmEps && mud > 0.0 ? mud / fn[m] : rmd;
          const T Pm = ((const T*)S.pmat[m])[c] + Q;
          const T Wm = dtT * sde - Pm * jm1;
          const T rdm = tmax((T)rmm, GT::rho_ref(g) * T(kRhoDenFloor));
          oILm[m] = (S.Im[m][c] + (double)N::div(Wm, rdm)) + (double)hL;
          if (kb >= 0 || kr >= 0) oILm[m] = oILm[m] - dt * (psi2 / rt);
          // the printed placement's phi1 removes the same fraction of every
          // material's mass (the quotient only where it acted)
          double muE = mud;
          if (rhoE != rho) muE = mud * (rho > 0.0 ? rhoE / rho : 0.0);
          oMuL[m] = muE / iJ;
        }
      }
      // Jm / J, which is exactly 1 where the material follows the cell (Jm = J)
      double fr = (Jm == J && J > T(0)) ? 1.0 : (double)N::div(Jm, J);
      double fLv[NM];
#pragma unroll
      for (int m = 0; m < NM; m++) fLv[m] = (m == 0 || m < g.nmat) ? fn[m] * fr : 0.0;
      if (owns_cell(i, j)) {
        if (db > 0.0) {
          T Wr = ((s0rr * kn.err + stt * kn.ett) + s0rz * kn.dvz_dr) - P * kn.Dr;
          pn.b_psi2[kb] = po.b_psi2[kb] - dt * db * (double)(phi * Wr);
        }
        if (drr > 0.0) {
          T Wz = (s0zz * kn.ezz + s0rz * kn.dvr_dz) - P * kn.Dz;
          pn.r_psi2[kr] = po.r_psi2[kr] - dt * drr * (double)(phi * Wz);
        }
      }
      oRhoL = rhoE / (double)J;
      if (rhoE != rho) s_rho[kA(i, j)] = rhoE;  // E2 and F start from it (B is done with rho^n)
      oIL = IL;
      os0 = srr;
      os1 = szz;
      os2 = srz;
#pragma unroll
      for (int m = 0; m < NM; m++) of[m] = fLv[m];
      // donor outflow limiter: volume leaving through the four faces vs V^L = V J
      {
        T dW = dv_r(i, j), dE = dv_r(i + 1, j), dS = dv_z(i, j), dN = dv_z(i, j + 1);
        T O = (tmax(-dW, T(0)) + tmax(dE, T(0))) + (tmax(-dS, T(0)) + tmax(dN, T(0)));
        T VL = volT(i, j) * J;
        oLam = O > VL ? N::div(tmax(VL, T(0)), O) : T(1);
      }
    }
    int kc = kC(i, j);
    if constexpr (DM) {
      cd[kDo * R::NC + kc] = oDL;
      cd[(kDo + 1) * R::NC + kc] = oVib;
    }
    if constexpr (PM) {
#pragma unroll
      for (int m = 0; m < NM; m++) {
        cd[m * R::NC + kc] = oMuL[m];
        cd[(NM + m) * R::NC + kc] = oILm[m];
      }
    } else {
      cd[0 * R::NC + kc] = oRhoL;
      cd[1 * R::NC + kc] = oIL;
    }
#pragma unroll
    for (int m = 0; m < NM; m++) cd[(kFo + m) * R::NC + kc] = of[m];
    ct[0 * R::NC + kc] = oLam;
    ct[1 * R::NC + kc] = os0;
    ct[2 * R::NC + kc] = os1;
    ct[3 * R::NC + kc] = os2;
  }
  __syncthreads();

  // ------------------------------------------------------- face mass fluxes
  // mass flux of a face (0 where there is no face): e = dV lambda of the
  // donor d; the flux is e rho^L(d), or with the per-material closure the
  // sum of every material's e mu_m^L(d) (E2 recomputes the same terms per
  // material). Each E2 position forms the fluxes of its four faces and leaves
  // those F needs in LDS: its west and south faces, the east faces of the
  // last column and the north faces of the last row.
  auto face_flux = [&](T dV, int d) -> double {
    if (!(dV > T(0) || dV < T(0))) return 0.0;
    const double e = (double)dV * (double)ct[0 * R::NC + d];
    if constexpr (PM) {
      double F = 0.0;
#pragma unroll
      for (int m = 0; m < NM; m++)
        if (m < g.nmat) F += e * cd[m * R::NC + d];
      return F;
    } else {
      return e * cd[0 * R::NC + d];
    }
  };

  // ------------------------------------------------------------------ E2
  // (the new density, energy and volume fractions of owned cells reach G,
  // which uses the same cell-to-thread map, through memory: this workgroup
  // wrote them, and holding them in registers across F costs spills)
  unsigned flags = 0;
  constexpr int UE = (R::NE + NT - 1) / NT;
#pragma unroll 1
  for (int u = 0; u < UE; u++) {
    int k = tid + u * NT;
    if (k >= R::NE) continue;
    int i, j;
    e_cell(k, i, j);
    double rho1 = 0.0;
    const T dV[4] = {dv_r(i, j), dv_r(i + 1, j), dv_z(i, j), dv_z(i, j + 1)};
    const int dk[4] = {kC(i - 1, j), kC(i + 1, j), kC(i, j - 1), kC(i, j + 1)};
    const bool inq[4] = {dV[0] > T(0), dV[1] < T(0), dV[2] > T(0), dV[3] < T(0)};
    const int kc = kC(i, j);
    const bool face[4] = {i >= 0 && i <= g.NR && j >= 0 && j < g.NZ, i + 1 >= 0 && i + 1 <= g.NR && j >= 0 && j < g.NZ,
                          i >= 0 && i < g.NR && j >= 0 && j <= g.NZ, i >= 0 && i < g.NR && j + 1 >= 0 && j + 1 <= g.NZ};
    double F[4];
#pragma unroll
    for (int q = 0; q < 4; q++) F[q] = face[q] ? face_flux(dV[q], inq[q] ? dk[q] : kc) : 0.0;
    s_Fr[kR(i, j)] = F[0];
    s_Fz[kZ(i, j)] = F[2];
    if (i == i0 + TW) s_Fr[kR(i + 1, j)] = F[1];
    if (j == j0 + TH) s_Fz[kZ(i, j + 1)] = F[3];
    if (in_cells(g, i, j)) {
      // the cell's damping rates (LDS, or memory ahead of the flux sums)
      const double dbl = DL ? s_dcz[j - (j0 - 2)] : (g.pml_on ? pm.dcz : S.rho)[g.pml_on ? j : 0];
      const double drl = DL ? s_dcr[i - (i0 - 2)] : (g.pml_on ? pm.dcr : S.rho)[g.pml_on ? i : 0];
      bool own = owns_cell(i, j);
      double V = volD(i, j);
      double netin = (F[0] - F[1]) + (F[2] - F[3]);
      const Over<T> byV(V);
      rho1 = s_rho[kA(i, j)] + byV(netin);
      double M1 = rho1 * V;
      double fL[NM];
#pragma unroll
      for (int m = 0; m < NM; m++) fL[m] = cd[(kFo + m) * R::NC + kc];
      // per-material closure: every material's face mass fluxes (the terms face_flux
      // summed), its new partial density, and rho as their sum
      double Fm[PM ? NM : 1][4], mu1[PM ? NM : 1];
      if constexpr (PM) {
        rho1 = 0.0;
#pragma unroll
        for (int m = 0; m < NM; m++) {
          mu1[m] = 0.0;
#pragma unroll
          for (int q = 0; q < 4; q++) Fm[m][q] = 0.0;
          if (m >= g.nmat) continue;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            const int d = inq[q] ? dk[q] : kc;
            if (dV[q] > T(0) || dV[q] < T(0))
              Fm[m][q] = ((double)dV[q] * (double)ct[0 * R::NC + d]) * cd[m * R::NC + d];
          }
          const double nin = (Fm[m][0] - Fm[m][1]) + (Fm[m][2] - Fm[m][3]);
          double mu0 = S.mu[m][cidx(g, i, j)];
          if (g.pml_place) {  // the printed placement's phi1 in the Lagrangian step
            const double rn = S.rho[cidx(g, i, j)], rE = s_rho[kA(i, j)];
            if (rE != rn) mu0 = mu0 * (rn > 0.0 ? rE / rn : 0.0);
          }
          mu1[m] = mu0 + byV(nin);
          rho1 += mu1[m];
        }
        M1 = rho1 * V;
      }
      double IL = PM ? 0.0 : cd[1 * R::NC + kc];
      double sL0 = (double)ct[1 * R::NC + kc], sL1 = (double)ct[2 * R::NC + kc], sL2 = (double)ct[3 * R::NC + kc];
      // per-face inflow terms (zero on outflow faces), each sum pairing the
      // r faces and the z faces
      double ed[4];
      FaceAcc am, aI, as0, as1, as2, acut, af[NM];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // e = dV * lambda of the donor (the own cell on outflow faces)
        int d = inq[q] ? dk[q] : kc;
        double tm = 0.0, tI = 0.0, ts0 = 0.0, ts1 = 0.0, ts2 = 0.0, tcut = 0.0, tf[NM];
#pragma unroll
        for (int m = 0; m < NM; m++) tf[m] = 0.0;
        if (inq[q]) {
          double adV = fabs((double)dV[q] * (double)ct[0 * R::NC + d]);
          double aF = fabs(F[q]);
          tcut = fabs((double)dV[q]) - adV;
          double Id = PM ? 0.0 : cd[1 * R::NC + d];
          tm = aF;
          tI = aF * (Id - IL);
          ts0 = aF * ((double)ct[1 * R::NC + d] - sL0);
          ts1 = aF * ((double)ct[2 * R::NC + d] - sL1);
          ts2 = aF * ((double)ct[3 * R::NC + d] - sL2);
#pragma unroll
          for (int m = 0; m < NM; m++)
            if (m == 0 || m < g.nmat) tf[m] = adV * (cd[(kFo + m) * R::NC + d] - fL[m]);
          ed[q] = F[q] * Id;
        } else {
          ed[q] = F[q] * IL;
        }
        am.put(q, tm);
        aI.put(q, tI);
        as0.put(q, ts0);
        as1.put(q, ts1);
        as2.put(q, ts2);
        acut.put(q, tcut);
#pragma unroll
        for (int m = 0; m < NM; m++) af[m].put(q, tf[m]);
      }
      const double min_ = am.sum(), nI = aI.sum(), vcut = acut.sum();
      const double nsrr = as0.sum(), nszz = as1.sum(), nsrz = as2.sum();
      double nf[NM];
#pragma unroll
      for (int m = 0; m < NM; m++) nf[m] = af[m].sum();
      double lam = (double)ct[0 * R::NC + kc];
      double O = (double)((tmax(-dV[0], T(0)) + tmax(dV[1], T(0))) + (tmax(-dV[2], T(0)) + tmax(dV[3], T(0))));
      double den = dmax(dmax(M1, min_), kMRemapFloor * g.rho_ref * V);
      const Over<T> byDen(den);
      double I1 = IL + byDen(nI);
      // damage and vibration speed travel with the mass (donor values, the
      // faces paired as above)
      double Dn = 0.0, Vn = 0.0;
      if constexpr (DM) {
        const double DLc = cd[kDo * R::NC + kc], VLc = cd[(kDo + 1) * R::NC + kc];
        FaceAcc aD, aV;
#pragma unroll
        for (int q = 0; q < 4; q++) {
          double tD = 0.0, tV = 0.0;
          if (inq[q]) {
            const double aF = fabs(F[q]);
            tD = aF * (cd[kDo * R::NC + dk[q]] - DLc);
            tV = aF * (cd[(kDo + 1) * R::NC + dk[q]] - VLc);
          }
          aD.put(q, tD);
          aV.put(q, tV);
        }
        Dn = DLc + byDen(aD.sum());
        Vn = VLc + byDen(aV.sum());
      }
      // per-material closure: every material's specific energy remapped with
      // its own mass fluxes (donor values); the energy fluxes are the sums
      // over materials
      double I1m[PM ? NM : 1];
      if constexpr (PM) {
#pragma unroll
        for (int q = 0; q < 4; q++) ed[q] = 0.0;
#pragma unroll
        for (int m = 0; m < NM; m++) {
          I1m[m] = 0.0;
          if (m >= g.nmat) continue;
          const double ILc = cd[(NM + m) * R::NC + kc];
          FaceAcc amm, aIm;
#pragma unroll
          for (int q = 0; q < 4; q++) {
            double tmm = 0.0, tIm = 0.0;
            if (inq[q]) {
              const double Id = cd[(NM + m) * R::NC + dk[q]];
              const double aF = fabs(Fm[m][q]);
              tmm = aF;
              tIm = aF * (Id - ILc);
              ed[q] += Fm[m][q] * Id;
            } else {
              ed[q] += Fm[m][q] * ILc;
            }
            amm.put(q, tmm);
            aIm.put(q, tIm);
          }
          const double minm = amm.sum(), nIm = aIm.sum();
          const double denm = dmax(dmax(mu1[m] * V, minm), kMRemapFloor * g.rho_ref * V);
          I1m[m] = ILc + nIm / denm;
        }
      }
      double ex = (1.0 - lam) * O - vcut;
      double f1v[NM];
#pragma unroll
      for (int m = 0; m < NM; m++) f1v[m] = (m == 0 || m < g.nmat) ? dmax(fL[m] + byV(nf[m] + fL[m] * ex), 0.0) : 0.0;
      double fs = f1v[0];
#pragma unroll
      for (int m = 1; m < NM; m++)
        if (m < g.nmat) fs = fs + f1v[m];
      double sdamp = 0.0;  // the layer's rate, when it also relaxes the stress
      if (g.pml_on) {
        double db = dbl, drr = drl;
        if (db > 0.0 || drr > 0.0) {
          long long kb = j < g.pml_b ? pml_bc(g, i, j) : -1;
          long long kr = i >= g.n_r ? pml_rc(g, i, j) : -1;
          long long ku = pml_cell_union(g, i, j);
          double dsum = db + drr;
          if (g.damp_stress) sdamp = dsum;
          double p1b = kb >= 0 ? po.b_phi1[kb] : 0.0, p1r = kr >= 0 ? po.r_phi1[kr] : 0.0;
          double p3b = kb >= 0 ? po.b_phi3[kb] : 0.0, p3r = kr >= 0 ? po.r_phi3[kr] : 0.0;
          // the auxiliaries this step applies: phi1 and phi3, or only psi2
          // (on the energy) as printed
          double a1 = p1b + p1r, a3 = p3b + p3r;
          if (g.pml_place) {
            a1 = 0.0;
            a3 = (kb >= 0 ? po.b_psi2[kb] : 0.0) + (kr >= 0 ? po.r_psi2[kr] : 0.0);
          }
          double rho2 = dmax(rho1 - dt * (dsum * (rho1 - pm.rref[ku]) + a1), 0.0);
          double rt = dmax(rho1, g.rho_ref * kPmlRhoFloor);
          double I2 = I1 - dt * (dsum * I1 + a3 / rt);
          if constexpr (PM) {
            // every material loses the same fraction of its mass and the same
            // specific energy
            const double kap = rho1 > 0.0 ? rho2 / rho1 : 0.0;
            double r2 = 0.0;
#pragma unroll
            for (int m = 0; m < NM; m++) {
              if (m >= g.nmat) continue;
              mu1[m] = mu1[m] * kap;
              r2 += mu1[m];
              I1m[m] = I1m[m] - dt * (dsum * I1m[m] + a3 / rt);
            }
            rho2 = r2;
          }
          if (own) {
            double sink = pm.msink[ku];
            // the printed placement's phi1 left the cell in the Lagrangian step
            if (g.pml_place) sink = sink + V * (S.rho[cidx(g, i, j)] - s_rho[kA(i, j)]);
            pm.msink[ku] = sink + V * (rho1 - rho2);
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
        double fv[NM];
        // fractions summing above 1 are scaled back (x / 1 = x below that)
        const Over<T> byFs(dmax(fs, 1.0));
#pragma unroll
        for (int m = 0; m < NM; m++) {
          fv[m] = fs > 1.0 ? byFs(f1v[m]) : f1v[m];
          if (m == 0 || m < g.nmat) D.f[m][c] = fv[m];
        }
        T s0n = (T)(sL0 + byDen(nsrr)), s1n = (T)(sL1 + byDen(nszz)), s2n = (T)(sL2 + byDen(nsrz));
        if (sdamp > 0.0) {  // extension: relax toward the initial (zero) deviator
          const double a0 = (double)s0n, a1 = (double)s1n, a2 = (double)s2n;
          s0n = (T)(a0 - dt * (sdamp * a0));
          s1n = (T)(a1 - dt * (sdamp * a1));
          s2n = (T)(a2 - dt * (sdamp * a2));
        }
        if (g.any_strength) {
          ((T*)D.s[0])[c] = s0n;
          ((T*)D.s[1])[c] = s1n;
          ((T*)D.s[2])[c] = s2n;
        }
        if (j == g.NZ - 1) {
          in.mout[i] += F[3];
          in.eout[i] += ed[3];
        }
        double chk = rho1;
        if constexpr (!PM) {
          D.I[c] = I1;  // before the remap heat, which G adds
          chk += I1;
        } else {
          // G adds the remap heat and forms I
#pragma unroll
          for (int m = 0; m < NM; m++) {
            if (m >= g.nmat) continue;
            D.mu[m][c] = mu1[m];
            D.Im[m][c] = I1m[m];
            chk += mu1[m] + I1m[m];
          }
        }
        if (g.any_strength) chk += (double)s0n + (double)s1n + (double)s2n;
#pragma unroll
        for (int m = 0; m < NM; m++)
          if (m == 0 || m < g.nmat) chk += fv[m];
        if constexpr (DM) {
          // G excites the vibration speed and reads both back
          D.dmg[c] = Dn;
          D.vib[c] = Vn;
          chk += Dn + Vn;
        }
        if (!((chk - chk) == 0.0)) flags |= kFlagNonFinite;
        if (rho1 < -kNegMassTol * g.rho_ref) flags |= kFlagNegMass;
      }
    }
    s_rho1[kE(i, j)] = rho1;
  }
  __syncthreads();

  // ------------------------------------------------------------------ F
  for (int k = tid; k < R::NF; k += NT) {
    int i = i0 + k % R::FW, j = j0 + k / R::FW;
    if (i > g.NR || j > g.NZ) continue;
    // the node's damping rates (LDS, or memory ahead of the flux sums)
    const double dbl = DL ? s_dnz[j - (j0 - 2)] : (g.pml_on ? pm.dnz : S.rho)[g.pml_on ? j : 0];
    const double drl = DL ? s_dnr[i - (i0 - 2)] : (g.pml_on ? pm.dnr : S.rho)[g.pml_on ? i : 0];
    // node mass: a quarter of the four cell masses (SW, SE, NW, NE)
    const int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
    double M[4] = {0, 0, 0, 0};
    bool qok[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      qok[q] = in_cells(g, qi[q], qj[q]);
      if (qok[q]) M[q] = s_rho[kA(qi[q], qj[q])] * volD(qi[q], qj[q]);
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
    const bool inq[4] = {FD[0] > 0.0, FD[1] < 0.0, FD[2] > 0.0, FD[3] < 0.0};
    double m1 = mL + ((FD[0] - FD[1]) + (FD[2] - FD[3]));
    int kb0 = kB(i, j);
    T vLr = s_vL[kb0], vLz = s_vL[R::NB + kb0];
    T upr[4], upz[4];
    FaceAcc am, ar_, az_, ak;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const bool ok = ni[q] >= 0 && ni[q] <= g.NR && nj[q] >= 0 && nj[q] <= g.NZ;
      double tm = 0.0, tr = 0.0, tz = 0.0, tk = 0.0;
      if (inq[q] && ok) {
        int d = kB(ni[q], nj[q]);
        double aF = fabs(FD[q]);
        T ur = s_vL[d], uz = s_vL[R::NB + d];
        tm = aF;
        tr = aF * (double)(ur - vLr);
        tz = aF * (double)(uz - vLz);
        // the kinetic energy the donor flux carries in, relative to v^L
        T dr_ = ur - vLr, dz_ = uz - vLz;
        tk = aF * (double)(dr_ * dr_ + dz_ * dz_);
        upr[q] = ur;
        upz[q] = uz;
      } else {
        upr[q] = vLr;
        upz[q] = vLz;
      }
      am.put(q, tm);
      ar_.put(q, tr);
      az_.put(q, tz);
      ak.put(q, tk);
    }
    const double min_ = am.sum(), nr = ar_.sum(), nz = az_.sum();
    double aE = i < g.NR ? colD(i).aw : 0.0;
    double aW = i > 0 ? colD(i - 1).ae : 0.0;
    double hN = j < g.NZ ? 0.5 * dzD(j) : 0.0;
    double hS = j > 0 ? 0.5 * dzD(j - 1) : 0.0;
    double Vd = (aE + aW) * (hN + hS);
    double den = dmax(dmax(m1, min_), kMRemapFloor * g.rho_ref * Vd);
    const Over<T> byDen(den);
    double v1r = (double)vLr + byDen(nr);
    double v1z = (double)vLz + byDen(nz);
    const double kin = ak.sum();
    double dKE = 0.5 * (kin - byDen(nr * nr + nz * nz));
    double Mq1[4];
#pragma unroll
    for (int q = 0; q < 4; q++) Mq1[q] = qok[q] ? s_rho1[kE(qi[q], qj[q])] * volD(qi[q], qj[q]) : 0.0;
    const double Mn = face_sum(Mq1);
    double h = Mn > kMRemapFloor * g.rho_ref * Vd ? dmax(dKE, 0.0) / Mn : 0.0;
    bool own = owns_node(i, j);
    if (g.pml_on) {
      double db = dbl, drr = drl;
      if (db > 0.0 || drr > 0.0) {
        long long kb = j < g.pml_b ? pml_bn(g, i, j) : -1;
        long long kr = i > g.n_r ? pml_rn(g, i, j) : -1;
        double dsum = db + drr;
        double mt = dmax(m1, kMAccEps * g.rho_ref * Vd);
        double bpr = kb >= 0 ? po.b_phi2r[kb] : 0.0, bpz = kb >= 0 ? po.b_phi2z[kb] : 0.0;
        double rpr = kr >= 0 ? po.r_phi2r[kr] : 0.0, rpz = kr >= 0 ? po.r_phi2z[kr] : 0.0;
        // the auxiliary this step applies: phi2, or psi1 as printed
        double pr = bpr + rpr, pz = bpz + rpz;
        if (g.pml_place) {
          pr = (kb >= 0 ? po.b_psi1r[kb] : 0.0) + (kr >= 0 ? po.r_psi1r[kr] : 0.0);
          pz = (kb >= 0 ? po.b_psi1z[kb] : 0.0) + (kr >= 0 ? po.r_psi1z[kr] : 0.0);
        }
        double v2r = v1r - dt * (dsum * v1r + (pr * Vd) / mt);
        double v2z = v1z - dt * (dsum * v1z + (pz * Vd) / mt);
        if (own) {
          if (db > 0.0) {
            pn.b_phi2r[kb] = bpr + db * ((FD[1] * (double)upr[1] - FD[0] * (double)upr[0]) / Vd);
            pn.b_phi2z[kb] = bpz + db * ((FD[1] * (double)upz[1] - FD[0] * (double)upz[0]) / Vd);
          }
          if (drr > 0.0) {
            pn.r_phi2r[kr] = rpr + drr * ((FD[3] * (double)upr[3] - FD[2] * (double)upr[2]) / Vd);
            pn.r_phi2z[kr] = rpz + drr * ((FD[3] * (double)upz[3] - FD[2] * (double)upz[2]) / Vd);
          }
        }
        v1r = v2r;
        v1z = v2z;
      }
    }
    T vr = (T)v1r, vz = (T)v1z;
    if (i == 0 || i == g.NR) vr = T(0);
    if (j == 0) {
      vr = T(0);
      vz = T(0);
    }
    if (g.top_closed && j == g.NZ) vz = T(0);
    if (own) {
      long long n = nidx(g, i, j);
      ((T*)D.v[0])[n] = vr;
      ((T*)D.v[1])[n] = vz;
    }
    heat[k] = h;
    speed[k] = N::sqr(vr * vr + vz * vz);
    // a non-finite velocity makes the speed non-finite and is caught in G
  }
  __syncthreads();

  // ------------------------------------------------------------------ G
  double cand = __builtin_huge_val();
#pragma unroll
  for (int u = 0; u < UE; u++) {
    int k = tid + u * NT;
    if (k >= TH * R::EW) continue;
    int i, j;
    e_cell(k, i, j);
    if (!owns_cell(i, j)) continue;
    long long c = cidx(g, i, j);
    // the cell's loads first, ahead of its stores (which the compiler may not
    // move them past) and with no branch among them (as in A)
    double f[kMaxMat];
#pragma unroll
    for (int m = 0; m < kMaxMat; m++) {
      if (m < NM) {
        const double x = D.f[m < g.nmat ? m : 0][c];
        f[m] = m < g.nmat ? x : 0.0;
      } else {
        f[m] = 0.0;
      }
    }
    const double rhoG = D.rho[c];
    double Ig = 0.0;
    if constexpr (!PM) Ig = D.I[c];
    const int nf[4] = {kF(i, j), kF(i + 1, j), kF(i, j + 1), kF(i + 1, j + 1)};
    double h = (heat[nf[0]] + heat[nf[1]]) + (heat[nf[2]] + heat[nf[3]]);
    double I1;
    // per-material closure: each material takes the heat; I is the
    // mass-weighted energy of the partial densities, rho their sum
    double mu[kMaxMat], Imv[kMaxMat];
    if constexpr (PM) {
      double r = 0.0, e = 0.0;
#pragma unroll
      for (int m = 0; m < kMaxMat; m++) {
        mu[m] = Imv[m] = 0.0;
        if (m >= NM || m >= g.nmat) continue;
        mu[m] = D.mu[m][c];
        Imv[m] = D.Im[m][c] + h;
        D.Im[m][c] = Imv[m];
        r += mu[m];
      }
#pragma unroll
      for (int m = 0; m < kMaxMat; m++)
        if (m < NM && m < g.nmat) e += mu[m] * Imv[m];
      I1 = r > 0.0 ? e / r : 0.0;
    } else {
      I1 = Ig + h;
    }
    D.I[c] = I1;
    if (!((I1 - I1) == 0.0)) flags |= kFlagNonFinite;
    T u4 = T(0);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      T sp = speed[nf[q]];
      if (!((sp - sp) == T(0))) flags |= kFlagNonFinite;
      u4 = tmax(u4, sp);
    }
    // block model: the vibration speed decays as exp(-dt / T_vib) over the
    // step and is excited to c_vib times the largest corner speed of the new
    // velocities (volume-fraction weighted constants of the damaging
    // materials); the new state's yield sees it and the new damage
    double Dg = 0.0, Vg = 0.0;
    if constexpr (DM) {
      Dg = D.dmg[c];
      double phin = 0.0;
#pragma unroll
      for (int m = 0; m < kMaxMat; m++)
        if (m < NM && m < g.nmat) phin += f[m];
      const double dn = phin > kPhiEps ? phin : kPhiEps;
      double kdec = 0.0, cv = 0.0;
#pragma unroll
      for (int m = 0; m < kMaxMat; m++) {
        if (!(m < NM && m < g.nmat) || !g.m[m].damage) continue;
        const double w = f[m] / dn;
        kdec += w * (g.m[m].Tvib > 0.0 ? exp_cw(-dt / g.m[m].Tvib) : 0.0);
        cv += w * g.m[m].c_vib;
      }
      Vg = dmax(D.vib[c] * kdec, cv * (double)u4);
      D.vib[c] = Vg;
      if (!((Vg - Vg) == 0.0)) flags |= kFlagNonFinite;
    }
    Mix<T> mx;
    if constexpr (PM) {
      T pmv[kMaxMat];
      mx = mixture_pm<T, DM>(g, rhoG, f, mu, Imv, pmv, Dg, Vg);
#pragma unroll
      for (int m = 0; m < NM; m++)
        if (m < g.nmat) ((T*)D.pmat[m])[c] = pmv[m];
    } else {
      mx = mixture<T, DM>(g, rhoG, I1, f, Dg, Vg);
    }
    store_eos(D, c, mx);
    cand = dmin(cand, cell_dt(g, mx, u4, dmin(colD(i).dr, dzD(j))));
  }
  if (flags) atomicOr(&sc->flags, flags);
  double m = block_min<NT>(cand, s_min);
  if (tid == 0) in.dtpart[tile] = m;
}

template <int TW, int TH, int NT, int WPE, class T, bool GEO, int NM, bool PM, bool DM = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_cycle(const Inst* __restrict__ insts, const TileRef* __restrict__ sched,
                                              int nsched) {
  using R = Regions<TW, TH>;
  using SM = Smem<TW, TH, T, NM, PM, DM>;
  __shared__ double s_rho[R::NA];     // rho^n over A (0 outside the grid)
  __shared__ double s_bigd[SM::kBigD];  // A..B stress; C..E2 Lagrangian state; F..G heat, speed
  __shared__ T s_vL[2 * R::NB];       // v^L over B
  __shared__ double s_F[R::NRF + R::NZF];  // B..C: node KE defect; E2..F: face mass fluxes
  __shared__ double s_rho1[R::NE];    // rho^{n+1} over E (0 outside the grid)
  __shared__ double s_min[NT / 64];
  __shared__ double s_geo[GEO ? GeoLds<TW, TH>::N : 1];  // a stretched tile's geometry
  // the tile's damping profiles (where they fit)
  constexpr bool kDampLds = SM::kRest + 8 * (NT / 64 + (GEO ? GeoLds<TW, TH>::N : 1) + SM::kDamp) <= 163840 - 64;
  __shared__ double s_damp[kDampLds ? SM::kDamp : 1];
  // Descriptors and schedule are read-only for the whole launch: reading them
  // through the constant address space lets the compiler keep or re-issue
  // those scalar loads freely across the workgroup barriers below.
  using CInst = const __attribute__((address_space(4))) Inst;
  using CTile = const __attribute__((address_space(4))) TileRef;
  CInst* cinst = (CInst*)insts;
  CTile* csched = (CTile*)sched;
  for (int e = blockIdx.x; e < nsched; e += gridDim.x) {
    const TileRef tr{csched[e].inst, csched[e].tile};
    if (tr.inst < 0) continue;
    const Inst* in = (const Inst*)(cinst + tr.inst);
    tile_cycle<TW, TH, NT, WPE, T, GEO, NM, PM, DM, kDampLds>(*in, tr.tile, s_rho, s_bigd, s_vL, s_F, s_F + R::NRF, s_rho1, s_min,
                                            s_geo, s_damp);
    __syncthreads();  // LDS is reused by the next entry
  }
}

// EoS cache and Courant candidates of the current state of one instance (the
// first step of a run, after the state was set).
template <class T>
__global__ void k_prime(Inst in) {
  const Geo& g = in.g;
  Scal* sc = in.sc;
  const int par = (int)(sc->cycle & 1);
  const State& S = in.S[par];
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double cand = __builtin_huge_val();
  if (t < (long long)g.NR * g.NZ) {
    int j = (int)(t / g.NR), i = (int)(t - (long long)j * g.NR);
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
      mx = g.dmg ? mixture_pm<T, true>(g, S.rho[c], f, mu, Im, pmv, S.dmg[c], S.vib[c])
                 : mixture_pm<T>(g, S.rho[c], f, mu, Im, pmv);
      for (int m = 0; m < g.nmat; m++) ((T*)S.pmat[m])[c] = pmv[m];
    } else {
      mx = g.dmg ? mixture<T, true>(g, S.rho[c], S.I[c], f, S.dmg[c], S.vib[c]) : mixture<T>(g, S.rho[c], S.I[c], f);
    }
    store_eos(S, c, mx);
    const long long nd[4] = {nidx(g, i, j), nidx(g, i + 1, j), nidx(g, i, j + 1), nidx(g, i + 1, j + 1)};
    T u4 = T(0);
    for (int q = 0; q < 4; q++) {
      T a = ((const T*)S.v[0])[nd[q]], b = ((const T*)S.v[1])[nd[q]];
      u4 = tmax(u4, Num<T>::sqr(a * a + b * b));
    }
    cand = cell_dt(g, mx, u4, dmin(col_of<double>(g, in.geo, i).dr, dz_of(g, in.geo, j)));
  }
  for (int off = 32; off > 0; off >>= 1) cand = dmin(cand, __shfl_down(cand, off, 64));
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = cand;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = dmin(dmin(part[0], part[1]), dmin(part[2], part[3]));
    atomicMin(&sc->dtmin, (unsigned long long)__double_as_longlong(m));
  }
}

// Instantiates the cycle kernel of every tile shape and the priming kernel
// for one bulk type (one translation unit per type keeps builds parallel).
#define SALEC_CYCLE_TABLE(T, suffix)                                                         \
  static CycleFn cycle_uni2_##suffix(int v) {                                                \
    switch (v) {                                                                             \
      case 0: return k_cycle<64, 14, 768, 3, T, false, 2, false>;                            \
      case 1: return k_cycle<40, 16, 512, 4, T, false, 2, false>;                            \
      case 2: return k_cycle<32, 20, 512, 4, T, false, 2, false>;                            \
      case 3: return k_cycle<64, 15, 768, 3, T, false, 2, false>;                            \
      case 4: return k_cycle<64, 16, 768, 3, T, false, 2, false>;                            \
      case 5: return k_cycle<48, 20, 768, 3, T, false, 2, false>;                            \
      case 6: return k_cycle<40, 24, 768, 3, T, false, 2, false>;                            \
      case 7: return k_cycle<28, 18, 512, 4, T, false, 2, false>;                            \
      case 8: return k_cycle<64, 16, 1024, 4, T, false, 2, false>;                           \
      case 9: return k_cycle<32, 32, 1024, 4, T, false, 2, false>;                           \
      case 10: return k_cycle<20, 13, 256, 3, T, false, 2, false>;                           \
      case 12: return k_cycle<35, 31, 768, 3, T, false, 2, false>;                           \
      case 13: return k_cycle<32, 34, 768, 3, T, false, 2, false>;                           \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_uni3_##suffix(int v) {                                                \
    switch (v) {                                                                             \
      case 0: return k_cycle<64, 14, 768, 3, T, false, 3, false>;                            \
      case 1: return k_cycle<40, 16, 512, 4, T, false, 3, false>;                            \
      case 2: return k_cycle<32, 20, 512, 4, T, false, 3, false>;                            \
      case 3: return k_cycle<64, 15, 768, 3, T, false, 3, false>;                            \
      case 5: return k_cycle<48, 20, 768, 3, T, false, 3, false>;                            \
      case 6: return k_cycle<40, 24, 768, 3, T, false, 3, false>;                            \
      case 7: return k_cycle<28, 18, 512, 4, T, false, 3, false>;                            \
      case 9: return k_cycle<32, 32, 1024, 4, T, false, 3, false>;                           \
      case 10: return k_cycle<20, 13, 256, 3, T, false, 3, false>;                           \
      case 11: return k_cycle<48, 14, 768, 3, T, false, 3, false>;                           \
      case 12: return k_cycle<35, 31, 768, 3, T, false, 3, false>;                           \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_uni2pm_##suffix(int v) {                                              \
    switch (v) {                                                                             \
      case 0: return k_cycle<64, 14, 768, 3, T, false, 2, true>;                             \
      case 1: return k_cycle<40, 16, 512, 4, T, false, 2, true>;                             \
      case 7: return k_cycle<28, 18, 512, 4, T, false, 2, true>;                             \
      case 10: return k_cycle<20, 13, 256, 3, T, false, 2, true>;                            \
      case 11: return k_cycle<48, 14, 768, 3, T, false, 2, true>;                            \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_uni3pm_##suffix(int v) {                                              \
    switch (v) {                                                                             \
      case 1: return k_cycle<40, 16, 512, 4, T, false, 3, true>;                             \
      case 7: return k_cycle<28, 18, 512, 4, T, false, 3, true>;                             \
      case 10: return k_cycle<20, 13, 256, 3, T, false, 3, true>;                            \
      case 11: return k_cycle<48, 14, 768, 3, T, false, 3, true>;                            \
      case 14: return k_cycle<27, 27, 768, 3, T, false, 3, true>;                            \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_geo2_##suffix(int v) {                                                \
    switch (v) {                                                                             \
      case 0: return k_cycle<64, 14, 768, 3, T, true, 2, false>;                             \
      case 1: return k_cycle<40, 16, 512, 4, T, true, 2, false>;                             \
      case 2: return k_cycle<32, 20, 512, 4, T, true, 2, false>;                             \
      case 3: return k_cycle<64, 15, 768, 3, T, true, 2, false>;                             \
      case 4: return k_cycle<64, 16, 768, 3, T, true, 2, false>;                             \
      case 5: return k_cycle<48, 20, 768, 3, T, true, 2, false>;                             \
      case 6: return k_cycle<40, 24, 768, 3, T, true, 2, false>;                             \
      case 7: return k_cycle<28, 18, 512, 4, T, true, 2, false>;                             \
      case 8: return k_cycle<64, 16, 1024, 4, T, true, 2, false>;                            \
      case 9: return k_cycle<32, 32, 1024, 4, T, true, 2, false>;                            \
      case 10: return k_cycle<20, 13, 256, 3, T, true, 2, false>;                            \
      case 12: return k_cycle<35, 31, 768, 3, T, true, 2, false>;                            \
      case 13: return k_cycle<32, 34, 768, 3, T, true, 2, false>;                            \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_geo3_##suffix(int v) {                                                \
    switch (v) {                                                                             \
      case 0: return k_cycle<64, 14, 768, 3, T, true, 3, false>;                             \
      case 1: return k_cycle<40, 16, 512, 4, T, true, 3, false>;                             \
      case 2: return k_cycle<32, 20, 512, 4, T, true, 3, false>;                             \
      case 3: return k_cycle<64, 15, 768, 3, T, true, 3, false>;                             \
      case 5: return k_cycle<48, 20, 768, 3, T, true, 3, false>;                             \
      case 6: return k_cycle<40, 24, 768, 3, T, true, 3, false>;                             \
      case 7: return k_cycle<28, 18, 512, 4, T, true, 3, false>;                             \
      case 9: return k_cycle<32, 32, 1024, 4, T, true, 3, false>;                            \
      case 10: return k_cycle<20, 13, 256, 3, T, true, 3, false>;                            \
      case 11: return k_cycle<48, 14, 768, 3, T, true, 3, false>;                            \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_geo2pm_##suffix(int v) {                                              \
    switch (v) {                                                                             \
      case 0: return k_cycle<64, 14, 768, 3, T, true, 2, true>;                              \
      case 1: return k_cycle<40, 16, 512, 4, T, true, 2, true>;                              \
      case 7: return k_cycle<28, 18, 512, 4, T, true, 2, true>;                              \
      case 10: return k_cycle<20, 13, 256, 3, T, true, 2, true>;                             \
      case 11: return k_cycle<48, 14, 768, 3, T, true, 2, true>;                             \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  static CycleFn cycle_geo3pm_##suffix(int v) {                                              \
    switch (v) {                                                                             \
      case 1: return k_cycle<40, 16, 512, 4, T, true, 3, true>;                              \
      case 7: return k_cycle<28, 18, 512, 4, T, true, 3, true>;                              \
      case 10: return k_cycle<20, 13, 256, 3, T, true, 3, true>;                             \
      case 11: return k_cycle<48, 14, 768, 3, T, true, 3, true>;                             \
      case 14: return k_cycle<27, 27, 768, 3, T, true, 3, true>;                             \
      default: return nullptr;                                                               \
    }                                                                                        \
  }                                                                                          \
  CycleFn cycle_kernel_##suffix(int v, bool geo, int nm, bool pm) {                          \
    if (pm) {                                                                                \
      if (nm <= 2) return geo ? cycle_geo2pm_##suffix(v) : cycle_uni2pm_##suffix(v);         \
      return geo ? cycle_geo3pm_##suffix(v) : cycle_uni3pm_##suffix(v);                      \
    }                                                                                        \
    if (nm <= 2) return geo ? cycle_geo2_##suffix(v) : cycle_uni2_##suffix(v);               \
    return geo ? cycle_geo3_##suffix(v) : cycle_uni3_##suffix(v);                            \
  }                                                                                          \
  hipError_t launch_prime_##suffix(const Inst& in, hipStream_t st) {                           \
    long long nc = (long long)in.g.NR * in.g.NZ;                                               \
    hipLaunchKernelGGL(k_prime<T>, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, in); \
    return hipGetLastError();                                                                  \
  }

// The damage family (damage and the block model of acoustic fluidization):
// the same cycle with two more FP64 records per cell in LDS, so only the
// shapes whose tiles still fit beside them (40 x 16 and 28 x 18 at 512
// threads, 20 x 13 at 256, 48 x 14 at 768) are built.
#define SALEC_CYCLE_DM_SHAPES(T, GEO, NM, PM)                 \
  switch (v) {                                                \
    case 1: return k_cycle<40, 16, 512, 4, T, GEO, NM, PM, true>;  \
    case 7: return k_cycle<28, 18, 512, 4, T, GEO, NM, PM, true>;  \
    case 10: return k_cycle<20, 13, 256, 3, T, GEO, NM, PM, true>; \
    case 11: return k_cycle<48, 14, 768, 3, T, GEO, NM, PM, true>; \
    default: return nullptr;                                  \
  }
#define SALEC_CYCLE_DM_TABLE(T, suffix)                                           \
  CycleFn cycle_kernel_dm_##suffix(int v, bool geo, int nm, bool pm) {            \
    if (geo) {                                                                    \
      if (pm) {                                                                   \
        if (nm <= 2) SALEC_CYCLE_DM_SHAPES(T, true, 2, true)                      \
        SALEC_CYCLE_DM_SHAPES(T, true, 3, true)                                   \
      }                                                                           \
      if (nm <= 2) SALEC_CYCLE_DM_SHAPES(T, true, 2, false)                       \
      SALEC_CYCLE_DM_SHAPES(T, true, 3, false)                                    \
    }                                                                             \
    if (pm) {                                                                     \
      if (nm <= 2) SALEC_CYCLE_DM_SHAPES(T, false, 2, true)                       \
      SALEC_CYCLE_DM_SHAPES(T, false, 3, true)                                    \
    }                                                                             \
    if (nm <= 2) SALEC_CYCLE_DM_SHAPES(T, false, 2, false)                        \
    SALEC_CYCLE_DM_SHAPES(T, false, 3, false)                                     \
  }

}  // namespace salec
