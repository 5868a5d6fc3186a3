/*
 * salec_oracle.c -- plain FP64 CPU oracle of one explicit cycle of a
 * SALE-type axisymmetric (r-z) impact hydrocode with perfectly matched layers.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. This is the slow, obviously
 * correct reference against which the HIP library is checked. It is written
 * for reading: whole-grid loops, one phase after another, in the order of the
 * SALE operator split (Lagrangian step, then Eulerian step), with full-size
 * temporary arrays and no blocking, fusion or reordering. It shares no code
 * with the HIP library. Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it.
 *
 * Built with -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 * OpenMP only splits independent per-cell / per-node loops over rows; the
 * arithmetic of every cell is independent of the thread count and the time
 * step minimum is exact, so results do not depend on the thread count.
 *
 * Paper: Li, Yue, Zhang, Zhang, Miao, "Parallel numerical simulation of
 * impact crater with perfect matched layers" (SALEc-2D).
 *   Sec. 2, eqs. (1)-(2): Lagrangian momentum and internal energy.
 *   Sec. 2, eqs. (3)-(5): Eulerian advection of mass, momentum, energy.
 *   Sec. 3: PML -- complex stretching, auxiliary variables phi1..3, psi1..2,
 *           damped control equations and the damping profile d(y).
 *   Sec. 4: boundary conditions (free-slip sides, outflow top, no-slip bottom).
 *   Table 1: pressure-dependent strength (cohesion, friction, limit).
 *   Sec. 7: Courant condition dt <= C0 min(dx, dy) / (|v| + c).
 * The paper defers the discretisation, equation of state, artificial
 * viscosity, strength update and remap to SALE; the discrete choices made
 * here are the documented readings of those silent points (staggered grid,
 * Tillotson EoS, compression-only linear+quadratic viscosity, Jaumann rate
 * with radial return, first-order donor-cell remap, volume-fraction
 * multi-material cells).
 */
#include "salec_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* regularisation constants (dimensionless; scaled by reference values) */
#define PHI_EPS 1e-12       /* volume fraction below which a cell is void     */
#define RHO_EOS_FLOOR 1e-6  /* EoS density floor, fraction of rho0            */
#define RHO_DEN_FLOOR 1e-6  /* energy-update density floor, fraction of rho_ref */
#define PML_RHO_FLOOR 1e-3  /* PML density floor, fraction of rho_ref        */
#define M_ACC_EPS 1e-3      /* node mass floor for accelerations             */
#define M_REMAP_FLOOR 1e-9  /* mass floor of remap denominators              */
#define W_LO 1e-3           /* volume fraction where the CFL weight starts   */
#define W_HI 1e-2           /* volume fraction where the CFL weight is 1     */
#define NEG_MASS_TOL 1e-9   /* density below -tol*rho_ref is an error        */
#define PCAV_FRAC 1e-4      /* pressure ramp of the cavitation rule, fraction of A */
#define F_PM_EPS 1e-6       /* closure 1: a material below this volume fraction
                               takes the cell's matter density in its EoS  */
#define VIB_ON 1e-3         /* block model: vibration speed (m/s) above which its
                               viscosity acts fully (linear ramp below)     */

struct orc_ctx {
    orc_grid g;
    orc_mat m[ORC_MAX_MAT];
    orc_pml pml;
    int NR, NZ, NC, NN, nmat, any_strength;
    int pm; /* closure 1: per-material density and specific energy */
    double rho_ref, Gm[ORC_MAX_MAT]; /* shear / bulk modulus ratio per material */
    /* damage and acoustic fluidization: some material accumulates damage; per
     * material the longitudinal speed at rest, the block model's kinematic
     * viscosity gamma_eta c h and vibration decay time gamma_T h / c */
    int dmg;
    double cL0[ORC_MAX_MAT], nub[ORC_MAX_MAT], Tvib[ORC_MAX_MAT];
    double *D, *vib, *D_n, *vib_n, *DL, *vibL, *etab;

    /* state at the start of the cycle */
    double *rho, *I, *f[ORC_MAX_MAT], *srr, *szz, *srz, *vr, *vz;
    double t, dt, dt_prev;
    int64_t cycle;
    int err, err_cycle;

    /* initial (lithostatic) pressure per cell row */
    double *p0;

    /* geometry tables: node and centre radii, column widths and the
     * r-weighted areas of each column's west and east halves; node and centre
     * heights and row heights */
    double *rn, *rcn, *drc, *awc, *aec, *azc, *zn, *zcn, *dzr;

    /* PML: damping profiles and auxiliary fields (zero outside the strips) */
    double *dcz, *dnz, *dcr, *dnr;
    double *phi1b, *phi3b, *psi2b, *phi1r, *phi3r, *psi2r, *rref, *msink;
    double *phi2b_r, *phi2b_z, *psi1b_r, *psi1b_z;
    double *phi2r_r, *phi2r_z, *psi1r_r, *psi1r_z;
    double *mout_col, *eout_col;
    /* placement 1: level-n sums of psi1 (node, r and z) and psi2 (cell) kept
     * for the Eulerian step, and the mass the Eulerian step starts from (rho
     * and, with closure 1, mu after phi1) */
    double *psi1n_r, *psi1n_z, *psi2n, *rho_t, *mu_t[ORC_MAX_MAT];
    double *rhoE, *muE[ORC_MAX_MAT];

    /* per-cycle work arrays */
    double *p, *c2, *G, *Y, *rmat, *phi, *sx, *Q, *sgrr, *sgzz, *sgtt, *sgrz;
    double *vLr, *vLz, *heat;
    double *J, *IL, *sLrr, *sLzz, *sLrz, *fL[ORC_MAX_MAT];
    double *dVr, *Fr, *dVz, *Fz, *dVre, *dVze, *lam, *outv;
    double *rho_n, *I_n, *f_n[ORC_MAX_MAT], *srr_n, *szz_n, *srz_n, *vr_n, *vz_n;

    /* closure 1: partial densities mu_m (mass of material m per cell volume)
     * and specific energies I_m (state), the material pressures and densities
     * the cycle's EoS used, Lagrangian energies, per-material face mass fluxes;
     * rho and I then hold sum(mu_m) and the mass-weighted energy */
    double *mu[ORC_MAX_MAT], *Im[ORC_MAX_MAT], *mu_n[ORC_MAX_MAT], *Im_n[ORC_MAX_MAT];
    double *pmm[ORC_MAX_MAT], *rhm[ORC_MAX_MAT], *ILm[ORC_MAX_MAT];
    double *Fmr[ORC_MAX_MAT], *Fmz[ORC_MAX_MAT];
};

#define CI(i, j) ((j) * NR + (i))
#define NI(i, j) ((j) * (NR + 1) + (i))
#define RF(i, j) ((j) * (NR + 1) + (i)) /* radial face at r_i, row j, i in [0,NR] */
#define AF(i, j) ((j) * NR + (i))       /* axial face at z_j, column i, j in [0,NZ] */

static double dmax(double a, double b) { return a > b ? a : b; }
static double dmin(double a, double b) { return a < b ? a : b; }

/* Sum of four per-face (or per-corner) terms ordered W, E, S, N (or SW, SE,
 * NW, NE): the r pair plus the z pair. The divergence of Sec. 2's equations is
 * an r part plus a z part; summing it that way also keeps the discrete scheme
 * exactly symmetric under a reflection in z (the pair (S, N) becomes (N, S)). */
static double face_sum(const double t[4]) { return (t[0] + t[1]) + (t[2] + t[3]); }

/* ---- geometry (per radian): radial face area, cell volume ---- */
static double area_r(const orc_ctx *x, int i, int j) { return x->rn[i] * x->dzr[j]; }
static double vol_c(const orc_ctx *x, int i, int j) { return x->azc[i] * x->dzr[j]; }

/* exp(x) by a fixed published method so that every implementation of this
 * algorithm rounds identically: Cody & Waite range reduction
 * x = k ln2 + r, |r| <= ln2/2, with ln2 split into a 32-bit head and a tail,
 * then the Taylor polynomial of e^r to degree 13 in Horner form (truncation
 * below 1e-17 relative), then scaling by 2^k. Results below e^-700 are
 * flushed to 0 and above e^709 overflow to +inf. */
static double exp_cw(double x)
{
    if (x != x) return x;
    if (x < -700.0) return 0.0;
    if (x > 709.0) return INFINITY;
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
    int k = (int)kd;
    uint64_t bits = (uint64_t)(k + 1023) << 52;
    double scale;
    memcpy(&scale, &bits, sizeof scale);
    return q * scale;
}

double orc_exp(double x) { return exp_cw(x); }

/* ========================================================================
 * Equation of state (the paper's EoS module is inherited from SALEc, Sec. 2;
 * the form used is the four-region Tillotson equation of state).
 * ======================================================================== */
void orc_tillotson(const orc_mat *m, double rho, double e, double *p_out, double *c2_out)
{
    double rf = m->rho0 * RHO_EOS_FLOOR;
    double r = rho > rf ? rho : rf;
    double E = e > 0.0 ? e : 0.0;
    double eta = r / m->rho0;
    double mu = eta - 1.0;
    double w = E / (m->E0 * eta * eta) + 1.0;

    /* compressed / cold branch */
    double pc = (m->a + m->b / w) * r * E + m->A * mu + m->B * mu * mu;
    double pc_E = r * (m->a + m->b / w - m->b * (w - 1.0) / (w * w));
    double pc_r = (m->a + m->b / w) * E + 2.0 * m->b * E * (w - 1.0) / (w * w)
                + (m->A + 2.0 * m->B * mu) / m->rho0;
    double p, dpdE, dpdr;
    if (r >= m->rho0 || E <= m->Eiv) {
        p = pc;
        dpdE = pc_E;
        dpdr = pc_r;
    } else {
        /* expanded branch */
        double z = 1.0 / eta - 1.0;
        double ea = exp_cw(-m->alpha * z * z);
        double eb = exp_cw(-m->beta * z);
        double pe = m->a * r * E + (m->b * r * E / w + m->A * mu * eb) * ea;
        double pe_E = m->a * r + ea * m->b * r * (1.0 / w - (w - 1.0) / (w * w));
        double pe_r = m->a * E
                    + ea * (m->b * E / w + 2.0 * m->b * E * (w - 1.0) / (w * w)
                            + (m->A / m->rho0) * eb + m->A * mu * m->beta * eb * m->rho0 / (r * r))
                    + (m->b * r * E / w + m->A * mu * eb) * ea * 2.0 * m->alpha * z * m->rho0 / (r * r);
        if (E >= m->Ecv) {
            p = pe;
            dpdE = pe_E;
            dpdr = pe_r;
        } else {
            /* partial vaporisation: energy-weighted blend */
            double x = (E - m->Eiv) / (m->Ecv - m->Eiv);
            p = x * pe + (1.0 - x) * pc;
            dpdE = x * pe_E + (1.0 - x) * pc_E + (pe - pc) / (m->Ecv - m->Eiv);
            dpdr = x * pe_r + (1.0 - x) * pc_r;
        }
    }
    *p_out = p;
    *c2_out = dpdr + p / (r * r) * dpdE;
}

/* intact-rock yield strength (Table 1 parameters Y_i0, mu_i, Y_im) */
double orc_yield(const orc_mat *m, double p)
{
    if (!m->strength) return 0.0;
    if (p >= 0.0) {
        double mp = m->mu_f * p;
        return m->Y0 + mp / (1.0 + mp / (m->Ylim - m->Y0));
    }
    return dmax(0.0, m->Y0 + m->mu_f * p);
}

double orc_shear_modulus(const orc_mat *m)
{
    if (!m->strength) return 0.0;
    return 3.0 * m->A * (1.0 - 2.0 * m->poisson) / (2.0 * (1.0 + m->poisson));
}

/* thermal softening of strength: full below the incipient-vaporisation
 * energy, none above complete vaporisation, linear in between */
double orc_softening(const orc_mat *m, double e)
{
    double E = e > 0.0 ? e : 0.0;
    return dmin(dmax((m->Ecv - E) / (m->Ecv - m->Eiv), 0.0), 1.0);
}

/* Damaged strength (Table 1's Y_d0, mu_d, Y_dm): Y_d = min(Y_d0 + mu_d q, Y_dm)
 * at the effective pressure q = max(p - p_vib, 0) of the block model for
 * p >= 0, max(0, Y_d0 + mu_d p) in tension, never above the intact curve;
 * the cell's strength blends the two by its damage D. */
double orc_yield_damaged(const orc_mat *m, double p, double D, double p_vib)
{
    double Yi = orc_yield(m, p);
    if (!m->strength || !m->damage) return Yi;
    double Yd;
    if (p >= 0.0)
        Yd = dmin(m->Yd0 + m->mu_d * dmax(p - p_vib, 0.0), m->Ydm);
    else
        Yd = dmax(0.0, m->Yd0 + m->mu_d * p);
    Yd = dmin(Yd, Yi);
    return (1.0 - D) * Yi + D * Yd;
}

/* plastic strain at failure of the damage law, eps_f = max(eps_fb, B (p - p_bd))
 * (brittle below the transition pressure p_bd, increasingly ductile above) */
double orc_failure_strain(const orc_mat *m, double p)
{
    return dmax(m->eps_fb, m->B_dmg * (p - m->p_bd));
}

/* mixture state of cell c: shared material density and energy, weights f_m/phi */
static void mixture(const orc_ctx *x, int c, const double *rho, const double *I,
                    double *const *f, double Dc, double vibc, double *p_o, double *c2_o, double *G_o,
                    double *Y_o, double *rmat_o, double *phi_o, double *sx_o)
{
    double phi = 0.0;
    for (int m = 0; m < x->nmat; m++) phi += f[m][c];
    double den = phi > PHI_EPS ? phi : PHI_EPS;
    double rm = rho[c] / den;
    double p = 0.0, c2 = 0.0, G = 0.0;
    double wm[ORC_MAX_MAT];
    for (int m = 0; m < x->nmat; m++) {
        double pm, c2m;
        wm[m] = f[m][c] / den;
        orc_tillotson(&x->m[m], rm, I[c], &pm, &c2m);
        pm = dmax(pm, x->m[m].p_min);
        c2m = dmax(c2m, x->m[m].c_floor_frac * x->m[m].A / x->m[m].rho0);
        p += wm[m] * pm;
        c2 += wm[m] * c2m;
        /* shear modulus from the local bulk modulus K = rho c^2 at a fixed
         * Poisson ratio (equals the reference value at rho0, E = 0) */
        G += wm[m] * (orc_softening(&x->m[m], I[c]) * (x->Gm[m] * (rm * c2m)));
    }
    double Y = 0.0, pmin = 0.0, ps = 0.0;
    for (int m = 0; m < x->nmat; m++) {
        /* the block model's vibration pressure rho c v_vib */
        double Ym = x->dmg ? orc_yield_damaged(&x->m[m], p, Dc, rm * x->cL0[m] * vibc) : orc_yield(&x->m[m], p);
        Y += wm[m] * (orc_softening(&x->m[m], I[c]) * Ym);
        pmin += wm[m] * x->m[m].p_min;
        ps += wm[m] * (PCAV_FRAC * x->m[m].A);
    }
    /* expansion weight of the material: 1 above its tension floor + ps */
    double d = p - pmin;
    *sx_o = d >= ps ? 1.0 : (ps > 0.0 ? dmax(d, 0.0) / ps : 0.0);
    *p_o = p;
    *c2_o = c2;
    *G_o = G;
    *Y_o = Y;
    *rmat_o = rm;
    *phi_o = phi;
}

/* Closure 1: the same volume-fraction average, each material at its own
 * density rho_m = mu_m / f_m and its own specific energy I_m (materials below
 * F_PM_EPS, or without mass, at the cell's matter density). Also returns the
 * material pressures (after the floor) and densities the energy update uses. */
static void mixture_pm(const orc_ctx *x, int c, const double *rho, double *const *f, double *const *mu,
                       double *const *Im, double Dc, double vibc, double *p_o, double *c2_o, double *G_o,
                       double *Y_o, double *rmat_o, double *phi_o, double *sx_o, double *pm_o, double *rhm_o)
{
    double phi = 0.0;
    for (int m = 0; m < x->nmat; m++) phi += f[m][c];
    double den = phi > PHI_EPS ? phi : PHI_EPS;
    double rm = rho[c] / den;
    double p = 0.0, c2 = 0.0, G = 0.0;
    double wm[ORC_MAX_MAT], sf[ORC_MAX_MAT], rmv[ORC_MAX_MAT];
    for (int m = 0; m < x->nmat; m++) {
        double fm = f[m][c], mm = mu[m][c];
        double rmm = fm > F_PM_EPS && mm > 0.0 ? mm / fm : rm;
        rmv[m] = rmm;
        double pm, c2m;
        wm[m] = fm / den;
        sf[m] = 0.0;
        if (pm_o) pm_o[m] = 0.0;
        if (rhm_o) rhm_o[m] = rmm;
        /* a material absent from the cell has no pressure and adds nothing */
        if (fm == 0.0) continue;
        orc_tillotson(&x->m[m], rmm, Im[m][c], &pm, &c2m);
        pm = dmax(pm, x->m[m].p_min);
        c2m = dmax(c2m, x->m[m].c_floor_frac * x->m[m].A / x->m[m].rho0);
        p += wm[m] * pm;
        c2 += wm[m] * c2m;
        sf[m] = orc_softening(&x->m[m], Im[m][c]);
        G += wm[m] * (sf[m] * (x->Gm[m] * (rmm * c2m)));
        if (pm_o) pm_o[m] = pm;
    }
    double Y = 0.0, pmin = 0.0, ps = 0.0;
    for (int m = 0; m < x->nmat; m++) {
        if (f[m][c] == 0.0) continue;
        double Ym = x->dmg ? orc_yield_damaged(&x->m[m], p, Dc, rmv[m] * x->cL0[m] * vibc) : orc_yield(&x->m[m], p);
        Y += wm[m] * (sf[m] * Ym);
        pmin += wm[m] * x->m[m].p_min;
        ps += wm[m] * (PCAV_FRAC * x->m[m].A);
    }
    double d = p - pmin;
    *sx_o = d >= ps ? 1.0 : (ps > 0.0 ? dmax(d, 0.0) / ps : 0.0);
    *p_o = p;
    *c2_o = c2;
    *G_o = G;
    *Y_o = Y;
    *rmat_o = rm;
    *phi_o = phi;
}

/* the cell's mixture under the context's closure (state at the cycle start) */
static void cell_mixture(const orc_ctx *x, int c, double *p_o, double *c2_o, double *G_o, double *Y_o,
                         double *rmat_o, double *phi_o, double *sx_o, double *pm_o, double *rhm_o)
{
    double Dc = x->dmg ? x->D[c] : 0.0, vc = x->dmg ? x->vib[c] : 0.0;
    if (x->pm)
        mixture_pm(x, c, x->rho, x->f, x->mu, x->Im, Dc, vc, p_o, c2_o, G_o, Y_o, rmat_o, phi_o, sx_o, pm_o, rhm_o);
    else
        mixture(x, c, x->rho, x->I, x->f, Dc, vc, p_o, c2_o, G_o, Y_o, rmat_o, phi_o, sx_o);
}

/* closure 1: rho = sum of the partial densities, I = their mass-weighted
 * specific energy (0 where there is no mass) */
static void derive_cell(const orc_ctx *x, double *const *mu, double *const *Im, double *rho, double *I, int c)
{
    double r = 0.0, e = 0.0;
    for (int m = 0; m < x->nmat; m++) r += mu[m][c];
    for (int m = 0; m < x->nmat; m++) e += mu[m][c] * Im[m][c];
    rho[c] = r;
    I[c] = r > 0.0 ? e / r : 0.0;
}

/* ========================================================================
 * Cell kinematics: face-mean velocities, flux-form divergence and the
 * strain-rate / spin components of cell (i, j) in r-z.
 * ======================================================================== */
typedef struct {
    double ur_w, ur_e, uz_s, uz_n; /* face-mean normal velocities */
    double Ur_w, Ur_e, Uz_s, Uz_n; /* face volume rates (area x velocity) */
    double D, Dr, Dz;              /* flux-form divergence and its r / z parts */
    double err, ezz, ett, erz, om, dvr_dz, dvz_dr;
} kin_t;

/* Axial faces weight their two nodes by the r-weighted areas of the node
 * dual cells they cut, a_E(i) = (r_{i+1/2}^2 - r_i^2)/2 and
 * a_W(i+1) = (r_{i+1}^2 - r_{i+1/2}^2)/2 (which sum to the face area); this
 * makes the control-volume node force the exact gradient of the discrete
 * cell volumes, so stress work and kinetic energy balance, also on the axis. */
/* one column's geometry: node radii rw, re, centre radius rc, width dr, the
 * r-weighted areas aw, ae of its halves and its area per unit height az */
typedef struct {
    double rw, re, rc, dr, aw, ae, az;
} col_t;

/* column i of a uniform grid; a stretched column takes rc = rw + dr / 2 and
 * re = rw + dr from the running sum of widths instead */
static col_t col_uniform(double dr, int i)
{
    col_t c;
    c.rw = (double)i * dr;
    c.re = (double)(i + 1) * dr;
    c.rc = ((double)i + 0.5) * dr;
    c.dr = dr;
    c.aw = 0.5 * (c.rc * c.rc - c.rw * c.rw);
    c.ae = 0.5 * (c.re * c.re - c.rc * c.rc);
    c.az = c.rc * c.dr;
    return c;
}

static col_t col_at(const orc_ctx *x, int i)
{
    col_t c;
    c.rw = x->rn[i];
    c.re = x->rn[i + 1];
    c.rc = x->rcn[i];
    c.dr = x->drc[i];
    c.aw = x->awc[i];
    c.ae = x->aec[i];
    c.az = x->azc[i];
    return c;
}

static void kinematics(const col_t *cg, double dz, const double *vr, const double *vz, kin_t *k)
{
    /* vr, vz ordered SW, SE, NW, NE (nodes (i,j), (i+1,j), (i,j+1), (i+1,j+1)) */
    double Arw = cg->rw * dz, Are = cg->re * dz, Az = cg->az, V = Az * dz;
    double aw = cg->aw, ae = cg->ae;
    k->ur_w = 0.5 * (vr[0] + vr[2]);
    k->ur_e = 0.5 * (vr[1] + vr[3]);
    k->Ur_w = Arw * k->ur_w;
    k->Ur_e = Are * k->ur_e;
    k->Uz_s = aw * vz[0] + ae * vz[1];
    k->Uz_n = aw * vz[2] + ae * vz[3];
    k->uz_s = k->Uz_s / Az;
    k->uz_n = k->Uz_n / Az;
    k->Dr = (k->Ur_e - k->Ur_w) / V;
    k->Dz = (k->Uz_n - k->Uz_s) / V;
    k->D = ((k->Ur_e - k->Ur_w) + (k->Uz_n - k->Uz_s)) / V;
    k->err = (k->ur_e - k->ur_w) / cg->dr;
    k->ezz = (k->Uz_n - k->Uz_s) / V;
    k->ett = (0.5 * (k->ur_w + k->ur_e)) / cg->rc;
    k->dvr_dz = ((aw * vr[2] + ae * vr[3]) - (aw * vr[0] + ae * vr[1])) / V;
    k->dvz_dr = (0.5 * (vz[1] + vz[3]) - 0.5 * (vz[0] + vz[2])) / cg->dr;
    k->erz = 0.5 * (k->dvr_dz + k->dvz_dr);
    k->om = 0.5 * (k->dvr_dz - k->dvz_dr);
}

void orc_cell_kinematics(const orc_grid *g, int32_t i, int32_t j, const double *vr, const double *vz, double *out)
{
    kin_t k;
    col_t c;
    double dz;
    if (g->dr_col) {
        double rw = 0.0;
        for (int q = 0; q < i; q++) rw += g->dr_col[q];
        c.rw = rw;
        c.dr = g->dr_col[i];
        c.re = rw + c.dr;
        c.rc = rw + 0.5 * c.dr;
        c.aw = 0.5 * (c.rc * c.rc - c.rw * c.rw);
        c.ae = 0.5 * (c.re * c.re - c.rc * c.rc);
        c.az = c.rc * c.dr;
    } else {
        c = col_uniform(g->dr, i);
    }
    dz = g->dz_row ? g->dz_row[j] : g->dz;
    kinematics(&c, dz, vr, vz, &k);
    out[0] = k.err;
    out[1] = k.ezz;
    out[2] = k.ett;
    out[3] = k.erz;
    out[4] = k.om;
    out[5] = k.D;
}

/* Jaumann-rate elastic trial stress and radial return onto Y (strength model,
 * Table 1). rates = (e_rr, e_zz, e_tt, e_rz, omega); s = (s_rr, s_zz, s_rz). */
static double stress_update(double G, double Y, double dt, const double *rt, double *s);

void orc_stress_update(double G, double Y, double dt, const double *rt, double *s)
{
    (void)stress_update(G, Y, dt, rt, s);
}

/* the same, returning the equivalent stress of the elastic trial state */
static double stress_update(double G, double Y, double dt, const double *rt, double *s)
{
    double srr = s[0], szz = s[1], srz = s[2];
    double tr3 = ((rt[0] + rt[1]) + rt[2]) / 3.0;
    double om = rt[4];
    double dsrr = 2.0 * G * (rt[0] - tr3) + 2.0 * om * srz;
    double dszz = 2.0 * G * (rt[1] - tr3) - 2.0 * om * srz;
    double dsrz = 2.0 * G * rt[3] + om * (szz - srr);
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
    s[0] = srr;
    s[1] = szz;
    s[2] = srz;
    return seq;
}

/* Material volume ratio over a Lagrangian step whose cell volume ratio is J,
 * for a cell whose material fills the fraction phi. Compression closes the
 * void first and only then compresses the material. Expansion stretches the
 * material only while its pressure is above its tension floor (weight s in
 * [0, 1], a ramp over a small pressure scale); at the floor the void opens
 * instead (cavitation / spall). Full cells with s = 1 give exactly J. */
static double material_ratio(double J, double phi, double s)
{
    if (J < 1.0) return dmin(1.0, J / dmax(phi, PHI_EPS));
    return 1.0 + (J - 1.0) * s;
}

/* ========================================================================
 * Construction
 * ======================================================================== */
static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* PML damping d(y) = (3c / 2 delta) (y / delta)^2 log(1/R)  (Sec. 3) */
static double pml_d(double c, double delta, double y, double R)
{
    return 1.5 * c / delta * (y / delta) * (y / delta) * log(1.0 / R);
}

orc_ctx *orc_create(const orc_grid *g, const orc_mat *mats, const orc_pml *pml)
{
    if (!g || !mats || !pml) return NULL;
    if (g->n_r < 1 || g->n_z < 1 || g->pml_r < 0 || g->pml_b < 0) return NULL;
    if (g->nmat < 1 || g->nmat > ORC_MAX_MAT) return NULL;
    if (g->closure != 0 && g->closure != 1) return NULL;
    if (pml->damp_stress != 0 && pml->damp_stress != 1) return NULL;
    if (pml->placement != 0 && pml->placement != 1) return NULL;
    if (pml->form != 0 && pml->form != 1) return NULL;
    if (pml->form == 1 && (pml->placement != 0 || g->closure != 0)) return NULL;
    if (!(g->dr > 0) || !(g->dz > 0) || !(g->cfl > 0) || g->cfl > 1.0) return NULL;
    for (int i = 0; g->dr_col && i < g->n_r + g->pml_r; i++)
        if (!(g->dr_col[i] > 0) || !isfinite(g->dr_col[i])) return NULL;
    for (int j = 0; g->dz_row && j < g->n_z + g->pml_b; j++)
        if (!(g->dz_row[j] > 0) || !isfinite(g->dz_row[j])) return NULL;
    for (int m = 0; m < g->nmat; m++) {
        const orc_mat *M = &mats[m];
        if (M->damage != 0 && M->damage != 1) return NULL;
        if (M->damage && (!M->strength || !(M->Yd0 >= 0) || !(M->Ydm >= M->Yd0) || !(M->mu_d >= 0) ||
                          !(M->eps_fb > 0) || !(M->B_dmg >= 0) || !(M->gamma_eta >= 0) || !(M->gamma_T >= 0) ||
                          !(M->c_vib >= 0) || ((M->gamma_eta > 0 || M->gamma_T > 0) && !(M->af_h > 0))))
            return NULL;
    }
    orc_ctx *x = (orc_ctx *)calloc(1, sizeof(orc_ctx));
    x->g = *g;
    x->pml = *pml;
    x->nmat = g->nmat;
    x->pm = g->closure == 1;
    for (int m = 0; m < g->nmat; m++) {
        const orc_mat *M = &mats[m];
        x->m[m] = mats[m];
        x->Gm[m] = mats[m].strength ? 3.0 * (1.0 - 2.0 * mats[m].poisson) / (2.0 * (1.0 + mats[m].poisson)) : 0.0;
        if (mats[m].strength) x->any_strength = 1;
        if (mats[m].rho0 > x->rho_ref) x->rho_ref = mats[m].rho0;
        if (M->damage) {
            x->dmg = 1;
            x->cL0[m] = sqrt((M->A + (4.0 / 3.0) * orc_shear_modulus(M)) / M->rho0);
            x->nub[m] = M->gamma_eta * x->cL0[m] * M->af_h;
            x->Tvib[m] = M->gamma_T * M->af_h / x->cL0[m];
        }
    }
    int NR = g->n_r + g->pml_r, NZ = g->n_z + g->pml_b;
    x->NR = NR;
    x->NZ = NZ;
    x->NC = NR * NZ;
    x->NN = (NR + 1) * (NZ + 1);
    size_t NC = x->NC, NN = x->NN, NRF = (size_t)(NR + 1) * NZ, NAF = (size_t)NR * (NZ + 1);

    /* geometry tables; a stretched grid sums its widths outward from the
     * axis and its heights upward from the bottom, centres halfway */
    x->rn = zalloc((size_t)NR + 1);
    x->rcn = zalloc(NR);
    x->drc = zalloc(NR);
    x->awc = zalloc(NR);
    x->aec = zalloc(NR);
    x->azc = zalloc(NR);
    x->zn = zalloc((size_t)NZ + 1);
    x->zcn = zalloc(NZ);
    x->dzr = zalloc(NZ);
    for (int i = 0; i < NR; i++) {
        col_t c;
        if (g->dr_col) {
            c.rw = x->rn[i];
            c.dr = g->dr_col[i];
            c.re = c.rw + c.dr;
            c.rc = c.rw + 0.5 * c.dr;
            c.aw = 0.5 * (c.rc * c.rc - c.rw * c.rw);
            c.ae = 0.5 * (c.re * c.re - c.rc * c.rc);
            c.az = c.rc * c.dr;
        } else {
            c = col_uniform(g->dr, i);
        }
        x->rn[i] = c.rw;
        x->rn[i + 1] = c.re;
        x->rcn[i] = c.rc;
        x->drc[i] = c.dr;
        x->awc[i] = c.aw;
        x->aec[i] = c.ae;
        x->azc[i] = c.az;
    }
    for (int j = 0; j < NZ; j++) {
        if (g->dz_row) {
            x->dzr[j] = g->dz_row[j];
            x->zn[j + 1] = x->zn[j] + x->dzr[j];
            x->zcn[j] = x->zn[j] + 0.5 * x->dzr[j];
        } else {
            x->dzr[j] = g->dz;
            x->zn[j] = (double)j * g->dz;
            x->zn[j + 1] = (double)(j + 1) * g->dz;
            x->zcn[j] = ((double)j + 0.5) * g->dz;
        }
    }
    x->g.dr_col = x->g.dz_row = NULL; /* the tables hold them now */

    x->rho = zalloc(NC);
    x->I = zalloc(NC);
    x->srr = zalloc(NC);
    x->szz = zalloc(NC);
    x->srz = zalloc(NC);
    x->vr = zalloc(NN);
    x->vz = zalloc(NN);
    x->rho_n = zalloc(NC);
    x->I_n = zalloc(NC);
    x->srr_n = zalloc(NC);
    x->szz_n = zalloc(NC);
    x->srz_n = zalloc(NC);
    x->vr_n = zalloc(NN);
    x->vz_n = zalloc(NN);
    for (int m = 0; m < ORC_MAX_MAT; m++) {
        x->f[m] = zalloc(NC);
        x->f_n[m] = zalloc(NC);
        x->fL[m] = zalloc(NC);
        x->mu[m] = zalloc(NC);
        x->Im[m] = zalloc(NC);
        x->mu_n[m] = zalloc(NC);
        x->Im_n[m] = zalloc(NC);
        x->pmm[m] = zalloc(NC);
        x->rhm[m] = zalloc(NC);
        x->ILm[m] = zalloc(NC);
        x->Fmr[m] = zalloc(NRF);
        x->Fmz[m] = zalloc(NAF);
        x->mu_t[m] = zalloc(NC);
    }
    x->psi1n_r = zalloc(NN);
    x->psi1n_z = zalloc(NN);
    x->psi2n = zalloc(NC);
    x->rho_t = zalloc(NC);
    double **dmga[] = {&x->D, &x->vib, &x->D_n, &x->vib_n, &x->DL, &x->vibL, &x->etab};
    for (size_t k = 0; k < sizeof(dmga) / sizeof(dmga[0]); k++) *dmga[k] = zalloc(NC);
    x->p0 = zalloc(NZ);
    x->dcz = zalloc(NZ);
    x->dnz = zalloc(NZ + 1);
    x->dcr = zalloc(NR);
    x->dnr = zalloc(NR + 1);
    double **cellaux[] = {&x->phi1b, &x->phi3b, &x->psi2b, &x->phi1r, &x->phi3r, &x->psi2r,
                          &x->rref, &x->msink, &x->p, &x->c2, &x->G, &x->Y, &x->rmat, &x->phi, &x->sx,
                          &x->Q, &x->sgrr, &x->sgzz, &x->sgtt, &x->sgrz, &x->J, &x->IL,
                          &x->sLrr, &x->sLzz, &x->sLrz};
    for (size_t k = 0; k < sizeof(cellaux) / sizeof(cellaux[0]); k++) *cellaux[k] = zalloc(NC);
    double **nodeaux[] = {&x->phi2b_r, &x->phi2b_z, &x->psi1b_r, &x->psi1b_z, &x->phi2r_r,
                          &x->phi2r_z, &x->psi1r_r, &x->psi1r_z, &x->vLr, &x->vLz, &x->heat};
    for (size_t k = 0; k < sizeof(nodeaux) / sizeof(nodeaux[0]); k++) *nodeaux[k] = zalloc(NN);
    x->dVr = zalloc(NRF);
    x->Fr = zalloc(NRF);
    x->dVre = zalloc(NRF);
    x->dVz = zalloc(NAF);
    x->Fz = zalloc(NAF);
    x->dVze = zalloc(NAF);
    x->lam = zalloc(NC);
    x->outv = zalloc(NC);
    x->mout_col = zalloc(NR);
    x->eout_col = zalloc(NR);

    /* damping profiles; y is measured from the inner face of each layer,
     * at cell centres for cell quantities and at nodes for node quantities */
    if (pml->enabled) {
        /* Sec. 3: c is the largest acoustic speed; by default the largest
         * longitudinal speed at rest over the materials */
        double c = pml->c_ref;
        if (!(c > 0)) {
            c = 0.0;
            for (int m = 0; m < g->nmat; m++) {
                const orc_mat *mm = &mats[m];
                double cm = sqrt((mm->A + (4.0 / 3.0) * orc_shear_modulus(mm)) / mm->rho0);
                if (cm > c) c = cm;
            }
        }
        if (g->pml_b > 0) {
            double zf = x->zn[g->pml_b], delta = zf - x->zn[0];
            for (int j = 0; j < g->pml_b; j++)
                x->dcz[j] = pml_d(c, delta, zf - x->zcn[j], pml->R);
            for (int j = 0; j < g->pml_b; j++)
                x->dnz[j] = pml_d(c, delta, zf - x->zn[j], pml->R);
        }
        if (g->pml_r > 0) {
            double rf = x->rn[g->n_r], delta = x->rn[NR] - rf;
            for (int i = g->n_r; i < NR; i++)
                x->dcr[i] = pml_d(c, delta, x->rcn[i] - rf, pml->R);
            for (int i = g->n_r + 1; i <= NR; i++)
                x->dnr[i] = pml_d(c, delta, x->rn[i] - rf, pml->R);
        }
    }
    return x;
}

void orc_destroy(orc_ctx *x)
{
    if (!x) return;
    double *all[] = {x->rho, x->I, x->srr, x->szz, x->srz, x->vr, x->vz, x->rho_n, x->I_n, x->p0,
                     x->rn, x->rcn, x->drc, x->awc, x->aec, x->azc, x->zn, x->zcn, x->dzr,
                     x->srr_n, x->szz_n, x->srz_n, x->vr_n, x->vz_n, x->dcz, x->dnz, x->dcr,
                     x->dnr, x->phi1b, x->phi3b, x->psi2b, x->phi1r, x->phi3r, x->psi2r,
                     x->rref, x->msink, x->p, x->c2, x->G, x->Y, x->rmat, x->phi, x->sx, x->Q,
                     x->sgrr, x->sgzz, x->sgtt, x->sgrz, x->J, x->IL, x->sLrr, x->sLzz,
                     x->sLrz, x->phi2b_r, x->phi2b_z, x->psi1b_r, x->psi1b_z, x->phi2r_r,
                     x->phi2r_z, x->psi1r_r, x->psi1r_z, x->vLr, x->vLz, x->heat, x->dVr, x->Fr,
                     x->dVz, x->Fz, x->dVre, x->dVze, x->lam, x->outv, x->mout_col, x->eout_col};
    for (size_t k = 0; k < sizeof(all) / sizeof(all[0]); k++) free(all[k]);
    free(x->psi1n_r);
    free(x->psi1n_z);
    free(x->psi2n);
    free(x->rho_t);
    double *dmga[] = {x->D, x->vib, x->D_n, x->vib_n, x->DL, x->vibL, x->etab};
    for (size_t k = 0; k < sizeof(dmga) / sizeof(dmga[0]); k++) free(dmga[k]);
    for (int m = 0; m < ORC_MAX_MAT; m++) {
        free(x->f[m]);
        free(x->f_n[m]);
        free(x->fL[m]);
        double *pa[] = {x->mu[m], x->Im[m], x->mu_n[m], x->Im_n[m], x->pmm[m], x->rhm[m], x->ILm[m],
                        x->Fmr[m], x->Fmz[m], x->mu_t[m]};
        for (size_t k = 0; k < sizeof(pa) / sizeof(pa[0]); k++) free(pa[k]);
    }
    free(x);
}

/* ========================================================================
 * Time step (Sec. 7): dt <= C0 min(dr, dz) / (|v| + c), evaluated per cell
 * with the longitudinal speed and the largest corner speed; cells whose
 * volume fraction is below W_LO are ignored, with a continuous ramp to W_HI.
 * ======================================================================== */
static double dt_candidate_min(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
    double best = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : best)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double p, c2, G, Y, rm, phi, sx;
            cell_mixture(x, c, &p, &c2, &G, &Y, &rm, &phi, &sx, NULL, NULL);
            double cl2 = c2 + (4.0 / 3.0) * G / dmax(rm, x->rho_ref * RHO_DEN_FLOOR);
            double cl = sqrt(cl2);
            int nd[4] = {NI(i, j), NI(i + 1, j), NI(i, j + 1), NI(i + 1, j + 1)};
            double u = 0.0;
            for (int k = 0; k < 4; k++) {
                double s = sqrt(x->vr[nd[k]] * x->vr[nd[k]] + x->vz[nd[k]] * x->vz[nd[k]]);
                u = dmax(u, s);
            }
            double w = dmin(dmax((phi - W_LO) / (W_HI - W_LO), 0.0), 1.0);
            if (w > 0.0) {
                double L = dmin(x->drc[i], x->dzr[j]);
                double cand = x->g.cfl * L / ((cl + u) * w);
                if (cand < best) best = cand;
            }
        }
    }
    return best;
}

static void start_run(orc_ctx *x)
{
    int NR = x->NR;
    memcpy(x->rref, x->rho, sizeof(double) * x->NC);
    double **cz[] = {&x->phi1b, &x->phi3b, &x->psi2b, &x->phi1r, &x->phi3r, &x->psi2r, &x->msink};
    for (size_t k = 0; k < sizeof(cz) / sizeof(cz[0]); k++) memset(*cz[k], 0, sizeof(double) * x->NC);
    double **nz[] = {&x->phi2b_r, &x->phi2b_z, &x->psi1b_r, &x->psi1b_z,
                     &x->phi2r_r, &x->phi2r_z, &x->psi1r_r, &x->psi1r_z};
    for (size_t k = 0; k < sizeof(nz) / sizeof(nz[0]); k++) memset(*nz[k], 0, sizeof(double) * x->NN);
    memset(x->mout_col, 0, sizeof(double) * NR);
    memset(x->eout_col, 0, sizeof(double) * NR);
    x->t = 0.0;
    x->cycle = 0;
    x->err = 0;
    x->err_cycle = -1;
    double dt = dmin(dt_candidate_min(x), x->g.dt_max);
    if (x->g.t_stop > 0) dt = dmin(dt, x->g.t_stop);
    x->dt = dt;
    x->dt_prev = 0.0;
}

/* boundary conditions (Sec. 4): symmetry axis and outer side free-slip
 * (v_r = 0), bottom no-slip (v = 0), top open unless closed */
static void apply_bc(orc_ctx *x, double *vr, double *vz)
{
    int NR = x->NR, NZ = x->NZ;
    for (int j = 0; j <= NZ; j++) {
        vr[NI(0, j)] = 0.0;
        vr[NI(NR, j)] = 0.0;
    }
    for (int i = 0; i <= NR; i++) {
        vr[NI(i, 0)] = 0.0;
        vz[NI(i, 0)] = 0.0;
        if (x->g.top_closed) vz[NI(i, NZ)] = 0.0;
    }
}

/* Lithostatic column of the target rows below surface_j (the initial
 * pressure p0 of Sec. 3's momentum equation, with -grad p0 + rho g = 0).
 * Cell-centre pressures are integrated down from p = 0 at the surface over
 * the piecewise-constant density: p(top row) = g rho dz / 2, p(j) = p(j+1)
 * + g (rho(j+1) dz(j+1) / 2 + rho(j) dz(j) / 2). Each row's density is the cold (E = 0) compressed
 * state at its pressure: with p = A mu + B mu^2, mu = 2p / (A + sqrt(A^2 +
 * 4Bp)); since p(j) depends on rho(j) too, the two are iterated to a fixed
 * point (at most 50 times). p0(j) is then set to the equation of state's own
 * pressure at that density and E = 0, so the column is in exact discrete
 * equilibrium: p - p0 = 0 in every target cell. mat_row[j] is the row's
 * material. */
static void lithostatic(orc_ctx *x, int surface_j, const int *mat_row, double g, double *rho_row)
{
    for (int j = surface_j - 1; j >= 0; j--) {
        const orc_mat *m = &x->m[mat_row[j]];
        int top = j == surface_j - 1;
        double p_up = top ? 0.0 : x->p0[j + 1];
        /* weight per unit area between the two row centres */
        double w_up = top ? 0.0 : g * (0.5 * x->dzr[j + 1]) * rho_row[j + 1];
        double hj = g * (0.5 * x->dzr[j]);
        double r = m->rho0;
        for (int it = 0; it < 50; it++) {
            double p = p_up + (w_up + hj * r);
            double mu = 2.0 * p / (m->A + sqrt(m->A * m->A + 4.0 * m->B * p));
            double rn = m->rho0 * (1.0 + mu);
            if (rn == r) break;
            r = rn;
        }
        double p, c2;
        orc_tillotson(m, r, 0.0, &p, &c2);
        rho_row[j] = r;
        x->p0[j] = p;
    }
}

/* scene: target half-space below surface_j (material 0; with two materials
 * the rows below layer_j are material 1, with three the rows below layer2_j
 * material 2 and those from layer2_j to layer_j material 1), with an
 * optional lithostatic column (gravity > 0), and a spherical projectile of
 * the last material (that of the deepest layer) resting on the surface at the
 * axis and moving downward (radius 0: none); momentum-exact nodal velocities */
int orc_init_scene(orc_ctx *x, const orc_scene *s)
{
    if (!x || !s || s->subsample < 1 || !(s->radius >= 0) || !(s->gravity >= 0)) return ORC_E_INVALID;
    if (s->surface_j < 0 || s->surface_j > x->NZ || s->layer_j < 0 || s->layer_j > s->surface_j) return ORC_E_INVALID;
    if (s->layer2_j < 0 || s->layer2_j > s->layer_j || (x->nmat < 3 && s->layer2_j != 0)) return ORC_E_INVALID;
    int NR = x->NR, NZ = x->NZ, S = s->subsample;
    int mp = x->nmat - 1;
    double R = s->radius, zc = x->zn[s->surface_j] + R;
    double *fp = zalloc(x->NC);
    for (int j = 0; j < NZ && R > 0; j++) {
        for (int i = 0; i < NR; i++) {
            double num = 0.0, den = 0.0;
            for (int l = 0; l < S; l++) {
                double zl = x->zn[j] + (((double)l + 0.5) / (double)S) * x->dzr[j];
                for (int k = 0; k < S; k++) {
                    double rk = x->rn[i] + (((double)k + 0.5) / (double)S) * x->drc[i];
                    double dzl = zl - zc;
                    if (rk * rk + dzl * dzl <= R * R) num += rk;
                    den += rk;
                }
            }
            fp[CI(i, j)] = num / den;
        }
    }
    /* material and density of each target row */
    int *mat_row = (int *)calloc((size_t)NZ + 1, sizeof(int));
    double *rho_row = zalloc((size_t)NZ + 1);
    for (int j = 0; j < s->surface_j; j++) {
        mat_row[j] = x->nmat == 3 && j < s->layer2_j ? 2 : (x->nmat > 1 && j < s->layer_j ? 1 : 0);
        rho_row[j] = x->m[mat_row[j]].rho0;
    }
    memset(x->p0, 0, sizeof(double) * (size_t)NZ);
    if (s->gravity > 0) lithostatic(x, s->surface_j, mat_row, s->gravity, rho_row);
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            for (int m = 0; m < x->nmat; m++) x->f[m][c] = 0.0;
            double rho = 0.0;
            if (j < s->surface_j) {
                x->f[mat_row[j]][c] = 1.0;
                rho = rho_row[j];
            } else {
                x->f[mp][c] = fp[c];
                rho = fp[c] * x->m[mp].rho0;
            }
            x->rho[c] = rho;
            x->I[c] = 0.0;
            /* closure 1: each cell holds one material's mass */
            for (int m = 0; m < x->nmat; m++) {
                int own = j < s->surface_j ? m == mat_row[j] : m == mp;
                x->mu[m][c] = own ? rho : 0.0;
                x->Im[m][c] = 0.0;
            }
            x->srr[c] = x->szz[c] = x->srz[c] = 0.0;
            x->D[c] = x->vib[c] = 0.0;
        }
    }
    /* node velocity = -v_imp * (projectile mass) / (total mass) over the four
     * cells around the node (quadrants SW, SE, NW, NE) */
    for (int j = 0; j <= NZ; j++) {
        for (int i = 0; i <= NR; i++) {
            double Mt = 0.0, Mp = 0.0;
            int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
            for (int q = 0; q < 4; q++) {
                if (qi[q] < 0 || qi[q] >= NR || qj[q] < 0 || qj[q] >= NZ) continue;
                int c = CI(qi[q], qj[q]);
                double V = vol_c(x, qi[q], qj[q]);
                Mt += x->rho[c] * V;
                Mp += fp[c] * x->m[mp].rho0 * V;
            }
            x->vr[NI(i, j)] = 0.0;
            x->vz[NI(i, j)] = Mt > 0.0 ? -s->v_imp * (Mp / Mt) : 0.0;
        }
    }
    free(fp);
    free(mat_row);
    free(rho_row);
    apply_bc(x, x->vr, x->vz);
    start_run(x);
    return ORC_OK;
}

int orc_get_geometry(orc_ctx *x, double *r_node, double *r_cell, double *z_node, double *z_cell)
{
    if (!x) return ORC_E_INVALID;
    if (r_node) memcpy(r_node, x->rn, sizeof(double) * ((size_t)x->NR + 1));
    if (r_cell) memcpy(r_cell, x->rcn, sizeof(double) * (size_t)x->NR);
    if (z_node) memcpy(z_node, x->zn, sizeof(double) * ((size_t)x->NZ + 1));
    if (z_cell) memcpy(z_cell, x->zcn, sizeof(double) * (size_t)x->NZ);
    return ORC_OK;
}

int orc_set_p0(orc_ctx *x, const double *p0)
{
    if (!x || !p0) return ORC_E_INVALID;
    memcpy(x->p0, p0, sizeof(double) * (size_t)x->NZ);
    return ORC_OK;
}

int orc_get_p0(orc_ctx *x, double *p0)
{
    if (!x || !p0) return ORC_E_INVALID;
    memcpy(p0, x->p0, sizeof(double) * (size_t)x->NZ);
    return ORC_OK;
}

int orc_set_fields(orc_ctx *x, const double *rho, const double *I, const double *f,
                   const double *s, const double *v)
{
    if (!x || !rho || !I || !f || !v) return ORC_E_INVALID;
    size_t NC = x->NC, NN = x->NN;
    memcpy(x->rho, rho, sizeof(double) * NC);
    memcpy(x->I, I, sizeof(double) * NC);
    for (int m = 0; m < x->nmat; m++) memcpy(x->f[m], f + m * NC, sizeof(double) * NC);
    if (s) {
        memcpy(x->srr, s, sizeof(double) * NC);
        memcpy(x->szz, s + NC, sizeof(double) * NC);
        memcpy(x->srz, s + 2 * NC, sizeof(double) * NC);
    } else {
        memset(x->srr, 0, sizeof(double) * NC);
        memset(x->szz, 0, sizeof(double) * NC);
        memset(x->srz, 0, sizeof(double) * NC);
    }
    memcpy(x->vr, v, sizeof(double) * NN);
    memcpy(x->vz, v + NN, sizeof(double) * NN);
    memset(x->D, 0, sizeof(double) * NC);
    memset(x->vib, 0, sizeof(double) * NC);
    /* closure 1: every material of a cell at the cell's matter density and
     * specific energy */
    for (size_t c = 0; c < NC; c++) {
        double phi = 0.0;
        for (int m = 0; m < x->nmat; m++) phi += x->f[m][c];
        double den = phi > PHI_EPS ? phi : PHI_EPS;
        for (int m = 0; m < x->nmat; m++) {
            x->mu[m][c] = x->rho[c] * (x->f[m][c] / den);
            x->Im[m][c] = x->I[c];
        }
    }
    start_run(x);
    return ORC_OK;
}

int orc_set_damage(orc_ctx *x, const double *D, const double *vib)
{
    if (!x) return ORC_E_INVALID;
    if (D) memcpy(x->D, D, sizeof(double) * (size_t)x->NC);
    if (vib) memcpy(x->vib, vib, sizeof(double) * (size_t)x->NC);
    return ORC_OK;
}

int orc_get_damage(orc_ctx *x, double *D, double *vib)
{
    if (!x) return ORC_E_INVALID;
    if (D) memcpy(D, x->D, sizeof(double) * (size_t)x->NC);
    if (vib) memcpy(vib, x->vib, sizeof(double) * (size_t)x->NC);
    return ORC_OK;
}

int orc_set_materials(orc_ctx *x, const double *mu, const double *Im)
{
    if (!x || !mu || !Im || !x->pm) return ORC_E_INVALID;
    size_t NC = x->NC;
    for (int m = 0; m < x->nmat; m++) {
        memcpy(x->mu[m], mu + m * NC, sizeof(double) * NC);
        memcpy(x->Im[m], Im + m * NC, sizeof(double) * NC);
    }
    for (size_t c = 0; c < NC; c++) derive_cell(x, x->mu, x->Im, x->rho, x->I, (int)c);
    start_run(x);
    return ORC_OK;
}

int orc_get_materials(orc_ctx *x, double *mu, double *Im)
{
    if (!x || !x->pm) return ORC_E_INVALID;
    size_t NC = x->NC;
    for (int m = 0; m < x->nmat; m++) {
        if (mu) memcpy(mu + m * NC, x->mu[m], sizeof(double) * NC);
        if (Im) memcpy(Im + m * NC, x->Im[m], sizeof(double) * NC);
    }
    return ORC_OK;
}

/* ========================================================================
 * One cycle
 * ======================================================================== */

/* (a) per cell: EoS, artificial viscosity from the start-of-cycle velocity
 * divergence, total stress sigma = phi (s - (p + Q - p0) I), p0 the initial
 * pressure of the cell's row (Sec. 3: the momentum balance and psi1 carry
 * p - p0; the energy equation keeps p) */
static void phase_cell_stress(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double L = dmin(x->drc[i], x->dzr[j]);
            double p, c2, G, Y, rm, phi, sx, pmv[ORC_MAX_MAT], rhv[ORC_MAX_MAT];
            cell_mixture(x, c, &p, &c2, &G, &Y, &rm, &phi, &sx, pmv, rhv);
            for (int m = 0; x->pm && m < x->nmat; m++) {
                x->pmm[m][c] = pmv[m];
                x->rhm[m][c] = rhv[m];
            }
            double vr4[4] = {x->vr[NI(i, j)], x->vr[NI(i + 1, j)], x->vr[NI(i, j + 1)], x->vr[NI(i + 1, j + 1)]};
            double vz4[4] = {x->vz[NI(i, j)], x->vz[NI(i + 1, j)], x->vz[NI(i, j + 1)], x->vz[NI(i + 1, j + 1)]};
            kin_t k;
            col_t cg = col_at(x, i);
            kinematics(&cg, x->dzr[j], vr4, vz4, &k);
            /* compression felt by the material (void closes first) */
            double Jn = 1.0 + x->dt * k.D;
            double Dm = Jn < 1.0 ? (1.0 - material_ratio(Jn, phi, sx)) / x->dt : 0.0;
            double Ld = L * Dm;
            double Q = rm * (x->g.q_quad * Ld * Ld + x->g.q_lin * sqrt(c2) * Ld);
            double P = p + Q;
            double Pf = P - x->p0[j];
            double stt = -(x->srr[c] + x->szz[c]);
            x->p[c] = p;
            x->c2[c] = c2;
            x->G[c] = G;
            x->Y[c] = Y;
            x->rmat[c] = rm;
            x->phi[c] = phi;
            x->sx[c] = sx;
            x->Q[c] = Q;
            x->sgrr[c] = phi * (x->srr[c] - Pf);
            x->sgzz[c] = phi * (x->szz[c] - Pf);
            x->sgtt[c] = phi * (stt - Pf);
            x->sgrz[c] = phi * x->srz[c];
            if (x->dmg) {
                /* block model: dynamic viscosity rho gamma_eta c h of the damaged
                 * rock (weight D) while it vibrates (ramp to full at VIB_ON) */
                double nu = 0.0;
                for (int m = 0; m < x->nmat; m++)
                    if (x->m[m].damage) nu += (x->f[m][c] / dmax(phi, PHI_EPS)) * x->nub[m];
                x->etab[c] = (x->D[c] * dmin(x->vib[c] / VIB_ON, 1.0)) * (rm * nu);
            }
        }
    }
}

/* (b) per node: control-volume force of eq. (1) over the dual cell, with the
 * hoop stress, acceleration, PML psi1 (Sec. 3), boundary conditions -> v^L */
static void phase_node_force(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
    double dt = x->dt;
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= NZ; j++) {
        for (int i = 0; i <= NR; i++) {
            /* quadrant cells: NE = (i,j), NW = (i-1,j), SE = (i,j-1), SW = (i-1,j-1) */
            double srr[4] = {0, 0, 0, 0}, szz[4] = {0, 0, 0, 0}, stt[4] = {0, 0, 0, 0},
                   srz[4] = {0, 0, 0, 0}, rh[4] = {0, 0, 0, 0};
            int qi[4] = {i, i - 1, i, i - 1}, qj[4] = {j, j, j - 1, j - 1}; /* NE NW SE SW */
            for (int q = 0; q < 4; q++) {
                if (qi[q] < 0 || qi[q] >= NR || qj[q] < 0 || qj[q] >= NZ) continue;
                int c = CI(qi[q], qj[q]);
                srr[q] = x->sgrr[c];
                szz[q] = x->sgzz[c];
                stt[q] = x->sgtt[c];
                srz[q] = x->sgrz[c];
                rh[q] = x->rho[c];
            }
            /* dual cell: from the west cell's centre rW to the east cell's
             * centre rE, half the row above (hN) and half the row below (hS) */
            double rN = x->rn[i];
            double rE = i < NR ? x->rcn[i] : 0.0;
            double rW = i > 0 ? x->rcn[i - 1] : 0.0;
            double aE = i < NR ? x->awc[i] : 0.0;
            double aW = i > 0 ? x->aec[i - 1] : 0.0;
            double hN = j < NZ ? 0.5 * x->dzr[j] : 0.0;
            double hS = j > 0 ? 0.5 * x->dzr[j - 1] : 0.0;
            /* r-direction (radial faces + hoop) and z-direction (axial faces) parts */
            double Frr = (hN * (rE * (srr[0] - stt[0]) + rN * stt[0]) + hS * (rE * (srr[2] - stt[2]) + rN * stt[2]))
                       - (hN * (rW * (srr[1] - stt[1]) + rN * stt[1]) + hS * (rW * (srr[3] - stt[3]) + rN * stt[3]));
            double Frz = (aW * srz[1] + aE * srz[0]) - (aW * srz[3] + aE * srz[2]);
            double Fzr = rE * (hN * srz[0] + hS * srz[2]) - rW * (hN * srz[1] + hS * srz[3]);
            double Fzz = (aW * szz[1] + aE * szz[0]) - (aW * szz[3] + aE * szz[2]);
            double Fr = Frr + Frz, Fz = Fzr + Fzz;
            double macc = (aE * hN * rh[0] + aW * hN * rh[1]) + (aE * hS * rh[2] + aW * hS * rh[3]);
            double Vd = (aE + aW) * (hN + hS);
            double mt = dmax(macc, M_ACC_EPS * x->rho_ref * Vd);
            int n = NI(i, j);
            double db = x->dnz[j], drr = x->dnr[i];
            double psr = x->psi1b_r[n] + x->psi1r_r[n];
            double psz = x->psi1b_z[n] + x->psi1r_z[n];
            /* the auxiliary this step applies: psi1, or phi2 as printed */
            double apr = psr, apz = psz;
            if (x->pml.placement) {
                apr = x->phi2b_r[n] + x->phi2r_r[n];
                apz = x->phi2b_z[n] + x->phi2r_z[n];
                x->psi1n_r[n] = psr; /* for the momentum remap */
                x->psi1n_z[n] = psz;
            }
            double Fer = Fr - Vd * apr, Fez = Fz - Vd * apz;
            x->vLr[n] = x->vr[n] + dt * (Fer / mt);
            x->vLz[n] = x->vz[n] + dt * (Fez / mt);
            if (db > 0.0) {
                x->psi1b_r[n] = x->psi1b_r[n] - dt * db * (Frr / Vd);
                x->psi1b_z[n] = x->psi1b_z[n] - dt * db * (Fzr / Vd);
            }
            if (drr > 0.0) {
                x->psi1r_r[n] = x->psi1r_r[n] - dt * drr * (Frz / Vd);
                x->psi1r_z[n] = x->psi1r_z[n] - dt * drr * (Fzz / Vd);
            }
        }
    }
    apply_bc(x, x->vLr, x->vLz);
}

/* (c) per cell: Lagrangian update -- strain rates from v^L, deviatoric stress
 * (Jaumann rate + radial return), internal energy of eq. (2) with PML psi2,
 * Lagrangian volume ratio J = V^L / V */
static void phase_cell_lagrange(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
    double dt = x->dt;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double vr4[4] = {x->vLr[NI(i, j)], x->vLr[NI(i + 1, j)], x->vLr[NI(i, j + 1)], x->vLr[NI(i + 1, j + 1)]};
            double vz4[4] = {x->vLz[NI(i, j)], x->vLz[NI(i + 1, j)], x->vLz[NI(i, j + 1)], x->vLz[NI(i + 1, j + 1)]};
            kin_t k;
            col_t cg = col_at(x, i);
            kinematics(&cg, x->dzr[j], vr4, vz4, &k);
            double s[3] = {x->srr[c], x->szz[c], x->srz[c]};
            double DLc = x->dmg ? x->D[c] : 0.0;
            if (x->any_strength) {
                double rt[5] = {k.err, k.ezz, k.ett, k.erz, k.om};
                double Yr = x->Y[c];
                if (x->dmg) {
                    /* the block model's viscous resistance (Bingham): the flow
                     * stress exceeds Y by 3 eta times the equivalent strain rate
                     * sqrt(2/3 e':e') of this step */
                    double tr3 = ((k.err + k.ezz) + k.ett) / 3.0;
                    double dr_ = k.err - tr3, dz_ = k.ezz - tr3, dt_ = k.ett - tr3;
                    double e2 = ((dr_ * dr_ + dz_ * dz_) + dt_ * dt_) + 2.0 * (k.erz * k.erz);
                    Yr = Yr + 3.0 * x->etab[c] * sqrt((2.0 / 3.0) * e2);
                }
                double seq = stress_update(x->G[c], Yr, dt, rt, s);
                if (x->dmg) {
                    /* damage grows by the equivalent plastic strain of the
                     * return, (trial - yield) / 3G, over the failure strain at
                     * the cell's pressure (volume-fraction weighted rate) */
                    double G = x->G[c];
                    double dep = G > 0.0 ? dmax(seq - Yr, 0.0) / (3.0 * G) : 0.0;
                    double rate = 0.0;
                    for (int m = 0; m < x->nmat; m++)
                        if (x->m[m].damage)
                            rate += (x->f[m][c] / dmax(x->phi[c], PHI_EPS)) / orc_failure_strain(&x->m[m], x->p[c]);
                    DLc = dmin(x->D[c] + dep * rate, 1.0);
                }
            }
            x->DL[c] = DLc;
            x->vibL[c] = x->dmg ? x->vib[c] : 0.0;
            /* the deviatoric power uses s^n, the stress that produced the node
             * forces, so the step's work equals the forces' work exactly */
            double s0rr = x->srr[c], s0zz = x->szz[c], s0rz = x->srz[c];
            double stt = -(s0rr + s0zz);
            double P = x->p[c] + x->Q[c];
            double sde = ((s0rr * k.err + s0zz * k.ezz) + stt * k.ett) + 2.0 * s0rz * k.erz;
            double J = 1.0 + dt * k.D;
            double Jm = material_ratio(J, x->phi[c], x->sx[c]);
            /* specific work over the step: deviatoric power minus P dV, with the
             * cell's volume change (the work of the phi-scaled stress) */
            double Wdt = dt * sde - P * (J - 1.0);
            double rden = dmax(x->rmat[c], x->rho_ref * RHO_DEN_FLOOR);
            double rt_ = dmax(x->rho[c], x->rho_ref * PML_RHO_FLOOR);
            double psi2 = x->psi2b[c] + x->psi2r[c];
            /* the auxiliary this step applies to the energy: psi2, or phi3 as
             * printed (which then also applies phi1 to the mass below) */
            double a3 = x->pml.placement ? x->phi3b[c] + x->phi3r[c] : psi2;
            if (x->pml.placement) x->psi2n[c] = psi2; /* for the cell remap */
            /* Symplectic Euler (the grid moves with v^L) makes the p dV work
             * fall short of the kinetic-energy change by m |v^L - v^n|^2 / 2
             * per node; each corner mass of the node keeps its share, so the
             * cell gains sum over corners |dv|^2 / 2 * (corner volume / V). */
            double kd[4];
            int nd[4] = {NI(i, j), NI(i + 1, j), NI(i, j + 1), NI(i + 1, j + 1)}; /* SW SE NW NE */
            for (int q = 0; q < 4; q++) {
                double dvr = x->vLr[nd[q]] - x->vr[nd[q]], dvz = x->vLz[nd[q]] - x->vz[nd[q]];
                kd[q] = 0.5 * (dvr * dvr + dvz * dvz);
            }
            double V = vol_c(x, i, j), hdz = 0.5 * x->dzr[j];
            double wW = (cg.aw * hdz) / V;
            double wE = (cg.ae * hdz) / V;
            double hL = wW * (kd[0] + kd[2]) + wE * (kd[1] + kd[3]);
            x->IL[c] = ((x->I[c] + Wdt / rden) + hL) - dt * (a3 / rt_);
            /* closure 1: each material does the deviatoric work and its own
             * p dV work on the cell's volume change (the sum over materials of
             * mu_m times the specific work is the cell's work above) */
            for (int m = 0; x->pm && m < x->nmat; m++) {
                double Pm = x->pmm[m][c] + x->Q[c];
                double Wm = dt * sde - Pm * (J - 1.0);
                double rdm = dmax(x->rhm[m][c], x->rho_ref * RHO_DEN_FLOOR);
                x->ILm[m][c] = ((x->Im[m][c] + Wm / rdm) + hL) - dt * (a3 / rt_);
            }
            for (int m = 0; m < x->nmat; m++) x->fL[m][c] = x->f[m][c] * (Jm / J);
            double db = x->dcz[j], drr = x->dcr[i];
            if (db > 0.0) {
                double Wr = ((s0rr * k.err + stt * k.ett) + s0rz * k.dvz_dr) - P * k.Dr;
                x->psi2b[c] = x->psi2b[c] - dt * db * (x->phi[c] * Wr);
            }
            if (drr > 0.0) {
                double Wz = (s0zz * k.ezz + s0rz * k.dvr_dz) - P * k.Dz;
                x->psi2r[c] = x->psi2r[c] - dt * drr * (x->phi[c] * Wz);
            }
            x->sLrr[c] = s[0];
            x->sLzz[c] = s[1];
            x->sLrz[c] = s[2];
            x->J[c] = J;
            /* the mass the Eulerian step starts from: phi1 as printed leaves
             * the layer here (a sink that never leaves negative mass, whose
             * loss the sink budget records; with closure 1 every material
             * loses the same fraction) */
            if (x->pml.placement) {
                double rt = x->rho[c];
                if (db > 0.0 || drr > 0.0) {
                    rt = dmax(x->rho[c] - dt * (x->phi1b[c] + x->phi1r[c]), 0.0);
                    x->msink[c] = x->msink[c] + V * (x->rho[c] - rt);
                }
                x->rho_t[c] = rt;
                double kap = x->rho[c] > 0.0 ? rt / x->rho[c] : 0.0;
                for (int m = 0; x->pm && m < x->nmat; m++)
                    x->mu_t[m][c] = rt == x->rho[c] ? x->mu[m][c] : x->mu[m][c] * kap;
            }
        }
    }
    x->rhoE = x->pml.placement ? x->rho_t : x->rho;
    for (int m = 0; m < ORC_MAX_MAT; m++) x->muE[m] = x->pml.placement ? x->mu_t[m] : x->mu[m];
}

/* Lagrangian density and outflow limiter of cell (i, j); outside the grid: void */
static double rhoL(const orc_ctx *x, int i, int j)
{
    int NR = x->NR;
    if (i < 0 || i >= NR || j < 0 || j >= x->NZ) return 0.0;
    return x->rhoE[CI(i, j)] / x->J[CI(i, j)];
}
/* closure 1: Lagrangian partial density of material m (mass per Lagrangian volume) */
static double muL(const orc_ctx *x, int m, int i, int j)
{
    int NR = x->NR;
    if (i < 0 || i >= NR || j < 0 || j >= x->NZ) return 0.0;
    return x->muE[m][CI(i, j)] / x->J[CI(i, j)];
}
static double lam_at(const orc_ctx *x, int i, int j)
{
    int NR = x->NR;
    if (i < 0 || i >= NR || j < 0 || j >= x->NZ) return 1.0;
    return x->lam[CI(i, j)];
}

/* (d) per face: volume swept by the face-mean Lagrangian velocity and the
 * donor-cell (upwind) mass flux -- eqs. (3)-(5). A donor never gives away
 * more than its Lagrangian volume: when the volume leaving a cell through its
 * four faces exceeds V^L, all its outflows are scaled by V^L / outflow. */
static void phase_faces(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
    double dt = x->dt;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i <= NR; i++) {
            double u = 0.5 * (x->vLr[NI(i, j)] + x->vLr[NI(i, j + 1)]);
            x->dVr[RF(i, j)] = dt * (area_r(x, i, j) * u);
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= NZ; j++) {
        for (int i = 0; i < NR; i++) {
            x->dVz[AF(i, j)] = dt * (x->awc[i] * x->vLz[NI(i, j)] + x->aec[i] * x->vLz[NI(i + 1, j)]);
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double O = (dmax(-x->dVr[RF(i, j)], 0.0) + dmax(x->dVr[RF(i + 1, j)], 0.0))
                     + (dmax(-x->dVz[AF(i, j)], 0.0) + dmax(x->dVz[AF(i, j + 1)], 0.0));
            double VL = vol_c(x, i, j) * x->J[c];
            x->outv[c] = O;
            x->lam[c] = O > VL ? dmax(VL, 0.0) / O : 1.0;
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i <= NR; i++) {
            double dV = x->dVr[RF(i, j)], e = 0.0, F = 0.0;
            int di = i;
            if (dV > 0.0) {
                di = i - 1;
                e = dV * lam_at(x, i - 1, j);
                F = e * rhoL(x, i - 1, j);
            } else if (dV < 0.0) {
                e = dV * lam_at(x, i, j);
                F = e * rhoL(x, i, j);
            }
            if (x->pm) {
                /* closure 1: each material carries its own donor mass; the
                 * face's mass flux is their sum */
                F = 0.0;
                for (int m = 0; m < x->nmat; m++) {
                    double Fm = dV != 0.0 ? e * muL(x, m, di, j) : 0.0;
                    x->Fmr[m][RF(i, j)] = Fm;
                    F += Fm;
                }
            }
            x->dVre[RF(i, j)] = e;
            x->Fr[RF(i, j)] = F;
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= NZ; j++) {
        for (int i = 0; i < NR; i++) {
            double dV = x->dVz[AF(i, j)], e = 0.0, F = 0.0;
            int dj = j;
            if (dV > 0.0) {
                dj = j - 1;
                e = dV * lam_at(x, i, j - 1);
                F = e * rhoL(x, i, j - 1);
            } else if (dV < 0.0) {
                e = dV * lam_at(x, i, j);
                F = e * rhoL(x, i, j);
            }
            if (x->pm) {
                F = 0.0;
                for (int m = 0; m < x->nmat; m++) {
                    double Fm = dV != 0.0 ? e * muL(x, m, i, dj) : 0.0;
                    x->Fmz[m][AF(i, j)] = Fm;
                    F += Fm;
                }
            }
            x->dVze[AF(i, j)] = e;
            x->Fz[AF(i, j)] = F;
        }
    }
}

/* (e) per cell: conservative donor-cell remap back to the Eulerian cell of
 * mass, specific internal energy, deviatoric stress and volume fractions,
 * then the PML mass / energy damping with phi1, phi3 (Sec. 3) */
static void phase_cell_remap(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ, nm = x->nmat;
    double dt = x->dt;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double V = vol_c(x, i, j);
            /* faces W, E, S, N: flux (positive along +r / +z), donor cell, inflow flag */
            double F[4] = {x->Fr[RF(i, j)], x->Fr[RF(i + 1, j)], x->Fz[AF(i, j)], x->Fz[AF(i, j + 1)]};
            double dV[4] = {x->dVr[RF(i, j)], x->dVr[RF(i + 1, j)], x->dVz[AF(i, j)], x->dVz[AF(i, j + 1)]};
            double dVe[4] = {x->dVre[RF(i, j)], x->dVre[RF(i + 1, j)], x->dVze[AF(i, j)], x->dVze[AF(i, j + 1)]};
            int di[4] = {i - 1, i + 1, i, i}, dj[4] = {j, j, j - 1, j + 1};
            int in[4] = {dV[0] > 0.0, dV[1] < 0.0, dV[2] > 0.0, dV[3] < 0.0};
            double netin = (F[0] - F[1]) + (F[2] - F[3]);
            double rho1 = x->rhoE[c] + netin / V;
            /* closure 1: each partial density takes its own net inflow; rho is
             * their sum */
            double mu1[ORC_MAX_MAT], I1m[ORC_MAX_MAT], Fm[ORC_MAX_MAT][4];
            if (x->pm) {
                rho1 = 0.0;
                for (int m = 0; m < nm; m++) {
                    Fm[m][0] = x->Fmr[m][RF(i, j)];
                    Fm[m][1] = x->Fmr[m][RF(i + 1, j)];
                    Fm[m][2] = x->Fmz[m][AF(i, j)];
                    Fm[m][3] = x->Fmz[m][AF(i, j + 1)];
                    double nin = (Fm[m][0] - Fm[m][1]) + (Fm[m][2] - Fm[m][3]);
                    mu1[m] = x->muE[m][c] + nin / V;
                    rho1 += mu1[m];
                }
            }
            double M1 = rho1 * V;
            double IL = x->IL[c];
            double ed[4] = {0.0, 0.0, 0.0, 0.0}; /* energy flux through each face */
            /* per-face inflow terms (zero on outflow faces), summed below with
             * opposite faces paired */
            double tm[4] = {0}, tI[4] = {0}, tsrr[4] = {0}, tszz[4] = {0}, tsrz[4] = {0}, tcut[4] = {0};
            double tf[ORC_MAX_MAT][4] = {{0}};
            double tD[4] = {0}, tV[4] = {0};
            for (int q = 0; q < 4; q++) {
                int dc_ok = di[q] >= 0 && di[q] < NR && dj[q] >= 0 && dj[q] < NZ;
                int dc = dc_ok ? CI(di[q], dj[q]) : -1;
                if (in[q]) {
                    double aF = fabs(F[q]), adV = fabs(dVe[q]);
                    if (x->dmg) {
                        /* damage and vibration speed travel with the mass */
                        tD[q] = aF * ((dc_ok ? x->DL[dc] : 0.0) - x->DL[c]);
                        tV[q] = aF * ((dc_ok ? x->vibL[dc] : 0.0) - x->vibL[c]);
                    }
                    tcut[q] = fabs(dV[q]) - adV;
                    double Id = dc_ok ? x->IL[dc] : 0.0;
                    tm[q] = aF;
                    tI[q] = aF * (Id - IL);
                    tsrr[q] = aF * ((dc_ok ? x->sLrr[dc] : 0.0) - x->sLrr[c]);
                    tszz[q] = aF * ((dc_ok ? x->sLzz[dc] : 0.0) - x->sLzz[c]);
                    tsrz[q] = aF * ((dc_ok ? x->sLrz[dc] : 0.0) - x->sLrz[c]);
                    for (int m = 0; m < nm; m++)
                        tf[m][q] = adV * ((dc_ok ? x->fL[m][dc] : 0.0) - x->fL[m][c]);
                    ed[q] = F[q] * Id;
                } else {
                    ed[q] = F[q] * IL;
                }
            }
            double min_ = face_sum(tm), nI = face_sum(tI), vcut = face_sum(tcut);
            double nsrr = face_sum(tsrr), nszz = face_sum(tszz), nsrz = face_sum(tsrz);
            double nf[ORC_MAX_MAT] = {0.0, 0.0};
            for (int m = 0; m < nm; m++) nf[m] = face_sum(tf[m]);
            double den = dmax(dmax(M1, min_), M_REMAP_FLOOR * x->rho_ref * V);
            double I1 = IL + nI / den;
            if (x->dmg) {
                x->D_n[c] = x->DL[c] + face_sum(tD) / den;
                x->vib_n[c] = x->vibL[c] + face_sum(tV) / den;
            }
            x->srr_n[c] = x->sLrr[c] + nsrr / den;
            x->szz_n[c] = x->sLzz[c] + nszz / den;
            x->srz_n[c] = x->sLrz[c] + nsrz / den;
            double fs = 0.0;
            double f1[ORC_MAX_MAT];
            /* volume the limiter kept from leaving this cell, minus void that
             * arrived in place of limited inflow (both zero without limiting) */
            double ex = (1.0 - x->lam[c]) * x->outv[c] - vcut;
            for (int m = 0; m < nm; m++) {
                f1[m] = dmax(x->fL[m][c] + (nf[m] + x->fL[m][c] * ex) / V, 0.0);
                fs += f1[m];
            }
            for (int m = 0; m < nm; m++) x->f_n[m][c] = f1[m] / dmax(fs, 1.0);

            /* closure 1: each material's specific energy is remapped with its
             * own mass fluxes (donor values, as I above); the energy fluxes
             * are the sums over materials */
            if (x->pm) {
                for (int q = 0; q < 4; q++) ed[q] = 0.0;
                for (int m = 0; m < nm; m++) {
                    double ILc = x->ILm[m][c], tmm[4] = {0}, tIm[4] = {0};
                    for (int q = 0; q < 4; q++) {
                        int dc_ok = di[q] >= 0 && di[q] < NR && dj[q] >= 0 && dj[q] < NZ;
                        if (in[q]) {
                            double Id = dc_ok ? x->ILm[m][CI(di[q], dj[q])] : 0.0;
                            double aF = fabs(Fm[m][q]);
                            tmm[q] = aF;
                            tIm[q] = aF * (Id - ILc);
                            ed[q] += Fm[m][q] * Id;
                        } else {
                            ed[q] += Fm[m][q] * ILc;
                        }
                    }
                    double minm = face_sum(tmm), nIm = face_sum(tIm);
                    double denm = dmax(dmax(mu1[m] * V, minm), M_REMAP_FLOOR * x->rho_ref * V);
                    I1m[m] = ILc + nIm / denm;
                }
            }

            /* PML: damping of the fluctuation about the initial state plus the
             * unstretched-direction auxiliary terms; r-faces feed the bottom
             * layer's phi, z-faces feed the right layer's phi */
            double db = x->dcz[j], drr = x->dcr[i];
            if (db > 0.0 || drr > 0.0) {
                double dsum = db + drr;
                /* the layer is a sink that never leaves negative mass (ejecta
                 * crossing the void part of a layer violate the small-fluctuation
                 * assumption of the derivation) */
                /* the auxiliaries this step applies: phi1 and phi3, or only
                 * psi2 (on the energy) as printed */
                double a1 = x->pml.placement ? 0.0 : x->phi1b[c] + x->phi1r[c];
                double a3 = x->pml.placement ? x->psi2n[c] : x->phi3b[c] + x->phi3r[c];
                double rho2 = dmax(rho1 - dt * (dsum * (rho1 - x->rref[c]) + a1), 0.0);
                double rt_ = dmax(rho1, x->rho_ref * PML_RHO_FLOOR);
                double I2 = I1 - dt * (dsum * I1 + a3 / rt_);
                if (x->pml.form) {
                    /* rho I damped toward zero, then divided by the damped mass */
                    double e1 = rho1 * I1;
                    I2 = (e1 - dt * (dsum * e1 + a3)) / dmax(rho2, x->rho_ref * PML_RHO_FLOOR);
                }
                if (x->pm) {
                    /* every material loses the same fraction of its mass and
                     * the same specific energy */
                    double kap = rho1 > 0.0 ? rho2 / rho1 : 0.0;
                    double r2 = 0.0;
                    for (int m = 0; m < nm; m++) {
                        mu1[m] = mu1[m] * kap;
                        r2 += mu1[m];
                        I1m[m] = I1m[m] - dt * (dsum * I1m[m] + a3 / rt_);
                    }
                    rho2 = r2;
                }
                x->msink[c] = x->msink[c] + V * (rho1 - rho2);
                /* extension: the deviatoric stress relaxes toward its initial
                 * value (zero) at the layer's rate, like the velocity */
                if (x->pml.damp_stress) {
                    x->srr_n[c] = x->srr_n[c] - dt * (dsum * x->srr_n[c]);
                    x->szz_n[c] = x->szz_n[c] - dt * (dsum * x->szz_n[c]);
                    x->srz_n[c] = x->srz_n[c] - dt * (dsum * x->srz_n[c]);
                }
                if (db > 0.0) {
                    x->phi1b[c] = x->phi1b[c] + db * ((F[1] - F[0]) / V);
                    x->phi3b[c] = x->phi3b[c] + db * ((ed[1] - ed[0]) / V);
                }
                if (drr > 0.0) {
                    x->phi1r[c] = x->phi1r[c] + drr * ((F[3] - F[2]) / V);
                    x->phi3r[c] = x->phi3r[c] + drr * ((ed[3] - ed[2]) / V);
                }
                rho1 = rho2;
                I1 = I2;
            }
            x->rho_n[c] = rho1;
            x->I_n[c] = I1;
            for (int m = 0; x->pm && m < nm; m++) {
                x->mu_n[m][c] = mu1[m];
                x->Im_n[m][c] = I1m[m];
            }
            if (j == NZ - 1) {
                x->mout_col[i] += F[3];
                x->eout_col[i] += ed[3];
            }
        }
    }
}

/* (f) per node: momentum remap over the dual cell with dual mass fluxes built
 * as quarter-sums of the four neighbouring primal fluxes (eq. (4)), donor
 * velocity, PML phi2 and velocity damping (Sec. 3), boundary conditions */
static double Fr_at(const orc_ctx *x, int i, int j)
{
    int NR = x->NR;
    if (i < 0 || i > NR || j < 0 || j >= x->NZ) return 0.0;
    return x->Fr[RF(i, j)];
}
static double Fz_at(const orc_ctx *x, int i, int j)
{
    int NR = x->NR;
    if (i < 0 || i >= NR || j < 0 || j > x->NZ) return 0.0;
    return x->Fz[AF(i, j)];
}

static void phase_node_remap(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
    double dt = x->dt;
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= NZ; j++) {
        for (int i = 0; i <= NR; i++) {
            int n = NI(i, j);
            /* node mass: quarter of the four cell masses (SW, SE, NW, NE) */
            double M[4] = {0, 0, 0, 0};
            int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
            for (int q = 0; q < 4; q++) {
                if (qi[q] < 0 || qi[q] >= NR || qj[q] < 0 || qj[q] >= NZ) continue;
                M[q] = x->rhoE[CI(qi[q], qj[q])] * vol_c(x, qi[q], qj[q]);
            }
            double mL = 0.25 * ((M[0] + M[1]) + (M[2] + M[3]));
            /* dual faces W, E, S, N */
            double FD[4];
            FD[0] = 0.25 * ((Fr_at(x, i - 1, j - 1) + Fr_at(x, i, j - 1)) + (Fr_at(x, i - 1, j) + Fr_at(x, i, j)));
            FD[1] = 0.25 * ((Fr_at(x, i, j - 1) + Fr_at(x, i + 1, j - 1)) + (Fr_at(x, i, j) + Fr_at(x, i + 1, j)));
            FD[2] = 0.25 * ((Fz_at(x, i - 1, j - 1) + Fz_at(x, i, j - 1)) + (Fz_at(x, i - 1, j) + Fz_at(x, i, j)));
            FD[3] = 0.25 * ((Fz_at(x, i - 1, j) + Fz_at(x, i, j)) + (Fz_at(x, i - 1, j + 1) + Fz_at(x, i, j + 1)));
            if (i == 0) FD[0] = 0.0;
            if (i == NR) FD[1] = 0.0;
            if (j == 0) FD[2] = 0.0;
            int ni[4] = {i - 1, i + 1, i, i}, nj[4] = {j, j, j - 1, j + 1};
            int in[4] = {FD[0] > 0.0, FD[1] < 0.0, FD[2] > 0.0, FD[3] < 0.0};
            double m1 = mL + ((FD[0] - FD[1]) + (FD[2] - FD[3]));
            double vLr = x->vLr[n], vLz = x->vLz[n];
            double upr[4], upz[4], tm[4] = {0}, tr[4] = {0}, tz[4] = {0};
            for (int q = 0; q < 4; q++) {
                int ok = ni[q] >= 0 && ni[q] <= NR && nj[q] >= 0 && nj[q] <= NZ;
                if (in[q] && ok) {
                    int d = NI(ni[q], nj[q]);
                    double aF = fabs(FD[q]);
                    tm[q] = aF;
                    tr[q] = aF * (x->vLr[d] - vLr);
                    tz[q] = aF * (x->vLz[d] - vLz);
                    upr[q] = x->vLr[d];
                    upz[q] = x->vLz[d];
                } else {
                    upr[q] = vLr;
                    upz[q] = vLz;
                }
            }
            double min_ = face_sum(tm), nr = face_sum(tr), nz = face_sum(tz);
            double aE = i < NR ? x->awc[i] : 0.0;
            double aW = i > 0 ? x->aec[i - 1] : 0.0;
            double hN = j < NZ ? 0.5 * x->dzr[j] : 0.0;
            double hS = j > 0 ? 0.5 * x->dzr[j - 1] : 0.0;
            double Vd = (aE + aW) * (hN + hS);
            double den = dmax(dmax(m1, min_), M_REMAP_FLOOR * x->rho_ref * Vd);
            double v1r = vLr + nr / den;
            double v1z = vLz + nz / den;
            /* kinetic energy the donor-cell mixing destroyed, in shift-invariant
             * form (exactly zero for a uniform field, >= 0 by Cauchy-Schwarz),
             * returned as specific heat to the surrounding cells by mass */
            double tk[4] = {0};
            for (int q = 0; q < 4; q++) {
                int ok = ni[q] >= 0 && ni[q] <= NR && nj[q] >= 0 && nj[q] <= NZ;
                if (in[q] && ok) {
                    double ar = upr[q] - vLr, az = upz[q] - vLz;
                    tk[q] = fabs(FD[q]) * (ar * ar + az * az);
                }
            }
            double kin = face_sum(tk);
            double dKE = 0.5 * (kin - (nr * nr + nz * nz) / den);
            double Mq1[4] = {0, 0, 0, 0};
            for (int q = 0; q < 4; q++) {
                if (qi[q] < 0 || qi[q] >= NR || qj[q] < 0 || qj[q] >= NZ) continue;
                Mq1[q] = x->rho_n[CI(qi[q], qj[q])] * vol_c(x, qi[q], qj[q]);
            }
            double Mn = (Mq1[0] + Mq1[1]) + (Mq1[2] + Mq1[3]);
            x->heat[n] = Mn > M_REMAP_FLOOR * x->rho_ref * Vd ? dmax(dKE, 0.0) / Mn : 0.0;
            double db = x->dnz[j], drr = x->dnr[i];
            if (db > 0.0 || drr > 0.0) {
                double dsum = db + drr;
                double mt = dmax(m1, M_ACC_EPS * x->rho_ref * Vd);
                /* the auxiliary this step applies: phi2, or psi1 as printed */
                double pr = x->phi2b_r[n] + x->phi2r_r[n];
                double pz = x->phi2b_z[n] + x->phi2r_z[n];
                if (x->pml.placement) {
                    pr = x->psi1n_r[n];
                    pz = x->psi1n_z[n];
                }
                double v2r = v1r - dt * (dsum * v1r + (pr * Vd) / mt);
                double v2z = v1z - dt * (dsum * v1z + (pz * Vd) / mt);
                if (x->pml.form) {
                    /* m v damped toward zero, then divided by the damped node
                     * mass (a quarter of the four damped cell masses) */
                    double m2 = dmax(0.25 * Mn, M_ACC_EPS * x->rho_ref * Vd);
                    double pr1 = mt * v1r, pz1 = mt * v1z;
                    v2r = (pr1 - dt * (dsum * pr1 + pr * Vd)) / m2;
                    v2z = (pz1 - dt * (dsum * pz1 + pz * Vd)) / m2;
                }
                if (db > 0.0) {
                    x->phi2b_r[n] = x->phi2b_r[n] + db * ((FD[1] * upr[1] - FD[0] * upr[0]) / Vd);
                    x->phi2b_z[n] = x->phi2b_z[n] + db * ((FD[1] * upz[1] - FD[0] * upz[0]) / Vd);
                }
                if (drr > 0.0) {
                    x->phi2r_r[n] = x->phi2r_r[n] + drr * ((FD[3] * upr[3] - FD[2] * upr[2]) / Vd);
                    x->phi2r_z[n] = x->phi2r_z[n] + drr * ((FD[3] * upz[3] - FD[2] * upz[2]) / Vd);
                }
                v1r = v2r;
                v1z = v2z;
            }
            x->vr_n[n] = v1r;
            x->vz_n[n] = v1z;
        }
    }
    apply_bc(x, x->vr_n, x->vz_n);
}

/* (g) per cell: add the specific heat of the remap's kinetic-energy loss
 * from the four corner nodes */
static void phase_cell_heat(orc_ctx *x)
{
    int NR = x->NR, NZ = x->NZ;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < NZ; j++) {
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double h = (x->heat[NI(i, j)] + x->heat[NI(i + 1, j)]) + (x->heat[NI(i, j + 1)] + x->heat[NI(i + 1, j + 1)]);
            x->I_n[c] = x->I_n[c] + h;
            if (x->dmg) {
                /* block model: the vibration decays as exp(-dt / T) over the
                 * step and is excited to c_vib times the largest corner speed
                 * of the new velocities (volume-fraction weighted constants) */
                double phin = 0.0;
                for (int m = 0; m < x->nmat; m++) phin += x->f_n[m][c];
                double den = phin > PHI_EPS ? phin : PHI_EPS;
                double kdec = 0.0, cv = 0.0;
                for (int m = 0; m < x->nmat; m++) {
                    if (!x->m[m].damage) continue;
                    double w = x->f_n[m][c] / den;
                    kdec += w * (x->Tvib[m] > 0.0 ? exp_cw(-x->dt / x->Tvib[m]) : 0.0);
                    cv += w * x->m[m].c_vib;
                }
                int nd[4] = {NI(i, j), NI(i + 1, j), NI(i, j + 1), NI(i + 1, j + 1)};
                double u = 0.0;
                for (int q = 0; q < 4; q++)
                    u = dmax(u, sqrt(x->vr_n[nd[q]] * x->vr_n[nd[q]] + x->vz_n[nd[q]] * x->vz_n[nd[q]]));
                x->vib_n[c] = dmax(x->vib_n[c] * kdec, cv * u);
            }
            if (x->pm) {
                for (int m = 0; m < x->nmat; m++) x->Im_n[m][c] = x->Im_n[m][c] + h;
                derive_cell(x, x->mu_n, x->Im_n, x->rho_n, x->I_n, c);
            }
        }
    }
}

static void swap(double **a, double **b)
{
    double *t = *a;
    *a = *b;
    *b = t;
}

static int check_state(orc_ctx *x)
{
    int bad = 0, neg = 0;
    size_t NC = x->NC, NN = x->NN;
    double tol = -NEG_MASS_TOL * x->rho_ref;
    for (size_t c = 0; c < NC; c++) {
        double s = x->rho[c] + x->I[c] + x->srr[c] + x->szz[c] + x->srz[c];
        for (int m = 0; m < x->nmat; m++) s += x->f[m][c];
        for (int m = 0; x->pm && m < x->nmat; m++) s += x->mu[m][c] + x->Im[m][c];
        if (x->dmg) s += x->D[c] + x->vib[c];
        if (!isfinite(s)) bad = 1;
        if (x->rho[c] < tol) neg = 1;
    }
    for (size_t n = 0; n < NN; n++)
        if (!isfinite(x->vr[n] + x->vz[n])) bad = 1;
    if (bad) return ORC_E_NONFINITE;
    if (neg) return ORC_E_NEG_MASS;
    return ORC_OK;
}

static int one_cycle(orc_ctx *x)
{
    phase_cell_stress(x);
    phase_node_force(x);
    phase_cell_lagrange(x);
    phase_faces(x);
    phase_cell_remap(x);
    phase_node_remap(x);
    phase_cell_heat(x);
    swap(&x->rho, &x->rho_n);
    swap(&x->I, &x->I_n);
    for (int m = 0; m < x->nmat; m++) swap(&x->f[m], &x->f_n[m]);
    for (int m = 0; x->pm && m < x->nmat; m++) {
        swap(&x->mu[m], &x->mu_n[m]);
        swap(&x->Im[m], &x->Im_n[m]);
    }
    swap(&x->srr, &x->srr_n);
    swap(&x->szz, &x->szz_n);
    swap(&x->srz, &x->srz_n);
    if (x->dmg) {
        swap(&x->D, &x->D_n);
        swap(&x->vib, &x->vib_n);
    }
    swap(&x->vr, &x->vr_n);
    swap(&x->vz, &x->vz_n);
    x->t = x->t + x->dt;
    x->cycle += 1;
    int e = check_state(x);
    /* next time step: Courant limit, growth cap, maximum, stop time */
    double dt = dmin(dmin(dt_candidate_min(x), x->g.dt_grow * x->dt), x->g.dt_max);
    if (x->g.t_stop > 0) dt = dmin(dt, dmax(x->g.t_stop - x->t, 0.0));
    x->dt_prev = x->dt;
    x->dt = dt;
    int stopped = x->g.t_stop > 0 && x->t >= x->g.t_stop;
    if (e == ORC_OK && !stopped && dt < x->g.dt_floor) e = ORC_E_DT_FLOOR;
    return e;
}

int orc_step(orc_ctx *x, int32_t n)
{
    if (!x || n < 0) return ORC_E_INVALID;
    if (x->err) return x->err;
    for (int32_t k = 0; k < n; k++) {
        int e = one_cycle(x);
        if (e) {
            x->err = e;
            x->err_cycle = (int)x->cycle;
            return e;
        }
    }
    return ORC_OK;
}

int orc_get_fields(orc_ctx *x, double *rho, double *I, double *f, double *s, double *v,
                   double *p, double *c2)
{
    if (!x) return ORC_E_INVALID;
    size_t NC = x->NC, NN = x->NN;
    if (rho) memcpy(rho, x->rho, sizeof(double) * NC);
    if (I) memcpy(I, x->I, sizeof(double) * NC);
    if (f)
        for (int m = 0; m < x->nmat; m++) memcpy(f + m * NC, x->f[m], sizeof(double) * NC);
    if (s) {
        memcpy(s, x->srr, sizeof(double) * NC);
        memcpy(s + NC, x->szz, sizeof(double) * NC);
        memcpy(s + 2 * NC, x->srz, sizeof(double) * NC);
    }
    if (v) {
        memcpy(v, x->vr, sizeof(double) * NN);
        memcpy(v + NN, x->vz, sizeof(double) * NN);
    }
    if (p || c2) {
        for (size_t c = 0; c < NC; c++) {
            double pp, cc, G, Y, rm, phi, sx;
            cell_mixture(x, (int)c, &pp, &cc, &G, &Y, &rm, &phi, &sx, NULL, NULL);
            if (p) p[c] = pp;
            if (c2) c2[c] = cc;
        }
    }
    return ORC_OK;
}

int orc_get_pml(orc_ctx *x, double *ca, double *na)
{
    if (!x) return ORC_E_INVALID;
    size_t NC = x->NC, NN = x->NN;
    if (ca) {
        const double *src[8] = {x->phi1b, x->phi3b, x->psi2b, x->phi1r, x->phi3r, x->psi2r, x->rref, x->msink};
        for (int k = 0; k < 8; k++) memcpy(ca + k * NC, src[k], sizeof(double) * NC);
    }
    if (na) {
        const double *src[8] = {x->phi2b_r, x->phi2b_z, x->psi1b_r, x->psi1b_z,
                                x->phi2r_r, x->phi2r_z, x->psi1r_r, x->psi1r_z};
        for (int k = 0; k < 8; k++) memcpy(na + k * NN, src[k], sizeof(double) * NN);
    }
    return ORC_OK;
}

/* Inverse of orc_get_pml: the PML auxiliary fields, reference density and
 * sink of the current state, in the same full-grid layouts. */
int orc_set_pml(orc_ctx *x, const double *ca, const double *na)
{
    if (!x) return ORC_E_INVALID;
    size_t NC = x->NC, NN = x->NN;
    if (ca) {
        double *dst[8] = {x->phi1b, x->phi3b, x->psi2b, x->phi1r, x->phi3r, x->psi2r, x->rref, x->msink};
        for (int k = 0; k < 8; k++) memcpy(dst[k], ca + k * NC, sizeof(double) * NC);
    }
    if (na) {
        double *dst[8] = {x->phi2b_r, x->phi2b_z, x->psi1b_r, x->psi1b_z,
                          x->phi2r_r, x->phi2r_z, x->psi1r_r, x->psi1r_z};
        for (int k = 0; k < 8; k++) memcpy(dst[k], na + k * NN, sizeof(double) * NN);
    }
    return ORC_OK;
}

/* Time of the state and the step of the next cycle (Sec. 7's step is chosen
 * at the end of the cycle before; a continued run takes it over). */
int orc_set_clock(orc_ctx *x, double t, double dt)
{
    if (!x || !isfinite(t) || t < 0.0 || !isfinite(dt) || !(dt > 0.0) || dt > x->g.dt_max)
        return ORC_E_INVALID;
    if (x->g.t_stop > 0 && dt > x->g.t_stop - t) return ORC_E_INVALID;
    x->t = t;
    x->dt = dt;
    return ORC_OK;
}

int orc_get_profiles(orc_ctx *x, double *dcz, double *dnz, double *dcr, double *dnr)
{
    if (!x) return ORC_E_INVALID;
    if (dcz) memcpy(dcz, x->dcz, sizeof(double) * x->NZ);
    if (dnz) memcpy(dnz, x->dnz, sizeof(double) * (x->NZ + 1));
    if (dcr) memcpy(dcr, x->dcr, sizeof(double) * x->NR);
    if (dnr) memcpy(dnr, x->dnr, sizeof(double) * (x->NR + 1));
    return ORC_OK;
}

/* compensated (Neumaier) summation in a fixed order */
typedef struct {
    double s, c;
} ksum;
static void kadd(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static double kval(const ksum *k) { return k->s + k->c; }

int orc_diag(orc_ctx *x, double *out)
{
    if (!x || !out) return ORC_E_INVALID;
    int NR = x->NR, NZ = x->NZ;
    ksum mass = {0, 0}, ie = {0, 0}, ke = {0, 0}, mo = {0, 0}, mp = {0, 0}, eo = {0, 0};
    for (int j = 0; j < NZ; j++)
        for (int i = 0; i < NR; i++) {
            int c = CI(i, j);
            double M = x->rho[c] * vol_c(x, i, j);
            kadd(&mass, M);
            kadd(&ie, M * x->I[c]);
            kadd(&mp, x->msink[c]);
        }
    for (int j = 0; j <= NZ; j++)
        for (int i = 0; i <= NR; i++) {
            double M = 0.0;
            int qi[4] = {i - 1, i, i - 1, i}, qj[4] = {j - 1, j - 1, j, j};
            double Mq[4] = {0, 0, 0, 0};
            for (int q = 0; q < 4; q++) {
                if (qi[q] < 0 || qi[q] >= NR || qj[q] < 0 || qj[q] >= NZ) continue;
                Mq[q] = x->rho[CI(qi[q], qj[q])] * vol_c(x, qi[q], qj[q]);
            }
            M = 0.25 * ((Mq[0] + Mq[1]) + (Mq[2] + Mq[3]));
            int n = NI(i, j);
            kadd(&ke, 0.5 * M * (x->vr[n] * x->vr[n] + x->vz[n] * x->vz[n]));
        }
    for (int i = 0; i < NR; i++) {
        kadd(&mo, x->mout_col[i]);
        kadd(&eo, x->eout_col[i]);
    }
    out[0] = x->t;
    out[1] = x->dt;
    out[2] = (double)x->cycle;
    out[3] = kval(&mass);
    out[4] = kval(&ie);
    out[5] = kval(&ke);
    out[6] = kval(&mo);
    out[7] = kval(&mp);
    out[8] = kval(&eo);
    out[9] = (double)x->err;
    out[10] = (double)x->err_cycle;
    out[11] = x->dt_prev;
    return ORC_OK;
}
