/*
 * salec_oracle.h -- C interface of the plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. The oracle is the slow,
 * obviously-correct reference the HIP library is checked against. Only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or helper with the HIP library.
 *
 * Method: Li et al., "Parallel numerical simulation of impact crater with
 * perfect matched layers" (SALEc-2D), Sec. 2 eqs. (1)-(5) (SALE operator
 * split), Sec. 3 (PML), Sec. 4 (boundary conditions), Table 1 (strength
 * parameters), Sec. 7 (Courant condition). Every point where the paper is
 * silent is resolved by the readings listed in the repository's design notes;
 * the oracle and the HIP path follow the same readings.
 *
 * Layout: cell (i, j) with i = 0..NR-1 outward from the symmetry axis and
 * j = 0..NZ-1 upward from the bottom is element j*NR + i. Node (i, j),
 * i = 0..NR, j = 0..NZ, is element j*(NR+1) + i. NR = n_r + pml_r,
 * NZ = n_z + pml_b. All quantities are SI; volumes and areas are per radian.
 */
#ifndef SALEC_ORACLE_H
#define SALEC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAX_MAT 3

/* error codes (negative), shared meaning with the product library */
#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_NONFINITE (-4)
#define ORC_E_NEG_MASS (-5)
#define ORC_E_DT_FLOOR (-6)

typedef struct {
    int32_t n_r, n_z;   /* physical cells in r and z                        */
    int32_t pml_r;      /* PML cells to the right of the physical region    */
    int32_t pml_b;      /* PML cells below the physical region              */
    int32_t nmat;       /* 1 to 3 materials                                 */
    int32_t top_closed; /* 0: open (outflow) top, 1: rigid top wall         */
    int32_t closure;    /* mixed cells: 0 shared material density and      */
                        /* specific energy, 1 per-material density and      */
                        /* specific energy (partial densities advected)     */
    double dr, dz;      /* cell size, m                                     */
    double cfl;         /* Courant constant C0                               */
    double dt_grow;     /* max growth factor of dt per cycle                */
    double dt_max, dt_floor;
    double t_stop;      /* >0: clip the step so that t never passes t_stop  */
    double q_lin, q_quad; /* artificial viscosity coefficients C1, C2       */
    /* stretched grid (Table 2's extension zones): per-column widths (NR
     * values) and per-row heights (NZ values), or NULL for uniform dr / dz */
    const double *dr_col, *dz_row;
} orc_grid;

typedef struct {
    double rho0, A, B, E0, a, b, alpha, beta, Eiv, Ecv; /* Tillotson       */
    double p_min;        /* pressure floor, Pa                              */
    double c_floor_frac; /* c^2 floor = c_floor_frac * A / rho0             */
    int32_t strength;    /* 0: hydrodynamic, 1: elasto-plastic              */
    double Y0, mu_f, Ylim, poisson;
    /* Damage and acoustic fluidization (Table 1's damaged-material and
     * block-model constants; the equations are readings, see the source):
     * with damage = 1 the yield strength blends from the intact curve to the
     * damaged one, Y_d = min(Yd0 + mu_d p, Ydm) (never above the intact), by
     * the cell's damage D, which grows by the plastic strain of the radial
     * return over the failure strain max(eps_fb, B_dmg (p - p_bd)); the
     * damaged friction sees the pressure less the vibration pressure
     * rho c v_vib of the block model, whose vibration speed decays with time
     * constant gamma_T h / c and is excited to c_vib times the local flow
     * speed, and whose viscosity gamma_eta rho c h resists the flow of
     * damaged, vibrating rock (c: longitudinal speed at rest, h: block size) */
    int32_t damage;
    double Yd0, mu_d, Ydm;
    double eps_fb, B_dmg, p_bd;
    double gamma_eta, gamma_T, c_vib, af_h;
} orc_mat;

typedef struct {
    int32_t enabled;
    int32_t damp_stress; /* 1: the layers also relax the deviatoric stress */
                         /* toward zero at the rate d (an extension: Sec. 3 */
                         /* damps mass, momentum and energy only)           */
    double R;     /* theoretical reflection coefficient                    */
    double c_ref; /* <=0: the largest longitudinal speed at rest over the  */
                  /* materials                                             */
    /* Which step applies each auxiliary (Sec. 3 names psi1, psi2 for the
     * Eulerian step and phi1, phi2, phi3 for the Lagrangian step):
     *   0 (derived): psi1 in the node force, psi2 in the Lagrangian energy,
     *     phi1, phi3 in the cell remap, phi2 in the momentum remap;
     *   1 (as printed): phi2 in the node force, phi1 on the mass and phi3 on
     *     the energy at the end of the Lagrangian step, psi2 in the cell
     *     remap, psi1 in the momentum remap.
     * Every application uses the auxiliary's value at the start of the cycle. */
    int32_t placement;
    /* Damped quantity of the momentum and energy equations:
     *   0: the specific velocity and energy (v -= dt (d v + ...), I likewise);
     *   1: the conserved densities as Sec. 3 prints them (rho v, rho I damped,
     *      then divided by the damped mass). Oracle only, placement 0 and the
     *      shared closure only; it pins that the two forms differ at second
     *      order in the fluctuation. */
    int32_t form;
} orc_pml;

typedef struct {
    int32_t surface_j;  /* first void row above the target                  */
    int32_t subsample;  /* S x S sub-samples per cell for the disc fraction */
    double radius;      /* projectile radius, m (0: no projectile)          */
    double v_imp;       /* impact speed, m/s (downwards)                    */
    double gravity;     /* g, m/s^2 (0: no lithostatic pressure)            */
    int32_t layer_j;    /* rows below it are material 1 (nmat >= 2), the    */
                        /* rows from it up to the surface material 0        */
    int32_t layer2_j;   /* nmat = 3: rows below it are material 2           */
                        /* (<= layer_j); the projectile is material nmat-1  */
} orc_scene;

typedef struct orc_ctx orc_ctx;

orc_ctx *orc_create(const orc_grid *g, const orc_mat *mats, const orc_pml *pml);
void orc_destroy(orc_ctx *x);
int orc_set_threads(int n); /* OpenMP thread count; returns threads in use */

int orc_init_scene(orc_ctx *x, const orc_scene *s);
/* f: nmat*NC values (material-major); s: 3*NC (rr, zz, rz) or NULL;
 * v: 2*NN (r then z). Starts a new run at t = 0. */
int orc_set_fields(orc_ctx *x, const double *rho, const double *I,
                   const double *f, const double *s, const double *v);
/* initial pressure p0 per cell row (NZ values, Pa): the momentum balance
 * and the PML's psi1 use p - p0 (Sec. 3 momentum equation with -grad p0 +
 * rho g = 0). Zero unless a scene with gravity or this call sets it; kept
 * across orc_set_fields. */
int orc_set_p0(orc_ctx *x, const double *p0);
/* per-material state (closure 1): mu = partial densities (mass of material m
 * per cell volume, nmat*NC, material-major), Im = specific internal energies
 * (nmat*NC). Setting them also sets rho = sum of mu and I = the mass-weighted
 * energy; orc_set_fields in this mode gives every material of a cell the
 * cell's matter density and its specific energy. */
int orc_set_materials(orc_ctx *x, const double *mu, const double *Im);
int orc_get_materials(orc_ctx *x, double *mu, double *Im);
int orc_get_p0(orc_ctx *x, double *p0);
/* damage D and block-model vibration speed v_vib per cell (NC values each;
 * zero after orc_set_fields and orc_init_scene); either pointer may be NULL */
int orc_set_damage(orc_ctx *x, const double *D, const double *vib);
int orc_get_damage(orc_ctx *x, double *D, double *vib);
int orc_step(orc_ctx *x, int32_t n);
/* any pointer may be NULL; p and c2 are evaluated from the current state */
int orc_get_fields(orc_ctx *x, double *rho, double *I, double *f, double *s,
                   double *v, double *p, double *c2);
/* cell_aux: 8*NC = phi1_b, phi3_b, psi2_b, phi1_r, phi3_r, psi2_r, rho_ref, msink
 * node_aux: 8*NN = phi2_b(r,z), psi1_b(r,z), phi2_r(r,z), psi1_r(r,z) */
int orc_get_pml(orc_ctx *x, double *cell_aux, double *node_aux);
/* Continuing a run: the PML auxiliaries (layouts of orc_get_pml) and the
 * clock (t, and the dt of the next cycle) of a state set with
 * orc_set_fields / orc_set_materials, which start a run at t = 0. */
int orc_set_pml(orc_ctx *x, const double *cell_aux, const double *node_aux);
int orc_set_clock(orc_ctx *x, double t, double dt);
/* out[0..11]: t, dt, cycle, mass, internal energy, kinetic energy,
 * mass_out, mass_pml, ie_out, err, err_cycle, dt_prev */
int orc_diag(orc_ctx *x, double *out);
/* damping profiles: dcz[NZ], dnz[NZ+1], dcr[NR], dnr[NR+1] */
int orc_get_profiles(orc_ctx *x, double *dcz, double *dnz, double *dcr, double *dnr);

/* point functions, exposed for the pins */
double orc_exp(double x);
void orc_tillotson(const orc_mat *m, double rho, double e, double *p, double *c2);
double orc_yield(const orc_mat *m, double p);
double orc_shear_modulus(const orc_mat *m);
/* strength factor in [0, 1] from the specific internal energy */
double orc_softening(const orc_mat *m, double e);
/* yield strength of damage D at pressure p and vibration pressure p_vib
 * (before softening; the intact curve when damage is off) */
double orc_yield_damaged(const orc_mat *m, double p, double D, double p_vib);
/* failure strain max(eps_fb, B_dmg (p - p_bd)) of the damage law */
double orc_failure_strain(const orc_mat *m, double p);
/* one constitutive update: s[3] in/out, rates = (e_rr, e_zz, e_tt, e_rz, omega) */
void orc_stress_update(double G, double Y, double dt, const double *rates, double *s);
/* strain rates of cell (i, j) from its four node velocities
 * vr[4], vz[4] ordered SW, SE, NW, NE -> out = (e_rr, e_zz, e_tt, e_rz, omega, D) */
void orc_cell_kinematics(const orc_grid *g, int32_t i, int32_t j, const double *vr,
                         const double *vz, double *out);
/* geometry tables: r_node[NR+1], r_cell[NR], z_node[NZ+1], z_cell[NZ] */
int orc_get_geometry(orc_ctx *x, double *r_node, double *r_cell, double *z_node, double *z_cell);

#ifdef __cplusplus
}
#endif
#endif
