/*
 * salec.h -- C ABI of libsalec: the per-cycle grid update of a SALE-type
 * axisymmetric (r-z) impact hydrocode with perfectly matched layers, on one
 * AMD Instinct MI355X (gfx950).
 *
 * Method (Li et al., "Parallel numerical simulation of impact crater with
 * perfect matched layers"): each cycle is the SALE operator split of Sec. 2 --
 * a Lagrangian step for momentum and internal energy (eqs. (1)-(2)) followed by
 * an Eulerian advection step for mass, momentum and energy (eqs. (3)-(5)) --
 * with the PML auxiliary variables and damping of Sec. 3 in the right and
 * bottom layers, the boundary conditions of Sec. 4 (free-slip symmetry axis
 * and outer side, no-slip bottom, open top) and the Courant time step of
 * Sec. 7. Material laws: Tillotson equation of state and the pressure-
 * dependent intact-rock strength whose parameters Table 1 lists.
 *
 * Conventions
 *   Cell (i, j): i = 0..NR-1 outward from the axis, j = 0..NZ-1 upward, with
 *   NR = n_r + pml_r and NZ = n_z + pml_b. Node (i, j): i = 0..NR, j = 0..NZ.
 *   Host arrays exchanged through this ABI are FP64, row-major with r
 *   fastest: cells NZ x NR, nodes (NZ+1) x (NR+1). SI units; volumes and
 *   areas per radian.
 *
 * Ownership
 *   Device memory is owned by the caller: salec_plan() gives the byte count,
 *   the caller allocates it (e.g. a torch uint8 tensor on the GPU) and passes
 *   its address to salec_init(); the library never allocates device memory
 *   and the caller keeps the buffer alive until salec_destroy(). The stream
 *   (a hipStream_t, or NULL for the default stream) is also the caller's.
 *   Host arrays are owned by the caller and only read/written during a call.
 *   A context may be used by one host thread at a time.
 *
 * Errors
 *   Every int-returning call returns SALEC_OK (0) or a negative code. Device-
 *   detected errors (non-finite field, negative mass, collapsed time step)
 *   are sticky: salec_step() returns them until a new state is set with
 *   salec_set_fields(), salec_init() or salec_set_state(); the state after
 *   such an error is undefined. salec_last_error() returns a message for the
 *   most recent failure of the context.
 */
#ifndef SALEC_H
#define SALEC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SALEC_OK 0
#define SALEC_E_INVALID (-1)   /* bad sizes or parameters                       */
#define SALEC_E_BUFFER (-2)    /* device buffer or host blob too small          */
#define SALEC_E_HIP (-3)       /* HIP runtime error (message in last_error)      */
#define SALEC_E_NONFINITE (-4) /* a field became NaN or infinite                 */
#define SALEC_E_NEG_MASS (-5)  /* a density fell below -1e-9 rho_ref             */
#define SALEC_E_DT_FLOOR (-6)  /* the time step fell below dt_floor              */

#define SALEC_FP64 0  /* every field and all arithmetic in FP64                  */
#define SALEC_MIXED 1 /* FP32 stencil, EoS, stress and velocity arithmetic and
                         storage; FP64 density, volume fractions, internal
                         energy, every mass / volume / energy flux and its sums,
                         and the Courant reduction                               */

#define SALEC_MAX_MAT 3

/* Closure of mixed cells (a reading of Sec. 2's volume-fraction cells; the
 * paper's layered target mixes materials with different equations of state):
 *  SALEC_CLOSURE_SHARED: the materials of a cell share one material density
 *    rho / phi and one specific energy I; the cell pressure is the
 *    volume-fraction average of the materials' pressures at that state.
 *  SALEC_CLOSURE_PER_MATERIAL: each material keeps its partial density mu_m
 *    (its mass per cell volume) and its specific energy I_m. Its equation of
 *    state sees rho_m = mu_m / f_m (below a volume fraction of 1e-6, or
 *    without mass, the cell's matter density) and I_m; the cell pressure is
 *    the same volume-fraction average. In the Lagrangian step every material
 *    does the deviatoric work and its own p dV work on the cell's volume
 *    change; in the remap (eqs. (3)-(5)) each material carries its own donor
 *    mass and energy through the face's volume flux, and the face mass flux
 *    is their sum. rho and I hold sum(mu_m) and the mass-weighted energy. A
 *    material absent from a cell (f_m = 0) has no pressure there. Every
 *    member of a context uses the same closure. */
#define SALEC_CLOSURE_SHARED 0
#define SALEC_CLOSURE_PER_MATERIAL 1

typedef struct salec_grid {
    int32_t n_r, n_z;    /* physical cells in r and z (>= 1)                      */
    int32_t pml_r;       /* PML cells right of the physical region (>= 0)        */
    int32_t pml_b;       /* PML cells below the physical region (>= 0)           */
    int32_t nmat;        /* 1 to 3 materials                                     */
    int32_t top_closed;  /* 0: open top (void ghost), 1: rigid top wall          */
    int32_t precision;   /* SALEC_FP64 or SALEC_MIXED                            */
    int32_t closure;     /* mixed cells: SALEC_CLOSURE_SHARED or                 */
                         /* SALEC_CLOSURE_PER_MATERIAL (see below)               */
    double dr, dz;       /* cell size, m (> 0)                                   */
    double cfl;          /* Courant constant C0 in (0, 1] (Sec. 7)               */
    double dt_grow;      /* largest dt growth factor per cycle (>= 1)            */
    double dt_max;       /* largest time step, s                                 */
    double dt_floor;     /* dt below this is an error (0 disables)               */
    double t_stop;       /* > 0: the step is clipped so t never passes t_stop    */
    double q_lin, q_quad;/* artificial viscosity coefficients C1, C2 (>= 0)       */
    /* Stretched grid (Table 2's extension zones), or NULL for uniform dr / dz:
     * dr_col[NR] column widths outward from the axis, dz_row[NZ] row heights
     * upward from the bottom (m, > 0, host arrays read at init). Node radii
     * and heights are their running sums, cell centres halfway between. */
    const double *dr_col, *dz_row;
} salec_grid;

typedef struct salec_material {
    double rho0, A, B, E0, a, b, alpha, beta, Eiv, Ecv; /* Tillotson constants  */
    double p_min;        /* pressure floor, Pa                                   */
    double c_floor_frac; /* c^2 >= c_floor_frac * A / rho0                       */
    int32_t strength;    /* 0: hydrodynamic, 1: elasto-plastic (Table 1 form)     */
    int32_t damage;      /* 0: intact strength only; 1: damage and the block     */
                         /* model of acoustic fluidization (needs strength;      */
                         /* the fields below; Table 1 lists their parameters     */
                         /* and the paper gives no equations, so the laws are    */
                         /* the library's documented readings)                   */
    double Y0, mu_f, Ylim, poisson; /* cohesion, friction, limit strength, nu   */
    /* damage = 1 only: the yield blends (1 - D) Y_intact(p) + D Y_damaged,     */
    /* Y_damaged = min(Yd0 + mu_d max(p - p_vib, 0), Ydm) for p >= 0 (never     */
    /* above the intact curve), and D (per cell, in [0, 1], advected with the   */
    /* mass) grows by the radial return's plastic strain (trial - Y) / 3G over  */
    /* the failure strain max(eps_fb, B_dmg (p - p_bd))                         */
    double Yd0, mu_d, Ydm;  /* damaged cohesion (Pa), friction, limit (Pa)      */
    double eps_fb;       /* failure strain of brittle rock (> 0)                 */
    double B_dmg;        /* its growth with pressure, 1/Pa (>= 0)                */
    double p_bd;         /* brittle-ductile transition pressure, Pa              */
    /* block model: a vibration speed v_vib per cell decays as exp(-dt / T),   */
    /* T = gamma_T h / c, is excited to c_vib times the largest corner speed,   */
    /* relieves the damaged friction by p_vib = rho c v_vib, and the viscosity  */
    /* rho gamma_eta c h raises the flow stress of damaged, vibrating rock by   */
    /* 3 eta times its equivalent strain rate (c: longitudinal speed at rest)   */
    double gamma_eta, gamma_T, c_vib; /* >= 0 each (zeros: no fluidization)     */
    double af_h;         /* block size h, m (> 0 when gamma_eta or gamma_T > 0)  */
} salec_material;

typedef struct salec_pml {
    int32_t enabled;     /* 0: plain walls, 1: damping layers (Sec. 3)           */
    int32_t damp_stress; /* 0: Sec. 3's layers (mass, momentum and energy are    */
                         /* damped); 1: an extension that also relaxes the       */
                         /* deviatoric stress toward zero at the layer's rate d  */
                         /* (s -= dt d s after the remap), which absorbs the     */
                         /* elastic shear waves of strong, confined rock         */
    double R;            /* theoretical reflection coefficient (0, 1)            */
    double c_ref;        /* damping speed c of Sec. 3's profile (the largest     */
                         /* acoustic speed); <= 0: the largest longitudinal      */
                         /* speed at rest over the materials                     */
    int32_t placement;   /* which step applies each auxiliary variable of        */
                         /* Sec. 3 (every application uses its value at the      */
                         /* start of the cycle):                                 */
                         /* 0 (derived from the auxiliaries' definitions): psi1  */
                         /*   in the node force and psi2 in the internal energy  */
                         /*   of the Lagrangian step; phi1, phi3 in the cell     */
                         /*   remap and phi2 in the momentum remap (Eulerian);   */
                         /* 1 (Sec. 3's sentence as printed: psi1, psi2 in the   */
                         /*   Eulerian step, phi1, phi2, phi3 in the Lagrangian  */
                         /*   step): phi2 in the node force; phi1 on the mass    */
                         /*   and phi3 on the energy at the end of the Lagrangian */
                         /*   step (the remap starts from that mass; the sink    */
                         /*   budget records it); psi2 in the cell remap, psi1   */
                         /*   in the momentum remap                              */
    int32_t reserved;    /* must be 0                                            */
} salec_pml;

typedef struct salec_scene {
    int32_t surface_j;   /* first void row above the target half-space           */
    int32_t subsample;   /* S x S sub-samples per cell for the sphere's fraction  */
    double radius;       /* projectile radius, m (0: no projectile)              */
    double v_imp;        /* vertical impact speed, m/s (downwards)               */
    double gravity;      /* g, m/s^2; > 0: lithostatic target (see below)        */
    int32_t layer_j;     /* two or three materials: target rows below it are     */
                         /* material 1, rows from it up to the surface material 0 */
    int32_t layer2_j;    /* three materials: rows below it are material 2        */
                         /* (<= layer_j; 0 otherwise). The projectile is the last */
                         /* material, that of the deepest layer.                  */
} salec_scene;

/* Host FP64 arrays; any pointer may be NULL to skip that field.
 *   rho, I, p, c2 : NZ*NR        f : nmat*NZ*NR (material-major)
 *   s             : 3*NZ*NR (s_rr, s_zz, s_rz)       v : 2*(NZ+1)*(NR+1) (v_r, v_z)
 * p and c2 are outputs only (evaluated from the state). */
typedef struct salec_fields {
    double *rho, *I, *f, *s, *v, *p, *c2;
} salec_fields;

typedef struct salec_diag {
    double t, dt, dt_prev;
    int64_t cycle;
    double mass, ie, ke;   /* compensated totals: sum rho V, sum rho V I, node KE */
    double mass_out, mass_pml, ie_out; /* outflow through the top, PML sink      */
    int32_t err, err_cycle;
} salec_diag_t;

/* One member of an ensemble (salec_init_batch). Every member of a context
 * uses the same precision. scene is used when has_scene != 0. */
typedef struct salec_instance {
    salec_grid grid;
    salec_material mats[SALEC_MAX_MAT];
    salec_pml pml;
    salec_scene scene;
    int32_t has_scene;
    int32_t reserved;    /* must be 0                                            */
} salec_instance;

/* Launch schedule of the cycle kernel: tile shape (cells per workgroup tile,
 * threads per workgroup), workgroups per launch and the time the tuner
 * measured for it (0 if not timed). */
typedef struct salec_schedule {
    int32_t variant;     /* index of the tile shape, 0 .. salec_num_variants()-1 */
    int32_t tile_r, tile_z, threads;
    int32_t grid;        /* workgroups per launch (0: one per tile)              */
    int32_t reserved;
    double ms_per_cycle; /* measured by salec_tune(), else 0                     */
} salec_schedule;

typedef struct salec_ctx salec_ctx;

/* Bytes of device memory salec_init() needs for this problem (the grid with
 * its PML zones of Table 2, the materials of Table 1, the layers of Sec. 3);
 * 0 if invalid. */
size_t salec_plan(const salec_grid *grid, const salec_material *mats, const salec_pml *pml);

/* Sets up the problem Sec. 4 states (a vertical impact of a sphere on a
 * target half-space with PML layers right and below, Table 2), with Table 1's
 * strength, the equation of state of Sec. 2 and the damping profile of
 * Sec. 3. Lays out the state in dev_buf (dev_bytes >= salec_plan(), 256-byte
 * aligned), uploads the constants and, if scene is not NULL, builds the
 * impact scene (target half-space of material 0, spherical projectile of
 * material nmat-1) on the device; otherwise the state is zero until
 * salec_set_fields(). Computes the first time step (Sec. 7's Courant
 * condition). SALEC_E_INVALID for a bad description (message in
 * salec_last_error), SALEC_E_BUFFER for a small or misaligned buffer,
 * SALEC_E_HIP for a runtime error; *out is set in every case but a null
 * argument and must be passed to salec_destroy(). stream: hipStream_t or
 * NULL (a stream of the library's own is created). A context made here is
 * an ensemble of one: instance index 0 below. */
int salec_init(const salec_grid *grid, const salec_material *mats, const salec_pml *pml,
               const salec_scene *scene, void *dev_buf, size_t dev_bytes, void *stream,
               salec_ctx **out);

/* Ensembles: n >= 1 independent impacts of any sizes, each the problem of
 * Sec. 4 as salec_init describes it (the paper runs one impact at a time;
 * ensembles are an extension), advanced together, one kernel launch per
 * cycle for all of them (captured in HIP graphs); each member keeps its own
 * time step (Sec. 7), time and cycle count and its own sticky error. Same
 * ownership, layout and error rules as salec_plan/salec_init; instance
 * indices below are 0..n-1. */
size_t salec_plan_batch(const salec_instance *inst, int32_t n);
int salec_init_batch(const salec_instance *inst, int32_t n, void *dev_buf, size_t dev_bytes,
                     void *stream, salec_ctx **out);
int32_t salec_num_instances(const salec_ctx *ctx);

/* Advances every member n >= 0 cycles of Sec. 2's operator split: the
 * Lagrangian step (eqs. (1)-(2): stress divergence, velocity, internal energy
 * with the Table 1 strength model), then the Eulerian step (eqs. (3)-(5):
 * advection of mass, momentum and energy), with Sec. 3's PML control
 * equations in the layers, Sec. 4's boundary conditions, and the next time
 * step from Sec. 7's Courant condition. Replays captured HIP graphs, then
 * synchronises the stream once and returns the first sticky device error
 * among the members, if any (members without an error keep advancing);
 * SALEC_E_INVALID for a null context or n < 0, SALEC_E_HIP for a runtime
 * error. */
int salec_step(salec_ctx *ctx, int32_t n);

/* The cycles of salec_step() (same passages), enqueued without
 * synchronising or checking errors (for timing loops); errors surface at the
 * next salec_step() or salec_diag(). */
int salec_enqueue(salec_ctx *ctx, int32_t n);

/* Copies the current state of member `instance` -- the variables of Sec. 2's
 * conservation equations: density, specific internal energy, volume
 * fractions, deviatoric stress tau, node velocity -- and, if requested, the
 * pressure and squared sound speed of the equation of state at that state, to
 * host FP64 arrays (layout above; the mixed mode's FP32 fields are widened).
 * SALEC_E_INVALID for a bad context, instance or pointer. */
int salec_get_fields(salec_ctx *ctx, int32_t instance, const salec_fields *out);

/* Replaces the state of member `instance` with host arrays (rho, I, f, v
 * required; s optional, zero if NULL) and starts a new run of that member at
 * t = 0: PML auxiliaries and budgets are cleared, the PML reference density
 * (the initial state Sec. 3 measures the fluctuation against) is taken from
 * rho, dt recomputed by Sec. 7's condition, its error cleared.
 * SALEC_E_INVALID for a bad context, instance or pointer (the values are
 * not checked; a non-finite one surfaces as SALEC_E_NONFINITE at the next
 * cycle). */
int salec_set_fields(salec_ctx *ctx, int32_t instance, const salec_fields *in);

/* The auxiliary variables phi1, phi2, phi3, psi1, psi2 of Sec. 3 (one set
 * per damped direction), the reference density and the mass sink of member
 * `instance`, expanded to full grids (zero outside the layers):
 *   cell_aux 8*NZ*NR: phi1_b, phi3_b, psi2_b, phi1_r, phi3_r, psi2_r, rho_ref, msink
 *   node_aux 8*(NZ+1)*(NR+1): phi2_b (r, z), psi1_b (r, z), phi2_r (r, z), psi1_r (r, z) */
int salec_get_pml(salec_ctx *ctx, int32_t instance, double *cell_aux, double *node_aux);

/* Continuing a run in another context (same problem, possibly another
 * precision), e.g. an FP64 start handed to the mixed mode. The state of the
 * scheme between cycles (Sec. 2's staggered fields, the auxiliary fields of
 * Sec. 3's PML and the clock) is: salec_get_fields (eos = NULL), with
 * salec_get_materials under the per-material closure, salec_get_pml and
 * salec_diag's t and dt. Restore it in this order: salec_set_fields,
 * salec_set_materials (per-material closure), salec_set_pml, salec_set_clock.
 * An FP64 member continued this way repeats the uninterrupted run bit for bit;
 * the cycle counter and the outflow budgets restart from zero.
 *
 * salec_set_pml writes the current level of member `instance`'s PML
 * auxiliaries, reference density and sink from the layouts salec_get_pml
 * returns (entries outside the layers are ignored; a NULL array leaves its
 * group unchanged; nothing happens without a PML). SALEC_E_INVALID if an
 * entry inside the layers is not finite.
 *
 * salec_set_clock sets the member's time t and the step dt of its next cycle
 * (salec_diag's t and dt). SALEC_E_INVALID unless t >= 0 and 0 < dt <=
 * dt_max, and, with a stop time, dt <= t_stop - t. */
int salec_set_pml(salec_ctx *ctx, int32_t instance, const double *cell_aux, const double *node_aux);
int salec_set_clock(salec_ctx *ctx, int32_t instance, double t, double dt);

/* Checkpoint (runtime support, no passage): the whole device state of every
 * member (fields, EoS cache, PML, budgets, t, dt, cycle, errors) as an opaque
 * host blob of salec_state_bytes() bytes; salec_set_state restores it into a
 * context made from the same descriptions. SALEC_E_BUFFER if the blob is too
 * small, SALEC_E_INVALID if it belongs to another layout. */
size_t salec_state_bytes(const salec_ctx *ctx);
int salec_get_state(salec_ctx *ctx, void *host_blob, size_t bytes);
int salec_set_state(salec_ctx *ctx, const void *host_blob, size_t bytes);

/* Time, step (Sec. 7), cycle, and the compensated totals of the quantities
 * eqs. (3)-(5) conserve -- mass, internal and kinetic energy -- with the
 * budgets of what left through the open top (Sec. 4) and what the PML sink
 * of Sec. 3 removed; sticky error of one member. SALEC_E_INVALID for a bad
 * context, instance or pointer. */
int salec_diag(salec_ctx *ctx, int32_t instance, salec_diag_t *out);

/* For callers that cannot allocate or synchronise (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * compensated totals of salec_diag (mass, ie, ke, mass_out, mass_pml, ie_out,
 * in this order) of member `instance`, written to dev_totals, 6 FP64 values in
 * device memory owned by the caller. Only enqueues the reduction on the
 * context's stream: no allocation of any kind, no memset, no host
 * synchronisation; the values are ready when the stream reaches that point,
 * and equal salec_diag's bit for bit. Its partial sums live in one scratch
 * array per GPU that the library holds for the life of the process (the
 * 240 x 6 compensated partials of the fixed reduction tree, 23 KB; every
 * instance size reduces into them, so no size is refused). Every call on one
 * GPU shares that array, so calls that overlap on one GPU (other streams,
 * other contexts, other host threads) race; successive calls on one stream do
 * not. SALEC_E_INVALID for a bad context, instance or pointer. */
int salec_diag_totals(salec_ctx *ctx, int32_t instance, double *dev_totals);

/* Measurement (no passage; the paper times whole runs, Sec. 6): device time
 * of the cycle kernels over the last salec_step() call, measured with HIP
 * events on the context's stream, in milliseconds. */
int salec_last_step_ms(salec_ctx *ctx, double *ms);

/* Initial pressure p0 per cell row of member `instance` (NZ host values, Pa;
 * row 0 at the bottom). Sec. 3 writes the momentum balance with
 * div(tau - p + p0), p0 the pressure of the state before impact with
 * -grad p0 + rho g = 0, and carries p - p0 into the PML auxiliary psi1: the
 * node force and psi1 use p - p0; the energy equation and psi2 keep p. A
 * scene with gravity > 0 sets it to a lithostatic column (trapezoid-rule
 * integral of rho g from the surface, each row's density the cold compressed
 * Tillotson state of its pressure, p0 re-evaluated by the equation of state
 * so that a target at rest stays at rest exactly in FP64); otherwise it is 0.
 * salec_set_p0 replaces it (values must be finite; the state is untouched;
 * checkpoints do not include it). Both return SALEC_E_INVALID for a bad
 * context, instance or pointer. */
int salec_set_p0(salec_ctx *ctx, int32_t instance, const double *p0);
int salec_get_p0(salec_ctx *ctx, int32_t instance, double *p0);

/* Per-material state of member `instance` under SALEC_CLOSURE_PER_MATERIAL
 * (the closure above): mu = partial densities (kg/m^3 of cell volume) and
 * Im = specific internal energies (J/kg), each nmat*NZ*NR host FP64 values,
 * material-major, row-major with r fastest. salec_set_materials replaces them
 * in the current state (values must be finite), sets rho = sum of mu and
 * I = the mass-weighted energy, keeps f, s and v, and starts a new run at
 * t = 0 like salec_set_fields (which, under this closure, gives every
 * material of a cell the cell's matter density rho f_m / phi and the cell's
 * I). salec_get_materials reads the current state; either pointer may be
 * NULL. Both return SALEC_E_INVALID for a bad context, instance or pointer,
 * or when the member uses SALEC_CLOSURE_SHARED. */
int salec_set_materials(salec_ctx *ctx, int32_t instance, const double *mu, const double *Im);
int salec_get_materials(salec_ctx *ctx, int32_t instance, double *mu, double *Im);

/* Damage D and block-model vibration speed v_vib (m/s) of member `instance`
 * (Table 1's damaged-material and acoustic-fluidization rows), NZ*NR host
 * FP64 values each, row-major with r fastest. They exist when some material
 * of the context has damage = 1 (then every member carries them); the scene
 * set-up and salec_set_fields leave intact, quiet rock (0, 0). salec_set_damage
 * replaces either (a NULL pointer keeps it; D in [0, 1], v_vib finite and
 * >= 0), keeps the rest of the current state and starts a new run at t = 0
 * like salec_set_fields. salec_get_damage reads the current state; either
 * pointer may be NULL. Checkpoints include both. Both return
 * SALEC_E_INVALID for a bad context, instance or value, or when no material
 * has damage. */
int salec_set_damage(salec_ctx *ctx, int32_t instance, const double *D, const double *vib);
int salec_get_damage(salec_ctx *ctx, int32_t instance, double *D, double *vib);

/* Measurement (no passage): advances every member by n cycles
 * (1 <= n <= 100000) like salec_step(),
 * but launches each cycle's two kernels directly (no graph) with a HIP event
 * after each on the context's stream, queues all n cycles before waiting,
 * and returns the mean time between consecutive events: per cycle kernel and
 * per finalize kernel, in milliseconds (each includes its launch gap). Same
 * kernels, same results; meant for measurement. Returns the first member
 * error like salec_step(). */
int salec_time_kernels(salec_ctx *ctx, int32_t n, double *cycle_ms, double *finalize_ms);

/* Launch schedules (runtime; no passage: the paper's parallel decomposition
 * of Sec. 2's grid over MPI ranks becomes tiles over workgroups here). Every
 * tile shape computes bit-identical results, so the
 * schedule only changes speed. A new context starts on the shape measured
 * fastest for its precision on a filled device, with as many workgroups as
 * fit at once when that is fewer than the tiles. salec_set_schedule() selects a shape and a
 * workgroup count (grid 0: one workgroup per tile; otherwise that many
 * workgroups walk the tiles). salec_tune() times each shape, with one
 * workgroup per tile and with as many workgroups as fit on the device at
 * once, over `cycles` real cycles of the run after one warm-up cycle each
 * (the members advance by (cycles + 1) cycles per candidate, at most
 * 2 * salec_num_variants() candidates), keeps the fastest and reports it in
 * out (may be NULL). Not every shape is built for every context: three
 * material slots and the per-material closure need more LDS per cell, so
 * the larger tiles are not built for them, and shapes 11 and 14 are built
 * only for them. salec_set_schedule() refuses a shape
 * the context cannot run with SALEC_E_INVALID and leaves the context as it
 * was; salec_tune() skips such shapes. A HIP error while switching leaves
 * the context unusable (SALEC_E_HIP). */
int32_t salec_num_variants(void);
int salec_get_schedule(const salec_ctx *ctx, salec_schedule *out);
int salec_set_schedule(salec_ctx *ctx, int32_t variant, int32_t grid);
int salec_tune(salec_ctx *ctx, int32_t cycles, salec_schedule *out);

const char *salec_last_error(const salec_ctx *ctx);
void salec_destroy(salec_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
