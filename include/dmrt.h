/*
 * dmrt.h -- C ABI of the MI355X double-MRT lattice Boltzmann solver for
 * solid-liquid phase change with natural convection in porous media
 * (Liu & He, arXiv:1503.08406).
 *
 * One time step is one fused pass over the lattice: pull-streaming of the
 * D2Q9 flow populations (Eq. 21) and D2Q5 temperature populations (Eq. 36),
 * non-equilibrium-extrapolation walls and the moving solid-liquid interface
 * (Sec. 4, first paragraph), the iterated enthalpy update with the latent
 * source (Eqs. 38, 40-42), the velocity closure and porous force (Eqs. 4-6,
 * 24-28), the D2Q9 MRT collision with forcing (Eqs. 17-20, 22-23) and the
 * D2Q5 MRT collision (Eqs. 32-35, 37, 39).
 *
 * Units: lattice units, dx = dt = c = 1, rho0 = 1 (Sec. 4).  Temperatures are
 * the dimensionless theta of Eq. (9) (Delta T = 1, so L_a/c_p = 1/St).
 *
 * Conventions for every entry point:
 *  - Return 0 (DMRT_OK) on success or a negative DMRT_E* code; nothing is
 *    thrown and nothing aborts.  dmrt_last_error() gives a thread-local text
 *    for the last failure on the calling thread.
 *  - Scalar fields are [ny][nx] float32 with index y*nx + x; population arrays
 *    are planar [q][ny][nx].  Every field pointer may be host memory or device
 *    memory of the handle's device (the library asks the HIP runtime which).
 *  - The library copies what it needs at create time; the caller keeps
 *    ownership of every pointer it passes.  All device state belongs to the
 *    handle and is released by dmrt_destroy.
 *  - Work is enqueued on the stream given in dmrt_opts (NULL: the null
 *    stream).  Calls that return data to the caller synchronise that stream.
 *  - A handle is not thread-safe; different handles are independent.
 */
#ifndef DMRT_H
#define DMRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DMRT_OK 0
#define DMRT_EINVAL (-1)     /* bad argument, size or parameter            */
#define DMRT_ENOMEM (-2)     /* device or host allocation failed           */
#define DMRT_EDEVICE (-3)    /* a HIP runtime call failed                  */
#define DMRT_ENONFINITE (-4) /* the state holds NaN/Inf (see check_every)  */
#define DMRT_ESIZE (-5)      /* caller buffer too small                    */

/* Boundary kinds; every wall is a no-slip wall for the flow (Sec. 4). */
typedef enum {
    DMRT_PERIODIC = 0,       /* both sides of the axis must be periodic     */
    DMRT_WALL_T = 1,         /* wall held at T_wall (Secs. 4.1-4.3)         */
    DMRT_WALL_ADIABATIC = 2  /* wall at the receiving node's temperature    */
} dmrt_bc_kind;

/* Lattice of nx * ny evolving nodes.  A non-periodic side has its wall one
 * lattice unit outside the first/last node.  H is the characteristic length
 * of Eq. (9); H <= 0 means H = ny (Sec. 4.3). */
typedef struct {
    int32_t nx, ny;
    double H;
} dmrt_grid;

/* Sides are ordered x-, x+, y-, y+.  Gravity points to -y (buoyancy +y, Eq. 5). */
typedef struct {
    int32_t kind[4];
    double T_wall[4];
} dmrt_bc;

/* Model options; dmrt_opts_default() fills the paper's values (Sec. 4). */
typedef struct {
    double Ma;          /* Mach number fixing tau_nu and g beta DT (Sec. 4.3), 0.1      */
    double J;           /* viscosity ratio nu_e/nu_l, Eq. (9), 1                        */
    double lambda;      /* alpha_e/alpha_l, Eq. (9), 1                                  */
    double alpha_ratio; /* alpha_l/alpha_s (Sec. 4.1), 1                                */
    double sigma_s;     /* heat-capacity ratio of Eq. (7) in the solid, 1               */
    double sigma_l;     /* ... in the liquid, 1                                         */
    double T_s, T_l;    /* solidus / liquidus, Eqs. (41)-(42), -0.02 / 0.02             */
    double T0;          /* Boussinesq reference temperature, Eq. (5), 0                 */
    double T_init;      /* uniform initial temperature, 0                               */
    double alpha_l;     /* liquid diffusivity (lattice) used when Ra == 0, 0.02         */
    double varpi;       /* D2Q5 parameter of Eq. (34), -2                               */
    double s_e, s_eps, s_q;   /* D2Q9 rates of Eq. (23): 1.1, 1.1, 1.2                  */
    double zeta_e, zeta_nu;   /* D2Q5 rates zeta_3, zeta_4 of Eq. (37): 1.5, 1.5        */
    double ergun_c;     /* constant of Eq. (6), 175                                     */
    double fl_tol;      /* enthalpy iteration stops when |df_l| <= fl_tol, 1e-6         */
    int32_t fl_maxit;   /* enthalpy iteration cap, 64                                   */
    int32_t convective; /* vartheta of Eq. (34): 1 convection, 0 conduction, 1          */
    int32_t check_every;/* >0: dmrt_step checks the state for NaN/Inf every this many
                           steps and returns DMRT_ENONFINITE; 0: never                 */
    int32_t graph_steps;/* >0: dmrt_step replays a captured HIP graph of this many
                           steps (even); 0: plain launches, default 0                  */
    int32_t block_rows; /* rows per step-kernel block: 4 or 8; 0 = 4                   */
    int32_t cells_per_lane; /* nodes per lane in the step kernel: 1 or 2; 0 = 1       */
    void *stream;       /* hipStream_t for all work; NULL = null stream                 */
    /* Literal variants of the thermal model (single lattices only; the batch
     * and the adjoint reject them with DMRT_EINVAL):                          */
    int32_t sigma_mode; /* 0: sigma = sigma_s + f_l (sigma_l - sigma_s); 1: sigma of each
                           node from Eq. (7), phi (f_l + (1 - f_l) cps_ratio) + (1 - phi)
                           cm_ratio, with cps_ratio also in the enthalpy of
                           Eqs. (40)-(41) (c_p = f_l + (1 - f_l) cps_ratio,
                           En_s = cps_ratio T_s); default 0                    */
    int32_t ke_mode;    /* 0: alpha_e = lambda (alpha_l f_l + alpha_s (1 - f_l));
                           1: alpha_e = alpha_l k_e / k_l with k_e the root of Eq. (8)
                           for the node's porosity, k_p = f_l + (1 - f_l) ks_ratio,
                           k_m = km_ratio (lambda, alpha_ratio unused); default 0 */
    int32_t latent_mode;/* 0: latent source after streaming at the receiving node,
                           per-node iteration (R1); 1: source added before streaming
                           (Eq. 30), f_l of all nodes iterated together (R2), one
                           launch per sweep, so fl_maxit <= 4096; default 0      */
    int32_t store_hint; /* cache policy of the step's state stores: 0 by working set
                           (write-through the L2 when the double-buffered state fits
                           the 256 MB Infinity Cache, streaming otherwise), 1 plain
                           write-back, 2 write-through, 3 streaming; the results do
                           not depend on it; default 0                          */
    double cps_ratio;   /* c_ps / c_pl (sigma_mode 1), 1                        */
    double cm_ratio;    /* (rho c_p)_m / (rho c_pl) of the matrix (sigma_mode 1), 1 */
    double ks_ratio;    /* k_s / k_l (ke_mode 1), 1                             */
    double km_ratio;    /* k_m / k_l of the matrix (ke_mode 1), 1               */
    int32_t record_mode;/* what dmrt_record keeps for the adjoint: 0 every state of the
                           run when n + 1 states take at most half of the free device
                           memory, checkpoints otherwise; 1 checkpoints every
                           ceil(sqrt(n)) steps, the adjoint recomputing each segment;
                           2 every state (DMRT_ENOMEM if it does not fit); default 0.
                           The gradients are the same bits in every mode          */
    int32_t steps_per_launch; /* 0 or 1: one time step per launch; 2: two steps per
                           launch where the launch allows it (default thermal model,
                           R1, arrays within 4 GB, block_rows 4, one node per lane;
                           otherwise, and for a last odd step, one per launch):
                           the intermediate state stays in LDS, so a node update
                           moves half the bytes.  The results are the same bits;
                           default 2                                              */
    int32_t addressing; /* how the two-step kernels reach the state: 0 through one
                           buffer resource over the memory window that holds every
                           array of a launch, where that window is under 4 GB (a
                           batch: one per half of its state, under 4 GB each), else
                           one resource per array; 1 always one per array.  The
                           results are the same bits; default 0                   */
} dmrt_opts;

/* Lattice constants derived from the dimensionless inputs (Sec. 4.3). */
typedef struct {
    double H, tau_nu, nu_l, nu_e, alpha_l, alpha_s, gbeta, K_default;
    double tau_T_liquid, tau_T_solid, csT2;
} dmrt_derived;

/* On-demand diagnostics of the current state. */
typedef struct {
    double mass;        /* sum of rho over flow-active cells (Eq. 24)           */
    double enthalpy;    /* sum of sigma T + phi f_l / St (Eqs. 3, 40)           */
    double liquid;      /* sum of f_l                                           */
    double T_sum;       /* sum of T (Eq. 33)                                    */
    double u_max;       /* max |u| over the lattice                             */
    double front_mean;  /* mean over rows of the first f_l = 1/2 crossing from
                           x = 0 (interpolated, measured from the x- wall)     */
    double front_max;   /* max over rows of the same                            */
    int64_t active;     /* cells with f_l > 0 (flow solved there, Sec. 4)       */
    int64_t nonfinite;  /* NaN/Inf values found in the state                    */
    int64_t step;       /* time steps taken                                     */
} dmrt_diag_t;

typedef struct dmrt dmrt_t;

/* Fill o with the paper's defaults (Sec. 4). */
void dmrt_opts_default(dmrt_opts *o);

/* Host-only: lattice constants for (grid, Ra, Da, Pr, Ste, opts) following
 * Sec. 4.3 (Ra > 0) or the given alpha_l (Ra == 0).  opts may be NULL.
 * DMRT_EINVAL if a relaxation time is not above 1/2. No device work. */
int dmrt_derive(const dmrt_grid *grid, double Ra, double Da, double Pr, double Ste,
                const dmrt_opts *opts, dmrt_derived *out);

/* Create a solver on the current HIP device and initialise it at rest with
 * T = T_init, f_l = f_l(T_init) (Eq. 42), g = g^eq (Eq. 39), f = f^eq (Eq. 29).
 *   eps  : porosity per cell, (0, 1]; required.
 *   K    : permeability per cell at f_l = 1; NULL means Da * H^2 (Eq. 9).
 *   Feps : inertial coefficient per cell at f_l = 1; NULL means the Ergun
 *          relation 1.75 / sqrt(ergun_c eps^3) of Eq. (6).
 *   Ra   : Rayleigh number; Ra == 0 means no buoyancy (conduction cases).
 *   Da, Pr, Ste : Darcy, Prandtl and Stefan numbers of Eq. (9).
 * opts may be NULL (defaults).  On success *out owns the device state. */
int dmrt_create(const dmrt_grid *grid, const float *eps, const float *K, const float *Feps,
                double Ra, double Da, double Pr, double Ste, const dmrt_bc *bc,
                const dmrt_opts *opts, dmrt_t **out);

/* Advance n >= 0 time steps (enqueued; returns before they finish unless a
 * NaN check runs).  DMRT_ENONFINITE names the step in dmrt_last_error().
 * One step is one kernel launch; with latent_mode 1 it is 2 + fl_maxit
 * launches (the global iteration; sweeps after convergence return at once). */
int dmrt_step(dmrt_t *h, int64_t n);

/* Fields at the current time: T (Eq. 33), u (Eq. 26; 0 in solid cells) and
 * f_l.  Any pointer may be NULL; each takes nx*ny floats. */
int dmrt_fields(dmrt_t *h, float *T, float *ux, float *uy, float *fl);

/* Replace the state with the pre-collision populations f[9][ny][nx],
 * g[5][ny][nx] and liquid fraction fl[ny][nx].  f may be NULL (rest
 * equilibrium w_i rho0), g may be NULL (g^eq at T_init), fl may be NULL
 * (f_l(T) of Eq. 42 with T = sum g).  The time counter is not changed.
 * A given f switches a handle created without buoyancy (Ra = 0) to the
 * flow kernels for good, so that the given velocity field evolves. */
int dmrt_set_state(dmrt_t *h, const float *f, const float *g, const float *fl);

/* Post-collision populations of the current time step: fpost[9][ny][nx]
 * (0 in solid cells) and gpost[5][ny][nx]; either may be NULL. */
int dmrt_get_populations(dmrt_t *h, float *fpost, float *gpost);

/* Reductions of the current state (see dmrt_diag_t). */
int dmrt_diag(dmrt_t *h, dmrt_diag_t *out);

/* dmrt_diag for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * reductions, with the same bits, computed without any allocation, in a fixed
 * device scratch array of 4 MiB + 64 KiB that the library holds on each device
 * it runs on (set up by dmrt_create) until the process ends.  A lattice needs
 * 64 bytes per tile of 64 x 4 nodes plus 4 bytes per row (each rounded up to
 * 256 bytes) plus 128 bytes: 4096 x 4096 needs 4.02 MiB and fits; a lattice
 * that does not fit returns DMRT_ESIZE (dmrt_diag serves it).  Every call on a device shares that device's array:
 * calls that overlap on one device (from any handle or thread) race, so the
 * caller must serialise them.  Synchronises the handle's stream. */
int dmrt_diag_noalloc(dmrt_t *h, dmrt_diag_t *out);

/* Lattice constants the handle runs with. */
int dmrt_get_derived(const dmrt_t *h, dmrt_derived *out);

/* Time steps one launch of the step kernel advances: 2 where two steps per
 * launch are in effect (steps_per_launch 2 and a configuration that allows
 * it), else 1; a negative DMRT_* code for a null handle. */
int32_t dmrt_launch_steps(const dmrt_t *h);

/* Enthalpy-iteration statistics of the last step taken with counting on:
 * dmrt_step_counted(h, n) runs n steps and accumulates per-cell iteration
 * counts; max_it and mean_it (over cells and steps) are returned. */
int dmrt_step_counted(dmrt_t *h, int64_t n, int32_t *max_it, double *mean_it);

/* Checkpoint: dmrt_state_bytes() bytes hold the complete state and the time
 * counter; dmrt_save writes them to a host buffer of capacity cap
 * (DMRT_ESIZE if smaller), dmrt_load restores them into a handle created
 * with the same grid (DMRT_EINVAL otherwise).  A checkpoint of a handle that
 * ran the flow kernels switches the loading handle to them as well. */
int64_t dmrt_state_bytes(const dmrt_t *h);
int dmrt_save(dmrt_t *h, void *buf, size_t cap);
int dmrt_load(dmrt_t *h, const void *buf, size_t n);

/* Replace the porous fields (same meaning as in dmrt_create; K and Feps may
 * be NULL).  The state is kept; a recorded run is discarded. */
int dmrt_set_porous(dmrt_t *h, const float *eps, const float *K, const float *Feps);

/* Differentiation of a run (NEXT row f2: the discrete adjoint of the step).
 * dmrt_record advances n >= 1 steps like dmrt_step and keeps what the
 * adjoint needs (record_mode of dmrt_opts): either every state of the run,
 * each step writing its result into a slot of its own, or the state every
 * S = ceil(sqrt(n)) steps (checkpoints) plus room for one segment of S states
 * that the adjoint recomputes.  The launches of a recording are replayed from
 * a HIP graph captured at the first call for n (when the handle has a
 * stream).  Needs
 * uniform sigma and tau_T (sigma_s == sigma_l, alpha_ratio == 1).
 * dmrt_adjoint then returns, for a loss L of the fields at the end of the
 * recorded run with adjoints dL_dT and dL_dfl (nx*ny each; NULL = 0), the
 * gradients dL/dlog K and dL/deps per cell (nx*ny each; NULL = not wanted),
 * K being the permeability at f_l = 1 and Feps held fixed when it was given
 * (otherwise it follows eps through Eq. 6).  The enthalpy update is
 * differentiated at its converged fixed point (zero derivative where f_l is
 * clamped to 0 or 1); the flow mask and the liquid/solid status of pull
 * sources are held fixed; |v| has the subgradient 0 at v = 0.  The state of
 * the handle is not changed. */
int dmrt_record(dmrt_t *h, int64_t n);
int dmrt_adjoint(dmrt_t *h, const float *dL_dT, const float *dL_dfl, float *grad_logK,
                 float *grad_eps);

/* Time steps taken so far. */
int64_t dmrt_time(const dmrt_t *h);

/* Wait for the handle's stream. */
int dmrt_sync(dmrt_t *h);

/* Release the handle (NULL is ignored). */
void dmrt_destroy(dmrt_t *h);

/* ------------------------------------------------------------------------
 * Batches: many independent cavities of uneven size and parameters advance
 * together, one or two time steps per launch over all of them (see
 * dmrt_batch_set_launch).  Each cavity runs
 * exactly the step of a single lattice created by dmrt_create with the same
 * grid, boundary, dimensionless numbers and options and with uniform porous
 * fields (eps everywhere, K = Da H^2, F_eps from the Ergun relation of
 * Eq. 6), so its fields equal that lattice's bit for bit.  The flow part is
 * always solved (a cavity with Ra == 0 stays at rest).
 * ------------------------------------------------------------------------ */
typedef struct dmrt_batch dmrt_batch_t;

/* One cavity of a batch. */
typedef struct {
    dmrt_grid grid;
    dmrt_bc bc;
    double eps;                 /* uniform porosity, (0, 1]                  */
    double Ra, Da, Pr, Ste;     /* as for dmrt_create                        */
} dmrt_cavity;

/* Create a batch of ncav >= 1 cavities on the current HIP device, every one
 * initialised as dmrt_create does.  opts (may be NULL) applies to all
 * cavities; its graph_steps and check_every act on the batch, block_rows
 * picks the launch shape of the one-step kernel (see dmrt_batch_set_launch),
 * steps_per_launch 2 (the default) starts the batch on the two-step kernel
 * and cells_per_lane is ignored.  DMRT_EINVAL names the first bad cavity. */
int dmrt_batch_create(int32_t ncav, const dmrt_cavity *cav, const dmrt_opts *opts,
                      dmrt_batch_t **out);

/* Advance every cavity n >= 0 time steps (enqueued). */
int dmrt_batch_step(dmrt_batch_t *b, int64_t n);

/* Fields of cavity i, as dmrt_fields (each pointer nx*ny floats of that
 * cavity, any may be NULL). */
int dmrt_batch_fields(dmrt_batch_t *b, int32_t i, float *T, float *ux, float *uy, float *fl);

/* Per-cavity counts of liquid nodes (f_l > 0) and of NaN/Inf values in f_l
 * and g; either array (ncav entries) may be NULL. */
int dmrt_batch_check(dmrt_batch_t *b, int64_t *liquid, int64_t *nonfinite);

/* Launch shape of the batched step.  rows 4 or 8: one step per launch,
 * tiles of 64 x rows nodes, and the number of blocks (a multiple of 8; 0 =
 * as many as the device holds at once).  rows 0 (only for a batch created
 * with steps_per_launch 2; blocks is ignored): two steps per launch, tiles
 * of 62 x 6 nodes, one block per tile; a last odd step of dmrt_batch_step
 * then runs on the one-step shape set last.  dmrt_batch_get_launch gives
 * rows 0 and the two-step kernel's block count in that case.  The shape
 * changes speed only, never results. */
int dmrt_batch_set_launch(dmrt_batch_t *b, int32_t rows, int32_t blocks);
int dmrt_batch_get_launch(const dmrt_batch_t *b, int32_t *rows, int32_t *blocks);

/* Autotuner of the launch shape.  For every candidate (rows 4 and 8; as
 * many blocks as the device holds at once, twice that, one block per tile;
 * and rows 0, two steps per launch, where the batch allows it) run
 * trial_steps >= 1 untimed and then trial_steps timed steps from a copy of
 * the current state; keep the fastest (dmrt_batch_set_launch; the fastest
 * one-step shape stays the shape of single launches) and restore the state,
 * so results and the time counter are unchanged.  Any output pointer may be
 * NULL; ms_per_step is the winner's mean step time. */
int dmrt_batch_tune(dmrt_batch_t *b, int32_t trial_steps, int32_t *rows, int32_t *blocks,
                    double *ms_per_step);

/* Lattice constants of cavity i. */
int dmrt_batch_get_derived(const dmrt_batch_t *b, int32_t i, dmrt_derived *out);

/* Evolving nodes over all cavities (sum of nx * ny). */
int64_t dmrt_batch_cells(const dmrt_batch_t *b);

/* Time steps taken so far. */
int64_t dmrt_batch_time(const dmrt_batch_t *b);

/* Wait for the batch's stream. */
int dmrt_batch_sync(dmrt_batch_t *b);

/* Release the batch (NULL is ignored). */
void dmrt_batch_destroy(dmrt_batch_t *b);

/* Thread-local text of the last error ("" if none). */
const char *dmrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DMRT_H */
