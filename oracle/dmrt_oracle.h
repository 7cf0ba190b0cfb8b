/*
 * dmrt_oracle.h -- FP64 CPU oracle for the double-MRT lattice Boltzmann model
 * of solid-liquid phase change with natural convection in porous media
 * (Liu & He, arXiv:1503.08406).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, literal implementation of
 * the paper's time step, used to check the HIP library.  Only the tests, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code, header, table or constant with the HIP path.
 *
 * Units are lattice units: dx = dt = c = 1, rho0 = 1 (Sec. 4, first
 * paragraph).  Temperature is the dimensionless theta of Eq. (9) with
 * Delta T = 1, so L_a / c_pl = 1 / St and c_ps = c_pl = 1.
 *
 * Field layout used at this interface (not inside the oracle): planar,
 * f[i][y][x] with index (i*ny + y)*nx + x; scalar fields [y][x].
 */
#ifndef DMRT_ORACLE_H
#define DMRT_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

/* Side order for boundaries: 0 = x-, 1 = x+, 2 = y-, 3 = y+. */
enum { ORC_PERIODIC = 0, ORC_WALL_T = 1, ORC_WALL_ADIABATIC = 2 };

typedef struct {
    int nx, ny;
    double H;              /* characteristic length; <= 0 means ny (Sec. 4.3) */
    int bc_kind[4];        /* ORC_* per side; every wall is a no-slip wall     */
    double T_wall[4];      /* Dirichlet temperature of ORC_WALL_T sides        */
    double Ra, Da, Pr, Ste;/* dimensionless groups of Eq. (9)                  */
    double Ma;             /* Mach number used to fix tau_nu (Sec. 4.3)        */
    double J;              /* viscosity ratio nu_e / nu_l, Eq. (9)             */
    double lambda_;        /* alpha_e / alpha_l, Eq. (9)                        */
    double alpha_ratio;    /* alpha_l / alpha_s (Sec. 4.1)                      */
    double sigma_s, sigma_l; /* heat-capacity ratio in solid / liquid, Eq. (7) */
    double T_s, T_l;       /* solidus / liquidus temperatures, Eqs. (41)-(42)  */
    double T0;             /* Boussinesq reference temperature, Eq. (5)        */
    double T_init;         /* uniform initial temperature                      */
    double alpha_l;        /* liquid diffusivity used when Ra == 0 (lattice)   */
    double varpi;          /* D2Q5 parameter of Eq. (34)                        */
    double s_e, s_eps, s_q;/* D2Q9 rates of Eq. (23)                            */
    double zeta_e, zeta_nu;/* D2Q5 rates zeta_3, zeta_4 of Eq. (37)             */
    double ergun_c;        /* constant of the Ergun relation, Eq. (6) (175)     */
    double fl_tol;         /* enthalpy iteration tolerance                      */
    int fl_maxit;          /* enthalpy iteration cap                            */
    int convective;        /* vartheta of Eq. (34)                              */
    int nthreads;          /* OpenMP threads (<= 0: runtime default)            */
    /* Variants of the thermal model (ablations of the readings):            */
    int sigma_mode;        /* 0: sigma_s + f_l (sigma_l - sigma_s); 1: Eq. (7)  */
    double cps_ratio;      /* c_ps / c_pl (sigma_mode 1)                        */
    double cm_ratio;       /* (rho c_p)_m / (rho c_pl) of the matrix (mode 1)    */
    int ke_mode;           /* 0: alpha_e linear in f_l; 1: k_e of Eq. (8)       */
    double ks_ratio;       /* k_s / k_l (ke_mode 1)                             */
    double km_ratio;       /* k_m / k_l of the matrix (ke_mode 1)               */
    int latent_mode;       /* 0: source at the receiving node after streaming,
                              per-node iteration (R1); 1: source at the pre-
                              stream site, global iteration (R2, Eq. 30)       */
} orc_params;

/* Effective conductivity ratio k_e / k_l of Eq. (8) for porosity phi and
 * liquid fraction fl (k_p = fl k_l + (1 - fl) k_s). */
double orc_ke(double phi, double fl, double ks_ratio, double km_ratio);

/* Lattice constants derived from orc_params (Sec. 3, Sec. 4). */
typedef struct {
    double H, tau_nu, nu_l, nu_e, alpha_l, alpha_s, gbeta, K_default, cs2, csT2;
    double tau_T_liquid, tau_T_solid;
} orc_derived;

/* Fill p with the paper's defaults (Sec. 4 first paragraph). */
void orc_default_params(orc_params *p);
/* 0 on success, negative if a relaxation time is <= 1/2 or sizes are bad. */
int orc_derive(const orc_params *p, orc_derived *d);

/* ---- lattice tables (for the pins) ------------------------------------- */
/* ex9,ey9 [9]; w9 [9]; M,Minv [81] row-major; ex5,ey5 [5]; w5 [5] (for varpi);
 * N,Ninv [25] row-major. */
void orc_lattice(double varpi, int *ex9, int *ey9, double *w9, double *M,
                 double *Minv, int *ex5, int *ey5, double *w5, double *N,
                 double *Ninv);

/* ---- per-cell operators (for the pins) --------------------------------- */
void orc_feq(double rho, double ux, double uy, double phi, double *feq9);       /* Eq. (29) */
void orc_meq(double rho, double ux, double uy, double phi, double *meq9);       /* Eq. (19) */
void orc_force_moments(double ux, double uy, double Fx, double Fy, double phi,
                       double *S9);                                              /* Eq. (22) */
void orc_geq(double T, double ux, double uy, double sigma, double varpi,
             double *geq5);                                                      /* Eq. (39) */
void orc_neq(double T, double ux, double uy, double sigma, double varpi,
             int convective, double *neq5);                                      /* Eq. (34) */
/* Eq. (20) then f+ = M^-1 m+, with the nine rates s[9]. */
void orc_collide_f(const double *f9, double rho, double ux, double uy, double Fx,
                   double Fy, double phi, const double *s9, double *fpost9);
/* Eqs. (24)-(28) and (4): velocity and total force of one cell. */
void orc_closure(double jx, double jy, double phi, double nu_l, double Ke,
                 double Ce, double Gx, double Gy, double *u2, double *F2);
/* Iterated enthalpy update of one cell (cps = c_ps / c_pl in Eqs. 40-41);
 * returns iterations used. */
int orc_enthalpy(double Tstar, double fl_old, double eps, double Ste,
                 double sigma_s, double sigma_l, double cps, double T_s, double T_l,
                 double tol, int maxit, double *fl_new, double *T_new);

/* ---- whole-lattice simulation ------------------------------------------ */
typedef struct orc_sim orc_sim;
/* eps is required; K or Feps may be NULL (Da*H^2, Ergun of Eq. (6)). */
orc_sim *orc_create(const orc_params *p, const double *eps, const double *K,
                    const double *Feps);
void orc_destroy(orc_sim *s);
/* Replace the state: pre-collision f[9][ny][nx], g[5][ny][nx], fl[ny][nx]. */
void orc_set_state(orc_sim *s, const double *f, const double *g, const double *fl);
void orc_get_state(const orc_sim *s, double *f, double *g, double *fl);
void orc_step(orc_sim *s, long n);
long orc_time(const orc_sim *s);
/* Macroscopic fields of the current state; any pointer may be NULL. */
void orc_fields(const orc_sim *s, double *T, double *ux, double *uy, double *fl,
                double *rho);
/* Post-collision populations of the current state (f+ is 0 at inactive cells). */
void orc_post_collision(const orc_sim *s, double *fpost, double *gpost);
/* Enthalpy iteration counts of the last step: max and total. */
void orc_iter_stats(const orc_sim *s, long *max_it, long *sum_it);

/* ---- discrete derivatives of the step ----------------------------------- */
/* The step is differentiated at its converged enthalpy fixed point (zero where
 * f_l is clamped), with the flow mask and pull-source kinds held fixed and
 * the subgradient 0 of |v| at v = 0.  They need sigma_s == sigma_l,
 * alpha_ratio == 1 and the default thermal model; otherwise they return a
 * negative value.  Planar layouts as orc_set_state; the state is not changed.
 *
 * Tangent of one step at the current state along (df, dg, dfl) and the
 * per-cell parameter directions dlnK (of ln K) and deps (either may be NULL). */
int orc_step_tl(orc_sim *s, const double *df, const double *dg, const double *dfl,
                const double *dlnK, const double *deps, double *dfn, double *dgn, double *dfln);
/* Transpose of orc_step_tl: adjoints of the next state in, adjoints of the
 * current state out; the parameter adjoints are ADDED to blnK and beps. */
int orc_step_ad(orc_sim *s, const double *bfn, const double *bgn, const double *bfln,
                double *bf, double *bg, double *bfl, double *blnK, double *beps);
/* Gradients of a loss of the fields after n steps from the current state
 * (adjoints dL_dT, dL_dfl of T = sum g and f_l; either may be NULL) with
 * respect to ln K and eps per cell.  Keeps every state of the run (refused
 * beyond 4 GB); the state is left unchanged. */
int orc_adjoint_run(orc_sim *s, long n, const double *dL_dT, const double *dL_dfl,
                    double *grad_lnK, double *grad_eps);

#ifdef __cplusplus
}
#endif
#endif
