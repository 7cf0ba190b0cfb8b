/*
 * dmrt_oracle.c -- FP64 CPU oracle for the double-MRT lattice Boltzmann model
 * of Liu & He (arXiv:1503.08406): D2Q9 MRT flow with the generalized non-Darcy
 * force (Sec. 3.1), D2Q5 MRT temperature with the latent-heat source and the
 * iterated enthalpy method (Sec. 3.2), non-equilibrium-extrapolation walls and
 * a moving solid-liquid interface (Sec. 4, first paragraph).
 *
 * TEST INFRASTRUCTURE ONLY -- never linked into the product library.  It is
 * written to be checked against the paper by eye: dense matrices M, M^-1, N,
 * N^-1 exactly as printed, one function per equation, no fusion, no blocking.
 * OpenMP splits loops over cells; it never changes the arithmetic of a cell.
 *
 * Readings where the paper is silent or garbled (each is listed with its
 * reason in the design notes of the repository):
 *   - Lambda = diag(1, s_e, s_eps, 1, s_q, 1, s_q, s_nu, s_nu) (Eq. (23)).
 *   - Eq. (26) denominator starts with l_0 (the printed d_0 is a typo).
 *   - rho0 replaces rho in the force terms (incompressible approximation).
 *   - Eq. (6) is read in varphi = phi*f_l; the per-cell inputs K and F_eps are
 *     the values at f_l = 1, so K_e = K (varphi/phi)^3 ((1-phi)/(1-varphi))^2
 *     and C_e = F_eps (phi/varphi)^(3/2).  phi = 1 means clear fluid (no drag).
 *   - The flow is solved where f_l > 0.  A cell that becomes liquid restarts
 *     at rest at the mean density of its liquid neighbours (rho0 if none), so
 *     melting launches no pressure pulse; a cell that becomes solid drops its
 *     populations.
 *   - Boundaries: link-wise non-equilibrium extrapolation at the receiving
 *     node.  A wall lies one lattice unit outside the first node.  A missing
 *     population gets equilibrium(wall values) + (own post-collision value -
 *     own equilibrium), with the start-of-step values of the receiving node.
 *     Solid nodes act as no-slip walls for the flow.
 *   - The latent source of Eq. (38) is applied after streaming at the
 *     receiving node, so the enthalpy iteration is local to one cell.
 *   - Enthalpy: c_ps = c_pl = 1, En_s = T_s, En_l = T_l + 1/St.
 *   - sigma(f_l) = sigma_s + f_l (sigma_l - sigma_s) (Eq. (7) is linear in f_l);
 *     alpha_e(f_l) = lambda alpha_l (f_l + (1-f_l)/(alpha_l/alpha_s)).
 */
#include "dmrt_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q9 9
#define Q5 5

static const double RHO0 = 1.0; /* Sec. 4: rho0 = 1 */
static const double DT = 1.0;   /* Sec. 4: delta_t = 1 */
static const double CS2 = 1.0 / 3.0; /* c_s = c / sqrt(3), Sec. 3.1 */

/* Transformation matrix M, Eq. (18). */
static const double M18[Q9][Q9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* Transformation matrix N, Eq. (32). */
static const double N32[Q5][Q5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {-4, 1, 1, 1, 1},
    {0, 1, -1, 1, -1}};

typedef struct {
    int ex[Q9], ey[Q9];
    double w[Q9];
    double M[Q9][Q9], Minv[Q9][Q9];
} lat9;

typedef struct {
    int ex[Q5], ey[Q5];
    double w[Q5];
    double N[Q5][Q5], Ninv[Q5][Q5];
} lat5;

/* D2Q9: velocities from Eq. (15), weights below Eq. (29), M from Eq. (18),
 * M^-1 = M^T (M M^T)^-1 as stated under Eq. (18). */
static void build_lat9(lat9 *L)
{
    const double pi = acos(-1.0);
    for (int i = 0; i < Q9; ++i) {
        double ax = 0, ay = 0;
        if (i >= 1 && i <= 4) {
            ax = cos((i - 1) * pi / 2);
            ay = sin((i - 1) * pi / 2);
        } else if (i >= 5) {
            ax = sqrt(2.0) * cos((2 * i - 9) * pi / 4);
            ay = sqrt(2.0) * sin((2 * i - 9) * pi / 4);
        }
        L->ex[i] = (int)lround(ax);
        L->ey[i] = (int)lround(ay);
        L->w[i] = (i == 0) ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
    }
    double MMt[Q9][Q9];
    for (int a = 0; a < Q9; ++a)
        for (int b = 0; b < Q9; ++b) {
            double s = 0;
            for (int k = 0; k < Q9; ++k) s += M18[a][k] * M18[b][k];
            MMt[a][b] = s;
        }
    for (int a = 0; a < Q9; ++a)
        for (int k = 0; k < Q9; ++k) {
            L->M[a][k] = M18[a][k];
            L->Minv[k][a] = M18[a][k] / MMt[a][a]; /* M M^T is diagonal */
        }
}

/* D2Q5: velocities from Eq. (31), weights below Eq. (39), N from Eq. (32). */
static void build_lat5(lat5 *L, double varpi)
{
    const double pi = acos(-1.0);
    for (int i = 0; i < Q5; ++i) {
        double ax = 0, ay = 0;
        if (i >= 1) {
            ax = cos((i - 1) * pi / 2);
            ay = sin((i - 1) * pi / 2);
        }
        L->ex[i] = (int)lround(ax);
        L->ey[i] = (int)lround(ay);
        L->w[i] = (i == 0) ? (1.0 - varpi) / 5.0 : (4.0 + varpi) / 20.0;
    }
    double NNt[Q5][Q5];
    for (int a = 0; a < Q5; ++a)
        for (int b = 0; b < Q5; ++b) {
            double s = 0;
            for (int k = 0; k < Q5; ++k) s += N32[a][k] * N32[b][k];
            NNt[a][b] = s;
        }
    for (int a = 0; a < Q5; ++a)
        for (int k = 0; k < Q5; ++k) {
            L->N[a][k] = N32[a][k];
            L->Ninv[k][a] = N32[a][k] / NNt[a][a];
        }
}

void orc_lattice(double varpi, int *ex9, int *ey9, double *w9, double *M,
                 double *Minv, int *ex5, int *ey5, double *w5, double *N,
                 double *Ninv)
{
    lat9 L9;
    lat5 L5;
    build_lat9(&L9);
    build_lat5(&L5, varpi);
    for (int i = 0; i < Q9; ++i) {
        ex9[i] = L9.ex[i];
        ey9[i] = L9.ey[i];
        w9[i] = L9.w[i];
        for (int k = 0; k < Q9; ++k) {
            M[i * Q9 + k] = L9.M[i][k];
            Minv[i * Q9 + k] = L9.Minv[i][k];
        }
    }
    for (int i = 0; i < Q5; ++i) {
        ex5[i] = L5.ex[i];
        ey5[i] = L5.ey[i];
        w5[i] = L5.w[i];
        for (int k = 0; k < Q5; ++k) {
            N[i * Q5 + k] = L5.N[i][k];
            Ninv[i * Q5 + k] = L5.Ninv[i][k];
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Parameters                                                              */
/* ---------------------------------------------------------------------- */

void orc_default_params(orc_params *p)
{
    memset(p, 0, sizeof(*p));
    p->nx = p->ny = 0;
    p->H = 0;
    for (int k = 0; k < 4; ++k) {
        p->bc_kind[k] = ORC_WALL_ADIABATIC;
        p->T_wall[k] = 0;
    }
    p->Ra = 0;
    p->Da = 1e-4;
    p->Pr = 1;
    p->Ste = 1;
    p->Ma = 0.1;      /* Sec. 4.3 */
    p->J = 1;         /* Sec. 4 */
    p->lambda_ = 1;
    p->alpha_ratio = 1;
    p->sigma_s = p->sigma_l = 1;
    p->T_s = -0.02;   /* Sec. 4.1 / 4.2 mushy range around T_m = 0 */
    p->T_l = 0.02;
    p->T0 = 0;
    p->T_init = 0;
    p->alpha_l = 0.02; /* Sec. 4.1 */
    p->varpi = -2;     /* Sec. 4 */
    p->s_e = 1.1;      /* Sec. 4 */
    p->s_eps = 1.1;
    p->s_q = 1.2;
    p->zeta_e = 1.5;
    p->zeta_nu = 1.5;
    p->ergun_c = 175;  /* Eq. (6) as printed */
    p->fl_tol = 1e-12;
    p->fl_maxit = 200;
    p->convective = 1;
    p->nthreads = 0;
    p->sigma_mode = 0;
    p->cps_ratio = 1;
    p->cm_ratio = 1;
    p->ke_mode = 0;
    p->ks_ratio = 1;
    p->km_ratio = 1;
    p->latent_mode = 0;
}

/* c_ps / c_pl: the capacities differ only in the Eq. (7) variant. */
static double cps_of(const orc_params *p)
{
    return p->sigma_mode == 1 ? p->cps_ratio : 1.0;
}

/* Heat-capacity ratio of a cell.  Mode 0: linear between the given solid
 * and liquid values.  Mode 1: Eq. (7) with rho_s = rho_l, i.e.
 * sigma = phi (f_l + (1 - f_l) c_ps / c_pl) + (1 - phi) (rho c_p)_m / (rho c_pl). */
static double sigma_of(const orc_params *p, double eps, double fl)
{
    if (p->sigma_mode == 1)
        return eps * (fl + (1.0 - fl) * p->cps_ratio) + (1.0 - eps) * p->cm_ratio;
    return p->sigma_s + fl * (p->sigma_l - p->sigma_s);
}

/* Eq. (8) in units of k_l: with z = k_e^(1/3) it is the depressed cubic
 * z^3 + P z + Q = 0, P = phi (k_m - k_p) / k_p^(1/3), Q = -k_m, solved by
 * Cardano's formula (one real root when (Q/2)^2 + (P/3)^3 >= 0, otherwise
 * the largest of the three real roots, trigonometric form). */
double orc_ke(double phi, double fl, double ks_ratio, double km_ratio)
{
    double kp = fl + (1.0 - fl) * ks_ratio;
    double P = phi * (km_ratio - kp) / cbrt(kp);
    double Q = -km_ratio;
    double D = 0.25 * Q * Q + P * P * P / 27.0;
    double z;
    if (D >= 0) {
        double sD = sqrt(D);
        z = cbrt(-0.5 * Q + sD) + cbrt(-0.5 * Q - sD);
    } else {
        double r = sqrt(-P / 3.0);
        double th = acos(1.5 * Q / (P * r)) / 3.0;
        z = 2.0 * r * cos(th);
    }
    return z * z * z;
}

int orc_derive(const orc_params *p, orc_derived *d)
{
    if (p->nx <= 0 || p->ny <= 0) return -1;
    d->H = p->H > 0 ? p->H : (double)p->ny;
    d->cs2 = CS2;
    d->csT2 = (4.0 + p->varpi) / 10.0; /* below Eq. (39), c = 1 */
    if (p->Ra > 0) {
        /* Sec. 4.3: tau_nu = 1/2 + Ma J H sqrt(3 Pr) / (c dt sqrt(Ra)) */
        d->tau_nu = 0.5 + p->Ma * p->J * d->H * sqrt(3.0 * p->Pr) / (DT * sqrt(p->Ra));
        d->nu_e = CS2 * (d->tau_nu - 0.5) * DT; /* below Eq. (28) */
        d->nu_l = d->nu_e / p->J;               /* J = nu_e / nu_l, Eq. (9) */
        d->alpha_l = d->nu_l / p->Pr;           /* Pr = nu_l / alpha_l */
        /* Ma = u_c / c_s with u_c = sqrt(g beta DeltaT H), Sec. 4.3 */
        double uc = p->Ma * sqrt(CS2);
        d->gbeta = uc * uc / d->H;
    } else {
        d->alpha_l = p->alpha_l;
        d->nu_l = p->Pr * d->alpha_l;
        d->nu_e = p->J * d->nu_l;
        d->tau_nu = 0.5 + d->nu_e / (CS2 * DT);
        d->gbeta = 0;
    }
    d->alpha_s = d->alpha_l / p->alpha_ratio;
    d->K_default = p->Da * d->H * d->H; /* Da = K / H^2, Eq. (9) */
    /* tau_T = 1/2 + alpha_e / (sigma c_sT^2 dt), below Eq. (39) and Sec. 4.1 */
    d->tau_T_liquid = 0.5 + p->lambda_ * d->alpha_l / (p->sigma_l * d->csT2 * DT);
    d->tau_T_solid = 0.5 + p->lambda_ * d->alpha_s / (p->sigma_s * d->csT2 * DT);
    if (!(d->tau_nu > 0.5) || !(d->tau_T_liquid > 0.5) || !(d->tau_T_solid > 0.5))
        return -2;
    return 0;
}

/* tau_T = 1/2 + alpha_e / (sigma c_sT^2 dt).  Mode 0: alpha_e = lambda
 * (alpha_l f_l + alpha_s (1 - f_l)) (Sec. 4.1, 4.3); mode 1: alpha_e =
 * k_e / (rho c_pl) = alpha_l k_e / k_l with k_e from Eq. (8). */
static double tauT_of(const orc_params *p, const orc_derived *d, double eps, double fl)
{
    double alpha_e = p->ke_mode == 1
        ? d->alpha_l * orc_ke(eps, fl, p->ks_ratio, p->km_ratio)
        : p->lambda_ * (d->alpha_l * fl + d->alpha_s * (1.0 - fl));
    return 0.5 + alpha_e / (sigma_of(p, eps, fl) * d->csT2 * DT);
}

/* ---------------------------------------------------------------------- */
/* Per-cell operators                                                      */
/* ---------------------------------------------------------------------- */

static lat9 G9; /* D2Q9 tables, built once when the library is loaded */
static lat5 G5; /* D2Q5 velocities (weights depend on varpi: see w5_of) */

__attribute__((constructor)) static void build_tables(void)
{
    build_lat9(&G9);
    build_lat5(&G5, -2.0);
}

/* D2Q5 weights below Eq. (39). */
static double w5_of(int i, double varpi)
{
    return i == 0 ? (1.0 - varpi) / 5.0 : (4.0 + varpi) / 20.0;
}

/* Eq. (29) */
void orc_feq(double rho, double ux, double uy, double phi, double *feq9)
{
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < Q9; ++i) {
        double eu = G9.ex[i] * ux + G9.ey[i] * uy;
        feq9[i] = G9.w[i] * (rho + RHO0 * (eu / CS2 + eu * eu / (2 * CS2 * CS2 * phi) -
                                           uu / (2 * CS2 * phi)));
    }
}

/* Eq. (19) */
void orc_meq(double rho, double ux, double uy, double phi, double *m)
{
    double uu = ux * ux + uy * uy;
    m[0] = rho;
    m[1] = -2 * rho + 3 * RHO0 * uu / phi;
    m[2] = rho - 3 * RHO0 * uu / phi;
    m[3] = RHO0 * ux;
    m[4] = -RHO0 * ux;
    m[5] = RHO0 * uy;
    m[6] = -RHO0 * uy;
    m[7] = RHO0 * (ux * ux - uy * uy) / phi;
    m[8] = RHO0 * ux * uy / phi;
}

/* Eq. (22) */
void orc_force_moments(double ux, double uy, double Fx, double Fy, double phi, double *S)
{
    double uF = ux * Fx + uy * Fy;
    S[0] = 0;
    S[1] = 6 * RHO0 * uF / phi;
    S[2] = -6 * RHO0 * uF / phi;
    S[3] = RHO0 * Fx;
    S[4] = -RHO0 * Fx;
    S[5] = RHO0 * Fy;
    S[6] = -RHO0 * Fy;
    S[7] = 2 * RHO0 * (ux * Fx - uy * Fy) / phi;
    S[8] = RHO0 * (ux * Fy + uy * Fx) / phi;
}

/* Eq. (39) */
void orc_geq(double T, double ux, double uy, double sigma, double varpi, double *geq5)
{
    double csT2 = (4.0 + varpi) / 10.0;
    for (int i = 0; i < Q5; ++i) {
        double eu = G5.ex[i] * ux + G5.ey[i] * uy;
        geq5[i] = w5_of(i, varpi) * T * (1.0 + eu / (sigma * csT2));
    }
}

/* Eq. (34) */
void orc_neq(double T, double ux, double uy, double sigma, double varpi, int convective,
             double *n)
{
    double th = convective ? 1.0 : 0.0;
    n[0] = T;
    n[1] = th * ux * T / sigma;
    n[2] = th * uy * T / sigma;
    n[3] = varpi * T;
    n[4] = 0;
}

/* Eq. (20), then f+ = M^-1 m+ (text below Eq. (21)). */
void orc_collide_f(const double *f, double rho, double ux, double uy, double Fx, double Fy,
                   double phi, const double *s, double *fpost)
{
    double m[Q9], meq[Q9], S[Q9], mp[Q9];
    for (int a = 0; a < Q9; ++a) {
        double v = 0;
        for (int i = 0; i < Q9; ++i) v += G9.M[a][i] * f[i];
        m[a] = v; /* Eq. (16) */
    }
    orc_meq(rho, ux, uy, phi, meq);
    orc_force_moments(ux, uy, Fx, Fy, phi, S);
    for (int a = 0; a < Q9; ++a)
        mp[a] = m[a] - s[a] * (m[a] - meq[a]) + DT * (1.0 - s[a] / 2.0) * S[a];
    for (int i = 0; i < Q9; ++i) {
        double v = 0;
        for (int a = 0; a < Q9; ++a) v += G9.Minv[i][a] * mp[a];
        fpost[i] = v;
    }
}

/* Eqs. (27), (28), (26) and the total force Eq. (4). */
void orc_closure(double jx, double jy, double phi, double nu_l, double Ke, double Ce,
                 double Gx, double Gy, double *u, double *F)
{
    double vx = jx / RHO0 + DT / 2 * phi * Gx; /* Eq. (27) */
    double vy = jy / RHO0 + DT / 2 * phi * Gy;
    if (!(Ke > 0)) {
        /* Vanishing permeability: infinite drag, u = 0; Eq. (25) then fixes F. */
        u[0] = u[1] = 0;
        F[0] = -2 * jx / (DT * RHO0);
        F[1] = -2 * jy / (DT * RHO0);
        return;
    }
    double l0 = 0.5 * (1.0 + phi * DT / 2 * nu_l / Ke); /* Eq. (28) */
    double l1 = phi * DT / 2 * Ce / sqrt(Ke);
    double vmag = sqrt(vx * vx + vy * vy);
    double den = l0 + sqrt(l0 * l0 + l1 * vmag); /* Eq. (26) */
    u[0] = vx / den;
    u[1] = vy / den;
    double umag = sqrt(u[0] * u[0] + u[1] * u[1]);
    /* Eq. (4) */
    F[0] = -phi * nu_l / Ke * u[0] - phi * Ce / sqrt(Ke) * umag * u[0] + phi * Gx;
    F[1] = -phi * nu_l / Ke * u[1] - phi * Ce / sqrt(Ke) * umag * u[1] + phi * Gy;
}

/* Eq. (41): temperature from total enthalpy, in units with c_pl = 1 and
 * L_a / c_pl = 1/St; cps = c_ps / c_pl. */
static double T_of_En(double En, double T_s, double T_l, double Ste, double cps)
{
    double En_s = cps * T_s;       /* c_ps T_s */
    double En_l = T_l + 1.0 / Ste; /* c_pl T_l + L_a */
    if (En <= En_s) return En / cps;
    if (En >= En_l) return T_l + (En - En_l);
    return T_s + (En - En_s) / (En_l - En_s) * (T_l - T_s);
}

/* Eq. (42) */
static double fl_of_T(double T, double T_s, double T_l)
{
    if (T <= T_s) return 0.0;
    if (T >= T_l) return 1.0;
    return (T - T_s) / (T_l - T_s);
}

/* Eq. (40) with c_p of the mixture, f_l c_pl + (1 - f_l) c_ps. */
static double En_of(double T, double f, double Ste, double cps)
{
    return (f + (1.0 - f) * cps) * T + f / Ste;
}

/* Iterated enthalpy method (Sec. 3.2, end): the latent source of Eq. (38)
 * needs f_l(t+dt); iterate T <- T* + S0(f), En (Eq. 40), T(En) (Eq. 41),
 * f_l(T) (Eq. 42) until f_l stops changing.  sigma = sigma_s + f (sigma_l -
 * sigma_s); cps = c_ps / c_pl (1 unless the heat capacities differ). */
int orc_enthalpy(double Tstar, double fl_old, double eps, double Ste, double sigma_s,
                 double sigma_l, double cps, double T_s, double T_l, double tol, int maxit,
                 double *fl_new, double *T_new)
{
    double f = fl_old;
    int it = 0;
    while (it < maxit) {
        ++it;
        double sig = sigma_s + f * (sigma_l - sigma_s);
        double S0 = -(eps / (sig * Ste)) * (f - fl_old) / DT; /* Eq. (38) */
        double T = Tstar + DT * S0;                            /* zeroth moment of Eq. (35) */
        double En = En_of(T, f, Ste, cps);                     /* Eq. (40) */
        double fn = fl_of_T(T_of_En(En, T_s, T_l, Ste, cps), T_s, T_l);
        int done = fabs(fn - f) <= tol;
        f = fn;
        if (done) break;
    }
    double sig = sigma_s + f * (sigma_l - sigma_s);
    *fl_new = f;
    *T_new = Tstar - DT * (eps / (sig * Ste)) * (f - fl_old) / DT;
    return it;
}

/* ---------------------------------------------------------------------- */
/* Simulation                                                              */
/* ---------------------------------------------------------------------- */

struct orc_sim {
    orc_params p;
    orc_derived d;
    lat9 L9;
    lat5 L5;
    int nx, ny;
    long nc, t;
    double *eps, *K, *Feps;
    int feps_given;                   /* 0: F_eps follows eps through Eq. (6) */
    double *f, *g, *fl;               /* state: f[c*9+i], g[c*5+i], fl[c] */
    double *fpost, *gpost, *fnew, *gnew, *flnew;
    double *gstr;                     /* streamed g before the latent source */
    double *T, *ux, *uy, *rho, *Fx, *Fy;
    unsigned char *chi;
    int *iters;
};

#define NT(s) ((s)->p.nthreads > 0 ? (s)->p.nthreads : 1)

static double *dalloc(long n)
{
    double *a = (double *)calloc((size_t)n, sizeof(double));
    return a;
}

orc_sim *orc_create(const orc_params *p, const double *eps, const double *K,
                    const double *Feps)
{
    orc_derived d;
    if (!eps || orc_derive(p, &d) != 0) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->p = *p;
    s->d = d;
    build_lat9(&s->L9);
    build_lat5(&s->L5, p->varpi);
    s->nx = p->nx;
    s->ny = p->ny;
    s->nc = (long)p->nx * p->ny;
    long nc = s->nc;
    s->eps = dalloc(nc);
    s->K = dalloc(nc);
    s->Feps = dalloc(nc);
    s->f = dalloc(nc * Q9);
    s->g = dalloc(nc * Q5);
    s->fl = dalloc(nc);
    s->fpost = dalloc(nc * Q9);
    s->gpost = dalloc(nc * Q5);
    s->fnew = dalloc(nc * Q9);
    s->gnew = dalloc(nc * Q5);
    s->flnew = dalloc(nc);
    s->gstr = dalloc(nc * Q5);
    s->T = dalloc(nc);
    s->ux = dalloc(nc);
    s->uy = dalloc(nc);
    s->rho = dalloc(nc);
    s->Fx = dalloc(nc);
    s->Fy = dalloc(nc);
    s->chi = (unsigned char *)calloc((size_t)nc, 1);
    s->iters = (int *)calloc((size_t)nc, sizeof(int));
    s->feps_given = Feps != NULL;
    for (long c = 0; c < nc; ++c) {
        s->eps[c] = eps[c];
        s->K[c] = K ? K[c] : d.K_default;
        /* Eq. (6) at f_l = 1 */
        s->Feps[c] = Feps ? Feps[c] : 1.75 / sqrt(p->ergun_c * pow(eps[c], 3));
    }
    /* Initial state: uniform T_init at rest.  g = g^eq(T, 0) (Eq. 39),
     * f_l = f_l(T) (Eq. 42), f = f^eq(rho0, 0) (Eq. 29) where liquid. */
    for (long c = 0; c < nc; ++c) {
        double T = p->T_init;
        for (int i = 0; i < Q5; ++i) s->g[c * Q5 + i] = s->L5.w[i] * T;
        s->fl[c] = fl_of_T(T, p->T_s, p->T_l);
        for (int i = 0; i < Q9; ++i) s->f[c * Q9 + i] = s->fl[c] > 0 ? s->L9.w[i] * RHO0 : 0.0;
    }
    s->t = 0;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    free(s->eps); free(s->K); free(s->Feps);
    free(s->f); free(s->g); free(s->fl);
    free(s->fpost); free(s->gpost); free(s->fnew); free(s->gnew); free(s->flnew); free(s->gstr);
    free(s->T); free(s->ux); free(s->uy); free(s->rho); free(s->Fx); free(s->Fy);
    free(s->chi); free(s->iters);
    free(s);
}

void orc_set_state(orc_sim *s, const double *f, const double *g, const double *fl)
{
    long nc = s->nc;
    for (long c = 0; c < nc; ++c) {
        for (int i = 0; i < Q9; ++i) s->f[c * Q9 + i] = f[i * nc + c];
        for (int i = 0; i < Q5; ++i) s->g[c * Q5 + i] = g[i * nc + c];
        s->fl[c] = fl[c];
    }
}

void orc_get_state(const orc_sim *s, double *f, double *g, double *fl)
{
    long nc = s->nc;
    for (long c = 0; c < nc; ++c) {
        for (int i = 0; i < Q9; ++i) f[i * nc + c] = s->f[c * Q9 + i];
        for (int i = 0; i < Q5; ++i) g[i * nc + c] = s->g[c * Q5 + i];
        fl[c] = s->fl[c];
    }
}

long orc_time(const orc_sim *s) { return s->t; }

/* Effective permeability and inertial coefficient at varphi = eps*fl. */
static void porous_at(double eps, double K, double Feps, double fl, double *Ke, double *Ce)
{
    if (eps >= 1.0) { /* clear fluid: no porous drag */
        *Ke = INFINITY;
        *Ce = 0.0;
        return;
    }
    double phi = eps * fl;
    *Ke = K * pow(phi / eps, 3) * pow((1.0 - eps) / (1.0 - phi), 2);
    *Ce = Feps * pow(eps / phi, 1.5);
}

/* Step 1: macroscopic quantities of cell c from the state. */
static void macros_cell(const orc_sim *s, const double *f, const double *g,
                        const double *fl, long c, double *T, double *rho, double *ux,
                        double *uy, double *Fx, double *Fy, unsigned char *chi)
{
    double Tc = 0;
    for (int i = 0; i < Q5; ++i) Tc += g[c * Q5 + i]; /* Eq. (33) */
    *T = Tc;
    *chi = fl[c] > 0;
    if (!*chi) {
        *rho = 0;
        *ux = *uy = *Fx = *Fy = 0;
        return;
    }
    double r = 0, jx = 0, jy = 0;
    for (int i = 0; i < Q9; ++i) {
        double fi = f[c * Q9 + i];
        r += fi;                       /* Eq. (24) */
        jx += s->L9.ex[i] * fi;
        jy += s->L9.ey[i] * fi;
    }
    double phi = s->eps[c] * fl[c];
    double Ke, Ce;
    porous_at(s->eps[c], s->K[c], s->Feps[c], fl[c], &Ke, &Ce);
    double Gy = s->d.gbeta * (Tc - s->p.T0); /* Eq. (5), +y */
    double u[2], F[2];
    orc_closure(jx, jy, phi, s->d.nu_l, Ke, Ce, 0.0, Gy, u, F);
    *rho = r;
    *ux = u[0];
    *uy = u[1];
    *Fx = F[0];
    *Fy = F[1];
}

/* Steps 2-3: collisions of cell c (f only where chi). */
static void collide_cell(const orc_sim *s, const double *f, const double *g,
                         const double *fl, long c, double T, double rho, double ux,
                         double uy, double Fx, double Fy, int chi, double *fpost,
                         double *gpost)
{
    const orc_params *p = &s->p;
    if (chi) {
        double sv[Q9] = {1, p->s_e, p->s_eps, 1, p->s_q, 1, p->s_q,
                         1.0 / s->d.tau_nu, 1.0 / s->d.tau_nu}; /* Eq. (23), Sec. 4 */
        double phi = s->eps[c] * fl[c];
        orc_collide_f(&f[c * Q9], rho, ux, uy, Fx, Fy, phi, sv, &fpost[c * Q9]);
    } else {
        for (int i = 0; i < Q9; ++i) fpost[c * Q9 + i] = 0;
    }
    /* D2Q5, Eqs. (32), (34), (35), (37); the source is added after streaming. */
    double sig = sigma_of(p, s->eps[c], fl[c]);
    double za = 1.0 / tauT_of(p, &s->d, s->eps[c], fl[c]);
    double theta[Q5] = {1, za, za, p->zeta_e, p->zeta_nu};
    double n[Q5], neq[Q5], np[Q5];
    for (int a = 0; a < Q5; ++a) {
        double v = 0;
        for (int i = 0; i < Q5; ++i) v += s->L5.N[a][i] * g[c * Q5 + i];
        n[a] = v;
    }
    orc_neq(T, ux, uy, sig, p->varpi, p->convective, neq);
    for (int a = 0; a < Q5; ++a) np[a] = n[a] - theta[a] * (n[a] - neq[a]);
    for (int i = 0; i < Q5; ++i) {
        double v = 0;
        for (int a = 0; a < Q5; ++a) v += s->L5.Ninv[i][a] * np[a];
        gpost[c * Q5 + i] = v;
    }
}

/* Locate the source x - e_i of a pull.  Returns 1 and the wrapped node if it
 * is a lattice node; 0 and the wall side if it lies outside. */
static int source_node(const orc_sim *s, int x, int y, int ex, int ey, int *sx, int *sy,
                       int *side)
{
    int X = x - ex, Y = y - ey, out = 0;
    *side = -1;
    if (X < 0) {
        if (s->p.bc_kind[0] == ORC_PERIODIC) X += s->nx; else { out = 1; *side = 0; }
    } else if (X >= s->nx) {
        if (s->p.bc_kind[1] == ORC_PERIODIC) X -= s->nx; else { out = 1; *side = 1; }
    }
    if (Y < 0) {
        if (s->p.bc_kind[2] == ORC_PERIODIC) Y += s->ny; else { if (!out) *side = 2; out = 1; }
    } else if (Y >= s->ny) {
        if (s->p.bc_kind[3] == ORC_PERIODIC) Y -= s->ny; else { if (!out) *side = 3; out = 1; }
    }
    *sx = X;
    *sy = Y;
    return !out;
}

/* Heat-capacity bounds of cell c for the enthalpy iteration (sigma is
 * linear in f_l in both modes). */
static void sigma_pair(const orc_sim *s, long c, double *ss, double *sl)
{
    *ss = sigma_of(&s->p, s->eps[c], 0.0);
    *sl = sigma_of(&s->p, s->eps[c], 1.0);
}

/* Latent source w~_i S0 of Eq. (38) through N^-1, added to g of cell c. */
static void add_latent(orc_sim *s, long c, double S0)
{
    double St[Q5] = {0, 0, 0, 0, 0};
    St[0] = S0;
    St[3] = s->p.varpi * S0;
    for (int i = 0; i < Q5; ++i) {
        double v = 0;
        for (int a = 0; a < Q5; ++a) v += s->L5.Ninv[i][a] * St[a];
        s->gnew[c * Q5 + i] += DT * v;
    }
}

/* R1: the source at the receiving node after streaming; a per-node fixed
 * point (Z10). */
static void latent_r1(orc_sim *s)
{
    const orc_params *p = &s->p;
    const int nt = NT(s);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long c = 0; c < s->nc; ++c) {
        double Tstar = 0;
        for (int i = 0; i < Q5; ++i) Tstar += s->gnew[c * Q5 + i];
        double fln, Tn, ss, sl;
        sigma_pair(s, c, &ss, &sl);
        s->iters[c] = orc_enthalpy(Tstar, s->fl[c], s->eps[c], p->Ste, ss, sl, cps_of(p), p->T_s,
                                   p->T_l, p->fl_tol, p->fl_maxit, &fln, &Tn);
        double sig = sigma_of(p, s->eps[c], fln);
        add_latent(s, c, -(s->eps[c] / (sig * p->Ste)) * (fln - s->fl[c]) / DT); /* Eq. (38) */
        s->flnew[c] = fln;
    }
}

/* R2: the literal Eq. (30): the source S0(x) of a node, which needs f_l at
 * the new time, is added to its post-collision populations before they
 * stream, so node y receives w~_i S0(y - e_i) from each neighbour (its own
 * S0 for i = 0 and for directions whose source lies behind a wall, whose
 * extrapolation uses the node's own post-collision population).  The new
 * f_l of all nodes is found together: a Jacobi iteration of Eqs. (40)-(42)
 * over the lattice until the largest change of f_l is at most fl_tol. */
static void latent_r2(orc_sim *s)
{
    const orc_params *p = &s->p;
    const int nx = s->nx, ny = s->ny, nt = NT(s);
    const long nc = s->nc;
    double *f = dalloc(nc), *fn = dalloc(nc), *S0 = dalloc(nc), *Ts = dalloc(nc);
    for (long c = 0; c < nc; ++c) {
        double t = 0;
        for (int i = 0; i < Q5; ++i) t += s->gnew[c * Q5 + i];
        Ts[c] = t;
        f[c] = s->fl[c];
    }
    const double w0 = (1.0 - p->varpi) / 5.0, w1 = (4.0 + p->varpi) / 20.0; /* N^-1 (1,0,0,varpi,0) */
    int it = 0;
    for (;;) {
        ++it;
#pragma omp parallel for num_threads(nt) schedule(static)
        for (long c = 0; c < nc; ++c) {
            double sig = sigma_of(p, s->eps[c], f[c]);
            S0[c] = -(s->eps[c] / (sig * p->Ste)) * (f[c] - s->fl[c]) / DT;
        }
        double delta = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(max : delta)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = (long)y * nx + x;
                double T = Ts[c] + DT * w0 * S0[c];
                for (int i = 1; i < Q5; ++i) {
                    int sx, sy, side;
                    long sc = c;
                    if (source_node(s, x, y, s->L5.ex[i], s->L5.ey[i], &sx, &sy, &side))
                        sc = (long)sy * nx + sx;
                    T += DT * w1 * S0[sc];
                }
                double En = En_of(T, f[c], p->Ste, cps_of(p)); /* Eq. (40) */
                fn[c] = fl_of_T(T_of_En(En, p->T_s, p->T_l, p->Ste, cps_of(p)), p->T_s, p->T_l);
                double dd = fabs(fn[c] - f[c]);
                if (dd > delta) delta = dd;
            }
        double *tmp = f;
        f = fn;
        fn = tmp;
        if (delta <= p->fl_tol || it >= p->fl_maxit) break;
    }
    /* the streamed sources, with the converged f_l */
    for (long c = 0; c < nc; ++c) {
        double sig = sigma_of(p, s->eps[c], f[c]);
        S0[c] = -(s->eps[c] / (sig * p->Ste)) * (f[c] - s->fl[c]) / DT;
    }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            s->gnew[c * Q5 + 0] += DT * w0 * S0[c];
            for (int i = 1; i < Q5; ++i) {
                int sx, sy, side;
                long sc = c;
                if (source_node(s, x, y, s->L5.ex[i], s->L5.ey[i], &sx, &sy, &side))
                    sc = (long)sy * nx + sx;
                s->gnew[c * Q5 + i] += DT * w1 * S0[sc];
            }
            s->flnew[c] = f[c];
            s->iters[c] = it;
        }
    free(f);
    free(fn);
    free(S0);
    free(Ts);
}

/* One time step from the state (f, g, fl) into (fnew, gnew, flnew), keeping
 * the intermediate fields (macros, post-collision populations, streamed g)
 * in the simulation's work arrays. */
static void compute_step(orc_sim *s)
{
    const orc_params *p = &s->p;
    const int nx = s->nx, ny = s->ny;
    const long nc = s->nc;
    const int nt = NT(s);

    /* Step 1: macros at time k (chi^k = [f_l^k > 0]). */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long c = 0; c < nc; ++c)
        macros_cell(s, s->f, s->g, s->fl, c, &s->T[c], &s->rho[c], &s->ux[c], &s->uy[c],
                    &s->Fx[c], &s->Fy[c], &s->chi[c]);

    /* Steps 2-3: collisions. */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long c = 0; c < nc; ++c)
        collide_cell(s, s->f, s->g, s->fl, c, s->T[c], s->rho[c], s->ux[c], s->uy[c],
                     s->Fx[c], s->Fy[c], s->chi[c], s->fpost, s->gpost);

    /* Steps 4-5: streaming, Eqs. (21) and (36), pull form, with non-equilibrium
     * extrapolation for sources that are walls (g, f) or solid nodes (f). */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            int sx, sy, side;
            double sig = sigma_of(p, s->eps[c], s->fl[c]);
            double geq_x[Q5];
            orc_geq(s->T[c], s->ux[c], s->uy[c], sig, p->varpi, geq_x);
            for (int i = 0; i < Q5; ++i) {
                if (source_node(s, x, y, s->L5.ex[i], s->L5.ey[i], &sx, &sy, &side)) {
                    s->gnew[c * Q5 + i] = s->gpost[((long)sy * nx + sx) * Q5 + i];
                } else {
                    double Tw = p->bc_kind[side] == ORC_WALL_T ? p->T_wall[side] : s->T[c];
                    double geq_w[Q5];
                    orc_geq(Tw, 0, 0, sig, p->varpi, geq_w);
                    s->gnew[c * Q5 + i] = geq_w[i] + s->gpost[c * Q5 + i] - geq_x[i];
                }
            }
            if (!s->chi[c]) {
                for (int i = 0; i < Q9; ++i) s->fnew[c * Q9 + i] = 0;
                continue;
            }
            double phi = s->eps[c] * s->fl[c];
            double feq_x[Q9], feq_w[Q9];
            orc_feq(s->rho[c], s->ux[c], s->uy[c], phi, feq_x);
            orc_feq(s->rho[c], 0, 0, phi, feq_w);
            for (int i = 0; i < Q9; ++i) {
                long sc;
                if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side) &&
                    s->chi[sc = (long)sy * nx + sx]) {
                    s->fnew[c * Q9 + i] = s->fpost[sc * Q9 + i];
                } else {
                    s->fnew[c * Q9 + i] = feq_w[i] + s->fpost[c * Q9 + i] - feq_x[i];
                }
            }
        }
    }

    memcpy(s->gstr, s->gnew, sizeof(double) * (size_t)nc * Q5);

    /* Step 6: iterated enthalpy method and the latent source N^-1 dt S~
     * (Eqs. 30, 38, 40-42). */
    if (p->latent_mode == 1)
        latent_r2(s);
    else
        latent_r1(s);

    /* Step 7: flow mask update.  A node that became liquid starts at rest,
     * f_i = w_i rho_bar, with rho_bar the mean start-of-step density of its
     * liquid lattice neighbours (rho0 if it has none); a node that became
     * solid drops its populations. */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            long c = (long)y * nx + x;
            int was = s->fl[c] > 0, now = s->flnew[c] > 0;
            if (now && !was) {
                double rsum = 0;
                int cnt = 0;
                for (int i = 1; i < Q9; ++i) {
                    int sx, sy, side;
                    if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side)) {
                        long sc = (long)sy * nx + sx;
                        if (s->chi[sc]) {
                            rsum += s->rho[sc];
                            ++cnt;
                        }
                    }
                }
                double rbar = cnt ? rsum / cnt : RHO0;
                for (int i = 0; i < Q9; ++i) s->fnew[c * Q9 + i] = s->L9.w[i] * rbar;
            } else if (!now) {
                for (int i = 0; i < Q9; ++i) s->fnew[c * Q9 + i] = 0;
            }
        }
    }

}

static void one_step(orc_sim *s)
{
    compute_step(s);
    double *tmp;
    tmp = s->f; s->f = s->fnew; s->fnew = tmp;
    tmp = s->g; s->g = s->gnew; s->gnew = tmp;
    tmp = s->fl; s->fl = s->flnew; s->flnew = tmp;
    s->t += 1;
}

void orc_step(orc_sim *s, long n)
{
    for (long k = 0; k < n; ++k) one_step(s);
}

void orc_fields(const orc_sim *s, double *T, double *ux, double *uy, double *fl, double *rho)
{
    const long nc = s->nc;
#pragma omp parallel for num_threads(NT(s)) schedule(static)
    for (long c = 0; c < nc; ++c) {
        double t, r, a, b, fx, fy;
        unsigned char chi;
        macros_cell(s, s->f, s->g, s->fl, c, &t, &r, &a, &b, &fx, &fy, &chi);
        if (T) T[c] = t;
        if (ux) ux[c] = a;
        if (uy) uy[c] = b;
        if (fl) fl[c] = s->fl[c];
        if (rho) rho[c] = r;
    }
}

void orc_post_collision(const orc_sim *s, double *fpost, double *gpost)
{
    const long nc = s->nc;
    double *fp = dalloc(nc * Q9), *gp = dalloc(nc * Q5);
#pragma omp parallel for num_threads(NT(s)) schedule(static)
    for (long c = 0; c < nc; ++c) {
        double t, r, a, b, fx, fy;
        unsigned char chi;
        macros_cell(s, s->f, s->g, s->fl, c, &t, &r, &a, &b, &fx, &fy, &chi);
        collide_cell(s, s->f, s->g, s->fl, c, t, r, a, b, fx, fy, chi, fp, gp);
    }
    for (long c = 0; c < nc; ++c) {
        for (int i = 0; i < Q9; ++i) fpost[i * nc + c] = fp[c * Q9 + i];
        for (int i = 0; i < Q5; ++i) gpost[i * nc + c] = gp[c * Q5 + i];
    }
    free(fp);
    free(gp);
}

void orc_iter_stats(const orc_sim *s, long *max_it, long *sum_it)
{
    long mx = 0, sm = 0;
    for (long c = 0; c < s->nc; ++c) {
        if (s->iters[c] > mx) mx = s->iters[c];
        sm += s->iters[c];
    }
    *max_it = mx;
    *sum_it = sm;
}

/* ====================================================================== */
/* Discrete derivatives of one time step (tangent-linear and reverse)      */
/* ====================================================================== */
/*
 * The step above is differentiated as a map from the state (f, g, f_l) at
 * time k and the per-cell parameters (ln K, eps) to the state at time k+1,
 * line by line, in FP64.  Where the map is not smooth, the derivative is
 * taken as follows:
 *   - the enthalpy update (Eqs. 38, 40-42) at its converged fixed point: on
 *     the mushy branch f = (T* + a f^k - T_s) / (T_l - T_s + a), a =
 *     eps / (sigma St); zero where f_l is clamped to 0 or 1;
 *   - the flow mask, the liquid/solid status of every pull source and the
 *     branch of each cell (melted, solidified) are held fixed;
 *   - |v| in Eq. (26) has the subgradient 0 at v = 0.
 * The derivative needs sigma and tau_T independent of f_l (sigma_s ==
 * sigma_l, alpha_ratio == 1) and the default thermal model (R1, no
 * variants); other settings are refused.
 * F_eps follows eps through Eq. (6) unless it was given per cell.
 * Vectors are in the simulation's internal layout (f[c*9+i], g[c*5+i]).
 */

/* Forward values of the velocity closure of one liquid cell, recomputed as
 * macros_cell / orc_closure compute them. */
typedef struct {
    double fl, eps, phi, Ke, Ce, Gy, vx, vy, l0, l1, vm, R, den, ux, uy, um, A, B;
    int nodrag;
} clos_fw;

static void closure_forward(const orc_sim *s, long c, double T, double jx, double jy, clos_fw *w)
{
    w->fl = s->fl[c];
    w->eps = s->eps[c];
    w->phi = w->eps * w->fl;
    porous_at(w->eps, s->K[c], s->Feps[c], w->fl, &w->Ke, &w->Ce);
    w->nodrag = !(w->eps < 1.0);
    w->Gy = s->d.gbeta * (T - s->p.T0);
    w->vx = jx;
    w->vy = jy + 0.5 * w->phi * w->Gy;
    if (w->nodrag) {
        w->l0 = 0.5;
        w->l1 = 0.0;
        w->den = 1.0;
    } else {
        w->l0 = 0.5 * (1.0 + 0.5 * w->phi * s->d.nu_l / w->Ke);
        w->l1 = 0.5 * w->phi * w->Ce / sqrt(w->Ke);
    }
    w->vm = sqrt(w->vx * w->vx + w->vy * w->vy);
    w->R = sqrt(w->l0 * w->l0 + w->l1 * w->vm);
    if (!w->nodrag) w->den = w->l0 + w->R;
    w->ux = w->vx / w->den;
    w->uy = w->vy / w->den;
    w->um = sqrt(w->ux * w->ux + w->uy * w->uy);
    w->A = w->nodrag ? 0.0 : w->phi * s->d.nu_l / w->Ke;
    w->B = w->nodrag ? 0.0 : w->phi * w->Ce / sqrt(w->Ke);
}

/* Tangent of Eqs. (4)-(6), (26)-(28): from the tangents of jx, jy, T, f_l,
 * eps and ln K to those of u, F and varphi. */
static void closure_tl(const orc_sim *s, const clos_fw *w, double djx, double djy, double dT,
                       double dfl, double deps, double dlnK, double *dux, double *duy,
                       double *dFx, double *dFy, double *dphi)
{
    const double nu = s->d.nu_l, gb = s->d.gbeta;
    const double ph = w->eps * dfl + deps * w->fl;
    const double dGy = gb * dT;
    const double dvx = djx;
    const double dvy = djy + 0.5 * (ph * w->Gy + w->phi * dGy);
    *dphi = ph;
    if (w->nodrag) {
        *dux = dvx;
        *duy = dvy;
        *dFx = 0.0;
        *dFy = ph * w->Gy + w->phi * dGy;
        return;
    }
    const double dlnFe = s->feps_given ? 0.0 : -1.5 * deps / w->eps; /* Eq. (6) */
    const double dlnKe = dlnK + 3.0 * dfl / w->fl - 2.0 * deps / (1.0 - w->eps) +
                         2.0 * ph / (1.0 - w->phi);
    const double dlnCe = dlnFe - 1.5 * dfl / w->fl;
    const double q = 0.25 * nu * w->phi / w->Ke;
    const double dl0 = q * (ph / w->phi - dlnKe);
    const double dl1 = w->l1 * (ph / w->phi + dlnCe - 0.5 * dlnKe);
    const double dvm = w->vm > 0 ? (w->vx * dvx + w->vy * dvy) / w->vm : 0.0;
    const double dR = (2.0 * w->l0 * dl0 + dl1 * w->vm + w->l1 * dvm) / (2.0 * w->R);
    const double dden = dl0 + dR;
    const double ux_d = (dvx - w->ux * dden) / w->den;
    const double uy_d = (dvy - w->uy * dden) / w->den;
    const double dum = w->um > 0 ? (w->ux * ux_d + w->uy * uy_d) / w->um : 0.0;
    const double dA = w->A * (ph / w->phi - dlnKe);
    const double dB = w->B * (ph / w->phi + dlnCe - 0.5 * dlnKe);
    *dux = ux_d;
    *duy = uy_d;
    *dFx = -dA * w->ux - w->A * ux_d - dB * w->um * w->ux - w->B * dum * w->ux -
           w->B * w->um * ux_d;
    *dFy = -dA * w->uy - w->A * uy_d - dB * w->um * w->uy - w->B * dum * w->uy -
           w->B * w->um * uy_d + ph * w->Gy + w->phi * dGy;
}

/* Reverse of closure_tl: adjoints of u, F and varphi in, adjoints of jx, jy,
 * T, f_l, eps and ln K added to the outputs. */
static void closure_ad(const orc_sim *s, const clos_fw *w, double bux, double buy, double bFx,
                       double bFy, double bphi, double *bjx, double *bjy, double *bT,
                       double *bfl, double *beps, double *blnK)
{
    const double nu = s->d.nu_l, gb = s->d.gbeta;
    double bGy = 0.0, bvx = 0.0, bvy = 0.0;
    if (w->nodrag) {
        bphi += w->Gy * bFy;
        bGy += w->phi * bFy;
        bvx = bux;
        bvy = buy;
    } else {
        double bA = 0, bB = 0, bum = 0, blnKe = 0, blnCe = 0, bden = 0, bl0 = 0, bl1 = 0;
        double bR = 0, bvm = 0;
        /* F */
        bA += -w->ux * bFx - w->uy * bFy;
        bB += -w->um * w->ux * bFx - w->um * w->uy * bFy;
        bum += -w->B * w->ux * bFx - w->B * w->uy * bFy;
        bux += (-w->A - w->B * w->um) * bFx;
        buy += (-w->A - w->B * w->um) * bFy;
        bphi += w->Gy * bFy;
        bGy += w->phi * bFy;
        /* B, A */
        bphi += w->B / w->phi * bB + w->A / w->phi * bA;
        blnCe += w->B * bB;
        blnKe += -0.5 * w->B * bB - w->A * bA;
        /* |u| */
        if (w->um > 0) {
            bux += w->ux / w->um * bum;
            buy += w->uy / w->um * bum;
        }
        /* u = v / den */
        bvx += bux / w->den;
        bvy += buy / w->den;
        bden += -(w->ux * bux + w->uy * buy) / w->den;
        bl0 += bden;
        bR += bden;
        bl0 += w->l0 / w->R * bR;
        bl1 += w->vm / (2.0 * w->R) * bR;
        bvm += w->l1 / (2.0 * w->R) * bR;
        if (w->vm > 0) {
            bvx += w->vx / w->vm * bvm;
            bvy += w->vy / w->vm * bvm;
        }
        /* l1, l0 */
        bphi += w->l1 / w->phi * bl1;
        blnCe += w->l1 * bl1;
        blnKe += -0.5 * w->l1 * bl1;
        const double q = 0.25 * nu * w->phi / w->Ke;
        bphi += q / w->phi * bl0;
        blnKe += -q * bl0;
        /* ln C_e, ln K_e */
        *bfl += -1.5 / w->fl * blnCe;
        if (!s->feps_given) *beps += -1.5 / w->eps * blnCe;
        *blnK += blnKe;
        *bfl += 3.0 / w->fl * blnKe;
        *beps += -2.0 / (1.0 - w->eps) * blnKe;
        bphi += 2.0 / (1.0 - w->phi) * blnKe;
    }
    /* v */
    *bjx += bvx;
    *bjy += bvy;
    bphi += 0.5 * w->Gy * bvy;
    bGy += 0.5 * w->phi * bvy;
    *bT += gb * bGy;
    *beps += w->fl * bphi;
    *bfl += w->eps * bphi;
}

/* Rates of Eq. (23). */
static void rates9(const orc_sim *s, double *sv)
{
    const orc_params *p = &s->p;
    double r[Q9] = {1, p->s_e, p->s_eps, 1, p->s_q, 1, p->s_q, 1.0 / s->d.tau_nu,
                    1.0 / s->d.tau_nu};
    memcpy(sv, r, sizeof r);
}

/* Tangent of the D2Q9 collision (Eqs. 19, 20, 22) of one liquid cell. */
static void collide_f_tl(const orc_sim *s, const double *df, double drho, double ux, double uy,
                         double Fx, double Fy, double phi, double dux, double duy, double dFx,
                         double dFy, double dphi, double *dfp)
{
    double sv[Q9], dm[Q9], dmeq[Q9], dS[Q9], dmp[Q9];
    rates9(s, sv);
    for (int a = 0; a < Q9; ++a) {
        double v = 0;
        for (int i = 0; i < Q9; ++i) v += s->L9.M[a][i] * df[i];
        dm[a] = v;
    }
    const double q = (ux * ux + uy * uy) / phi;
    const double dq = (2 * ux * dux + 2 * uy * duy) / phi - q * dphi / phi;
    const double m7 = (ux * ux - uy * uy) / phi, m8 = ux * uy / phi;
    dmeq[0] = drho;
    dmeq[1] = -2 * drho + 3 * dq;
    dmeq[2] = drho - 3 * dq;
    dmeq[3] = dux;
    dmeq[4] = -dux;
    dmeq[5] = duy;
    dmeq[6] = -duy;
    dmeq[7] = (2 * ux * dux - 2 * uy * duy) / phi - m7 * dphi / phi;
    dmeq[8] = (dux * uy + ux * duy) / phi - m8 * dphi / phi;
    const double uF = ux * Fx + uy * Fy;
    const double duF = dux * Fx + ux * dFx + duy * Fy + uy * dFy;
    const double S1 = 6 * uF / phi, S7 = 2 * (ux * Fx - uy * Fy) / phi,
                 S8 = (ux * Fy + uy * Fx) / phi;
    dS[0] = 0;
    dS[1] = 6 * duF / phi - S1 * dphi / phi;
    dS[2] = -dS[1];
    dS[3] = dFx;
    dS[4] = -dFx;
    dS[5] = dFy;
    dS[6] = -dFy;
    dS[7] = 2 * (dux * Fx + ux * dFx - duy * Fy - uy * dFy) / phi - S7 * dphi / phi;
    dS[8] = (dux * Fy + ux * dFy + duy * Fx + uy * dFx) / phi - S8 * dphi / phi;
    for (int a = 0; a < Q9; ++a)
        dmp[a] = dm[a] - sv[a] * (dm[a] - dmeq[a]) + DT * (1.0 - sv[a] / 2.0) * dS[a];
    for (int i = 0; i < Q9; ++i) {
        double v = 0;
        for (int a = 0; a < Q9; ++a) v += s->L9.Minv[i][a] * dmp[a];
        dfp[i] = v;
    }
}

/* Reverse of collide_f_tl: adjoint of f+ in; adjoints of f, rho, u, F and
 * varphi added to the outputs. */
static void collide_f_ad(const orc_sim *s, const double *bfp, double ux, double uy, double Fx,
                         double Fy, double phi, double *bf, double *brho, double *bux,
                         double *buy, double *bFx, double *bFy, double *bphi)
{
    double sv[Q9], bmp[Q9], bm[Q9], bmeq[Q9], bS[Q9];
    rates9(s, sv);
    for (int a = 0; a < Q9; ++a) {
        double v = 0;
        for (int i = 0; i < Q9; ++i) v += s->L9.Minv[i][a] * bfp[i];
        bmp[a] = v;
    }
    for (int a = 0; a < Q9; ++a) {
        bm[a] = (1.0 - sv[a]) * bmp[a];
        bmeq[a] = sv[a] * bmp[a];
        bS[a] = DT * (1.0 - sv[a] / 2.0) * bmp[a];
    }
    for (int i = 0; i < Q9; ++i) {
        double v = 0;
        for (int a = 0; a < Q9; ++a) v += s->L9.M[a][i] * bm[a];
        bf[i] += v;
    }
    const double q = (ux * ux + uy * uy) / phi;
    const double m7 = (ux * ux - uy * uy) / phi, m8 = ux * uy / phi;
    *brho += bmeq[0] - 2 * bmeq[1] + bmeq[2];
    const double bq = 3 * bmeq[1] - 3 * bmeq[2];
    *bux += 2 * ux / phi * bq + bmeq[3] - bmeq[4] + 2 * ux / phi * bmeq[7] + uy / phi * bmeq[8];
    *buy += 2 * uy / phi * bq + bmeq[5] - bmeq[6] - 2 * uy / phi * bmeq[7] + ux / phi * bmeq[8];
    *bphi += -q / phi * bq - m7 / phi * bmeq[7] - m8 / phi * bmeq[8];
    const double uF = ux * Fx + uy * Fy;
    const double S1 = 6 * uF / phi, S7 = 2 * (ux * Fx - uy * Fy) / phi,
                 S8 = (ux * Fy + uy * Fx) / phi;
    const double b1 = bS[1] - bS[2];
    const double buF = 6 / phi * b1;
    *bphi += -S1 / phi * b1 - S7 / phi * bS[7] - S8 / phi * bS[8];
    *bFx += bS[3] - bS[4];
    *bFy += bS[5] - bS[6];
    *bux += 2 / phi * Fx * bS[7] + Fy / phi * bS[8] + Fx * buF;
    *bFx += 2 / phi * ux * bS[7] + uy / phi * bS[8] + ux * buF;
    *buy += -2 / phi * Fy * bS[7] + Fx / phi * bS[8] + Fy * buF;
    *bFy += -2 / phi * uy * bS[7] + ux / phi * bS[8] + uy * buF;
}

/* Tangent of the D2Q5 collision (Eqs. 34, 35, 37) with uniform sigma, tau_T. */
static void collide_g_tl(const orc_sim *s, long c, const double *dg, double dT, double T,
                         double ux, double uy, double dux, double duy, double *dgp)
{
    const orc_params *p = &s->p;
    const double sig = p->sigma_s, th = p->convective ? 1.0 : 0.0;
    const double za = 1.0 / tauT_of(p, &s->d, s->eps[c], s->fl[c]);
    const double theta[Q5] = {1, za, za, p->zeta_e, p->zeta_nu};
    double dn[Q5], dneq[Q5], dnp[Q5];
    for (int a = 0; a < Q5; ++a) {
        double v = 0;
        for (int i = 0; i < Q5; ++i) v += s->L5.N[a][i] * dg[i];
        dn[a] = v;
    }
    dneq[0] = dT;
    dneq[1] = th * (dux * T + ux * dT) / sig;
    dneq[2] = th * (duy * T + uy * dT) / sig;
    dneq[3] = p->varpi * dT;
    dneq[4] = 0;
    for (int a = 0; a < Q5; ++a) dnp[a] = dn[a] - theta[a] * (dn[a] - dneq[a]);
    for (int i = 0; i < Q5; ++i) {
        double v = 0;
        for (int a = 0; a < Q5; ++a) v += s->L5.Ninv[i][a] * dnp[a];
        dgp[i] = v;
    }
}

static void collide_g_ad(const orc_sim *s, long c, const double *bgp, double T, double ux,
                         double uy, double *bg, double *bT, double *bux, double *buy)
{
    const orc_params *p = &s->p;
    const double sig = p->sigma_s, th = p->convective ? 1.0 : 0.0;
    const double za = 1.0 / tauT_of(p, &s->d, s->eps[c], s->fl[c]);
    const double theta[Q5] = {1, za, za, p->zeta_e, p->zeta_nu};
    double bnp[Q5], bn[Q5], bneq[Q5];
    for (int a = 0; a < Q5; ++a) {
        double v = 0;
        for (int i = 0; i < Q5; ++i) v += s->L5.Ninv[i][a] * bgp[i];
        bnp[a] = v;
        bn[a] = (1.0 - theta[a]) * bnp[a];
        bneq[a] = theta[a] * bnp[a];
    }
    for (int i = 0; i < Q5; ++i) {
        double v = 0;
        for (int a = 0; a < Q5; ++a) v += s->L5.N[a][i] * bn[a];
        bg[i] += v;
    }
    *bT += bneq[0] + p->varpi * bneq[3] + th * (ux * bneq[1] + uy * bneq[2]) / sig;
    *bux += th * T / sig * bneq[1];
    *buy += th * T / sig * bneq[2];
}

/* The latent weights w~ = N^-1 (1, 0, 0, varpi, 0) of add_latent. */
static void latent_weights(const orc_sim *s, double *wt)
{
    for (int i = 0; i < Q5; ++i) wt[i] = s->L5.Ninv[i][0] + s->p.varpi * s->L5.Ninv[i][3];
}

static int adjoint_scope(const orc_sim *s)
{
    const orc_params *p = &s->p;
    if (p->latent_mode != 0 || p->sigma_mode != 0 || p->ke_mode != 0) return -1;
    if (p->sigma_s != p->sigma_l || p->alpha_ratio != 1.0) return -2;
    return 0;
}

/* Tangent of one step at the current state, internal layout; NULL parameter
 * tangents are zero. */
static void step_tl(orc_sim *s, const double *df, const double *dg, const double *dfl,
                    const double *dlnK, const double *deps, double *dfn, double *dgn,
                    double *dfln)
{
    const orc_params *p = &s->p;
    const int nx = s->nx, ny = s->ny;
    const long nc = s->nc;
    compute_step(s);
    double *dT = dalloc(nc), *dux = dalloc(nc), *duy = dalloc(nc), *dphi = dalloc(nc);
    double *drho = dalloc(nc), *dfp = dalloc(nc * Q9), *dgp = dalloc(nc * Q5);
    double *dgs = dalloc(nc * Q5), *dfs = dalloc(nc * Q9);
    for (long c = 0; c < nc; ++c) {
        double t = 0;
        for (int i = 0; i < Q5; ++i) t += dg[c * Q5 + i];
        dT[c] = t;
        if (s->chi[c]) {
            double r = 0, jx = 0, jy = 0, djx = 0, djy = 0;
            for (int i = 0; i < Q9; ++i) {
                const double fi = s->f[c * Q9 + i], di = df[c * Q9 + i];
                r += di;
                jx += s->L9.ex[i] * fi;
                jy += s->L9.ey[i] * fi;
                djx += s->L9.ex[i] * di;
                djy += s->L9.ey[i] * di;
            }
            drho[c] = r;
            clos_fw w;
            closure_forward(s, c, s->T[c], jx, jy, &w);
            double dFx, dFy;
            closure_tl(s, &w, djx, djy, t, dfl[c], deps ? deps[c] : 0.0, dlnK ? dlnK[c] : 0.0,
                       &dux[c], &duy[c], &dFx, &dFy, &dphi[c]);
            collide_f_tl(s, &df[c * Q9], drho[c], s->ux[c], s->uy[c], s->Fx[c], s->Fy[c],
                         s->eps[c] * s->fl[c], dux[c], duy[c], dFx, dFy, dphi[c], &dfp[c * Q9]);
        }
        collide_g_tl(s, c, &dg[c * Q5], dT[c], s->T[c], s->ux[c], s->uy[c], dux[c], duy[c],
                     &dgp[c * Q5]);
    }
    const double cu = 1.0 / (p->sigma_s * s->d.csT2);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            int sx, sy, side;
            for (int i = 0; i < Q5; ++i) {
                if (source_node(s, x, y, s->L5.ex[i], s->L5.ey[i], &sx, &sy, &side)) {
                    dgs[c * Q5 + i] = dgp[((long)sy * nx + sx) * Q5 + i];
                } else {
                    const double w5 = s->L5.w[i];
                    const double eu = s->L5.ex[i] * s->ux[c] + s->L5.ey[i] * s->uy[c];
                    const double deu = s->L5.ex[i] * dux[c] + s->L5.ey[i] * duy[c];
                    const double dTw = p->bc_kind[side] == ORC_WALL_T ? 0.0 : w5 * dT[c];
                    dgs[c * Q5 + i] = dTw + dgp[c * Q5 + i] -
                                      w5 * (dT[c] * (1.0 + eu * cu) + s->T[c] * deu * cu);
                }
            }
            if (!s->chi[c]) continue;
            const double ph = s->eps[c] * s->fl[c];
            const double ux = s->ux[c], uy = s->uy[c], uu = ux * ux + uy * uy;
            for (int i = 0; i < Q9; ++i) {
                long sc;
                if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side) &&
                    s->chi[sc = (long)sy * nx + sx]) {
                    dfs[c * Q9 + i] = dfp[sc * Q9 + i];
                } else {
                    const double eu = s->L9.ex[i] * ux + s->L9.ey[i] * uy;
                    const double deu = s->L9.ex[i] * dux[c] + s->L9.ey[i] * duy[c];
                    const double duu = 2 * (ux * dux[c] + uy * duy[c]);
                    dfs[c * Q9 + i] = dfp[c * Q9 + i] -
                        s->L9.w[i] * (3 * deu + 9 * eu * deu / ph - 4.5 * eu * eu * dphi[c] / (ph * ph) -
                                      1.5 * duu / ph + 1.5 * uu * dphi[c] / (ph * ph));
                }
            }
        }
    double wt[Q5];
    latent_weights(s, wt);
    const double dTm = p->T_l - p->T_s;
    for (long c = 0; c < nc; ++c) {
        double dTs = 0;
        for (int i = 0; i < Q5; ++i) dTs += dgs[c * Q5 + i];
        const double a = s->eps[c] / (p->sigma_s * p->Ste);
        const double da = (deps ? deps[c] : 0.0) / (p->sigma_s * p->Ste);
        const double fk = s->fl[c], fn = s->flnew[c];
        const double d1 = (fn > 0 && fn < 1) ? (dTs + a * dfl[c] + (fk - fn) * da) / (dTm + a) : 0.0;
        const double dS0 = -da * (fn - fk) - a * (d1 - dfl[c]);
        for (int i = 0; i < Q5; ++i) dgn[c * Q5 + i] = dgs[c * Q5 + i] + DT * wt[i] * dS0;
        dfln[c] = d1;
    }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            const int was = s->fl[c] > 0, now = s->flnew[c] > 0;
            if (now && !was) {
                double dsum = 0;
                int cnt = 0;
                for (int i = 1; i < Q9; ++i) {
                    int sx, sy, side;
                    if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side)) {
                        const long sc = (long)sy * nx + sx;
                        if (s->chi[sc]) {
                            dsum += drho[sc];
                            ++cnt;
                        }
                    }
                }
                for (int i = 0; i < Q9; ++i) dfn[c * Q9 + i] = cnt ? s->L9.w[i] * dsum / cnt : 0.0;
            } else if (!now) {
                for (int i = 0; i < Q9; ++i) dfn[c * Q9 + i] = 0.0;
            } else {
                for (int i = 0; i < Q9; ++i) dfn[c * Q9 + i] = dfs[c * Q9 + i];
            }
        }
    free(dT); free(dux); free(duy); free(dphi); free(drho); free(dfp); free(dgp); free(dgs);
    free(dfs);
}

/* Reverse of step_tl at the current state: adjoints of the next state in,
 * adjoints of the current state out, parameter adjoints added to blnK, beps. */
static void step_ad(orc_sim *s, const double *bfn, const double *bgn, const double *bfln,
                    double *bf, double *bg, double *bfl, double *blnK, double *beps)
{
    const orc_params *p = &s->p;
    const int nx = s->nx, ny = s->ny;
    const long nc = s->nc;
    compute_step(s);
    double *bT = dalloc(nc), *bux = dalloc(nc), *buy = dalloc(nc), *bphi = dalloc(nc);
    double *brho = dalloc(nc), *bfp = dalloc(nc * Q9), *bgp = dalloc(nc * Q5);
    double *bgs = dalloc(nc * Q5), *bfs = dalloc(nc * Q9);
    memset(bf, 0, sizeof(double) * (size_t)nc * Q9);
    memset(bg, 0, sizeof(double) * (size_t)nc * Q5);
    memset(bfl, 0, sizeof(double) * (size_t)nc);
    /* mask update */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            const int was = s->fl[c] > 0, now = s->flnew[c] > 0;
            if (now && !was) {
                double br = 0;
                for (int i = 0; i < Q9; ++i) br += s->L9.w[i] * bfn[c * Q9 + i];
                long nb[Q9];
                int cnt = 0;
                for (int i = 1; i < Q9; ++i) {
                    int sx, sy, side;
                    if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side)) {
                        const long sc = (long)sy * nx + sx;
                        if (s->chi[sc]) nb[cnt++] = sc;
                    }
                }
                for (int k = 0; k < cnt; ++k) brho[nb[k]] += br / cnt;
            } else if (now) {
                for (int i = 0; i < Q9; ++i) bfs[c * Q9 + i] = bfn[c * Q9 + i];
            }
        }
    /* latent source and enthalpy fixed point */
    double wt[Q5];
    latent_weights(s, wt);
    const double dTm = p->T_l - p->T_s;
    for (long c = 0; c < nc; ++c) {
        const double a = s->eps[c] / (p->sigma_s * p->Ste);
        const double fk = s->fl[c], fn = s->flnew[c];
        double bS0 = 0;
        for (int i = 0; i < Q5; ++i) {
            bgs[c * Q5 + i] = bgn[c * Q5 + i];
            bS0 += DT * wt[i] * bgn[c * Q5 + i];
        }
        double ba = -(fn - fk) * bS0;
        const double b1 = bfln[c] - a * bS0;
        bfl[c] += a * bS0;
        if (fn > 0 && fn < 1) {
            const double bTs = b1 / (dTm + a);
            bfl[c] += a * b1 / (dTm + a);
            ba += (fk - fn) * b1 / (dTm + a);
            for (int i = 0; i < Q5; ++i) bgs[c * Q5 + i] += bTs;
        }
        beps[c] += ba / (p->sigma_s * p->Ste);
    }
    /* streaming (adjoint of the gathers) */
    const double cu = 1.0 / (p->sigma_s * s->d.csT2);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const long c = (long)y * nx + x;
            int sx, sy, side;
            for (int i = 0; i < Q5; ++i) {
                const double b = bgs[c * Q5 + i];
                if (source_node(s, x, y, s->L5.ex[i], s->L5.ey[i], &sx, &sy, &side)) {
                    bgp[((long)sy * nx + sx) * Q5 + i] += b;
                } else {
                    const double w5 = s->L5.w[i];
                    const double eu = s->L5.ex[i] * s->ux[c] + s->L5.ey[i] * s->uy[c];
                    if (p->bc_kind[side] != ORC_WALL_T) bT[c] += w5 * b;
                    bgp[c * Q5 + i] += b;
                    bT[c] += -w5 * (1.0 + eu * cu) * b;
                    bux[c] += -w5 * s->T[c] * cu * s->L5.ex[i] * b;
                    buy[c] += -w5 * s->T[c] * cu * s->L5.ey[i] * b;
                }
            }
            if (!s->chi[c]) continue;
            const double ph = s->eps[c] * s->fl[c];
            const double ux = s->ux[c], uy = s->uy[c], uu = ux * ux + uy * uy;
            for (int i = 0; i < Q9; ++i) {
                const double b = bfs[c * Q9 + i];
                long sc;
                if (source_node(s, x, y, s->L9.ex[i], s->L9.ey[i], &sx, &sy, &side) &&
                    s->chi[sc = (long)sy * nx + sx]) {
                    bfp[sc * Q9 + i] += b;
                } else {
                    const double wi = s->L9.w[i];
                    const double eu = s->L9.ex[i] * ux + s->L9.ey[i] * uy;
                    bfp[c * Q9 + i] += b;
                    const double beu = -wi * (3 + 9 * eu / ph) * b;
                    const double buu = wi * 1.5 / ph * b;
                    bux[c] += s->L9.ex[i] * beu + 2 * ux * buu;
                    buy[c] += s->L9.ey[i] * beu + 2 * uy * buu;
                    bphi[c] += -wi * (-4.5 * eu * eu / (ph * ph) + 1.5 * uu / (ph * ph)) * b;
                }
            }
        }
    /* collisions and macros */
    for (long c = 0; c < nc; ++c) {
        collide_g_ad(s, c, &bgp[c * Q5], s->T[c], s->ux[c], s->uy[c], &bg[c * Q5], &bT[c],
                     &bux[c], &buy[c]);
        if (s->chi[c]) {
            double bFx = 0, bFy = 0;
            collide_f_ad(s, &bfp[c * Q9], s->ux[c], s->uy[c], s->Fx[c], s->Fy[c],
                         s->eps[c] * s->fl[c], &bf[c * Q9], &brho[c], &bux[c], &buy[c], &bFx,
                         &bFy, &bphi[c]);
            double jx = 0, jy = 0;
            for (int i = 0; i < Q9; ++i) {
                jx += s->L9.ex[i] * s->f[c * Q9 + i];
                jy += s->L9.ey[i] * s->f[c * Q9 + i];
            }
            clos_fw w;
            closure_forward(s, c, s->T[c], jx, jy, &w);
            double bjx = 0, bjy = 0;
            closure_ad(s, &w, bux[c], buy[c], bFx, bFy, bphi[c], &bjx, &bjy, &bT[c], &bfl[c],
                       &beps[c], &blnK[c]);
            for (int i = 0; i < Q9; ++i)
                bf[c * Q9 + i] += brho[c] + s->L9.ex[i] * bjx + s->L9.ey[i] * bjy;
        }
        for (int i = 0; i < Q5; ++i) bg[c * Q5 + i] += bT[c];
    }
    free(bT); free(bux); free(buy); free(bphi); free(brho); free(bfp); free(bgp); free(bgs);
    free(bfs);
}

static void to_internal(const orc_sim *s, const double *src, double *dst, int q)
{
    for (long c = 0; c < s->nc; ++c)
        for (int i = 0; i < q; ++i) dst[c * q + i] = src ? src[i * s->nc + c] : 0.0;
}

static void to_planar(const orc_sim *s, const double *src, double *dst, int q)
{
    for (long c = 0; c < s->nc; ++c)
        for (int i = 0; i < q; ++i) dst[i * s->nc + c] = src[c * q + i];
}

int orc_step_tl(orc_sim *s, const double *df, const double *dg, const double *dfl,
                const double *dlnK, const double *deps, double *dfn, double *dgn, double *dfln)
{
    if (adjoint_scope(s)) return -1;
    const long nc = s->nc;
    double *a = dalloc(nc * Q9), *b = dalloc(nc * Q5), *c = dalloc(nc);
    double *ao = dalloc(nc * Q9), *bo = dalloc(nc * Q5);
    to_internal(s, df, a, Q9);
    to_internal(s, dg, b, Q5);
    to_internal(s, dfl, c, 1);
    step_tl(s, a, b, c, dlnK, deps, ao, bo, dfln);
    to_planar(s, ao, dfn, Q9);
    to_planar(s, bo, dgn, Q5);
    free(a); free(b); free(c); free(ao); free(bo);
    return 0;
}

int orc_step_ad(orc_sim *s, const double *bfn, const double *bgn, const double *bfln,
                double *bf, double *bg, double *bfl, double *blnK, double *beps)
{
    if (adjoint_scope(s)) return -1;
    const long nc = s->nc;
    double *a = dalloc(nc * Q9), *b = dalloc(nc * Q5), *c = dalloc(nc);
    double *ao = dalloc(nc * Q9), *bo = dalloc(nc * Q5);
    to_internal(s, bfn, a, Q9);
    to_internal(s, bgn, b, Q5);
    to_internal(s, bfln, c, 1);
    step_ad(s, a, b, c, ao, bo, bfl, blnK, beps);
    to_planar(s, ao, bf, Q9);
    to_planar(s, bo, bg, Q5);
    free(a); free(b); free(c); free(ao); free(bo);
    return 0;
}

int orc_adjoint_run(orc_sim *s, long n, const double *dL_dT, const double *dL_dfl,
                    double *grad_lnK, double *grad_eps)
{
    if (adjoint_scope(s)) return -1;
    if (n < 1) return -2;
    const long nc = s->nc;
    const size_t per = (size_t)nc * (Q9 + Q5 + 1);
    if ((double)per * n * sizeof(double) > 4e9) return -3; /* keeps every state */
    double *hist = (double *)malloc(per * (size_t)n * sizeof(double));
    if (!hist) return -4;
    const long t0 = s->t;
    for (long k = 0; k < n; ++k) {
        double *h = hist + per * (size_t)k;
        memcpy(h, s->f, sizeof(double) * nc * Q9);
        memcpy(h + nc * Q9, s->g, sizeof(double) * nc * Q5);
        memcpy(h + nc * (Q9 + Q5), s->fl, sizeof(double) * nc);
        one_step(s);
    }
    double *bfn = dalloc(nc * Q9), *bgn = dalloc(nc * Q5), *bfln = dalloc(nc);
    double *bf = dalloc(nc * Q9), *bg = dalloc(nc * Q5), *bfl = dalloc(nc);
    for (long c = 0; c < nc; ++c) {
        for (int i = 0; i < Q5; ++i) bgn[c * Q5 + i] = dL_dT ? dL_dT[c] : 0.0; /* T = sum g */
        bfln[c] = dL_dfl ? dL_dfl[c] : 0.0;
        grad_lnK[c] = 0.0;
        grad_eps[c] = 0.0;
    }
    for (long k = n - 1; k >= 0; --k) {
        const double *h = hist + per * (size_t)k;
        memcpy(s->f, h, sizeof(double) * nc * Q9);
        memcpy(s->g, h + nc * Q9, sizeof(double) * nc * Q5);
        memcpy(s->fl, h + nc * (Q9 + Q5), sizeof(double) * nc);
        step_ad(s, bfn, bgn, bfln, bf, bg, bfl, grad_lnK, grad_eps);
        double *t;
        t = bfn; bfn = bf; bf = t;
        t = bgn; bgn = bg; bg = t;
        t = bfln; bfln = bfl; bfl = t;
    }
    /* the reverse sweep ended on the state of step 0, the initial state */
    s->t = t0;
    free(hist); free(bfn); free(bgn); free(bfln); free(bf); free(bg); free(bfl);
    return 0;
}
