/* Runs the FP64 oracle over small lattices that exercise every code path
 * (walls of each kind, periodic sides, melting and freezing with flow, the
 * thermal-model variants and the latent source before streaming) so that
 * the oracle can be built and checked under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exit status 0 when every run stays finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "dmrt_oracle.h"

static int run(int nx, int ny, const int kind[4], int sigma_mode, int ke_mode, int latent_mode,
               double Ra)
{
    orc_params p;
    orc_default_params(&p);
    p.nx = nx;
    p.ny = ny;
    p.H = ny;
    for (int k = 0; k < 4; ++k) {
        p.bc_kind[k] = kind[k];
        p.T_wall[k] = k == 0 ? 1.0 : 0.2;
    }
    p.Ra = Ra;
    p.Da = 5e-3;
    p.Pr = 1.0;
    p.Ste = 0.5;
    p.T_s = 0.38;
    p.T_l = 0.42;
    p.T_init = kind[0] == ORC_WALL_T ? 0.35 : 0.40; /* mushy start without a hot wall */
    p.fl_maxit = 300;
    p.sigma_mode = sigma_mode;
    p.cps_ratio = 0.93;
    p.cm_ratio = 1.2;
    p.ke_mode = ke_mode;
    p.ks_ratio = 2.0;
    p.km_ratio = 0.02;
    p.latent_mode = latent_mode;
    p.nthreads = 1;
    const long nc = (long)nx * ny;
    double *eps = malloc(nc * sizeof(double)), *K = malloc(nc * sizeof(double));
    for (long c = 0; c < nc; ++c) {
        eps[c] = 0.35 + 0.3 * (double)((c * 7919) % 101) / 101.0;
        K[c] = 5e-3 * ny * ny * (0.5 + (double)((c * 104729) % 97) / 97.0);
    }
    orc_sim *s = orc_create(&p, eps, K, NULL);
    if (!s) {
        fprintf(stderr, "orc_create failed\n");
        return 1;
    }
    orc_step(s, 150);
    double *T = malloc(nc * sizeof(double)), *ux = malloc(nc * sizeof(double));
    double *uy = malloc(nc * sizeof(double)), *fl = malloc(nc * sizeof(double));
    double *rho = malloc(nc * sizeof(double));
    orc_fields(s, T, ux, uy, fl, rho);
    double *f = malloc(9 * nc * sizeof(double)), *g = malloc(5 * nc * sizeof(double));
    orc_get_state(s, f, g, fl);
    orc_set_state(s, f, g, fl);
    orc_step(s, 2);
    orc_post_collision(s, f, g);
    long mx, sum;
    orc_iter_stats(s, &mx, &sum);
    int bad = 0;
    double melted = 0;
    for (long c = 0; c < nc; ++c) {
        bad += !isfinite(T[c]) + !isfinite(ux[c]) + !isfinite(uy[c]) + !isfinite(fl[c]);
        melted += fl[c];
    }
    printf("%dx%d kinds %d%d%d%d sigma %d ke %d latent %d: melted %.3f, max sweeps %ld, bad %d\n",
           nx, ny, kind[0], kind[1], kind[2], kind[3], sigma_mode, ke_mode, latent_mode,
           melted / nc, mx, bad);
    orc_destroy(s);
    free(eps); free(K); free(T); free(ux); free(uy); free(fl); free(rho); free(f); free(g);
    return bad != 0;
}

int main(void)
{
    const int box[4] = {ORC_WALL_T, ORC_WALL_T, ORC_WALL_ADIABATIC, ORC_WALL_ADIABATIC};
    const int mixed[4] = {ORC_WALL_ADIABATIC, ORC_WALL_T, ORC_WALL_T, ORC_WALL_ADIABATIC};
    const int per[4] = {ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC, ORC_PERIODIC};
    const int slab[4] = {ORC_WALL_T, ORC_WALL_ADIABATIC, ORC_PERIODIC, ORC_PERIODIC};
    int rc = 0;
    rc |= run(19, 13, box, 0, 0, 0, 2e5);
    rc |= run(17, 11, mixed, 1, 1, 0, 2e5);
    rc |= run(12, 9, per, 0, 0, 1, 1e5);
    rc |= run(23, 3, slab, 1, 0, 1, 0.0);
    rc |= run(1, 1, per, 0, 1, 0, 1e5);
    return rc;
}
