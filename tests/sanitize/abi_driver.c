/* Host-side paths of the C ABI that need no GPU (defaults, the lattice
 * constants, argument validation of create / batch_create and of calls on
 * null handles), for a build of the library under AddressSanitizer and
 * UndefinedBehaviorSanitizer.  Exit status 0 when every call answers as
 * documented. */
#include <stdio.h>
#include <string.h>

#include "dmrt.h"

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "line %d: %s\n", __LINE__, #cond);        \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void)
{
    dmrt_opts o;
    dmrt_opts_default(&o);
    dmrt_grid g = {16, 8, 0.0};
    dmrt_derived d;
    CHECK(dmrt_derive(&g, 1e5, 1e-3, 1.0, 1.0, &o, &d) == DMRT_OK && d.tau_nu > 0.5);
    CHECK(dmrt_derive(&g, 1e5, 1e-3, 1.0, 1.0, NULL, &d) == DMRT_OK);
    CHECK(dmrt_derive(NULL, 1e5, 1e-3, 1.0, 1.0, &o, &d) == DMRT_EINVAL);
    dmrt_bc bc;
    memset(&bc, 0, sizeof bc);
    bc.kind[0] = bc.kind[1] = DMRT_WALL_T;
    bc.kind[2] = bc.kind[3] = DMRT_WALL_ADIABATIC;
    float eps[16 * 8];
    for (int i = 0; i < 16 * 8; ++i) eps[i] = 0.5f;
    dmrt_t* h = (dmrt_t*)1;
    /* each of these is rejected before the device is touched */
    dmrt_opts bad = o;
    bad.T_l = bad.T_s;
    CHECK(dmrt_create(&g, eps, NULL, NULL, 1e5, 1e-3, 1.0, 1.0, &bc, &bad, &h) == DMRT_EINVAL && !h);
    bad = o;
    bad.sigma_mode = 3;
    CHECK(dmrt_create(&g, eps, NULL, NULL, 1e5, 1e-3, 1.0, 1.0, &bc, &bad, &h) == DMRT_EINVAL);
    bad = o;
    bad.store_hint = 9;
    CHECK(dmrt_create(&g, eps, NULL, NULL, 1e5, 1e-3, 1.0, 1.0, &bc, &bad, &h) == DMRT_EINVAL);
    CHECK(dmrt_create(&g, NULL, NULL, NULL, 1e5, 1e-3, 1.0, 1.0, &bc, &o, &h) == DMRT_EINVAL);
    dmrt_grid g0 = {0, 8, 0.0};
    CHECK(dmrt_create(&g0, eps, NULL, NULL, 1e5, 1e-3, 1.0, 1.0, &bc, &o, &h) == DMRT_EINVAL);
    CHECK(strlen(dmrt_last_error()) > 0);
    dmrt_cavity cav[2];
    for (int i = 0; i < 2; ++i) {
        cav[i].grid = g;
        cav[i].bc = bc;
        cav[i].eps = 0.5;
        cav[i].Ra = 1e5;
        cav[i].Da = 1e-3;
        cav[i].Pr = 1.0;
        cav[i].Ste = 1.0;
    }
    cav[1].eps = 1.5;
    dmrt_batch_t* b = (dmrt_batch_t*)1;
    CHECK(dmrt_batch_create(2, cav, &o, &b) == DMRT_EINVAL && !b);
    CHECK(strstr(dmrt_last_error(), "cavity 1") != NULL);
    CHECK(dmrt_batch_create(0, cav, &o, &b) == DMRT_EINVAL);
    /* null handles */
    CHECK(dmrt_step(NULL, 1) == DMRT_EINVAL);
    CHECK(dmrt_fields(NULL, NULL, NULL, NULL, NULL) == DMRT_EINVAL);
    CHECK(dmrt_record(NULL, 4) == DMRT_EINVAL);
    CHECK(dmrt_batch_step(NULL, 1) == DMRT_EINVAL);
    dmrt_destroy(NULL);
    dmrt_batch_destroy(NULL);
    printf("host ABI paths ok\n");
    return 0;
}
