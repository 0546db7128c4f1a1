/* A caller of the library written in plain C (no Python, no torch): a 32^3
 * periodic box with two spheres, 20 steps on the null stream, then the
 * forces and torques printed with full precision, one body per line, and
 * the status of a rejected call.  test_gpu_c_abi.py runs it and compares
 * the numbers with the same run through the Python binding. */
#include <stdio.h>
#include <string.h>

#include "lbm.h"

#define CHECK(call)                                                                     \
    do {                                                                                \
        lbm_status st_ = (call);                                                        \
        if (st_ != LBM_OK) {                                                            \
            fprintf(stderr, "%s failed: %d %s\n", #call, (int)st_, h ? lbm_last_error(h) : ""); \
            if (h) lbm_destroy(h);                                                      \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

int main(void)
{
    lbm_handle h = NULL;
    lbm_config c;
    memset(&c, 0, sizeof c);
    c.nx = c.ny = c.nz = 32;
    c.storage = LBM_STORE_F32;
    c.tau0 = 0.6;
    c.smag_c = 0.1;
    c.rho0 = 1.0;
    c.body_force[0] = 1e-5;
    c.bb_mode = LBM_BB_BOUZIDI;
    c.max_bodies = 2;
    c.stream = NULL;
    CHECK(lbm_create(&c, &h));
    const double X[6] = {10.3, 11.7, 12.2, 22.6, 20.1, 19.4};
    const double V[6] = {0.01, 0.0, -0.005, 0.0, 0.002, 0.0};
    const double W[6] = {0.0, 0.0, 0.001, 0.0, 0.0, 0.0};
    const double R[2] = {4.2, 3.6};
    CHECK(lbm_set_bodies(h, 2, X, V, W, R));
    CHECK(lbm_init_fields(h, NULL, NULL));
    CHECK(lbm_step(h, 20));
    double F[6], T[6];
    CHECK(lbm_get_forces(h, F, T));
    lbm_info info;
    CHECK(lbm_get_info(h, &info));
    printf("version %d steps %d bodies %d\n", (int)lbm_version(), (int)info.steps_done, (int)info.n_bodies);
    for (int b = 0; b < 2; ++b)
        printf("body %d %.17g %.17g %.17g %.17g %.17g %.17g\n", b, F[3 * b], F[3 * b + 1], F[3 * b + 2], T[3 * b],
               T[3 * b + 1], T[3 * b + 2]);
    printf("rejected %d\n", (int)lbm_step(h, -1));
    lbm_destroy(h);
    return 0;
}
