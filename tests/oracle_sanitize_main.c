/* Driver for the sanitizer build of the oracle (tests/test_oracle_sanitized.py):
 * a binary and a van der Waals capillary with walls, a body force and an
 * invalid input, run for a few hundred steps; every result must be finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lb_oracle.h"

static int run(int model) {
    orc_params p = {0};
    p.model = model;
    p.kappa = model == ORC_BINARY ? 0.04 : 0.02;
    p.a = 9.0 / 49.0; p.b = 2.0 / 21.0; p.T = 0.56;
    p.A = 0.04; p.B = 0.04; p.Gamma = 1.0;
    p.nu_l = model == ORC_BINARY ? 0.5 : 0.1;
    p.nu_g = model == ORC_BINARY ? 0.05 : 0.1;
    p.wall_grad = model == ORC_BINARY ? -0.2 : -0.144;
    p.force_x = 1e-6;
    orc_geom g = {61, 23, 20, 31, 9, 7};
    const int n = g.nx * g.ny;
    double* q = malloc(sizeof(double) * n);
    for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; ++x)
            q[y * g.nx + x] = model == ORC_BINARY ? (x < 20 ? 1.0 : -1.0) : (x < 20 ? 4.5 : 2.55);
    orc_state* s = NULL;
    if (orc_create(&p, &g, q, &s) != ORC_OK) { fprintf(stderr, "create failed\n"); return 1; }
    if (orc_step(s, 300) != ORC_OK) { fprintf(stderr, "step failed\n"); return 1; }
    double* f[4];
    for (int i = 0; i < 4; ++i) f[i] = malloc(sizeof(double) * n);
    orc_moments(s, f[0], f[1], f[2], f[3]);
    for (int i = 0; i < 4; ++i)
        for (int k = 0; k < n; ++k)
            if (!isfinite(f[i][k])) { fprintf(stderr, "non-finite field\n"); return 1; }
    double l, le;
    orc_interface_length(s, model == ORC_BINARY ? 0.0 : 3.52821, &l, &le);
    orc_free(s);
    /* invalid input: a tube wider than the lattice must be rejected, not read */
    orc_geom bad = {61, 23, 20, 31, 30, 7};
    if (orc_create(&p, &bad, q, &s) == ORC_OK) { fprintf(stderr, "bad geometry accepted\n"); return 1; }
    for (int i = 0; i < 4; ++i) free(f[i]);
    free(q);
    printf("model %d ok l=%.3f\n", model, l);
    return 0;
}

int main(void) { return run(ORC_BINARY) || run(ORC_VDW); }
