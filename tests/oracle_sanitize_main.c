/*
 * Drives the oracle through every entry point on small lattices, for a build
 * with AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure:
 * compiled and run by tests/test_oracle_sanitizers.py).  Inputs are a flat
 * space plus a deterministic perturbation; exit status 0 when every call
 * returns LBREF_OK and the results are finite.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/lbref.h"

static double perturb(unsigned *state)
{
    *state = *state * 1664525u + 1013904223u;
    return ((double)(*state >> 8) / 16777216.0 - 0.5) * 0.04;
}

static int run(int lattice, int nx, int ny, int nz, int slicing, int collision, int matter)
{
    const int nf = 16, nq = lattice;
    const size_t n = (size_t)nx * ny * nz;
    double *u = calloc(n * nf, sizeof(double));
    double *f = calloc(n * nf * nq, sizeof(double));
    double *m = calloc(n * 10, sizeof(double));
    unsigned st = 12345u + (unsigned)(lattice + slicing + collision + matter);
    if (!u || !f || !m) return 1;
    for (size_t s = 0; s < n; ++s) {
        for (int F = 0; F < nf; ++F) u[F * n + s] = perturb(&st);
        u[0 * n + s] += 1.0;
        u[1 * n + s] += 1.0;
        u[4 * n + s] += 1.0;
        u[6 * n + s] += 1.0;
        for (int c = 0; c < 10; ++c) m[c * n + s] = 0.01 * (perturb(&st) + 0.05);
    }
    lbref *h = NULL;
    int rc = lbref_create_lattice(lattice, nx, ny, nz, 0.8, slicing, &h);
    if (!rc) rc = lbref_set_collision(h, collision);
    if (!rc && matter == 1) rc = lbref_set_matter(h, LBREF_MATTER_TENSOR, m, 1);
    if (!rc && matter == 2) rc = lbref_set_matter(h, LBREF_MATTER_FLUID, m, 1);
    if (!rc && matter == 3) rc = lbref_set_matter(h, LBREF_MATTER_FLUID, m, 0);
    if (!rc) rc = lbref_init_fields(h, u);
    if (!rc) rc = lbref_step(h, 3);
    if (!rc) rc = lbref_get_distributions(h, f);
    if (!rc) rc = lbref_set_distributions(h, f);
    if (!rc) rc = lbref_step(h, 2);
    if (!rc) rc = lbref_moments(h, u);
    for (size_t i = 0; !rc && i < n * nf; ++i)
        if (!isfinite(u[i])) rc = 2;
    lbref_destroy(h);
    free(u);
    free(f);
    free(m);
    return rc;
}

int main(void)
{
    int rc = 0, c[57];
    double w[19], p[37] = {1.0, 1.0, 0.0, 0.0, 1.0, 0.0, 1.0}, out[34], feq[19], F3[3] = {0.1, 0.2, 0.3};
    lbref_lattice_d3q19(c, w);
    rc |= lbref_lattice(LBREF_D2Q9, c, w) != LBREF_D2Q9;
    rc |= lbref_point_rhs(p, LBREF_SLICING_HARMONIC, out);
    rc |= lbref_point_rhs_matter(p, LBREF_MATTER_FLUID, F3, LBREF_SLICING_ONE_PLUS_LOG, out);
    lbref_point_feq(1, 0.5, F3, feq);
    rc |= run(19, 5, 4, 3, LBREF_SLICING_HARMONIC, LBREF_COLLISION_BGK, 0);
    rc |= run(19, 3, 1, 2, LBREF_SLICING_GEODESIC, LBREF_COLLISION_REGULARIZED, 1);
    rc |= run(19, 4, 3, 2, LBREF_SLICING_ONE_PLUS_LOG, LBREF_COLLISION_BGK, 2);
    rc |= run(9, 6, 5, 1, LBREF_SLICING_HARMONIC, LBREF_COLLISION_REGULARIZED, 3);
    rc |= run(9, 1, 1, 1, LBREF_SLICING_GEODESIC, LBREF_COLLISION_BGK, 0);
    printf("oracle sanitizer run: %s\n", rc ? "FAILED" : "ok");
    return rc ? 1 : 0;
}
