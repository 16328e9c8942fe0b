/* Exercises every entry point of the FP64 oracle, valid and invalid calls,
 * on small 2D and 3D cavities; built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py.  Exit status 0
 * means every call returned what its header promises; the sanitizers abort
 * on any memory or undefined-behaviour error. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/lbmref.h"

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            return 1;                                              \
        }                                                          \
    } while (0)

static void fill(lbmref_params* p, int dim, int nx, int ny, int nz) {
    memset(p, 0, sizeof(*p));
    p->dim = dim;
    p->n[0] = nx;
    p->n[1] = ny;
    p->n[2] = nz;
    for (int f = 0; f < 6; ++f) p->bc[f] = f / 2 < dim ? LBMREF_BC_ADIABATIC : LBMREF_BC_PERIODIC;
    p->bc[2 * (dim - 1)] = p->bc[2 * (dim - 1) + 1] = LBMREF_BC_DIRICHLET;
    p->t_wall[2 * (dim - 1)] = 1.0;
    p->ra = 2e4;
    p->pr = 0.71;
    p->u_ff = 0.1;
    p->t_hot = 1.0;
    p->t_cold = 0.0;
    p->nu = p->alpha = p->gbeta = p->a_t = NAN;
    p->s_e = p->s_eps = p->s_q = p->s_pi = p->s_m = p->q_e = p->q_nu = NAN;
}

static int run(int dim, int nx, int ny, int nz) {
    lbmref_params p;
    fill(&p, dim, nx, ny, nz);
    double d[LBMREF_D_COUNT];
    CHECK(lbmref_derive(&p, d) == LBMREF_OK);
    lbmref_ctx* c = NULL;
    CHECK(lbmref_create(&p, &c) == LBMREF_OK && c);
    CHECK(lbmref_time(c) == -1);
    double rho_, T_;
    CHECK(lbmref_fields(c, &rho_, NULL, &T_) == LBMREF_E_STATE); /* before init */
    CHECK(lbmref_init(c, 7, 1e-2) == LBMREF_OK);
    CHECK(lbmref_step(c, 5) == LBMREF_OK);
    const size_t N = (size_t)nx * ny * nz;
    const int qf = dim == 2 ? 9 : 19, qg = dim == 2 ? 5 : 7;
    double* rho = malloc(N * sizeof(double));
    double* u = malloc(3 * N * sizeof(double));
    double* T = malloc(N * sizeof(double));
    double* f = malloc(qf * N * sizeof(double));
    double* g = malloc(qg * N * sizeof(double));
    CHECK(rho && u && T && f && g);
    CHECK(lbmref_fields(c, rho, u, T) == LBMREF_OK);
    double nh, nc;
    CHECK(lbmref_nusselt(c, &nh, &nc) == LBMREF_OK && isfinite(nh) && isfinite(nc));
    lbmref_diag dg;
    CHECK(lbmref_diagnostics(c, &dg) == LBMREF_OK && dg.t == 5);
    double last[6], prev[6];
    CHECK(lbmref_wall_flux(c, last, prev) == LBMREF_OK);
    CHECK(lbmref_get_populations(c, f, g) == LBMREF_OK);
    CHECK(lbmref_set_populations(c, f, g) == LBMREF_OK);
    CHECK(lbmref_init_fields(c, rho, u, T) == LBMREF_OK);
    CHECK(lbmref_init_fields(c, NULL, u, T) == LBMREF_OK);
    CHECK(lbmref_init_fields(c, NULL, NULL, T) != LBMREF_OK);
    CHECK(lbmref_step(c, 3) == LBMREF_OK && lbmref_time(c) == 3);
    CHECK(lbmref_derived(c, d) == LBMREF_OK);
    CHECK(strlen(lbmref_last_error(c)) < 256);
    lbmref_destroy(c);
    free(rho); free(u); free(T); free(f); free(g);
    return 0;
}

int main(void) {
    lbmref_set_threads(1);
    if (run(2, 9, 7, 1) || run(3, 5, 4, 6)) return 1;
    /* invalid parameters are rejected without touching memory */
    lbmref_params p;
    fill(&p, 2, 9, 7, 1);
    double d[LBMREF_D_COUNT];
    p.dim = 4;
    CHECK(lbmref_derive(&p, d) != LBMREF_OK);
    fill(&p, 2, 9, 7, 1);
    p.n[0] = 0;
    lbmref_ctx* c = NULL;
    CHECK(lbmref_create(&p, &c) != LBMREF_OK && c == NULL);
    fill(&p, 2, 9, 7, 1);
    p.bc[0] = LBMREF_BC_PERIODIC; /* unpaired periodic face */
    CHECK(lbmref_create(&p, &c) != LBMREF_OK);
    fill(&p, 2, 9, 7, 1);
    p.ra = -1;
    CHECK(lbmref_derive(&p, d) != LBMREF_OK);
    CHECK(lbmref_derive(NULL, d) != LBMREF_OK && lbmref_create(NULL, &c) != LBMREF_OK);
    CHECK(strlen(lbmref_last_error(NULL)) > 0);
    lbmref_destroy(NULL);
    int q;
    double e[19 * 3], w[19], M[19 * 19], Mi[19 * 19];
    for (int dim = 2; dim <= 3; ++dim)
        for (int which = 0; which <= 1; ++which)
            CHECK(lbmref_lattice(dim, which, &q, e, w, M, Mi) == LBMREF_OK);
    CHECK(lbmref_lattice(5, 0, &q, e, w, M, Mi) != LBMREF_OK);
    CHECK(lbmref_splitmix64(0) != 0);
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
