/*
 * lbmref.h -- FP64 CPU oracle of the double-distribution (DDF) thermal
 * lattice Boltzmann step of Xu & Li, "Multi-GPU thermal lattice Boltzmann
 * simulations using OpenACC and MPI" (arXiv:2211.03160), Section 2.
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
 * benchmark's CPU-baseline leg are the only code allowed to load this
 * library.  It shares no code, header, table or helper with the GPU
 * library under paper_2211_03160_amd/; the two agree only through the
 * paper and through the seeded inputs both are given.
 *
 * State convention: the oracle stores PRE-collision populations f(x,t),
 * g(x,t) and advances them in the paper's split order (Section 3.1,
 * Eqs. 8a-9b): macroscopic moments, collision of f, collision of g,
 * streaming with the wall rules of Section 2.2.
 *
 * All functions return LBMREF_OK (0) or a negative status; none aborts.
 */
#ifndef LBMREF_H
#define LBMREF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LBMREF_OK = 0,
    LBMREF_E_INVALID = -1,
    LBMREF_E_UNSTABLE = -3,
    LBMREF_E_STATE = -4
};

/* per-face boundary kinds; faces are ordered -x, +x, -y, +y, -z, +z */
enum {
    LBMREF_BC_PERIODIC = 0,
    LBMREF_BC_ADIABATIC = 1, /* no-slip wall, zero heat flux           */
    LBMREF_BC_DIRICHLET = 2  /* no-slip wall, fixed temperature t_wall */
};

typedef struct lbmref_params {
    int32_t dim;       /* 2: D2Q9 + D2Q5, 3: D3Q19 + D3Q7                  */
    int32_t n[3];      /* nodes along x, y, z (z = 1 when dim == 2)        */
    int32_t storage;   /* ignored by the oracle (always FP64)              */
    int32_t bc[6];     /* boundary kind per face                           */
    int32_t reserved;
    double t_wall[6];  /* wall temperature of DIRICHLET faces              */
    double ra, pr;     /* Rayleigh and Prandtl numbers (Eq. 4)             */
    double u_ff;       /* free-fall velocity in lattice units              */
    double t_hot, t_cold;
    double nu, alpha, gbeta; /* NaN: derived from ra, pr, u_ff (Eq. 3)     */
    double a_t;        /* NaN: -1.5 (D2Q5) or -0.75 (D3Q7)                 */
    double s_e, s_eps, s_q, s_pi, s_m; /* flow MRT rates, NaN: default     */
    double q_e, q_nu;  /* thermal even-moment rates, NaN: 1                */
} lbmref_params;

typedef struct lbmref_diag {
    int64_t t;
    double mass;     /* sum of rho over all nodes                  */
    double energy;   /* sum of T over all nodes                    */
    double umax;     /* max |u|                                    */
    double nu_vol;   /* 1 + H <u_g (T - T0)> / (alpha dT)          */
    double re;       /* sqrt(<|u|^2>) H / nu                       */
    int64_t nonfinite;
} lbmref_diag;

/* derived lattice parameters, in this order, returned by lbmref_derived */
enum {
    LBMREF_D_NU = 0, LBMREF_D_ALPHA, LBMREF_D_GBETA, LBMREF_D_TAU_F,
    LBMREF_D_TAU_G, LBMREF_D_S_NU, LBMREF_D_S_E, LBMREF_D_S_EPS,
    LBMREF_D_S_Q, LBMREF_D_S_PI, LBMREF_D_S_M, LBMREF_D_Q_J, LBMREF_D_Q_E,
    LBMREF_D_Q_NU, LBMREF_D_A_T, LBMREF_D_OMEGA, LBMREF_D_CS2_T,
    LBMREF_D_T0, LBMREF_D_H, LBMREF_D_COUNT
};

typedef struct lbmref_ctx lbmref_ctx;

int lbmref_create(const lbmref_params* p, lbmref_ctx** out);
void lbmref_destroy(lbmref_ctx* c);
const char* lbmref_last_error(const lbmref_ctx* c);

/* rho = 1, u = 0, T = conduction profile + amp * xi(seed, node) */
int lbmref_init(lbmref_ctx* c, uint64_t seed, double amp);
/* equilibrium populations from host fields; rho may be NULL (=1),
 * u is [dim][N] (component-major), T is [N]; x is the fastest index   */
int lbmref_init_fields(lbmref_ctx* c, const double* rho, const double* u,
                       const double* T);
int lbmref_step(lbmref_ctx* c, int64_t n);
/* moments of the current pre-collision state; each pointer may be NULL */
int lbmref_fields(lbmref_ctx* c, double* rho, double* u, double* T);
/* wall-flux Nusselt number averaged over the last two steps */
int lbmref_nusselt(lbmref_ctx* c, double* nu_hot, double* nu_cold);
int lbmref_diagnostics(lbmref_ctx* c, lbmref_diag* d);
int64_t lbmref_time(const lbmref_ctx* c);

/* heat entering the fluid through each face during the last step
 * (last[6]) and the step before it (prev[6]); either may be NULL      */
int lbmref_wall_flux(lbmref_ctx* c, double* last, double* prev);

/* raw pre-collision populations: f is [qf][N], g is [qg][N] */
int lbmref_get_populations(const lbmref_ctx* c, double* f, double* g);
int lbmref_set_populations(lbmref_ctx* c, const double* f, const double* g);

int lbmref_derived(const lbmref_ctx* c, double* out /* LBMREF_D_COUNT */);
/* the same values for parameters alone, without creating a state; errors
 * as lbmref_create (message in lbmref_last_error(NULL))                 */
int lbmref_derive(const lbmref_params* p, double* out /* LBMREF_D_COUNT */);

/* lattice tables the oracle builds for `dim`, for the pin tests.
 * which: 0 = flow, 1 = thermal.  Outputs (each may be NULL):
 * q; e[q][3] as doubles; w[q] (flow only; thermal returns the rest-state
 * equilibrium weights g_eq(T=1,u=0)); M[q][q] (row = moment);
 * Minv[q][q].                                                         */
int lbmref_lattice(int dim, int which, int* q, double* e, double* w,
                   double* M, double* Minv);

/* splitmix64 output for state x (exposed for the generator pin) */
uint64_t lbmref_splitmix64(uint64_t x);

/* OpenMP threads used by the step loops (1 when built without OpenMP) */
int lbmref_threads(void);
void lbmref_set_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
