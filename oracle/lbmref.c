/*
 * lbmref.c -- FP64 CPU oracle of the DDF thermal lattice Boltzmann step of
 * Xu & Li (arXiv:2211.03160), Section 2.2, advanced in the split order of
 * Section 3.1 (Eqs. 8a-9b).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and
 * the benchmark's CPU-baseline leg, never by the product path.  It shares
 * no code with the GPU library.  Build: -O2 -fno-fast-math
 * -ffp-contract=off, so every product and sum is rounded as written.
 *
 * Where the paper leaves a quantity to its prior work (the moment bases M
 * and N, the equilibria m_eq and n_eq, the relaxation rates, a_T, the
 * initial state, the Nusselt number) the reading taken is stated at the
 * place it is used.  Everything is plain loops over nodes; the only
 * parallelism is an OpenMP split of independent per-node loops, and every
 * reduction is serial in node order, so results do not depend on the
 * thread count.
 */
#include "lbmref.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QMAX 19

typedef struct {
    int q;
    int e[QMAX][3];
    double w[QMAX];          /* lattice weights (flow lattices only)     */
    int opp[QMAX];           /* index of -e_i                            */
    double M[QMAX][QMAX];    /* moment basis: row k, column i            */
    double Minv[QMAX][QMAX]; /* numerical inverse of M                   */
} lattice_t;

struct lbmref_ctx {
    lbmref_params p;
    int dim, gaxis;
    int n[3];
    size_t N;
    lattice_t lf, lg;
    double s[QMAX];  /* flow relaxation rate of each moment row     */
    double qr[QMAX]; /* thermal relaxation rate of each moment row  */
    double d[LBMREF_D_COUNT];
    double nu, alpha, gbeta, a_t, omega, t0, dT, H;
    double *f, *g, *fp, *gp;  /* pre- and post-collision populations */
    double *rho, *T, *u, *F;  /* moments; u and F are [3][N]         */
    double flux[2][6];        /* slot (t & 1): heat in during the step ending at t */
    int64_t t;
    char err[256];
};

static char g_create_err[256] = "";
static int g_threads = 0;

/* ------------------------------------------------------------------ */
/* Velocity sets (Section 2.2, Fig. 1).  D2Q9 order: rest, +x, +y, -x,
 * -y, then the diagonals (1,1), (-1,1), (-1,-1), (1,-1); this is the
 * order in which Section 3.1 names f_2,5,6 as the upward and f_4,7,8 as
 * the downward populations.  D2Q5 is the first five of those.  The 3D
 * sets list opposite pairs next to each other.                          */
static const int E_D2Q9[9][3] = {{0, 0, 0},  {1, 0, 0},  {0, 1, 0},
                                 {-1, 0, 0}, {0, -1, 0}, {1, 1, 0},
                                 {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const int E_D3Q19[19][3] = {
    {0, 0, 0},  {1, 0, 0},  {-1, 0, 0},  {0, 1, 0},  {0, -1, 0},
    {0, 0, 1},  {0, 0, -1}, {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},
    {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const int E_D3Q7[7][3] = {{0, 0, 0},  {1, 0, 0}, {-1, 0, 0},
                                 {0, 1, 0},  {0, -1, 0}, {0, 0, 1},
                                 {0, 0, -1}};

/* Moment bases, evaluated as polynomials of the velocity (the rows are the
 * reading of the MRT bases the paper takes from its prior work; they are
 * the bases whose forcing moments reproduce Eqs. 6a and 6b).             */
static double basis_d2q9(int k, const int* e) {
    double x = e[0], y = e[1], s = x * x + y * y;
    switch (k) {
    case 0: return 1.0;                          /* rho      */
    case 1: return 3.0 * s - 4.0;                /* e        */
    case 2: return (9.0 * s * s - 21.0 * s + 8.0) / 2.0; /* eps */
    case 3: return x;                            /* j_x      */
    case 4: return (3.0 * s - 5.0) * x;          /* q_x      */
    case 5: return y;                            /* j_y      */
    case 6: return (3.0 * s - 5.0) * y;          /* q_y      */
    case 7: return x * x - y * y;                /* p_xx     */
    default: return x * y;                       /* p_xy     */
    }
}

static double basis_d3q19(int k, const int* e) {
    double x = e[0], y = e[1], z = e[2], s = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * s - 30.0;
    case 2: return (21.0 * s * s - 53.0 * s + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * s - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * s - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * s - 9.0) * z;
    case 9: return 3.0 * x * x - s;
    case 10: return (3.0 * s - 5.0) * (3.0 * x * x - s);
    case 11: return y * y - z * z;
    case 12: return (3.0 * s - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}

static double basis_d2q5(int k, const int* e) {
    double x = e[0], y = e[1], s = x * x + y * y;
    switch (k) {
    case 0: return 1.0;             /* T          */
    case 1: return x;               /* j_x        */
    case 2: return y;               /* j_y        */
    case 3: return 5.0 * s - 4.0;   /* e          */
    default: return x * x - y * y;  /* p_xx       */
    }
}

static double basis_d3q7(int k, const int* e) {
    double x = e[0], y = e[1], z = e[2], s = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return 7.0 * s - 6.0;
    case 5: return 3.0 * x * x - s;
    default: return y * y - z * z;
    }
}

/* Gauss-Jordan inversion with partial pivoting; returns 0 on success. */
static int invert(int q, double A[QMAX][QMAX], double R[QMAX][QMAX]) {
    double W[QMAX][2 * QMAX];
    for (int r = 0; r < q; ++r)
        for (int c = 0; c < 2 * q; ++c)
            W[r][c] = c < q ? A[r][c] : (c - q == r ? 1.0 : 0.0);
    for (int c = 0; c < q; ++c) {
        int piv = c;
        for (int r = c + 1; r < q; ++r)
            if (fabs(W[r][c]) > fabs(W[piv][c])) piv = r;
        if (fabs(W[piv][c]) < 1e-12) return -1;
        if (piv != c)
            for (int k = 0; k < 2 * q; ++k) {
                double t = W[c][k];
                W[c][k] = W[piv][k];
                W[piv][k] = t;
            }
        double d = W[c][c];
        for (int k = 0; k < 2 * q; ++k) W[c][k] /= d;
        for (int r = 0; r < q; ++r) {
            if (r == c) continue;
            double m = W[r][c];
            if (m != 0.0)
                for (int k = 0; k < 2 * q; ++k) W[r][k] -= m * W[c][k];
        }
    }
    for (int r = 0; r < q; ++r)
        for (int c = 0; c < q; ++c) R[r][c] = W[r][c + q];
    return 0;
}

static int build_lattice(int dim, int thermal, lattice_t* L) {
    const int(*E)[3];
    double (*basis)(int, const int*);
    memset(L, 0, sizeof(*L));
    if (dim == 2 && !thermal) { L->q = 9; E = E_D2Q9; basis = basis_d2q9; }
    else if (dim == 2) { L->q = 5; E = E_D2Q9; basis = basis_d2q5; }
    else if (!thermal) { L->q = 19; E = E_D3Q19; basis = basis_d3q19; }
    else { L->q = 7; E = E_D3Q7; basis = basis_d3q7; }
    for (int i = 0; i < L->q; ++i) {
        int s = 0;
        for (int a = 0; a < 3; ++a) {
            L->e[i][a] = E[i][a];
            s += E[i][a] * E[i][a];
        }
        /* weights of the second-order flow equilibria: D2Q9 4/9, 1/9,
         * 1/36; D3Q19 1/3, 1/18, 1/36 (by |e|^2 = 0, 1, 2)            */
        if (!thermal) {
            if (dim == 2) L->w[i] = s == 0 ? 4.0 / 9.0 : s == 1 ? 1.0 / 9.0 : 1.0 / 36.0;
            else L->w[i] = s == 0 ? 1.0 / 3.0 : s == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
        }
    }
    for (int i = 0; i < L->q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < L->q; ++j)
            if (L->e[j][0] == -L->e[i][0] && L->e[j][1] == -L->e[i][1] &&
                L->e[j][2] == -L->e[i][2])
                L->opp[i] = j;
    }
    for (int k = 0; k < L->q; ++k)
        for (int i = 0; i < L->q; ++i) L->M[k][i] = basis(k, L->e[i]);
    return invert(L->q, L->M, L->Minv);
}

/* ------------------------------------------------------------------ */
/* Per-node pieces of the method.                                      */

/* second-order equilibrium with local density (reading of m_eq = M f_eq) */
static void f_equilibrium(const lattice_t* L, double rho, const double* u,
                          double* out) {
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; ++i) {
        double eu = L->e[i][0] * u[0] + L->e[i][1] * u[1] + L->e[i][2] * u[2];
        out[i] = L->w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* M F~ of Eq. 6a (D2Q9) and Eq. 6b (D3Q19).  The last entry of Eq. 6a is
 * read as u F_y + v F_x, the xy moment of Guo's force term (the printed
 * entry repeats the diagonal; Eq. 6b's xy entry has the read form).    */
static void force_moments(int dim, const double* u, const double* F,
                          double* mf) {
    double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    if (dim == 2) {
        mf[0] = 0.0;
        mf[1] = 6.0 * uF;
        mf[2] = -6.0 * uF;
        mf[3] = F[0];
        mf[4] = -F[0];
        mf[5] = F[1];
        mf[6] = -F[1];
        mf[7] = 2.0 * u[0] * F[0] - 2.0 * u[1] * F[1];
        mf[8] = u[0] * F[1] + u[1] * F[0];
    } else {
        mf[0] = 0.0;
        mf[1] = 38.0 * uF;
        mf[2] = -11.0 * uF;
        mf[3] = F[0];
        mf[4] = -2.0 / 3.0 * F[0];
        mf[5] = F[1];
        mf[6] = -2.0 / 3.0 * F[1];
        mf[7] = F[2];
        mf[8] = -2.0 / 3.0 * F[2];
        mf[9] = 4.0 * u[0] * F[0] - 2.0 * u[1] * F[1] - 2.0 * u[2] * F[2];
        mf[10] = -2.0 * u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        mf[11] = 2.0 * u[1] * F[1] - 2.0 * u[2] * F[2];
        mf[12] = -u[1] * F[1] + u[2] * F[2];
        mf[13] = u[0] * F[1] + u[1] * F[0];
        mf[14] = u[1] * F[2] + u[2] * F[1];
        mf[15] = u[0] * F[2] + u[2] * F[0];
        mf[16] = 0.0;
        mf[17] = 0.0;
        mf[18] = 0.0;
    }
}

/* thermal equilibrium moments n_eq = (T, uT, vT[, wT], a_T T, 0[, 0]) */
static void g_eq_moments(int dim, double a_t, double T, const double* u,
                         double* neq) {
    if (dim == 2) {
        neq[0] = T;
        neq[1] = u[0] * T;
        neq[2] = u[1] * T;
        neq[3] = a_t * T;
        neq[4] = 0.0;
    } else {
        neq[0] = T;
        neq[1] = u[0] * T;
        neq[2] = u[1] * T;
        neq[3] = u[2] * T;
        neq[4] = a_t * T;
        neq[5] = 0.0;
        neq[6] = 0.0;
    }
}

static void matvec(int q, double A[QMAX][QMAX], const double* x, double* y) {
    for (int k = 0; k < q; ++k) {
        double acc = 0.0;
        for (int i = 0; i < q; ++i) acc += A[k][i] * x[i];
        y[k] = acc;
    }
}

/* g_eq = N^-1 n_eq */
static void g_equilibrium(const lbmref_ctx* c, double T, const double* u,
                          double* out) {
    double neq[QMAX];
    g_eq_moments(c->dim, c->a_t, T, u, neq);
    matvec(c->lg.q, (double(*)[QMAX])c->lg.Minv, neq, out);
}

/* ------------------------------------------------------------------ */
/* Parameters.                                                         */

static int fail(char* buf, const char* msg) {
    snprintf(buf, 256, "%s", msg);
    return LBMREF_E_INVALID;
}

static int derive(lbmref_ctx* c, char* err) {
    const lbmref_params* p = &c->p;
    if (p->dim != 2 && p->dim != 3) return fail(err, "dim must be 2 or 3");
    c->dim = p->dim;
    c->gaxis = p->dim == 2 ? 1 : 2; /* gravity along -y (2D) / -z (3D) */
    for (int a = 0; a < 3; ++a) {
        c->n[a] = p->n[a];
        if (p->n[a] < 1) return fail(err, "n must be >= 1");
    }
    if (p->dim == 2 && p->n[2] != 1) return fail(err, "n[2] must be 1 in 2D");
    for (int a = 0; a < p->dim; ++a) {
        int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2)
            return fail(err, "unknown boundary kind");
        if ((lo == LBMREF_BC_PERIODIC) != (hi == LBMREF_BC_PERIODIC))
            return fail(err, "periodic faces must come in pairs");
        if (lo != LBMREF_BC_PERIODIC && p->n[a] < 2)
            return fail(err, "a walled axis needs n >= 2");
    }
    c->N = (size_t)p->n[0] * p->n[1] * p->n[2];
    c->H = p->n[c->gaxis];
    c->dT = p->t_hot - p->t_cold;
    c->t0 = 0.5 * (p->t_hot + p->t_cold);

    /* Eqs. 2-4 in lattice units: the free-fall velocity U = sqrt(g beta dT
     * H) is u_ff, so t_f = H/U steps and nu* = sqrt(Pr/Ra) gives
     * nu = U H sqrt(Pr/Ra), alpha = U H / sqrt(Pr Ra), g beta = U^2/(dT H) */
    int need_derived = isnan(p->nu) || isnan(p->alpha) || isnan(p->gbeta);
    if (need_derived) {
        if (!(p->ra > 0) || !(p->pr > 0)) return fail(err, "ra and pr must be > 0");
        if (!(p->u_ff > 0) || p->u_ff > 0.3) return fail(err, "u_ff must be in (0, 0.3]");
        if (!(c->dT > 0)) return fail(err, "t_hot must exceed t_cold");
    }
    c->nu = isnan(p->nu) ? p->u_ff * c->H * sqrt(p->pr / p->ra) : p->nu;
    c->alpha = isnan(p->alpha) ? p->u_ff * c->H / sqrt(p->pr * p->ra) : p->alpha;
    c->gbeta = isnan(p->gbeta) ? p->u_ff * p->u_ff / (c->dT * c->H) : p->gbeta;
    if (!(c->nu > 0) || !(c->alpha > 0) || !isfinite(c->gbeta))
        return fail(err, "nu and alpha must be > 0");

    c->a_t = isnan(p->a_t) ? (p->dim == 2 ? -1.5 : -0.75) : p->a_t;
    if (!(c->a_t < 1.0) || !(c->a_t > (p->dim == 2 ? -4.0 : -6.0)))
        return fail(err, "a_t out of range");
    /* the anti-bounce-back weight of Section 2.2 */
    c->omega = p->dim == 2 ? (4.0 + c->a_t) / 10.0 : (6.0 + c->a_t) / 21.0;

    if (build_lattice(p->dim, 0, &c->lf) || build_lattice(p->dim, 1, &c->lg))
        return fail(err, "singular moment basis");

    /* thermal sound speed: second moment of the rest-state equilibrium */
    double ge[QMAX], u0[3] = {0, 0, 0};
    g_equilibrium(c, 1.0, u0, ge);
    double cs2t = 0.0;
    for (int i = 0; i < c->lg.q; ++i) cs2t += ge[i] * c->lg.e[i][0] * c->lg.e[i][0];

    double tau_f = 3.0 * c->nu + 0.5;          /* nu = c_s^2 (tau - 1/2) */
    double tau_g = c->alpha / cs2t + 0.5;      /* alpha = c_sT^2 (tau_g - 1/2) */
    double s_nu = 1.0 / tau_f;
    /* default rates: even moments at the shear rate, odd moments at the
     * rate that makes Lambda = (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16       */
    double s_q = isnan(p->s_q) ? 8.0 * (2.0 - s_nu) / (8.0 - s_nu) : p->s_q;
    double s_e = isnan(p->s_e) ? s_nu : p->s_e;
    double s_eps = isnan(p->s_eps) ? s_nu : p->s_eps;
    double s_pi = isnan(p->s_pi) ? s_nu : p->s_pi;
    double s_m = isnan(p->s_m) ? s_q : p->s_m;
    double q_j = 1.0 / tau_g;
    double q_e = isnan(p->q_e) ? 1.0 : p->q_e;
    double q_nu = isnan(p->q_nu) ? 1.0 : p->q_nu;
    double rates[] = {s_nu, s_q, s_e, s_eps, s_pi, s_m, q_j, q_e, q_nu};
    for (unsigned k = 0; k < sizeof(rates) / sizeof(rates[0]); ++k)
        if (!(rates[k] > 0.0 && rates[k] < 2.0))
            return fail(err, "relaxation rates must lie in (0, 2): check tau_f, tau_g");

    /* S and Q, diagonal, in the row order of the bases above; conserved
     * rows (rho, j for f; T for g) take rate 1, which has no effect       */
    for (int k = 0; k < QMAX; ++k) c->s[k] = c->qr[k] = 1.0;
    if (p->dim == 2) {
        c->s[1] = s_e; c->s[2] = s_eps; c->s[4] = s_q; c->s[6] = s_q;
        c->s[7] = s_nu; c->s[8] = s_nu;
        c->qr[1] = q_j; c->qr[2] = q_j; c->qr[3] = q_e; c->qr[4] = q_nu;
    } else {
        c->s[1] = s_e; c->s[2] = s_eps;
        c->s[4] = s_q; c->s[6] = s_q; c->s[8] = s_q;
        c->s[9] = s_nu; c->s[10] = s_pi; c->s[11] = s_nu; c->s[12] = s_pi;
        c->s[13] = s_nu; c->s[14] = s_nu; c->s[15] = s_nu;
        c->s[16] = s_m; c->s[17] = s_m; c->s[18] = s_m;
        c->qr[1] = q_j; c->qr[2] = q_j; c->qr[3] = q_j;
        c->qr[4] = q_e; c->qr[5] = q_nu; c->qr[6] = q_nu;
    }
    double* d = c->d;
    d[LBMREF_D_NU] = c->nu; d[LBMREF_D_ALPHA] = c->alpha; d[LBMREF_D_GBETA] = c->gbeta;
    d[LBMREF_D_TAU_F] = tau_f; d[LBMREF_D_TAU_G] = tau_g; d[LBMREF_D_S_NU] = s_nu;
    d[LBMREF_D_S_E] = s_e; d[LBMREF_D_S_EPS] = s_eps; d[LBMREF_D_S_Q] = s_q;
    d[LBMREF_D_S_PI] = s_pi; d[LBMREF_D_S_M] = s_m; d[LBMREF_D_Q_J] = q_j;
    d[LBMREF_D_Q_E] = q_e; d[LBMREF_D_Q_NU] = q_nu; d[LBMREF_D_A_T] = c->a_t;
    d[LBMREF_D_OMEGA] = c->omega; d[LBMREF_D_CS2_T] = cs2t; d[LBMREF_D_T0] = c->t0;
    d[LBMREF_D_H] = c->H;
    return LBMREF_OK;
}

/* ------------------------------------------------------------------ */

int lbmref_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

void lbmref_set_threads(int n) { g_threads = n > 0 ? n : 0; }

uint64_t lbmref_splitmix64(uint64_t x) {
    /* Steele, Lea & Flood (2014), SplitMix64: one step from state x */
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

const char* lbmref_last_error(const lbmref_ctx* c) {
    return c ? c->err : g_create_err;
}

int lbmref_create(const lbmref_params* p, lbmref_ctx** out) {
    if (!p || !out) return fail(g_create_err, "null argument");
    *out = NULL;
    lbmref_ctx* c = (lbmref_ctx*)calloc(1, sizeof(lbmref_ctx));
    if (!c) return fail(g_create_err, "out of host memory");
    c->p = *p;
    int st = derive(c, g_create_err);
    if (st) { free(c); return st; }
    size_t N = c->N;
    c->f = (double*)calloc(N * c->lf.q, sizeof(double));
    c->fp = (double*)calloc(N * c->lf.q, sizeof(double));
    c->g = (double*)calloc(N * c->lg.q, sizeof(double));
    c->gp = (double*)calloc(N * c->lg.q, sizeof(double));
    c->rho = (double*)calloc(N, sizeof(double));
    c->T = (double*)calloc(N, sizeof(double));
    c->u = (double*)calloc(3 * N, sizeof(double));
    c->F = (double*)calloc(3 * N, sizeof(double));
    if (!c->f || !c->fp || !c->g || !c->gp || !c->rho || !c->T || !c->u || !c->F) {
        lbmref_destroy(c);
        return fail(g_create_err, "out of host memory");
    }
    c->t = -1; /* not initialised */
    g_create_err[0] = 0;
    *out = c;
    return LBMREF_OK;
}

/* The parameter mapping of lbmref_create (Eqs. 2-4 in lattice units, the
 * relaxation rates and the anti-bounce-back weight) without a state: no
 * allocation.  out receives LBMREF_D_COUNT values.                      */
int lbmref_derive(const lbmref_params* p, double* out) {
    if (!p || !out) return fail(g_create_err, "null argument");
    lbmref_ctx tmp;
    memset(&tmp, 0, sizeof(tmp));
    tmp.p = *p;
    int st = derive(&tmp, g_create_err);
    if (st) return st;
    memcpy(out, tmp.d, sizeof(tmp.d));
    g_create_err[0] = 0;
    return LBMREF_OK;
}

void lbmref_destroy(lbmref_ctx* c) {
    if (!c) return;
    free(c->f); free(c->fp); free(c->g); free(c->gp);
    free(c->rho); free(c->T); free(c->u); free(c->F);
    free(c);
}

int64_t lbmref_time(const lbmref_ctx* c) { return c ? c->t : -1; }

static void coords(const lbmref_ctx* c, size_t idx, int* x) {
    x[0] = (int)(idx % c->n[0]);
    x[1] = (int)((idx / c->n[0]) % c->n[1]);
    x[2] = (int)(idx / ((size_t)c->n[0] * c->n[1]));
}

/* the axis whose two faces are both Dirichlet (gravity axis first) */
static int conduction_axis(const lbmref_ctx* c) {
    int order[3] = {c->gaxis, 0, 1};
    for (int k = 0; k < 3; ++k) {
        int a = order[k];
        if (a >= c->dim) continue;
        if (c->p.bc[2 * a] == LBMREF_BC_DIRICHLET && c->p.bc[2 * a + 1] == LBMREF_BC_DIRICHLET)
            return a;
    }
    return -1;
}

int lbmref_init(lbmref_ctx* c, uint64_t seed, double amp) {
    if (!c) return LBMREF_E_INVALID;
    if (!isfinite(amp)) return fail(c->err, "amp must be finite");
    int a = conduction_axis(c);
    double tlo = a >= 0 ? c->p.t_wall[2 * a] : c->t0;
    double thi = a >= 0 ? c->p.t_wall[2 * a + 1] : c->t0;
    int na = a >= 0 ? c->n[a] : 1;
    double u0[3] = {0, 0, 0};
#pragma omp parallel for schedule(static) num_threads(lbmref_threads())
    for (long long ii = 0; ii < (long long)c->N; ++ii) {
        size_t idx = (size_t)ii;
        int x[3];
        coords(c, idx, x);
        /* conduction profile between the walls, walls half a link out */
        double T = a >= 0 ? tlo + (x[a] + 0.5) * (thi - tlo) / na : c->t0;
        uint64_t r = lbmref_splitmix64(seed ^ lbmref_splitmix64((uint64_t)idx));
        double xi = 2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0;
        T += amp * xi;
        double fe[QMAX], ge[QMAX];
        f_equilibrium(&c->lf, 1.0, u0, fe);
        g_equilibrium(c, T, u0, ge);
        for (int i = 0; i < c->lf.q; ++i) c->f[i * c->N + idx] = fe[i];
        for (int i = 0; i < c->lg.q; ++i) c->g[i * c->N + idx] = ge[i];
    }
    memset(c->flux, 0, sizeof(c->flux));
    c->t = 0;
    return LBMREF_OK;
}

int lbmref_init_fields(lbmref_ctx* c, const double* rho, const double* u,
                       const double* T) {
    if (!c) return LBMREF_E_INVALID;
    if (!u || !T) return fail(c->err, "u and T are required");
#pragma omp parallel for schedule(static) num_threads(lbmref_threads())
    for (long long ii = 0; ii < (long long)c->N; ++ii) {
        size_t idx = (size_t)ii;
        double r = rho ? rho[idx] : 1.0;
        double uu[3] = {0, 0, 0};
        for (int a = 0; a < c->dim; ++a) uu[a] = u[a * c->N + idx];
        double fe[QMAX], ge[QMAX];
        f_equilibrium(&c->lf, r, uu, fe);
        g_equilibrium(c, T[idx], uu, ge);
        for (int i = 0; i < c->lf.q; ++i) c->f[i * c->N + idx] = fe[i];
        for (int i = 0; i < c->lg.q; ++i) c->g[i * c->N + idx] = ge[i];
    }
    memset(c->flux, 0, sizeof(c->flux));
    c->t = 0;
    return LBMREF_OK;
}

/* Macroscopic moments (Section 2.2): rho = sum f, T = sum g,
 * F = rho g beta (T - T0) along the upward unit vector, and
 * u = (sum e f + F/2) / rho.                                           */
static void macros(lbmref_ctx* c) {
    const size_t N = c->N;
    const int qf = c->lf.q, qg = c->lg.q;
#pragma omp parallel for schedule(static) num_threads(lbmref_threads())
    for (long long ii = 0; ii < (long long)N; ++ii) {
        size_t idx = (size_t)ii;
        double rho = 0.0, j[3] = {0, 0, 0}, T = 0.0;
        for (int i = 0; i < qf; ++i) {
            double v = c->f[i * N + idx];
            rho += v;
            for (int a = 0; a < 3; ++a) j[a] += c->lf.e[i][a] * v;
        }
        for (int i = 0; i < qg; ++i) T += c->g[i * N + idx];
        double F[3] = {0, 0, 0};
        F[c->gaxis] = rho * c->gbeta * (T - c->t0);
        c->rho[idx] = rho;
        c->T[idx] = T;
        for (int a = 0; a < 3; ++a) {
            c->F[a * N + idx] = F[a];
            c->u[a * N + idx] = (j[a] + 0.5 * F[a]) / rho;
        }
    }
}

/* Eq. 8a: f+ = f - M^-1 S (m - m_eq) + M^-1 (I - S/2) M F~, evaluated
 * as m+ = m - S (m - m_eq) + (I - S/2) M F~ followed by f+ = M^-1 m+. */
static void collide_f(lbmref_ctx* c) {
    const size_t N = c->N;
    const int q = c->lf.q;
#pragma omp parallel for schedule(static) num_threads(lbmref_threads())
    for (long long ii = 0; ii < (long long)N; ++ii) {
        size_t idx = (size_t)ii;
        double f[QMAX], m[QMAX], fe[QMAX], meq[QMAX], mf[QMAX], mp[QMAX], fp[QMAX];
        double u[3], F[3];
        for (int a = 0; a < 3; ++a) {
            u[a] = c->u[a * N + idx];
            F[a] = c->F[a * N + idx];
        }
        for (int i = 0; i < q; ++i) f[i] = c->f[i * N + idx];
        matvec(q, c->lf.M, f, m);
        f_equilibrium(&c->lf, c->rho[idx], u, fe);
        matvec(q, c->lf.M, fe, meq);
        force_moments(c->dim, u, F, mf);
        for (int k = 0; k < q; ++k)
            mp[k] = m[k] - c->s[k] * (m[k] - meq[k]) + (1.0 - 0.5 * c->s[k]) * mf[k];
        matvec(q, c->lf.Minv, mp, fp);
        for (int i = 0; i < q; ++i) c->fp[i * N + idx] = fp[i];
    }
}

/* Eq. 9a: g+ = g - N^-1 Q (n - n_eq) */
static void collide_g(lbmref_ctx* c) {
    const size_t N = c->N;
    const int q = c->lg.q;
#pragma omp parallel for schedule(static) num_threads(lbmref_threads())
    for (long long ii = 0; ii < (long long)N; ++ii) {
        size_t idx = (size_t)ii;
        double g[QMAX], n[QMAX], neq[QMAX], np[QMAX], gp[QMAX], u[3];
        for (int a = 0; a < 3; ++a) u[a] = c->u[a * N + idx];
        for (int i = 0; i < q; ++i) g[i] = c->g[i * N + idx];
        matvec(q, c->lg.M, g, n);
        g_eq_moments(c->dim, c->a_t, c->T[idx], u, neq);
        for (int k = 0; k < q; ++k) np[k] = n[k] - c->qr[k] * (n[k] - neq[k]);
        matvec(q, c->lg.Minv, np, gp);
        for (int i = 0; i < q; ++i) c->gp[i * N + idx] = gp[i];
    }
}

/* Eqs. 8b and 9b as a pull: population i at x comes from x - e_i.  When
 * x - e_i lies beyond a periodic face it wraps; beyond a wall the link is
 * reflected at the half-way wall (Section 2.2): f_i(x) = f+_ibar(x)
 * (no-slip), g_i(x) = -g+_ibar(x) + omega T_w on a Dirichlet face and
 * g_i(x) = g+_ibar(x) on an adiabatic face.                            */
static void stream(lbmref_ctx* c, const lattice_t* L, double* dst,
                   const double* src, int thermal) {
    const size_t N = c->N;
    const int nx = c->n[0], ny = c->n[1], nz = c->n[2];
#pragma omp parallel for schedule(static) num_threads(lbmref_threads())
    for (long long zy = 0; zy < (long long)nz * ny; ++zy) {
        int z = (int)(zy / ny), y = (int)(zy % ny);
        for (int x = 0; x < nx; ++x) {
            size_t idx = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
            int xyz[3] = {x, y, z};
            for (int i = 0; i < L->q; ++i) {
                int s[3], out = 0, face = -1;
                for (int a = 0; a < 3; ++a) {
                    s[a] = xyz[a] - L->e[i][a];
                    if (s[a] < 0 || s[a] >= c->n[a]) {
                        if (c->p.bc[2 * a] == LBMREF_BC_PERIODIC) {
                            s[a] = (s[a] + c->n[a]) % c->n[a];
                        } else {
                            out = 1;
                            face = 2 * a + (s[a] < 0 ? 0 : 1);
                        }
                    }
                }
                double v;
                if (!out) {
                    size_t sidx = (size_t)s[0] + (size_t)nx * ((size_t)s[1] + (size_t)ny * s[2]);
                    v = src[i * N + sidx];
                } else {
                    v = src[L->opp[i] * N + idx];
                    if (thermal && c->p.bc[face] == LBMREF_BC_DIRICHLET)
                        v = -v + c->omega * c->p.t_wall[face];
                }
                dst[i * N + idx] = v;
            }
        }
    }
}

/* Heat entering the fluid through each Dirichlet face during the stream
 * just done: per wall link, the returned omega T_w - g+_out minus the
 * g+_out that left, i.e. omega T_w - 2 g+_out.  Summed serially in node
 * order.                                                               */
static void wall_flux(lbmref_ctx* c, double* flux) {
    const size_t N = c->N;
    for (int face = 0; face < 6; ++face) {
        flux[face] = 0.0;
        int a = face / 2, side = face % 2;
        if (a >= c->dim || c->p.bc[face] != LBMREF_BC_DIRICHLET) continue;
        int out = -1; /* thermal direction pointing into this face */
        for (int i = 0; i < c->lg.q; ++i)
            if (c->lg.e[i][a] == (side ? 1 : -1)) out = i;
        double acc = 0.0;
        for (size_t idx = 0; idx < N; ++idx) {
            int x[3];
            coords(c, idx, x);
            if (x[a] != (side ? c->n[a] - 1 : 0)) continue;
            acc += c->omega * c->p.t_wall[face] - 2.0 * c->gp[out * N + idx];
        }
        flux[face] = acc;
    }
}

int lbmref_step(lbmref_ctx* c, int64_t n) {
    if (!c) return LBMREF_E_INVALID;
    if (n < 0) return fail(c->err, "n must be >= 0");
    if (c->t < 0) { snprintf(c->err, 256, "not initialised"); return LBMREF_E_STATE; }
    for (int64_t s = 0; s < n; ++s) {
        macros(c);
        collide_f(c);
        collide_g(c);
        stream(c, &c->lf, c->f, c->fp, 0);
        stream(c, &c->lg, c->g, c->gp, 1);
        c->t += 1;
        wall_flux(c, c->flux[c->t & 1]);
    }
    return LBMREF_OK;
}

static int64_t count_nonfinite(const lbmref_ctx* c) {
    int64_t bad = 0;
    for (size_t k = 0; k < c->N * c->lf.q; ++k) bad += !isfinite(c->f[k]);
    for (size_t k = 0; k < c->N * c->lg.q; ++k) bad += !isfinite(c->g[k]);
    return bad;
}

int lbmref_fields(lbmref_ctx* c, double* rho, double* u, double* T) {
    if (!c) return LBMREF_E_INVALID;
    if (c->t < 0) { snprintf(c->err, 256, "not initialised"); return LBMREF_E_STATE; }
    macros(c);
    for (size_t idx = 0; idx < c->N; ++idx) {
        if (rho) rho[idx] = c->rho[idx];
        if (T) T[idx] = c->T[idx];
        if (u)
            for (int a = 0; a < c->dim; ++a) u[a * c->N + idx] = c->u[a * c->N + idx];
    }
    if (count_nonfinite(c)) { snprintf(c->err, 256, "non-finite populations"); return LBMREF_E_UNSTABLE; }
    return LBMREF_OK;
}

int lbmref_wall_flux(lbmref_ctx* c, double* last, double* prev) {
    if (!c) return LBMREF_E_INVALID;
    for (int f = 0; f < 6; ++f) {
        if (last) last[f] = c->flux[c->t & 1][f];
        if (prev) prev[f] = c->flux[(c->t + 1) & 1][f];
    }
    return LBMREF_OK;
}

/* Nusselt number at the isothermal walls.  The paper prints no formula;
 * this takes the conductive-flux normalisation Nu = q L / (alpha dT),
 * with q the mean heat flux per unit wall area from the anti-bounce-back
 * links and L the distance between the two walls of that axis, averaged
 * over the last two steps (one period of the even/odd lattice mode).
 * Hot faces: Dirichlet faces warmer than T0; cold: colder.             */
int lbmref_nusselt(lbmref_ctx* c, double* nu_hot, double* nu_cold) {
    if (!c) return LBMREF_E_INVALID;
    if (c->t < 2) { snprintf(c->err, 256, "need at least two steps"); return LBMREF_E_STATE; }
    double num[2] = {0, 0}, area[2] = {0, 0};
    for (int face = 0; face < 6; ++face) {
        int a = face / 2;
        if (a >= c->dim || c->p.bc[face] != LBMREF_BC_DIRICHLET) continue;
        double tw = c->p.t_wall[face];
        if (tw == c->t0) continue;
        int k = tw > c->t0 ? 0 : 1;
        double sign = k == 0 ? 1.0 : -1.0;
        double q = 0.5 * (c->flux[0][face] + c->flux[1][face]);
        num[k] += sign * c->n[a] * q;
        area[k] += (double)(c->N / c->n[a]);
    }
    if (area[0] == 0.0 || area[1] == 0.0) {
        snprintf(c->err, 256, "needs a hot and a cold Dirichlet face");
        return LBMREF_E_STATE;
    }
    double scale = 1.0 / (c->alpha * c->dT);
    if (nu_hot) *nu_hot = num[0] * scale / area[0];
    if (nu_cold) *nu_cold = num[1] * scale / area[1];
    if (count_nonfinite(c)) { snprintf(c->err, 256, "non-finite populations"); return LBMREF_E_UNSTABLE; }
    return LBMREF_OK;
}

int lbmref_diagnostics(lbmref_ctx* c, lbmref_diag* d) {
    if (!c || !d) return LBMREF_E_INVALID;
    if (c->t < 0) { snprintf(c->err, 256, "not initialised"); return LBMREF_E_STATE; }
    macros(c);
    double mass = 0, energy = 0, umax = 0, uT = 0, u2 = 0;
    const size_t N = c->N;
    for (size_t idx = 0; idx < N; ++idx) {
        double uu = 0;
        for (int a = 0; a < c->dim; ++a) uu += c->u[a * N + idx] * c->u[a * N + idx];
        mass += c->rho[idx];
        energy += c->T[idx];
        if (sqrt(uu) > umax) umax = sqrt(uu);
        u2 += uu;
        uT += c->u[c->gaxis * N + idx] * (c->T[idx] - c->t0);
    }
    d->t = c->t;
    d->mass = mass;
    d->energy = energy;
    d->umax = umax;
    d->nu_vol = 1.0 + c->H * (uT / N) / (c->alpha * c->dT);
    d->re = sqrt(u2 / N) * c->H / c->nu;
    d->nonfinite = count_nonfinite(c);
    return d->nonfinite ? LBMREF_E_UNSTABLE : LBMREF_OK;
}

int lbmref_get_populations(const lbmref_ctx* c, double* f, double* g) {
    if (!c) return LBMREF_E_INVALID;
    if (f) memcpy(f, c->f, c->N * c->lf.q * sizeof(double));
    if (g) memcpy(g, c->g, c->N * c->lg.q * sizeof(double));
    return LBMREF_OK;
}

int lbmref_set_populations(lbmref_ctx* c, const double* f, const double* g) {
    if (!c) return LBMREF_E_INVALID;
    if (f) memcpy(c->f, f, c->N * c->lf.q * sizeof(double));
    if (g) memcpy(c->g, g, c->N * c->lg.q * sizeof(double));
    if (c->t < 0) c->t = 0;
    return LBMREF_OK;
}

int lbmref_derived(const lbmref_ctx* c, double* out) {
    if (!c || !out) return LBMREF_E_INVALID;
    memcpy(out, c->d, sizeof(c->d));
    return LBMREF_OK;
}

int lbmref_lattice(int dim, int which, int* q, double* e, double* w,
                   double* M, double* Minv) {
    if ((dim != 2 && dim != 3) || (which != 0 && which != 1)) return LBMREF_E_INVALID;
    lattice_t L;
    if (build_lattice(dim, which, &L)) return LBMREF_E_INVALID;
    if (q) *q = L.q;
    for (int i = 0; i < L.q; ++i) {
        if (e)
            for (int a = 0; a < 3; ++a) e[i * 3 + a] = L.e[i][a];
        if (w) w[i] = L.w[i];
        for (int k = 0; k < L.q; ++k) {
            if (M) M[i * L.q + k] = L.M[i][k];
            if (Minv) Minv[i * L.q + k] = L.Minv[i][k];
        }
    }
    if (which == 1 && w) {
        /* rest-state thermal equilibrium weights g_eq(T = 1, u = 0) */
        lbmref_ctx tmp;
        memset(&tmp, 0, sizeof(tmp));
        tmp.dim = dim;
        tmp.a_t = dim == 2 ? -1.5 : -0.75;
        tmp.lg = L;
        double u0[3] = {0, 0, 0};
        g_equilibrium(&tmp, 1.0, u0, w);
    }
    return LBMREF_OK;
}
