/*
 * lbm.h -- C ABI of the MI355X (gfx950) thermal lattice Boltzmann library.
 *
 * The library advances the double-distribution-function (DDF) thermal
 * lattice Boltzmann model of Xu & Li, "Multi-GPU thermal lattice Boltzmann
 * simulations using OpenACC and MPI" (arXiv:2211.03160), Section 2:
 *   - flow populations f on D2Q9 (3D: D3Q19) with the multiple-relaxation-
 *     time collision of Eq. (5) / Eq. (8a) and the Guo forcing of
 *     Eqs. (6a)/(6b), driven by the Boussinesq buoyancy force
 *     F = rho g beta (T - T0) along the upward axis (Section 2.2);
 *   - temperature populations g on D2Q5 (3D: D3Q7) with the MRT collision
 *     of Eq. (7) / Eq. (9a);
 *   - half-way bounce-back on no-slip walls, half-way anti-bounce-back on
 *     isothermal (Dirichlet) walls and bounce-back of g on adiabatic walls
 *     (Section 2.2), or periodic faces.
 * Every time step is one fused pass: pull-streaming (Eqs. 8b, 9b) with the
 * wall rules, the moments, both collisions and the store of the
 * post-collision populations.  In 2D one kernel launch runs two to five
 * such steps (lbm_set_steps_per_launch), keeping the intermediate rows in
 * registers; in 3D one launch runs two (FP32 storage, the first step's
 * planes in LDS and registers) or one.
 *
 * Conventions
 *   - Every function returns an lbm_status (or a documented value); none
 *     throws, aborts or exits.  On failure lbm_last_error() describes it.
 *   - The library NEVER allocates device memory.  The caller provides one
 *     device workspace of lbm_workspace_bytes() bytes (e.g. a uint8 tensor)
 *     and a HIP stream; both must outlive the context.  Host memory of the
 *     context itself is owned by the library and freed by lbm_destroy().
 *   - All kernels run on the caller's stream, in stream order.  lbm_step()
 *     only enqueues; lbm_fields/lbm_nusselt/lbm_diagnostics/lbm_wall_flux/
 *     lbm_export_state synchronise the stream before returning.
 *   - A context is used by one host thread at a time.
 *   - Node (x, y, z) has flat index x + nx*(y + ny*z) (x fastest), the
 *     structure-of-arrays order of Section 3.1.  Faces are ordered
 *     -x, +x, -y, +y, -z, +z.  Gravity points along -y (2D) or -z (3D).
 *   - Field arrays: rho[N], T[N], u[dim][N] (component-major), FP64.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lbm_status;
#define LBM_OK 0
#define LBM_E_INVALID (-1)     /* bad argument or parameter                */
#define LBM_E_DEVICE (-2)      /* a HIP call failed                        */
#define LBM_E_UNSTABLE (-3)    /* non-finite populations, or a speed above
                                  the lattice sound speed c_s = 1/sqrt(3),
                                  found at a sync point                    */
#define LBM_E_STATE (-4)       /* call out of order                        */
#define LBM_E_UNSUPPORTED (-5) /* valid request this build cannot serve    */

/* Population storage.  Collision arithmetic is FP32 for every mode except
 * LBM_FP64, which computes in FP64 (the accuracy reference).  Every mode
 * stores deviations from a reference state: f_i - w_i, and g_i - G_i with
 * G the exact conduction state of the discrete step between the Dirichlet
 * faces of one axis (the gravity axis first; the linear profile and the
 * odd part that carries its heat flux), or w_i^T T0 where there is no such
 * axis (w_i^T: rest-state weights of the thermal equilibrium).  The
 * 16-bit modes round the deviations to nearest even; FP16 stores them
 * scaled by 2^14.                                                       */
#define LBM_FP32 0
#define LBM_FP64 1
#define LBM_FP16_SHIFTED 2
#define LBM_BF16_SHIFTED 3
#define LBM_MIXED_F16_G32 4 /* f as shifted FP16, g as FP32 */

/* Boundary kind per face */
#define LBM_BC_PERIODIC 0  /* both faces of an axis, or neither       */
#define LBM_BC_ADIABATIC 1 /* no-slip wall, zero heat flux             */
#define LBM_BC_DIRICHLET 2 /* no-slip wall at temperature t_wall[face] */

/* Run parameters, copied by lbm_create.  Any double documented as
 * "NaN: default" takes the default when set to NaN.                    */
typedef struct lbm_params {
    int32_t dim;      /* 2 (D2Q9 + D2Q5) or 3 (D3Q19 + D3Q7)               */
    int32_t n[3];     /* nodes along x, y, z; n[2] == 1 when dim == 2      */
    int32_t storage;  /* LBM_FP32 ... LBM_MIXED_F16_G32                    */
    int32_t bc[6];    /* LBM_BC_* per face                                 */
    int32_t reserved; /* must be 0                                         */
    double t_wall[6]; /* temperature of each DIRICHLET face                */
    double ra, pr;    /* Rayleigh and Prandtl numbers, Eq. (4)             */
    double u_ff;      /* free-fall velocity sqrt(g beta dT H), lattice units */
    double t_hot, t_cold; /* dT = t_hot - t_cold, T0 = (t_hot + t_cold)/2  */
    /* Transport coefficients in lattice units.  NaN: from Eqs. (2)-(4)
     * with H = n along gravity: nu = u_ff H sqrt(Pr/Ra),
     * alpha = u_ff H / sqrt(Pr Ra), g beta = u_ff^2 / (dT H).            */
    double nu, alpha, gbeta;
    double a_t; /* thermal-equilibrium constant a_T; NaN: -1.5 (2D), -0.75 (3D) */
    /* Flow MRT rates of the non-conserved moments; the shear rate is
     * s_nu = 1/(3 nu + 1/2).  NaN: s_e = s_eps = s_pi = s_nu and
     * s_q = s_m = 8 (2 - s_nu) / (8 - s_nu).                              */
    double s_e, s_eps, s_q, s_pi, s_m;
    /* Thermal MRT rates of the even non-conserved moments (NaN: 1); the
     * flux rate is q_j = 1/(alpha/c_sT^2 + 1/2), c_sT^2 = 2 w^T_moving.   */
    double q_e, q_nu;
} lbm_params;

typedef struct lbm_diag {
    int64_t t;         /* time step of the state                          */
    double mass;       /* sum over nodes of rho                           */
    double energy;     /* sum over nodes of T                             */
    double umax;       /* max over nodes of |u|                           */
    double nu_vol;     /* 1 + H <u_g (T - T0)> / (alpha dT), u_g upward   */
    double re;         /* sqrt(<|u|^2>) H / nu                            */
    int64_t nonfinite; /* number of non-finite stored populations         */
} lbm_diag;

/* Derived parameters returned by lbm_derive, in this order. */
#define LBM_D_NU 0
#define LBM_D_ALPHA 1
#define LBM_D_GBETA 2
#define LBM_D_TAU_F 3
#define LBM_D_TAU_G 4
#define LBM_D_S_NU 5
#define LBM_D_S_E 6
#define LBM_D_S_EPS 7
#define LBM_D_S_Q 8
#define LBM_D_S_PI 9
#define LBM_D_S_M 10
#define LBM_D_Q_J 11
#define LBM_D_Q_E 12
#define LBM_D_Q_NU 13
#define LBM_D_A_T 14
#define LBM_D_OMEGA 15 /* anti-bounce-back weight, Section 2.2 */
#define LBM_D_CS2_T 16
#define LBM_D_T0 17
#define LBM_D_H 18
#define LBM_D_COUNT 19

typedef struct lbm_ctx lbm_ctx;

/* Host only (no GPU needed).  Validates *p and fills out[LBM_D_COUNT]
 * (out may be NULL).  Returns LBM_E_INVALID with a message in
 * lbm_last_error(NULL) when the parameters are rejected: dim not 2/3,
 * n < 1, unpaired periodic faces, a walled axis with n < 2, more than
 * 2^31 - 1 nodes, non-positive nu/alpha, relaxation rates outside (0, 2)
 * (tau_f or tau_g <= 1/2), a_t outside (-4, 1) in 2D / (-6, 1) in 3D,
 * unknown storage.                                                       */
lbm_status lbm_derive(const lbm_params* p, double* out);

/* Host only.  Device workspace bytes needed for *p; 0 if *p is invalid. */
size_t lbm_workspace_bytes(const lbm_params* p);

/* Bytes moved to/from HBM per node and launch by the step kernels in
 * their algorithmic minimum (each population read once and written once):
 * per lattice update with one step per launch, per two updates with two. */
double lbm_bytes_per_update(const lbm_params* p);

/* Creates a context on the current HIP device.  d_workspace: device
 * pointer, 256-byte aligned, at least lbm_workspace_bytes(p) bytes, owned
 * by the caller.  hip_stream: a hipStream_t (NULL = default stream).
 * The state is undefined until lbm_init or lbm_init_fields.             */
lbm_status lbm_create(const lbm_params* p, void* d_workspace, size_t bytes,
                      void* hip_stream, lbm_ctx** out);

/* Resting start: rho = 1, u = 0, T = linear conduction profile between
 * the two Dirichlet faces of one axis (the gravity axis first; T0 when
 * there is none) plus amp * xi, xi in [-1, 1) drawn per node from
 * SplitMix64: xi = 2 * (s(seed ^ s(idx)) >> 11) * 2^-53 - 1, with s() one
 * SplitMix64 step from the given state and idx the flat node index.
 * Populations start at their equilibria.  Sets t = 0.  Asynchronous.   */
lbm_status lbm_init(lbm_ctx* c, uint64_t seed, double amp);

/* Start from host fields: populations at the equilibria of (rho, u, T).
 * rho may be NULL (rho = 1); u is [dim][N]; T is [N].  Sets t = 0.
 * Copies through the workspace staging area; returns after the copies.  */
lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* u,
                           const double* T);

/* Enqueues n fused steps (n = 0: no-op; n < 0: LBM_E_INVALID).  Several
 * steps go per launch (see lbm_set_steps_per_launch); a count that does
 * not divide n ends with shorter launches.                              */
lbm_status lbm_step(lbm_ctx* c, int64_t n);

/* Steps per kernel launch of lbm_step: 1 .. 5 in 2D (5 with FP32 storage
 * only), 1 or 2 in 3D.  A context starts with the count measured
 * fastest for its storage: in 2D 5 (FP32), 4 (FP16-f+FP32-g, BF16), 3
 * (FP16), 2 (FP64); in 3D 2 (FP32) and 1 (the others).
 * With k > 1 in 2D, each wavefront walks down a strip of columns row by
 * row, keeping the last rows of step t and of the intermediate steps in
 * registers, and writes step t+k; in 3D (k = 2) a block walks a 32 x 16
 * tile of columns along z, keeping three planes of the first step in LDS
 * and registers.  The update of every node is the same arithmetic on the
 * same stored values as with 1, so the results are bitwise identical;
 * only the global memory traffic per step drops.  A count of steps that k
 * does not divide ends with shorter launches.  LBM_E_INVALID for other
 * values, LBM_E_UNSUPPORTED for k > 2 in 3D, for k > 1 with FP64 storage in
 * 3D (its plane ring would not fit the LDS), for k > 2 with FP64 in 2D
 * (its deeper register rings do not fit) and for k = 5 with 16-bit
 * storage (slower than four there, so not built), LBM_E_STATE for a batch
 * member. */
lbm_status lbm_set_steps_per_launch(lbm_ctx* c, int32_t steps);
int32_t lbm_get_steps_per_launch(const lbm_ctx* c); /* 0 for NULL */

/* Debug mode (on = 1; off = 0, the default): before every kernel launch of
 * lbm_step, the population buffer the launch writes is filled with all-one
 * bits (NaN in every storage type; the padding beyond the last node stays
 * zero).  The pull scheme reads only the state and writes only the other
 * buffer, so a launch that leaves any population of any node unwritten
 * makes that value NaN in the new state, where lbm_diagnostics counts it
 * (nonfinite); with every node written the results are bitwise those of
 * the normal mode.  Costs one extra pass over the buffer per launch.
 * LBM_E_INVALID for other values of on, LBM_E_STATE for a batch member.  */
lbm_status lbm_set_debug_poison(lbm_ctx* c, int32_t on);
int32_t lbm_get_debug_poison(const lbm_ctx* c); /* 0 for NULL */

/* Moments of the current state at time t (the pre-collision moments
 * rho = sum f, u = (sum e f + F/2)/rho, T = sum g of Section 2.2),
 * computed in FP64 from the stored populations.  Each pointer may be
 * NULL, host or device memory.  Synchronises.  LBM_E_UNSTABLE (after
 * writing the outputs) if any stored population is non-finite or any
 * node's speed exceeds the lattice sound speed 1/sqrt(3).               */
lbm_status lbm_fields(lbm_ctx* c, double* rho, double* u, double* T);

/* Wall Nusselt numbers, FP64, averaged over the last two steps.  The heat
 * entering through a Dirichlet wall link per step is omega T_w - 2 g_out+
 * (anti-bounce-back, Section 2.2); Nu = L q / (alpha dT) with q the heat
 * flux per unit wall area and L the node count across that axis.  Hot
 * faces are Dirichlet faces warmer than T0, cold faces colder (their
 * outgoing flux is counted positive).  LBM_E_STATE if t < 2 or a hot or
 * cold face is missing; LBM_E_UNSTABLE (after writing the outputs) if a
 * result is not finite.  Synchronises.                                  */
lbm_status lbm_nusselt(lbm_ctx* c, double* nu_hot, double* nu_cold);

/* Heat entering through each face during the last step (last[6]) and the
 * step before (prev[6]); zero for non-Dirichlet faces.  Synchronises.   */
lbm_status lbm_wall_flux(lbm_ctx* c, double* last, double* prev);

/* FP64 reductions over all nodes.  Synchronises.  LBM_E_UNSTABLE (after
 * writing *d) if a stored population is non-finite or umax exceeds the
 * lattice sound speed 1/sqrt(3).                                        */
lbm_status lbm_diagnostics(lbm_ctx* c, lbm_diag* d);

/* For callers that cannot allocate device memory or wait on the host (code
 * under HIP graph capture, tight serving loops): lbm_diagnostics without
 * the context's workspace scratch and without synchronising.  Enqueues on
 * the context's stream the same FP64 reductions and writes the values of
 * lbm_diag, in field order and as doubles (t, mass, energy, umax, nu_vol,
 * re, nonfinite), to the caller's device buffer d_out[LBM_DIAG_VALUES].
 * The per-block partial sums live in a scratch array the library keeps per
 * device (48 KiB, statically, until the process ends); the call allocates
 * nothing, copies nothing to the host and issues no memset.  Calls that
 * overlap on one device (from several host threads, or on different
 * streams) share that scratch and race: the caller serialises them.
 * LBM_E_INVALID if d_out is NULL or not device memory, LBM_E_STATE before
 * init.  Non-finite populations are counted in d_out[6], not reported as
 * LBM_E_UNSTABLE (the call does not wait for the result).              */
#define LBM_DIAG_VALUES 7
lbm_status lbm_diagnostics_async(lbm_ctx* c, double* d_out);

/* Checkpoint: the stored populations, the wall-flux history and t.
 * lbm_state_bytes gives the size; export writes it to host memory and
 * synchronises; import reads a buffer exported by a context with the same
 * parameters.                                                           */
size_t lbm_state_bytes(const lbm_ctx* c);
lbm_status lbm_export_state(lbm_ctx* c, void* host, size_t bytes);
lbm_status lbm_import_state(lbm_ctx* c, const void* host, size_t bytes);

int64_t lbm_time(const lbm_ctx* c); /* -1 before init, -1 for NULL */
void lbm_destroy(lbm_ctx* c);       /* NULL-safe; does not synchronise    */

/* Last error of a context, or of lbm_derive/lbm_workspace_bytes/
 * lbm_create on this thread when c is NULL.  Never NULL.                */
const char* lbm_last_error(const lbm_ctx* c);

/* Host only.  The tables the kernels are compiled with.  which: 0 flow,
 * 1 thermal.  q: lattice size; e[q*3] velocities; M[q*q] moment basis
 * (row = moment, integer entries); w[q] flow weights (which = 0) or
 * rest-state thermal weights for a_T = default (which = 1).  Any output
 * may be NULL.                                                          */
lbm_status lbm_lattice(int32_t dim, int32_t which, int32_t* q, int32_t* e,
                       int32_t* M, double* w);

/* Host only.  Version string of the library build.                      */
const char* lbm_version(void);

/* HBM bandwidth probe: the ceiling a one-pass streaming kernel reaches on
 * this GPU, against which the step kernels are measured (the step is
 * bound by HBM bandwidth, Section 3.1).  One kernel launch on hip_stream
 * (a hipStream_t, NULL = default stream), asynchronous:
 *   kind 0: copy `bytes` from src to dst;
 *   kind 1: read `bytes` of src (dst receives at most one 16-byte vector);
 *   kind 2: write `bytes` of dst (src unused, may be NULL).
 * per_thread: 16-byte vectors per thread, 1, 2, 4 or 8 (a block of 256
 * threads moves 4 KiB x per_thread contiguous bytes); flags bit 0:
 * non-temporal loads and stores.  src and dst are device pointers owned by
 * the caller, 16-byte aligned, bytes a positive multiple of 16; the ranges
 * must not overlap.  LBM_E_INVALID for other arguments, LBM_E_DEVICE if
 * the launch fails.                                                      */
lbm_status lbm_probe_bandwidth(int32_t kind, const void* src, void* dst, size_t bytes, int32_t per_thread,
                               int32_t flags, void* hip_stream);

/* ------------------------------------------------------------- batches
 * Many independent cavities of different sizes and parameters (same dim
 * and storage) advanced together: every launch of lbm_batch_step updates
 * all nodes of all cavities, by 2-5 steps in 2D (the streaming kernel of
 * lbm_set_steps_per_launch, over the work units of every cavity) or by one,
 * with the per-node arithmetic of lbm_step, so each cavity evolves exactly
 * as it would alone (the physics is Section 2.2's, per cavity; batching is
 * a launch strategy).  All cavities share the time step counter.  The batch
 * workspace holds every cavity's state plus the work tables; the library
 * never allocates device memory.                                        */
typedef struct lbm_batch lbm_batch;

typedef struct lbm_batch_config {
    int32_t block;       /* threads per block: 128, 256 or 512                */
    int32_t grid_per_cu; /* 0: one block per work unit of `block` nodes;
                            k > 0: persistent grid of k blocks per compute
                            unit, looping over the units                      */
    int32_t graph_steps; /* 0: launch every time; G > 0 (even): capture the
                            launches of G steps once into a hipGraph and
                            replay it (needs a non-default stream; ignored on
                            the NULL stream)                                  */
    int32_t reserved;    /* 0                                                 */
    int32_t stream_rows;  /* rows per strip segment of the streaming kernel
                             (several steps per launch), 8 .. 256; 0: the
                             single-cavity default of the storage mode        */
    int32_t stream_waves; /* wavefronts per block of the streaming kernel:
                             1, 2, 4 or 8; 0: 4                               */
} lbm_batch_config;
#define LBM_BATCH_TUNE_MAX 80 /* most timings lbm_batch_tune reports */

/* Host only.  Device workspace bytes for `count` cavities with parameters
 * ps[0..count-1]; 0 if any is invalid or they differ in dim or storage. */
size_t lbm_batch_workspace_bytes(const lbm_params* ps, int32_t count);

/* count in [1, 65535].  Default config {256, 0, 0, 0, 0, 0}.  d_workspace: device
 * pointer, 256-byte aligned, caller-owned, at least
 * lbm_batch_workspace_bytes bytes.                                      */
lbm_status lbm_batch_create(const lbm_params* ps, int32_t count, void* d_workspace, size_t bytes,
                            void* hip_stream, lbm_batch** out);

/* lbm_init of every cavity k with seeds[k], amps[k]; clears the
 * instability flags; t = 0.  Synchronises.                              */
lbm_status lbm_batch_init(lbm_batch* b, const uint64_t* seeds, const double* amps);

/* lbm_init_fields of cavity k; only at t = 0, after lbm_batch_init.     */
lbm_status lbm_batch_init_fields(lbm_batch* b, int32_t k, const double* rho, const double* u,
                                 const double* T);

/* Enqueues n steps of every cavity (graph replays when configured, then
 * launches of lbm_batch_get_steps_per_launch steps, then one-step launches
 * for the remainder).  Asynchronous.                                    */
lbm_status lbm_batch_step(lbm_batch* b, int64_t n);

/* Steps per launch of lbm_batch_step: 1 (batch_step_kernel, the shape of
 * lbm_batch_config) or 2..5 (the streaming kernel; 2D batches whose
 * cavities' population arrays are each under 4 GiB; 5 with FP32 storage
 * only).  A batch starts with the count a single cavity of its storage
 * mode starts with, where streaming is available, else 1.  Results do not
 * depend on it (bitwise).  LBM_E_INVALID outside 1..5, LBM_E_UNSUPPORTED
 * for k > 1 where streaming is not available, for k > 2 with FP64 storage
 * and for k = 5 with 16-bit storage.  Synchronises the batch stream when
 * the count changes (the work tables are rewritten).                    */
lbm_status lbm_batch_set_steps_per_launch(lbm_batch* b, int32_t steps);
int32_t lbm_batch_get_steps_per_launch(const lbm_batch* b); /* 0 for NULL */

/* Borrowed view of cavity k, owned by the batch: lbm_fields, lbm_nusselt,
 * lbm_wall_flux, lbm_diagnostics and lbm_export_state work on it;
 * lbm_init, lbm_init_fields, lbm_step and lbm_import_state return
 * LBM_E_STATE; lbm_destroy ignores it.                                  */
lbm_status lbm_batch_cavity(lbm_batch* b, int32_t k, lbm_ctx** view);

/* Wall Nusselt numbers of every cavity (arrays of count; NaN where a
 * cavity has no hot or cold face or has diverged).  LBM_E_STATE if t < 2.
 * Synchronises.                                                         */
lbm_status lbm_batch_nusselt(lbm_batch* b, double* nu_hot, double* nu_cold);

/* flags[k] = 1 once cavity k produced a non-finite density or temperature
 * or a speed above the lattice sound speed 1/sqrt(3) (its divergence does
 * not affect the other cavities).  Synchronises.                        */
lbm_status lbm_batch_unstable(lbm_batch* b, int32_t* flags);

/* Autotuner: times `steps` launches of each candidate with HIP events on
 * the batch stream and keeps the fastest per step: the one-step kernel's
 * launch shapes (block 128/256/512 x grid_per_cu 0/2/4/8) and, where the
 * batch can stream several steps per launch, the streaming kernel at 2, 3
 * and 4 steps per launch (FP32: 2 to 5; FP64: 2) x segment rows
 * 16/24/32/48/64 x 2/4/8 wavefronts per block.  The winner sets the configuration and the steps
 * per launch (graph_steps is left as configured); results do not depend on
 * any of them (bitwise).  The timing steps are real steps: t advances by
 * (steps + 1) x the steps per launch of every candidate.  ms_per_step
 * (nullable) receives up to LBM_BATCH_TUNE_MAX timings in candidate order,
 * ncand their number.                                                   */
lbm_status lbm_batch_tune(lbm_batch* b, int32_t steps, lbm_batch_config* best, double* ms_per_step,
                          int32_t* ncand);

/* LBM_E_INVALID for a field outside its range.  Changing the streaming
 * shape rewrites the work tables (synchronises the batch stream).       */
lbm_status lbm_batch_set_config(lbm_batch* b, const lbm_batch_config* cfg);
lbm_status lbm_batch_get_config(const lbm_batch* b, lbm_batch_config* cfg);
int64_t lbm_batch_time(const lbm_batch* b);   /* -1 before init          */
void lbm_batch_destroy(lbm_batch* b);         /* NULL-safe               */
const char* lbm_batch_last_error(const lbm_batch* b); /* NULL: this thread */

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
