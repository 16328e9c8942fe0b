// lbm_api.hip -- host side of the C ABI declared in include/lbm.h.
//
// Validates and maps the run parameters (Section 2.1, Eqs. 2-4: the
// free-fall scaling gives nu = U H sqrt(Pr/Ra), alpha = U H / sqrt(Pr Ra),
// g beta = U^2 / (dT H) in lattice units), carves the caller's device
// workspace, and launches the kernels of kernels.hpp on the caller's stream.
// The library never allocates device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"

using namespace lbm;

namespace {

thread_local char g_err[512] = "";

constexpr size_t kAlign = 256;
constexpr int kDiagBlocks = 1024;
constexpr uint32_t kStagingNodes = 1u << 20;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

lbm_status set_err(char* buf, lbm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return st;
}

FastDiv make_div(uint32_t d) {
    FastDiv f{d, 0, 0};
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    return f;
}

bool div_ok(const FastDiv& f, uint32_t limit) {
    // spot-check the multiply-high division against the hardware divide
    const uint32_t probes[] = {0u, 1u, f.d - 1, f.d, f.d + 1, 2 * f.d - 1, 2 * f.d,
                               limit / 2, limit - 1, limit};
    for (uint32_t x : probes)
        if (x <= limit && f.div(x) != x / f.d) return false;
    for (uint32_t x = 0; x < 4096 && x <= limit; ++x)
        if (f.div(x) != x / f.d) return false;
    return true;
}

struct Derived {
    double v[LBM_D_COUNT];
};

int qf_of(int dim) { return dim == 2 ? Flow<2>::Q : Flow<3>::Q; }
int qg_of(int dim) { return dim == 2 ? Heat<2>::Q : Heat<3>::Q; }

size_t elem_f(int storage) {
    switch (storage) {
    case LBM_FP32: return 4;
    case LBM_FP64: return 8;
    default: return 2;
    }
}
size_t elem_g(int storage) {
    switch (storage) {
    case LBM_FP32: case LBM_MIXED_F16_G32: return 4;
    case LBM_FP64: return 8;
    default: return 2;
    }
}

lbm_status derive(const lbm_params* p, Derived* out, char* err) {
    if (!p) return set_err(err, LBM_E_INVALID, "null params");
    if (p->dim != 2 && p->dim != 3) return set_err(err, LBM_E_INVALID, "dim must be 2 or 3");
    if (p->storage < LBM_FP32 || p->storage > LBM_MIXED_F16_G32)
        return set_err(err, LBM_E_INVALID, "unknown storage %d", p->storage);
    if (p->reserved != 0) return set_err(err, LBM_E_INVALID, "reserved must be 0");
    for (int a = 0; a < 3; ++a)
        if (p->n[a] < 1) return set_err(err, LBM_E_INVALID, "n[%d] must be >= 1", a);
    if (p->dim == 2 && p->n[2] != 1) return set_err(err, LBM_E_INVALID, "n[2] must be 1 in 2D");
    const double Nd = (double)p->n[0] * p->n[1] * p->n[2];
    if (Nd > 2147483647.0) return set_err(err, LBM_E_INVALID, "more than 2^31-1 nodes");
    // population offsets are 32-bit element indices
    if ((Nd + kTile) * (p->dim == 2 ? Flow<2>::Q : Flow<3>::Q) > 4294967295.0)
        return set_err(err, LBM_E_INVALID, "too many nodes for 32-bit population offsets");
    for (int a = 0; a < p->dim; ++a) {
        const int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
        if (lo < 0 || lo > 2 || hi < 0 || hi > 2)
            return set_err(err, LBM_E_INVALID, "unknown boundary kind on axis %d", a);
        if ((lo == LBM_BC_PERIODIC) != (hi == LBM_BC_PERIODIC))
            return set_err(err, LBM_E_INVALID, "periodic faces of axis %d must be paired", a);
        if (lo != LBM_BC_PERIODIC && p->n[a] < 2)
            return set_err(err, LBM_E_INVALID, "walled axis %d needs n >= 2", a);
    }
    const int gaxis = p->dim - 1;
    const double H = p->n[gaxis];
    const double dT = p->t_hot - p->t_cold;
    const double T0 = 0.5 * (p->t_hot + p->t_cold);
    const bool derived = std::isnan(p->nu) || std::isnan(p->alpha) || std::isnan(p->gbeta);
    if (derived) {
        if (!(p->ra > 0) || !(p->pr > 0)) return set_err(err, LBM_E_INVALID, "ra and pr must be > 0");
        if (!(p->u_ff > 0) || p->u_ff > 0.3) return set_err(err, LBM_E_INVALID, "u_ff must lie in (0, 0.3]");
        if (!(dT > 0)) return set_err(err, LBM_E_INVALID, "t_hot must exceed t_cold");
    }
    const double nu = std::isnan(p->nu) ? p->u_ff * H * std::sqrt(p->pr / p->ra) : p->nu;
    const double alpha = std::isnan(p->alpha) ? p->u_ff * H / std::sqrt(p->pr * p->ra) : p->alpha;
    const double gbeta = std::isnan(p->gbeta) ? p->u_ff * p->u_ff / (dT * H) : p->gbeta;
    if (!(nu > 0) || !(alpha > 0) || !std::isfinite(gbeta))
        return set_err(err, LBM_E_INVALID, "nu and alpha must be > 0 and g beta finite");
    const double a_t = std::isnan(p->a_t) ? (p->dim == 2 ? Heat<2>::a_t_default : Heat<3>::a_t_default) : p->a_t;
    if (!(a_t < 1.0) || !(a_t > (p->dim == 2 ? -4.0 : -6.0)))
        return set_err(err, LBM_E_INVALID, "a_t must lie in (%d, 1)", p->dim == 2 ? -4 : -6);
    const double w_move = p->dim == 2 ? Heat<2>::w_move(a_t) : Heat<3>::w_move(a_t);
    const double omega = 2.0 * w_move;  // (4 + a_T)/10 or (6 + a_T)/21
    const double cs2_t = 2.0 * w_move;
    const double tau_f = 3.0 * nu + 0.5;
    const double tau_g = alpha / cs2_t + 0.5;
    const double s_nu = 1.0 / tau_f;
    const double s_q = std::isnan(p->s_q) ? 8.0 * (2.0 - s_nu) / (8.0 - s_nu) : p->s_q;
    const double s_e = std::isnan(p->s_e) ? s_nu : p->s_e;
    const double s_eps = std::isnan(p->s_eps) ? s_nu : p->s_eps;
    const double s_pi = std::isnan(p->s_pi) ? s_nu : p->s_pi;
    const double s_m = std::isnan(p->s_m) ? s_q : p->s_m;
    const double q_j = 1.0 / tau_g;
    const double q_e = std::isnan(p->q_e) ? 1.0 : p->q_e;
    const double q_nu = std::isnan(p->q_nu) ? 1.0 : p->q_nu;
    const double rates[] = {s_nu, s_q, s_e, s_eps, s_pi, s_m, q_j, q_e, q_nu};
    for (double r : rates)
        if (!(r > 0.0 && r < 2.0))
            return set_err(err, LBM_E_INVALID,
                           "relaxation rates must lie in (0, 2) (tau_f = %g, tau_g = %g)", tau_f, tau_g);
    double* v = out->v;
    v[LBM_D_NU] = nu; v[LBM_D_ALPHA] = alpha; v[LBM_D_GBETA] = gbeta;
    v[LBM_D_TAU_F] = tau_f; v[LBM_D_TAU_G] = tau_g; v[LBM_D_S_NU] = s_nu;
    v[LBM_D_S_E] = s_e; v[LBM_D_S_EPS] = s_eps; v[LBM_D_S_Q] = s_q;
    v[LBM_D_S_PI] = s_pi; v[LBM_D_S_M] = s_m; v[LBM_D_Q_J] = q_j;
    v[LBM_D_Q_E] = q_e; v[LBM_D_Q_NU] = q_nu; v[LBM_D_A_T] = a_t;
    v[LBM_D_OMEGA] = omega; v[LBM_D_CS2_T] = cs2_t; v[LBM_D_T0] = T0; v[LBM_D_H] = H;
    return LBM_OK;
}

struct Layout {
    size_t pop_bytes, f_bytes;     // one population buffer; its f part
    size_t off_pop[2], off_flux, off_red, off_stage, total;
    size_t area[6];                // face node counts (0 for unused faces)
    size_t flux_doubles;           // per slot
    size_t red_doubles, stage_nodes;
};

Layout layout(const lbm_params* p, size_t staging_cap = kStagingNodes) {
    Layout L{};
    const size_t N = (size_t)p->n[0] * p->n[1] * p->n[2];
    const size_t Np = (N + kTile - 1) / kTile * kTile;  // whole storage tiles
    L.f_bytes = align_up(Np * qf_of(p->dim) * elem_f(p->storage));
    L.pop_bytes = L.f_bytes + Np * qg_of(p->dim) * elem_g(p->storage);
    for (int f = 0; f < 6; ++f) {
        const int a = f / 2;
        L.area[f] = a < p->dim ? N / p->n[a] : 0;
        L.flux_doubles += L.area[f];
    }
    L.red_doubles = (size_t)kDiagBlocks * kDiagVals + 64;
    L.stage_nodes = N < staging_cap ? N : staging_cap;
    size_t off = 0;
    L.off_pop[0] = off; off = align_up(off + L.pop_bytes);
    L.off_pop[1] = off; off = align_up(off + L.pop_bytes);
    L.off_flux = off; off = align_up(off + 2 * L.flux_doubles * sizeof(double));
    L.off_red = off; off = align_up(off + L.red_doubles * sizeof(double));
    L.off_stage = off; off = align_up(off + L.stage_nodes * (2 + p->dim) * sizeof(double));
    L.total = off;
    return L;
}

}  // namespace

struct lbm_ctx {
    lbm_params p;
    Derived d;
    Layout lay;
    int device;
    hipStream_t stream;
    char* ws;
    int cur;      // population buffer holding the state
    int64_t t;    // time step of the state; -1 before init
    Geometry geo;
    int cond_axis;
    bool view;    // a cavity owned by a batch: the batch steps and initialises it
    int32_t steps_per_launch;  // time steps per launch of lbm_step (1-5 in 2D, 1-2 in 3D)
    int cus;                   // compute units of the device
    bool poison;               // debug: fill the destination state with NaN before every launch
    char err[512];

    void* pop(int k) const { return ws + lay.off_pop[k]; }
    double* flux(int slot, int face) const {
        double* base = (double*)(ws + lay.off_flux) + (size_t)slot * lay.flux_doubles;
        for (int f = 0; f < face; ++f) base += lay.area[f];
        return base;
    }
    double* red() const { return (double*)(ws + lay.off_red); }
    double* stage() const { return (double*)(ws + lay.off_stage); }
};

#define HIP_TRY(buf, call)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return set_err(buf, LBM_E_DEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

namespace {

// The thermal reference state G the stored g deviations are taken from:
// the exact conduction state of the discrete step between the two Dirichlet
// faces of the context's conduction axis a (n nodes, walls half a link
// outside), T_b(k) = T_lo + (k + 1/2) gr with gr = (T_hi - T_lo)/n.  Its
// populations are w_i T_b plus an odd part along a: pre-collision
// +/-delta on the two populations along +/-a, (1 - q_j) times that after
// the collision.  Streaming maps the post-collision state at k - 1 onto the
// pre-collision one at k when w gr + q_j delta = 0, so delta = -w gr / q_j
// (w: moving thermal weight, q_j: flux relaxation rate); the
// anti-bounce-back rule of Section 2.2 then holds exactly at both walls,
// and each wall link carries the conduction flux -alpha gr into the fluid
// at the T_lo face (alpha = 2 w (1/q_j - 1/2)), +alpha gr at the T_hi face.
// Without a conduction axis G is the uniform rest state w_i T0.
struct Reference {
    int axis;            // -1: uniform T0
    double tb0, tbg;     // T_b(k) = tb0 + tbg k
    double delta;        // odd part of the pre-collision populations along the axis
    double flux_lo;      // heat entering through one link of the T_lo face
};
Reference reference_state(const lbm_ctx* c) {
    const double* v = c->d.v;
    Reference r{c->cond_axis, v[LBM_D_T0], 0.0, 0.0, 0.0};
    if (r.axis < 0) return r;
    const double t_lo = c->p.t_wall[2 * r.axis], t_hi = c->p.t_wall[2 * r.axis + 1];
    const double gr = (t_hi - t_lo) / c->p.n[r.axis];
    const double w = 0.5 * v[LBM_D_OMEGA], qj = v[LBM_D_Q_J];
    r.tb0 = t_lo + 0.5 * gr;
    r.tbg = gr;
    r.delta = -w * gr / qj;
    r.flux_lo = -2.0 * w * (1.0 / qj - 0.5) * gr;
    return r;
}

template <class R> Coef<R> make_coef(const lbm_ctx* c) {
    Coef<R> k{};
    const double* v = c->d.v;
    auto flow_rate = [&](int kind) {
        switch (kind) {
        case kE: return v[LBM_D_S_E];
        case kEps: return v[LBM_D_S_EPS];
        case kQ: return v[LBM_D_S_Q];
        case kNu: return v[LBM_D_S_NU];
        case kPi: return v[LBM_D_S_PI];
        case kM: return v[LBM_D_S_M];
        default: return 0.0;
        }
    };
    auto heat_rate = [&](int kind) {
        switch (kind) {
        case kJx: case kJy: case kJz: return v[LBM_D_Q_J];
        case kE: return v[LBM_D_Q_E];
        case kNu: return v[LBM_D_Q_NU];
        default: return 0.0;
        }
    };
    // in 2D each kind's rate also carries 1/|M_k|^2 of its rows
    const bool fold = c->p.dim == 2;
    for (int kind = 0; kind < 10; ++kind) {
        const double s = flow_rate(kind);
        const int nf = fold ? kind_norm<Flow<2>>(kind) : 0, ng = fold ? kind_norm<Heat<2>>(kind) : 0;
        const double sf = nf > 0 ? 1.0 / nf : 1.0, sg = ng > 0 ? 1.0 / ng : 1.0;
        k.s[kind] = (R)(s * sf);
        k.b[kind] = (R)((1.0 - 0.5 * s) * sf);
        k.q[kind] = (R)(heat_rate(kind) * sg);
    }
    if (c->p.dim == 3) {
        // the factors of collide_store_d3: d_k / |M_k|^2 with d_k = -s (m_k
        // - m_k,eq) + (1 - s/2) (M F~)_k, the row's integer factors included
        auto nf = [](int row) { return (double)row_norm<Flow<3>>(row); };
        auto ng = [](int row) { return (double)row_norm<Heat<3>>(row); };
        auto b = [&](int kind) { return 1.0 - 0.5 * flow_rate(kind); };
        const double sE = flow_rate(kE), sEps = flow_rate(kEps), sQ = flow_rate(kQ), sNu = flow_rate(kNu),
                     sPi = flow_rate(kPi), sM = flow_rate(kM);
        k.k3[k3SE] = (R)(-19.0 * sE / nf(1));
        k.k3[k3BE] = (R)(38.0 * b(kE) / nf(1));
        k.k3[k3SEps] = (R)(-sEps / nf(2));
        k.k3[k3BEps] = (R)(-11.0 * b(kEps) / nf(2));
        k.k3[k3SQ] = (R)(-5.0 / 3.0 * sQ / nf(4));
        k.k3[k3BQ] = (R)(-(sQ + 2.0 * b(kQ)) / 3.0 / nf(4));
        k.k3[k3SP] = (R)(-sNu / nf(9));
        k.k3[k3BP] = (R)(-2.0 * b(kNu) / nf(9));
        k.k3[k3SPi] = (R)(-sPi / nf(10));
        k.k3[k3BPi] = (R)(b(kPi) / nf(10));
        k.k3[k3SW] = (R)(-sNu / nf(11));
        k.k3[k3BW] = (R)(-2.0 * b(kNu) / nf(11));
        k.k3[k3SWi] = (R)(-sPi / nf(12));
        k.k3[k3BWi] = (R)(b(kPi) / nf(12));
        k.k3[k3SO] = (R)(-sNu / nf(13));
        k.k3[k3BO] = (R)(b(kNu) / nf(13));
        k.k3[k3SM] = (R)(-sM / nf(16));
        k.k3[k3QJ] = (R)(-heat_rate(kJx) / ng(1));
        k.k3[k3QE] = (R)(-heat_rate(kE) / ng(4));
        k.k3[k3QP] = (R)(-heat_rate(kNu) / ng(5));
        k.k3[k3QW] = (R)(-heat_rate(kNu) / ng(6));
    }
    k.a_t = (R)v[LBM_D_A_T];
    k.gbeta = (R)v[LBM_D_GBETA];
    k.t0 = (R)v[LBM_D_T0];
    const Reference ref = reference_state(c);
    k.bt.axis = ref.axis < 0 ? 0 : ref.axis;
    k.bt.tb0 = (R)ref.tb0;
    k.bt.tbg = (R)ref.tbg;
    const double omega = v[LBM_D_OMEGA];
    for (int f = 0; f < 6; ++f) {
        k.abb_a[f] = k.abb_b[f] = R(0);
        k.flux_c[f] = 0.0;
        if (!c->geo.dirichlet[f]) continue;
        if (f / 2 == ref.axis) {
            k.flux_c[f] = f % 2 == 0 ? ref.flux_lo : -ref.flux_lo;
        } else {
            k.abb_a[f] = (R)(omega * c->p.t_wall[f]);
            k.abb_b[f] = (R)omega;
        }
    }
    return k;
}

// Calls fn(std::integral_constant<int, DIM>{}, St{}) for the context's
// lattice and storage.
template <class Fn> lbm_status dispatch(const lbm_ctx* c, Fn&& fn) {
    const int s = c->p.storage;
    if (c->p.dim == 2) {
        std::integral_constant<int, 2> d;
        switch (s) {
        case LBM_FP32: return fn(d, StF32{});
        case LBM_FP64: return fn(d, StF64{});
        case LBM_FP16_SHIFTED: return fn(d, StF16{});
        case LBM_BF16_SHIFTED: return fn(d, StBF16{});
        default: return fn(d, StMix{});
        }
    }
    std::integral_constant<int, 3> d;
    switch (s) {
    case LBM_FP32: return fn(d, StF32{});
    case LBM_FP64: return fn(d, StF64{});
    case LBM_FP16_SHIFTED: return fn(d, StF16{});
    case LBM_BF16_SHIFTED: return fn(d, StBF16{});
    default: return fn(d, StMix{});
    }
}

unsigned grid_for(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

lbm_status enter(lbm_ctx* c) {
    if (!c) return set_err(g_err, LBM_E_INVALID, "null context");
    HIP_TRY(c->err, hipSetDevice(c->device));
    return LBM_OK;
}

lbm_status require_state(lbm_ctx* c) {
    if (c->t < 0) return set_err(c->err, LBM_E_STATE, "state not initialised: call lbm_init first");
    return LBM_OK;
}

bool is_device_ptr(const void* p) {
    if (!p) return false;
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

// split population buffer k into typed f and g pointers
template <class St> struct Pops {
    typename St::TF* f;
    typename St::TG* g;
};
template <class St> Pops<St> pops(const lbm_ctx* c, int k) {
    char* base = (char*)c->pop(k);
    return {(typename St::TF*)base, (typename St::TG*)(base + c->lay.f_bytes)};
}

lbm_status launch_init(lbm_ctx* c, int mode, uint32_t n0, uint32_t cnt, uint64_t seed, double amp,
                       const double* rho, const double* u, const double* T) {
    return dispatch(c, [&](auto dimc, auto st) -> lbm_status {
        constexpr int DIM = decltype(dimc)::value;
        using St = decltype(st);
        InitArgs<St> a{};
        const auto P = pops<St>(c, c->cur);
        a.fdst = P.f;
        a.gdst = P.g;
        a.geo = c->geo;
        a.c = make_coef<typename St::R>(c);
        a.n0 = n0;
        a.cnt = cnt;
        a.mode = mode;
        a.axis = c->cond_axis;
        a.t_lo = c->cond_axis >= 0 ? c->p.t_wall[2 * c->cond_axis] : 0.0;
        a.t_hi = c->cond_axis >= 0 ? c->p.t_wall[2 * c->cond_axis + 1] : 0.0;
        a.t0 = c->d.v[LBM_D_T0];
        a.amp = amp;
        a.seed = seed;
        a.rho = rho;
        a.u = u;
        a.T = T;
        const double at = c->d.v[LBM_D_A_T];
        a.w_rest = DIM == 2 ? Heat<2>::w_rest(at) : Heat<3>::w_rest(at);
        a.w_move = DIM == 2 ? Heat<2>::w_move(at) : Heat<3>::w_move(at);
        a.delta = reference_state(c).delta;
        hipLaunchKernelGGL((init_kernel<DIM, St>), dim3(grid_for(cnt)), dim3(kBlock), 0, c->stream, a);
        HIP_TRY(c->err, hipGetLastError());
        return LBM_OK;
    });
}

// both population buffers: zero the bytes that hold no node (the lanes of
// the last storage tile beyond N, the alignment gap after the f arrays)
void clear_tails_of(lbm_ctx* c, int k) {
    const uint32_t N = c->geo.N;
    const uint32_t qf = qf_of(c->p.dim), qg = qg_of(c->p.dim);
    const uint32_t ef = (uint32_t)elem_f(c->p.storage), eg = (uint32_t)elem_g(c->p.storage);
    const size_t f_used = (size_t)(N + kTile - 1) / kTile * kTile * qf * ef;
    unsigned char* base = (unsigned char*)c->pop(k);
    if (N % kTile) {
        hipLaunchKernelGGL(clear_tail_kernel, dim3(1), dim3(kBlock), 0, c->stream, base, N, qf, ef);
        hipLaunchKernelGGL(clear_tail_kernel, dim3(1), dim3(kBlock), 0, c->stream, base + c->lay.f_bytes, N, qg,
                           eg);
    }
    if (c->lay.f_bytes > f_used)
        hipLaunchKernelGGL(zero_bytes_kernel, dim3(1), dim3(kBlock), 0, c->stream, base + f_used,
                           (uint32_t)(c->lay.f_bytes - f_used));
}

lbm_status clear_tails(lbm_ctx* c) {
    for (int k = 0; k < 2; ++k) clear_tails_of(c, k);
    HIP_TRY(c->err, hipGetLastError());
    return LBM_OK;
}

// Debug mode: before a launch writes the population buffer that is not the
// state, fill every node's populations there with all-one bits (NaN in
// every storage type) and restore the zero tails, so that a node the
// launch fails to write reads as NaN in the next state.  A fill kernel,
// not a memset, so that a captured graph replays it correctly.
void poison_dst(lbm_ctx* c) {
    if (!c->poison) return;
    const size_t words = c->lay.pop_bytes / 4;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)std::min<size_t>(grid_for(words), 4096)), dim3(kBlock), 0,
                       c->stream, (uint32_t*)c->pop(1 - c->cur), words, 0xFFFFFFFFu);
    clear_tails_of(c, 1 - c->cur);
}

lbm_status zero_flux(lbm_ctx* c) {
    const size_t n = 2 * c->lay.flux_doubles;
    if (n == 0) return LBM_OK;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::min<size_t>(grid_for(n), 4096)), dim3(kBlock), 0,
                       c->stream, (double*)(c->ws + c->lay.off_flux), n, 0.0);
    HIP_TRY(c->err, hipGetLastError());
    return LBM_OK;
}

// sums of the two flux slots of every face: out[slot * 6 + face]
lbm_status face_sums(lbm_ctx* c, double* host12) {
    FaceSumArgs a{};
    for (int slot = 0; slot < 2; ++slot)
        for (int f = 0; f < 6; ++f) {
            const int b = slot * 6 + f;
            a.buf[b] = c->geo.dirichlet[f] ? c->flux(slot, f) : nullptr;
            a.count[b] = (uint32_t)c->lay.area[f];
        }
    a.out = c->red();
    hipLaunchKernelGGL(face_sum_kernel, dim3(12), dim3(1024), 0, c->stream, a);
    HIP_TRY(c->err, hipGetLastError());
    HIP_TRY(c->err, hipMemcpyAsync(host12, c->red(), 12 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c->err, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

}  // namespace

// ======================================================================= ABI

namespace {

// Steps per launch a 2D context starts with: the fastest measured on the
// 8193^2 cell per storage mode (GLUPS at 1/2/3/4 steps, each with its best
// segment length, before the pipeline fill was skipped: FP32 51/69/113/137,
// FP16-f+FP32-g 74/98/146/155, FP16 103/125/152/153, BF16 99/119/136/110,
// FP64 25/38/30/-).
// FP64 streams at most two steps per launch: the rings of deeper launches
// (two registers per value) do not fit the 256 registers, the kernels spill
// heavily and run slower (28 and 18 GLUPS at three and four steps, against
// 39 at two), and at four steps on arrays over 4 GiB the results differed
// from single steps on the columns next to strip edges.
constexpr int kMaxStepsFp64 = 2;
// Five steps per launch only with FP32 populations: with 16-bit ones the
// five-step kernel ran slower than four (FP16 151 / 161 GLUPS, BF16 177 /
// 185, FP16-f+FP32-g 165 / 172 at five / four steps), so it is not built
// for them.
constexpr int kMaxSteps2d = 5;
template <class St> constexpr bool five_steps() {
    return sizeof(typename St::TF) == 4 && sizeof(typename St::TG) == 4 && sizeof(typename St::R) == 4;
}

// Measured on the 8193^2 cell once the 2D collision was written out with
// its shared terms (GLUPS, best segment length each): FP32 at three / four /
// five steps 103 / 149 / 171; FP16 169 / 161 / 151; BF16 169 / 185 / 177;
// FP16-f+FP32-g 172 (four) / 165 (five).
int32_t default_steps_per_launch(int32_t dim, int32_t storage) {
    // 3D: the two-step plane ring beats one step per launch with FP32
    // storage only (with 16-bit storage a one-step launch moves half the
    // bytes and is faster)
    if (dim == 3) return storage == LBM_FP32 ? 2 : 1;
    switch (storage) {
    case LBM_FP32: return 5;
    case LBM_MIXED_F16_G32: return 4;
    case LBM_BF16_SHIFTED: return 4;
    case LBM_FP64: return 2;
    default: return 3;  // FP16 (shifted)
    }
}

// every population array is under 4 GiB: 32-bit byte offsets suffice
bool fits_o32(const lbm_ctx* c) {
    const size_t Np = ((size_t)c->geo.N + kTile - 1) / kTile * kTile;
    const size_t lim = ((size_t)1 << 32) - 65536;  // room for the dropped-lane offsets
    return Np * qf_of(c->p.dim) * elem_f(c->p.storage) < lim && Np * qg_of(c->p.dim) * elem_g(c->p.storage) < lim;
}

// the streaming kernels address the wall-flux area and (for arrays of 4 GiB
// or more) one row of populations with 32-bit byte offsets
bool streamable(const lbm_ctx* c) {
    const size_t lim = ((size_t)1 << 32) - 65536;
    const size_t row = ((size_t)c->geo.nx / kTile + 2) * kTile * qf_of(c->p.dim) * 8;
    return 2 * c->lay.flux_doubles * sizeof(double) < lim && row < lim;
}

// the 3D two-step kernel addresses the wall-flux area and two rows of a
// plane with 32-bit byte offsets
bool streamable3(const lbm_ctx* c) {
    const size_t lim = ((size_t)1 << 32) - 65536;
    // node indices below 2^30 (24-bit tile numbers in the gather), the store
    // window of a wavefront's rows and the flux area under 4 GiB
    return (size_t)c->geo.N <= ((size_t)1 << 30) &&
           ((size_t)c->geo.nx * 2 / kTile + 3) * kTile * qf_of(3) * 8 < lim &&
           2 * c->lay.flux_doubles * sizeof(double) < lim;
}

#ifndef LBM_STREAM_WAVES
#define LBM_STREAM_WAVES 4
#endif
#ifndef LBM_STREAM_AHEAD
#define LBM_STREAM_AHEAD 1  // rows between a row's loads and their first use (two-step kernel)
#endif

// k launches of the register-row kernel of NS steps each (prefetch distance
// D rows), A -> B, advancing t by NS k
// Rows per strip segment (one wavefront each), by storage and steps per
// launch, measured on the 8193^2 cell.  Every segment repeats the rows of
// its dependency cone outside it and runs its last step over the pipeline
// fill, so longer segments waste less arithmetic; launches that move many
// bytes per update still run fastest with short ones (FP32 at three steps:
// 117 / 111 / 107 / 97 GLUPS at 16 / 24 / 32 / 64 rows; FP64 at two: 39 /
// 37 / 36 / 36).  FP32 at four steps: 147 / 147 / 143 / 128 at 16 / 24 /
// 32 / 64; FP16-f+FP32-g at four: 150 / 165 / 171 / 171 at 16 / 32 / 48 /
// 64; FP16 at three: 162 / 168 / 164 / 161 at 16 / 32 / 48 / 64, BF16 at
// three 139 / 147 / 149 / 148.
// With the written-out 2D collision: FP32 at four steps 149 / 145 / 138 /
// 130 at 16 / 24 / 32 / 48 rows, at five 162 / 171 / 166 / 158; FP16 at
// three 169 / 168 at 32 / 48; BF16 at four 185 at 48; FP16-f+FP32-g at
// four 172 / 170 at 48 / 64.
template <class St, int NS> constexpr uint32_t stream_seg_rows() {
    constexpr bool f32 = sizeof(typename St::TF) == 4 && sizeof(typename St::TG) == 4;
    constexpr bool f64 = sizeof(typename St::TF) == 8;
    constexpr bool half = sizeof(typename St::TF) == 2 && sizeof(typename St::TG) == 2;
    if constexpr (f64) return NS == 2 ? 16 : 64;
    else if constexpr (f32) return NS == 5 ? 24 : 16;
    else if constexpr (half) return NS == 2 ? 40 : NS == 3 ? 32 : 48;
    else return NS == 2 ? 16 : NS == 3 ? 40 : 48;  // FP16 f, FP32 g
}

template <class St, int NS, int D> void stream_launches(lbm_ctx* c, int64_t k) {
    constexpr int NWB = LBM_STREAM_WAVES;
    constexpr uint32_t W = strip_cols<NS>();
    StreamArgs<St> a{};
    a.geo = c->geo;
    a.c = make_coef<typename St::R>(c);
    a.strips = (c->geo.nx + W - 1) / W;
    a.seg_rows = stream_seg_rows<St, NS>();
    a.units = a.strips * ((c->geo.ny + a.seg_rows - 1) / a.seg_rows);
    const uint32_t blocks = (a.units + NWB - 1) / NWB;
    a.blocks_per_xcd = (blocks + kXcd - 1) / kXcd;
    const dim3 grid(a.blocks_per_xcd * kXcd), block(64 * NWB);
    const bool o32 = fits_o32(c);
    const size_t Np = ((size_t)c->geo.N + kTile - 1) / kTile * kTile;
    a.f_bytes = o32 ? (uint32_t)(Np * Flow<2>::Q * sizeof(typename St::TF)) : 0u;
    a.g_bytes = o32 ? (uint32_t)(Np * Heat<2>::Q * sizeof(typename St::TG)) : 0u;
    a.flux = c->flux(0, 0);
    a.slot[0] = 0;
    a.slot[1] = (uint32_t)c->lay.flux_doubles;
    a.flux_bytes = (uint32_t)(2 * c->lay.flux_doubles * sizeof(double));
    for (int64_t s = 0; s < k; ++s) {
        const auto A = pops<St>(c, c->cur), B = pops<St>(c, 1 - c->cur);
        a.fsrc = A.f;
        a.gsrc = A.g;
        a.fdst = B.f;
        a.gdst = B.g;
        a.t_parity = (int32_t)(c->t & 1);
        poison_dst(c);
        if (o32) hipLaunchKernelGGL((stream_kernel<St, NWB, true, NS, D>), grid, block, 0, c->stream, a);
        else hipLaunchKernelGGL((stream_kernel<St, NWB, false, NS, D>), grid, block, 0, c->stream, a);
        c->cur = 1 - c->cur;
        c->t += NS;
    }
}

// z segments of the 3D two-step kernel.  Each segment repeats the first
// step on one plane below and one above it, and its block holds a compute
// unit's LDS for the whole segment, so a launch runs in rounds: each XCD
// takes its share of blocks `resident` per compute unit at a time.  The
// count chosen minimises rounds x (planes per segment + 2), the plane
// steps of the slowest compute unit (fewer segments on a tie).
uint32_t stream3_segments(uint32_t nz, uint32_t tiles, int cus, int resident) {
    const uint64_t slots = (uint64_t)std::max(cus / kXcd, 1) * (uint64_t)std::max(resident, 1);
    uint32_t best = 1;
    uint64_t best_cost = UINT64_MAX;
    for (uint32_t segs = 1; segs <= nz; ++segs) {
        const uint64_t planes = (nz + segs - 1) / segs;
        if (segs > 1 && (nz + planes - 1) / planes < segs) continue;  // same split as fewer segments
        const uint64_t per_xcd = ((uint64_t)tiles * segs + kXcd - 1) / kXcd;
        const uint64_t cost = (per_xcd + slots - 1) / slots * (planes + 2);
        if (cost < best_cost) {
            best_cost = cost;
            best = segs;
        }
    }
    return best;
}

// k launches of the 3D two-step kernel, A -> B, advancing t by 2 k
template <class St> void stream3_launches(lbm_ctx* c, int64_t k) {
    Stream3Args<St> a{};
    a.geo = c->geo;
    a.c = make_coef<typename St::R>(c);
    a.tiles_x = (c->geo.nx + kT3OutX - 1) / kT3OutX;
    a.tiles_y = (c->geo.ny + kT3OutY - 1) / kT3OutY;
    static const int resident = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, stream3_kernel<St>, kT3Threads, 0) != hipSuccess) n = 1;
        return std::max(n, 1);
    }();
    const uint32_t segs = stream3_segments(c->geo.nz, a.tiles_x * a.tiles_y, c->cus, resident);
    a.seg_planes = (c->geo.nz + segs - 1) / segs;
    a.segs = (c->geo.nz + a.seg_planes - 1) / a.seg_planes;
    const uint32_t blocks = a.tiles_x * a.tiles_y * a.segs;
    a.blocks_per_xcd = (blocks + kXcd - 1) / kXcd;
    a.flux = c->flux(0, 0);
    a.flux_bytes = (uint32_t)(2 * c->lay.flux_doubles * sizeof(double));
    const dim3 grid(a.blocks_per_xcd * kXcd), block(kT3Threads);
    for (int64_t s = 0; s < k; ++s) {
        const auto A = pops<St>(c, c->cur), B = pops<St>(c, 1 - c->cur);
        a.fsrc = A.f;
        a.gsrc = A.g;
        a.fdst = B.f;
        a.gdst = B.g;
        // step j of the launch writes flux slot (t + j) mod 2
        a.slot1 = (uint32_t)(((c->t + 1) & 1) * c->lay.flux_doubles);
        a.slot2 = (uint32_t)((c->t & 1) * c->lay.flux_doubles);
        poison_dst(c);
        hipLaunchKernelGGL((stream3_kernel<St>), grid, block, 0, c->stream, a);
        c->cur = 1 - c->cur;
        c->t += 2;
    }
}

}  // namespace

extern "C" {

const char* lbm_version(void) { return "paper_2211_03160_amd lbm 1.0 (gfx950)"; }

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err : g_err; }

lbm_status lbm_derive(const lbm_params* p, double* out) {
    Derived d;
    const lbm_status st = derive(p, &d, g_err);
    if (st) return st;
    if (out) memcpy(out, d.v, sizeof(d.v));
    g_err[0] = 0;
    return LBM_OK;
}

size_t lbm_workspace_bytes(const lbm_params* p) {
    Derived d;
    if (derive(p, &d, g_err)) return 0;
    return layout(p).total;
}

double lbm_bytes_per_update(const lbm_params* p) {
    Derived d;
    if (derive(p, &d, g_err)) return 0.0;
    return 2.0 * (qf_of(p->dim) * (double)elem_f(p->storage) + qg_of(p->dim) * (double)elem_g(p->storage));
}

}  // extern "C"

namespace {
lbm_status create_ctx(const lbm_params* p, void* d_workspace, size_t bytes, void* hip_stream, size_t staging_cap,
                      bool view, lbm_ctx** out) {
    if (!out) return set_err(g_err, LBM_E_INVALID, "null output pointer");
    *out = nullptr;
    Derived d;
    lbm_status st = derive(p, &d, g_err);
    if (st) return st;
    const Layout lay = layout(p, staging_cap);
    if (!d_workspace) return set_err(g_err, LBM_E_INVALID, "null workspace");
    if ((uintptr_t)d_workspace % kAlign) return set_err(g_err, LBM_E_INVALID, "workspace not 256-byte aligned");
    if (bytes < lay.total)
        return set_err(g_err, LBM_E_INVALID, "workspace of %zu bytes is smaller than the %zu needed", bytes, lay.total);
    int dev = 0, cus = 0;
    HIP_TRY(g_err, hipGetDevice(&dev));
    if (!is_device_ptr(d_workspace)) return set_err(g_err, LBM_E_INVALID, "workspace is not device memory");
    HIP_TRY(g_err, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return set_err(g_err, LBM_E_INVALID, "out of host memory");
    c->p = *p;
    c->d = d;
    c->lay = lay;
    c->device = dev;
    c->cus = cus;
    c->poison = false;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char*)d_workspace;
    c->cur = 0;
    c->t = -1;
    c->steps_per_launch = view ? 1 : default_steps_per_launch(p->dim, p->storage);
    Geometry& g = c->geo;
    g.nx = p->n[0];
    g.ny = p->n[1];
    g.nz = p->n[2];
    g.N = g.nx * g.ny * g.nz;
    g.divx = make_div(g.nx);
    g.divy = make_div(g.ny);
    if (!div_ok(g.divx, g.N) || !div_ok(g.divy, g.N / g.nx)) {
        delete c;
        return set_err(g_err, LBM_E_UNSUPPORTED, "fast division self-check failed");
    }
    for (int a = 0; a < 3; ++a) g.periodic[a] = a >= p->dim || p->bc[2 * a] == LBM_BC_PERIODIC;
    for (int f = 0; f < 6; ++f) g.dirichlet[f] = f / 2 < p->dim && p->bc[f] == LBM_BC_DIRICHLET;
    const uint32_t blocks = (g.N + kBlock - 1) / kBlock;
    g.blocks_per_xcd = (blocks + kXcd - 1) / kXcd;
    c->cond_axis = -1;
    const int order[3] = {p->dim - 1, 0, 1};
    for (int k = 0; k < 3 && c->cond_axis < 0; ++k) {
        const int a = order[k];
        if (a < p->dim && g.dirichlet[2 * a] && g.dirichlet[2 * a + 1]) c->cond_axis = a;
    }
    c->view = view;
    c->err[0] = 0;
    g_err[0] = 0;
    *out = c;
    return LBM_OK;
}

lbm_status reject_view(lbm_ctx* c, const char* what) {
    return set_err(c->err, LBM_E_STATE, "%s: this cavity belongs to a batch; use the lbm_batch_* calls", what);
}
}  // namespace

extern "C" {

lbm_status lbm_create(const lbm_params* p, void* d_workspace, size_t bytes, void* hip_stream, lbm_ctx** out) {
    return create_ctx(p, d_workspace, bytes, hip_stream, kStagingNodes, false, out);
}

void lbm_destroy(lbm_ctx* c) {
    if (c && !c->view) delete c;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

static lbm_status init_impl(lbm_ctx* c, uint64_t seed, double amp);
static lbm_status init_fields_impl(lbm_ctx* c, const double* rho, const double* u, const double* T);

lbm_status lbm_init(lbm_ctx* c, uint64_t seed, double amp) {
    lbm_status st = enter(c);
    if (st) return st;
    if (c->view) return reject_view(c, "lbm_init");
    return init_impl(c, seed, amp);
}

lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* u, const double* T) {
    lbm_status st = enter(c);
    if (st) return st;
    if (c->view) return reject_view(c, "lbm_init_fields");
    return init_fields_impl(c, rho, u, T);
}

static lbm_status init_impl(lbm_ctx* c, uint64_t seed, double amp) {
    lbm_status st;
    if (!std::isfinite(amp)) return set_err(c->err, LBM_E_INVALID, "amp must be finite");
    c->cur = 0;
    st = launch_init(c, 0, 0, c->geo.N, seed, amp, nullptr, nullptr, nullptr);
    if (st) return st;
    st = zero_flux(c);
    if (!st) st = clear_tails(c);
    if (st) return st;
    c->t = 0;
    return LBM_OK;
}

static lbm_status init_fields_impl(lbm_ctx* c, const double* rho, const double* u, const double* T) {
    lbm_status st;
    if (!u || !T) return set_err(c->err, LBM_E_INVALID, "u and T are required");
    const int dim = c->p.dim;
    const size_t N = c->geo.N, S = c->lay.stage_nodes;
    c->cur = 0;
    double* sr = c->stage();
    double* su = sr + S;
    double* sT = su + (size_t)dim * S;
    for (size_t n0 = 0; n0 < N; n0 += S) {
        const size_t cnt = std::min(S, N - n0);
        if (rho) HIP_TRY(c->err, hipMemcpyAsync(sr, rho + n0, cnt * 8, hipMemcpyHostToDevice, c->stream));
        for (int a = 0; a < dim; ++a)
            HIP_TRY(c->err, hipMemcpyAsync(su + a * cnt, u + a * N + n0, cnt * 8, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(c->err, hipMemcpyAsync(sT, T + n0, cnt * 8, hipMemcpyHostToDevice, c->stream));
        st = launch_init(c, 1, (uint32_t)n0, (uint32_t)cnt, 0, 0.0, rho ? sr : nullptr, su, sT);
        if (st) return st;
        HIP_TRY(c->err, hipStreamSynchronize(c->stream));
    }
    st = zero_flux(c);
    if (!st) st = clear_tails(c);
    if (st) return st;
    HIP_TRY(c->err, hipStreamSynchronize(c->stream));
    c->t = 0;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, int64_t n) {
    lbm_status st = enter(c);
    if (st) return st;
    if (c->view) return reject_view(c, "lbm_step");
    if (n < 0) return set_err(c->err, LBM_E_INVALID, "n must be >= 0");
    if ((st = require_state(c))) return st;
    if (n == 0) return LBM_OK;
    return dispatch(c, [&](auto dimc, auto stc) -> lbm_status {
        constexpr int DIM = decltype(dimc)::value;
        using St = decltype(stc);
        if constexpr (DIM == 2) {
            constexpr bool deep = sizeof(typename St::R) == 4;  // FP64: at most two (kMaxStepsFp64)
            const int32_t spl = streamable(c) ? c->steps_per_launch : 1;
            if constexpr (five_steps<St>()) {
                if (spl == 5 && n >= 5) {
                    stream_launches<St, 5, 0>(c, n / 5);
                    n -= n / 5 * 5;
                }
            }
            if constexpr (deep) {
                if (spl >= 4 && n >= 4) {
                    stream_launches<St, 4, 0>(c, n / 4);
                    n -= n / 4 * 4;
                }
                if (spl >= 3 && n >= 3) {
                    stream_launches<St, 3, 0>(c, n / 3);
                    n -= n / 3 * 3;
                }
            }
            if (spl >= 2 && n >= 2) {
                stream_launches<St, 2, LBM_STREAM_AHEAD>(c, n / 2);
                n -= n / 2 * 2;
            }
        } else if constexpr (sizeof(typename St::R) == 4) {
            // 3D: two steps per launch through the LDS plane ring (FP64's
            // ring would not fit the LDS)
            if (c->steps_per_launch == 2 && n >= 2 && streamable3(c)) {
                stream3_launches<St>(c, n / 2);
                n -= n / 2 * 2;
            }
        }
        StepArgs<St> a{};
        a.geo = c->geo;
        a.c = make_coef<typename St::R>(c);
        const dim3 grid(c->geo.blocks_per_xcd * kXcd), block(kBlock);
        for (int64_t s = 0; s < n; ++s) {
            const auto A = pops<St>(c, c->cur), B = pops<St>(c, 1 - c->cur);
            a.fsrc = A.f;
            a.gsrc = A.g;
            a.fdst = B.f;
            a.gdst = B.g;
            const int slot = (int)((c->t + 1) & 1);
            for (int f = 0; f < 6; ++f) a.flux[f] = c->flux(slot, f);
            poison_dst(c);
            hipLaunchKernelGGL((step_kernel<DIM, St>), grid, block, 0, c->stream, a);
            c->cur = 1 - c->cur;
            c->t += 1;
        }
        HIP_TRY(c->err, hipGetLastError());
        return LBM_OK;
    });
}

lbm_status lbm_set_steps_per_launch(lbm_ctx* c, int32_t steps) {
    lbm_status st = enter(c);
    if (st) return st;
    if (c->view) return reject_view(c, "lbm_set_steps_per_launch");
    if (steps < 1 || steps > kMaxSteps2d)
        return set_err(c->err, LBM_E_INVALID, "steps per launch must lie in 1 .. %d", kMaxSteps2d);
    if (steps > 2 && c->p.dim != 2)
        return set_err(c->err, LBM_E_UNSUPPORTED, "3D runs at most two steps per launch");
    if (steps > 1 && c->p.dim == 3 && c->p.storage == LBM_FP64)
        return set_err(c->err, LBM_E_UNSUPPORTED, "3D FP64 runs one step per launch (its plane ring would not fit the LDS)");
    if (steps > kMaxStepsFp64 && c->p.storage == LBM_FP64)
        return set_err(c->err, LBM_E_UNSUPPORTED, "FP64 runs at most %d steps per launch", kMaxStepsFp64);
    if (steps == 5 && c->p.storage != LBM_FP32)
        return set_err(c->err, LBM_E_UNSUPPORTED, "five steps per launch need FP32 storage");
    c->steps_per_launch = steps;
    return LBM_OK;
}

int32_t lbm_get_steps_per_launch(const lbm_ctx* c) { return c ? c->steps_per_launch : 0; }

lbm_status lbm_set_debug_poison(lbm_ctx* c, int32_t on) {
    lbm_status st = enter(c);
    if (st) return st;
    if (c->view) return reject_view(c, "lbm_set_debug_poison");
    if (on != 0 && on != 1) return set_err(c->err, LBM_E_INVALID, "on must be 0 or 1");
    c->poison = on == 1;
    return LBM_OK;
}

int32_t lbm_get_debug_poison(const lbm_ctx* c) { return c && c->poison ? 1 : 0; }

lbm_status lbm_fields(lbm_ctx* c, double* rho, double* u, double* T) {
    lbm_status st = enter(c);
    if (st) return st;
    if ((st = require_state(c))) return st;
    const int dim = c->p.dim;
    const size_t N = c->geo.N;
    // two counters in the tail of the reduction area, after the diagnostics
    // partials: non-finite populations, nodes faster than c_s
    unsigned long long* bad = (unsigned long long*)(c->red() + (size_t)kDiagBlocks * kDiagVals + 32);
    HIP_TRY(c->err, hipMemsetAsync(bad, 0, 2 * sizeof(*bad), c->stream));
    const bool dev_rho = is_device_ptr(rho), dev_u = is_device_ptr(u), dev_T = is_device_ptr(T);
    const bool all_dev = (!rho || dev_rho) && (!u || dev_u) && (!T || dev_T);
    st = dispatch(c, [&](auto dimc, auto stc) -> lbm_status {
        constexpr int DIM = decltype(dimc)::value;
        using St = decltype(stc);
        const auto A = pops<St>(c, c->cur);
        FieldArgs<St> a{};
        a.fsrc = A.f;
        a.gsrc = A.g;
        a.geo = c->geo;
        a.gbeta = c->d.v[LBM_D_GBETA];
        a.bt = make_coef<typename St::R>(c).bt;
        a.t0 = c->d.v[LBM_D_T0];
        a.nonfinite = bad;
        if (all_dev) {
            a.n0 = 0;
            a.cnt = (uint32_t)N;
            a.rho = rho;
            a.u = u;
            a.T = T;
            hipLaunchKernelGGL((fields_kernel<DIM, St>), dim3(grid_for(N)), dim3(kBlock), 0, c->stream, a);
            HIP_TRY(c->err, hipGetLastError());
            return LBM_OK;
        }
        const size_t S = c->lay.stage_nodes;
        double* sr = c->stage();
        double* su = sr + S;
        double* sT = su + (size_t)dim * S;
        for (size_t n0 = 0; n0 < N; n0 += S) {
            const size_t cnt = std::min(S, N - n0);
            a.n0 = (uint32_t)n0;
            a.cnt = (uint32_t)cnt;
            a.rho = rho ? sr : nullptr;
            a.u = u ? su : nullptr;
            a.T = T ? sT : nullptr;
            hipLaunchKernelGGL((fields_kernel<DIM, St>), dim3(grid_for(cnt)), dim3(kBlock), 0, c->stream, a);
            HIP_TRY(c->err, hipGetLastError());
            const hipMemcpyKind k = hipMemcpyDefault;
            if (rho) HIP_TRY(c->err, hipMemcpyAsync(rho + n0, sr, cnt * 8, k, c->stream));
            if (u)
                for (int d = 0; d < DIM; ++d)
                    HIP_TRY(c->err, hipMemcpyAsync(u + d * N + n0, su + d * cnt, cnt * 8, k, c->stream));
            if (T) HIP_TRY(c->err, hipMemcpyAsync(T + n0, sT, cnt * 8, k, c->stream));
            HIP_TRY(c->err, hipStreamSynchronize(c->stream));
        }
        return LBM_OK;
    });
    if (st) return st;
    unsigned long long nbad[2] = {0, 0};
    HIP_TRY(c->err, hipMemcpyAsync(nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c->err, hipStreamSynchronize(c->stream));
    if (nbad[0])
        return set_err(c->err, LBM_E_UNSTABLE, "%llu non-finite populations at t = %lld", nbad[0], (long long)c->t);
    if (nbad[1])
        return set_err(c->err, LBM_E_UNSTABLE, "%llu nodes faster than the lattice sound speed at t = %lld", nbad[1],
                       (long long)c->t);
    return LBM_OK;
}

lbm_status lbm_wall_flux(lbm_ctx* c, double* last, double* prev) {
    lbm_status st = enter(c);
    if (st) return st;
    if ((st = require_state(c))) return st;
    double s[12];
    if ((st = face_sums(c, s))) return st;
    const int sl = (int)(c->t & 1), sp = 1 - sl;
    for (int f = 0; f < 6; ++f) {
        if (last) last[f] = s[sl * 6 + f];
        if (prev) prev[f] = s[sp * 6 + f];
    }
    return LBM_OK;
}

lbm_status lbm_nusselt(lbm_ctx* c, double* nu_hot, double* nu_cold) {
    lbm_status st = enter(c);
    if (st) return st;
    if ((st = require_state(c))) return st;
    if (c->t < 2) return set_err(c->err, LBM_E_STATE, "lbm_nusselt needs at least two steps (t = %lld)", (long long)c->t);
    double num[2] = {0, 0}, area[2] = {0, 0};
    const double T0 = c->d.v[LBM_D_T0];
    for (int f = 0; f < 6; ++f) {
        if (!c->geo.dirichlet[f] || c->p.t_wall[f] == T0) continue;
        const int k = c->p.t_wall[f] > T0 ? 0 : 1;
        area[k] += (double)c->lay.area[f];
    }
    if (area[0] == 0.0 || area[1] == 0.0)
        return set_err(c->err, LBM_E_STATE, "lbm_nusselt needs a hot and a cold Dirichlet face");
    double s[12];
    if ((st = face_sums(c, s))) return st;
    for (int f = 0; f < 6; ++f) {
        if (!c->geo.dirichlet[f] || c->p.t_wall[f] == T0) continue;
        const int k = c->p.t_wall[f] > T0 ? 0 : 1;
        const double q = 0.5 * (s[f] + s[6 + f]);  // mean of the two slots
        num[k] += (k == 0 ? 1.0 : -1.0) * c->p.n[f / 2] * q;
    }
    const double scale = 1.0 / (c->d.v[LBM_D_ALPHA] * (c->p.t_hot - c->p.t_cold));
    const double nh = num[0] * scale / area[0], nc = num[1] * scale / area[1];
    if (nu_hot) *nu_hot = nh;
    if (nu_cold) *nu_cold = nc;
    if (!std::isfinite(nh) || !std::isfinite(nc))
        return set_err(c->err, LBM_E_UNSTABLE, "non-finite wall heat flux at t = %lld", (long long)c->t);
    return LBM_OK;
}

static lbm_status run_diag(lbm_ctx* c, double* host6) {
    return dispatch(c, [&](auto dimc, auto stc) -> lbm_status {
        constexpr int DIM = decltype(dimc)::value;
        using St = decltype(stc);
        const auto A = pops<St>(c, c->cur);
        DiagArgs<St> a{};
        a.fsrc = A.f;
        a.gsrc = A.g;
        a.geo = c->geo;
        a.gbeta = c->d.v[LBM_D_GBETA];
        a.bt = make_coef<typename St::R>(c).bt;
        a.t0 = c->d.v[LBM_D_T0];
        a.partial = c->red();
        const int nblk = (int)std::min<size_t>(kDiagBlocks, grid_for(c->geo.N));
        double* out = c->red() + (size_t)kDiagBlocks * kDiagVals;
        hipLaunchKernelGGL((diag_kernel<DIM, St>), dim3(nblk), dim3(kBlock), 0, c->stream, a);
        HIP_TRY(c->err, hipGetLastError());
        hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(1024), 0, c->stream, (const double*)c->red(), nblk, out);
        HIP_TRY(c->err, hipGetLastError());
        HIP_TRY(c->err, hipMemcpyAsync(host6, out, kDiagVals * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c->err, hipStreamSynchronize(c->stream));
        return LBM_OK;
    });
}

lbm_status lbm_diagnostics(lbm_ctx* c, lbm_diag* d) {
    lbm_status st = enter(c);
    if (st) return st;
    if (!d) return set_err(c->err, LBM_E_INVALID, "null output");
    if ((st = require_state(c))) return st;
    double v[kDiagVals];
    if ((st = run_diag(c, v))) return st;
    const double N = (double)c->geo.N, H = c->d.v[LBM_D_H];
    const double alpha = c->d.v[LBM_D_ALPHA], nu = c->d.v[LBM_D_NU];
    const double dT = c->p.t_hot - c->p.t_cold;
    d->t = c->t;
    d->mass = v[0];
    d->energy = v[1];
    d->umax = v[4];
    d->nu_vol = 1.0 + H * (v[3] / N) / (alpha * dT);
    d->re = std::sqrt(v[2] / N) * H / nu;
    d->nonfinite = (int64_t)v[5];
    if (d->nonfinite) return set_err(c->err, LBM_E_UNSTABLE, "%lld non-finite populations", (long long)d->nonfinite);
    if (d->umax > 1.0 / std::sqrt(3.0))
        return set_err(c->err, LBM_E_UNSTABLE, "max |u| = %g exceeds the lattice sound speed", d->umax);
    return LBM_OK;
}

}  // extern "C"

// ------------------------------------------------ diagnostics, no allocation
// Scratch of lbm_diagnostics_async: the per-block partial sums of the
// diagnostics reduction and the reduced sums after them.  Each device the
// library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns on that
// device (the array's name is a host-side stand-in).
constexpr int kNoAllocScratchDoubles = (kDiagBlocks + 1) * kDiagVals;  // 48 KiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device, looked up once per
// device
lbm_status scratch_of_device(char* err, int dev, double** out) {
    if (dev < 0 || dev >= kMaxDevices)
        return set_err(err, LBM_E_UNSUPPORTED, "device %d: the no-allocation scratch covers devices 0 .. %d", dev,
                       kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(err, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_err(err, LBM_E_DEVICE, "hipGetSymbolAddress returned no address for the scratch");
        g_scratch_ptr[dev] = (double*)p;
    }
    *out = g_scratch_ptr[dev];
    return LBM_OK;
}
}  // namespace

extern "C" {

lbm_status lbm_diagnostics_async(lbm_ctx* c, double* d_out) {
    lbm_status st = enter(c);
    if (st) return st;
    if (!d_out || !is_device_ptr(d_out)) return set_err(c->err, LBM_E_INVALID, "d_out must be device memory");
    if ((st = require_state(c))) return st;
    double* ws = nullptr;
    if ((st = scratch_of_device(c->err, c->device, &ws))) return st;
    const int nblk = (int)std::min<size_t>(kDiagBlocks, grid_for(c->geo.N));
    if ((size_t)(nblk + 1) * kDiagVals > (size_t)kNoAllocScratchDoubles)
        return set_err(c->err, LBM_E_INVALID, "%d reduction blocks exceed the %d-double scratch", nblk,
                       kNoAllocScratchDoubles);
    double* sums = ws + (size_t)nblk * kDiagVals;
    st = dispatch(c, [&](auto dimc, auto stc) -> lbm_status {
        constexpr int DIM = decltype(dimc)::value;
        using St = decltype(stc);
        const auto A = pops<St>(c, c->cur);
        DiagArgs<St> a{};
        a.fsrc = A.f;
        a.gsrc = A.g;
        a.geo = c->geo;
        a.gbeta = c->d.v[LBM_D_GBETA];
        a.bt = make_coef<typename St::R>(c).bt;
        a.t0 = c->d.v[LBM_D_T0];
        a.partial = ws;
        hipLaunchKernelGGL((diag_kernel<DIM, St>), dim3(nblk), dim3(kBlock), 0, c->stream, a);
        HIP_TRY(c->err, hipGetLastError());
        return LBM_OK;
    });
    if (st) return st;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(1024), 0, c->stream, (const double*)ws, nblk, sums);
    HIP_TRY(c->err, hipGetLastError());
    const DiagScale sc{(double)c->t, (double)c->geo.N, c->d.v[LBM_D_H], c->d.v[LBM_D_ALPHA], c->d.v[LBM_D_NU],
                       c->p.t_hot - c->p.t_cold};
    hipLaunchKernelGGL(diag_values_kernel, dim3(1), dim3(64), 0, c->stream, (const double*)sums, sc, d_out);
    HIP_TRY(c->err, hipGetLastError());
    return LBM_OK;
}

// checkpoint: header, populations of the current buffer, both flux slots
struct StateHeader {
    uint64_t magic;
    int64_t t;
    int32_t dim, storage, n[3], pad;
    uint64_t pop_bytes, flux_bytes;
};
static const uint64_t kStateMagic = 0x31304d424c544d4full;

size_t lbm_state_bytes(const lbm_ctx* c) {
    if (!c) return 0;
    return sizeof(StateHeader) + c->lay.pop_bytes + 2 * c->lay.flux_doubles * sizeof(double);
}

lbm_status lbm_export_state(lbm_ctx* c, void* host, size_t bytes) {
    lbm_status st = enter(c);
    if (st) return st;
    if ((st = require_state(c))) return st;
    if (!host || bytes < lbm_state_bytes(c)) return set_err(c->err, LBM_E_INVALID, "buffer too small");
    StateHeader h{kStateMagic, c->t, c->p.dim, c->p.storage, {c->p.n[0], c->p.n[1], c->p.n[2]}, 0,
                  c->lay.pop_bytes, 2 * c->lay.flux_doubles * sizeof(double)};
    char* out = (char*)host;
    memcpy(out, &h, sizeof(h));
    HIP_TRY(c->err, hipMemcpyAsync(out + sizeof(h), c->pop(c->cur), h.pop_bytes, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c->err, hipMemcpyAsync(out + sizeof(h) + h.pop_bytes, c->ws + c->lay.off_flux, h.flux_bytes,
                                   hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c->err, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_import_state(lbm_ctx* c, const void* host, size_t bytes) {
    lbm_status st = enter(c);
    if (st) return st;
    if (c->view) return reject_view(c, "lbm_import_state");
    if (!host || bytes < sizeof(StateHeader)) return set_err(c->err, LBM_E_INVALID, "buffer too small");
    StateHeader h;
    memcpy(&h, host, sizeof(h));
    if (h.magic != kStateMagic || h.dim != c->p.dim || h.storage != c->p.storage || h.n[0] != c->p.n[0] ||
        h.n[1] != c->p.n[1] || h.n[2] != c->p.n[2] || h.pop_bytes != c->lay.pop_bytes ||
        h.flux_bytes != 2 * c->lay.flux_doubles * sizeof(double) || bytes < lbm_state_bytes(c) || h.t < 0)
        return set_err(c->err, LBM_E_INVALID, "state buffer does not match this context");
    const char* in = (const char*)host;
    c->cur = 0;
    HIP_TRY(c->err, hipMemcpyAsync(c->pop(0), in + sizeof(h), h.pop_bytes, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c->err, hipMemcpyAsync(c->ws + c->lay.off_flux, in + sizeof(h) + h.pop_bytes, h.flux_bytes,
                                   hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c->err, hipStreamSynchronize(c->stream));
    c->t = h.t;
    return LBM_OK;
}

lbm_status lbm_lattice(int32_t dim, int32_t which, int32_t* q, int32_t* e, int32_t* M, double* w) {
    if ((dim != 2 && dim != 3) || (which != 0 && which != 1))
        return set_err(g_err, LBM_E_INVALID, "dim must be 2 or 3 and which 0 or 1");
    auto emit = [&](auto L, bool flow, double at) {
        using T = decltype(L);
        if (q) *q = T::Q;
        for (int i = 0; i < T::Q; ++i) {
            if (e) {
                e[3 * i] = T::ex[i];
                e[3 * i + 1] = T::ey[i];
                e[3 * i + 2] = T::ez[i];
            }
            if (M)
                for (int k = 0; k < T::Q; ++k) M[k * T::Q + i] = T::M(k, i);
        }
        if (w) {
            if constexpr (std::is_same_v<T, Flow<2>> || std::is_same_v<T, Flow<3>>) {
                for (int i = 0; i < T::Q; ++i) w[i] = T::w[i];
            } else {
                for (int i = 0; i < T::Q; ++i) w[i] = i == 0 ? T::w_rest(at) : T::w_move(at);
            }
        }
        (void)flow;
    };
    if (dim == 2 && which == 0) emit(Flow<2>{}, true, 0.0);
    else if (dim == 2) emit(Heat<2>{}, false, Heat<2>::a_t_default);
    else if (which == 0) emit(Flow<3>{}, true, 0.0);
    else emit(Heat<3>{}, false, Heat<3>::a_t_default);
    return LBM_OK;
}

}  // extern "C"

#include "batch.inc"
