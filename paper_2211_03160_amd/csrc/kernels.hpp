// kernels.hpp -- gfx950 kernels of the fused DDF thermal LBM step.
//
// One launch of step_kernel advances every node by one time step of the
// model of Section 2.2 (Eqs. 5-7) in the collide/stream split of Section
// 3.1 (Eqs. 8a-9b), fused into a single pass:
//   pull: f_i(x) = f+_i(x - e_i) and g_i(x) = g+_i(x - e_i) from buffer A,
//         with half-way bounce-back / anti-bounce-back where x - e_i lies
//         beyond a wall (Section 2.2) and wrap-around on periodic faces;
//   moments: rho, T, buoyancy F = rho g beta (T - T0) e_up, u = (j + F/2)/rho;
//   collide f in moment space with Guo forcing (Eqs. 5, 6a/6b, 8a);
//   collide g in moment space (Eqs. 7, 9a);
//   store f+, g+ at x into buffer B.
// A and B hold POST-collision populations in a tiled structure-of-arrays
// order: nodes keep the flat index x + nx (y + ny z) of Section 3.1, and
// each tile of kTile consecutive nodes (one wavefront) stores its Q
// velocity planes back to back, [tile][i][lane].  A wavefront then reads
// and writes a few contiguous runs of Q x 64 values instead of Q separate
// streams N apart, which the HBM controllers serve at a higher rate.
//
// Every storage mode keeps deviations from a reference state and all
// arithmetic runs on them, so the order-one reference populations never
// swamp the small parts that carry the flow and the heat flux: h_i = f_i -
// w_i (flow, the rest state) and h^g_i = g_i - G_i(x) (thermal), where G is
// the exact discrete conduction state between the two Dirichlet faces of
// one axis -- the linear profile T_b(x) = T_lo + (k + 1/2) (T_hi - T_lo)/n
// at coordinate k along that axis, with the odd part that carries its
// constant heat flux (a fixed point of the step, Section 2.2's wall rules
// included) -- or the uniform T0 where no such axis exists.  Stored as f
// itself, an FP32 population near w rounds away any deviation below half an
// ulp of w (~1.5e-8) every step; stored relative to T0 alone, a 16-bit g
// loses the wall heat flux, whose share of the populations (~alpha dT / H)
// lies below its quantum.  Relative to G the conduction state is exactly
// zero and the wall links need no constant of their own.
// With orthogonal bases the collision is applied as an increment:
//   h+_i = h_i + sum_k M_ki dm_k / |M_k|^2.
//
// In 2D, stream_kernel advances two to five steps per launch: each
// wavefront walks down a strip of columns keeping the last rows of the
// input and of the intermediate steps in registers, so the intermediate
// states never go to memory; every node update is the same step_node
// arithmetic on the same (storage-rounded) values, so the result is
// bitwise that of single steps.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "lattice.hpp"

namespace lbm {

constexpr int kBlock = 256;  // threads per block of the node-parallel kernels
constexpr int kXcd = 8;      // accelerator complex dies of an MI355X
constexpr int kTile = 64;    // nodes per storage tile (one wavefront)

// element offset of population i of node `node` in a tiled array of Q planes
template <int Q> __host__ __device__ __forceinline__ uint32_t pop_at(uint32_t node, int i) {
    return (node / kTile) * (uint32_t)(Q * kTile) + (uint32_t)(i * kTile) + node % kTile;
}
// the same for node < 2^30, where the tile number fits the 24-bit multiply
// (a full-rate instruction; the 32-bit one issues at a quarter of the rate)
template <int Q> __device__ __forceinline__ uint32_t pop_at24(uint32_t node, int i) {
    return __umul24(node / kTile, (uint32_t)(Q * kTile)) + (uint32_t)(i * kTile) + node % kTile;
}

// ------------------------------------------------------------------ storage
// Element codecs: stored type T, dec() to the compute type, enc() from it.
// The 16-bit codecs round to nearest even.
struct E32 {
    using T = float;
    __device__ static float dec(T v) { return v; }
    __device__ static T enc(float v) { return v; }
};
struct E64 {
    using T = double;
    __device__ static double dec(T v) { return v; }
    __device__ static T enc(double v) { return v; }
};
// FP16 holds the deviations scaled by 2^14 (exact: a power of two), which
// keeps deviations down to ~4e-9 in its normal range (unscaled, those below
// 6.1e-5 would be subnormal, with an absolute quantum of 6e-8) while the
// largest ones (|h| < 1) stay far below its maximum of 65504.
constexpr float kF16Scale = 16384.0f;
struct E16 {
    using T = _Float16;
    // a fused multiply-add with -0 is the product itself, and lets the
    // conversion fold into it (v_fma_mix_f32)
    __device__ static float dec(T v) { return __builtin_fmaf((float)v, 1.0f / kF16Scale, -0.0f); }
    __device__ static T enc(float v) { return (T)(v * kF16Scale); }
};
struct EB16 {  // bfloat16 kept as raw bits
    using T = uint16_t;
    __device__ static float dec(T v) { return __uint_as_float((uint32_t)v << 16); }
    // the hardware conversion (v_cvt_pk_bf16_f32): nearest even under the
    // default rounding mode, FP32 denormals kept, NaN to a quiet NaN
    __device__ static T enc(float v) { return __builtin_bit_cast(T, (__bf16)v); }
};

// A storage mode: codecs of f and g and the compute type R.
template <class CF, class CG, class Real> struct Storage {
    using EF = CF;
    using EG = CG;
    using TF = typename CF::T;
    using TG = typename CG::T;
    using R = Real;
};
using StF32 = Storage<E32, E32, float>;
using StF64 = Storage<E64, E64, double>;
using StF16 = Storage<E16, E16, float>;
using StBF16 = Storage<EB16, EB16, float>;
using StMix = Storage<E16, E32, float>;

// --------------------------------------------------------------- parameters
// x / d for x < 2^31 by multiply-high (round-up method of Granlund and
// Montgomery, 1994): q = (umulhi(x, m) + x) >> l, l = ceil(log2 d).
struct FastDiv {
    uint32_t d, m, l;
    __host__ __device__ __forceinline__ uint32_t div(uint32_t x) const {
#if defined(__HIP_DEVICE_COMPILE__)
        return (__umulhi(x, m) + x) >> l;
#else
        return (uint32_t)((((uint64_t)x * m) >> 32) + x) >> l;
#endif
    }
};

struct Geometry {
    uint32_t N, nx, ny, nz;
    FastDiv divx, divy;
    int32_t periodic[3];
    int32_t dirichlet[6];
    uint32_t blocks_per_xcd;  // logical blocks handled by each XCD
};

// Relaxation rates are indexed by row kind (RowKind), not by row: rows of
// one kind share a rate, so a kernel holds only the distinct values.  In 2D
// every kind's rows also share |M_k|^2, and s, b and q come divided by it,
// which saves the scaling of each relaxed moment before the inverse
// transform.  In 3D two kinds have rows of different norms, and the
// collision takes per-row factors instead (k3, below).
// Temperature of the thermal reference state at a node: T_b = tb0 + tbg k
// with k the node's coordinate along `axis` (tbg = 0 where the reference is
// the uniform T0).
template <class R> struct BaseTemp {
    R tb0, tbg;
    int32_t axis;
};
template <class R>
__host__ __device__ __forceinline__ R base_temp(const BaseTemp<R>& b, uint32_t x, uint32_t y, uint32_t z) {
    const uint32_t k = b.axis == 0 ? x : b.axis == 1 ? y : z;
    return b.tb0 + b.tbg * (R)k;
}

// entries of Coef::k3: S* multiply a row's non-equilibrium part, B* its
// forcing term; flow rows e, eps, q, 3p_xx, 3pi_xx, p_ww, pi_ww, the three
// off-diagonal stresses (O), the third-order rows m; heat rows j, e, 3p_xx,
// p_ww
enum K3 : int {
    k3SE, k3BE, k3SEps, k3BEps, k3SQ, k3BQ, k3SP, k3BP, k3SPi, k3BPi,
    k3SW, k3BW, k3SWi, k3BWi, k3SO, k3BO, k3SM, k3QJ, k3QE, k3QP, k3QW, kK3Count
};

template <class R> struct Coef {
    R s[10];     // flow rate per row kind (0 on conserved kinds)
    R b[10];     // 1 - s/2 per row kind
    R q[10];     // thermal rate per row kind
    R a_t;       // thermal equilibrium constant a_T
    R gbeta;     // g beta
    R t0;        // T0 of the buoyancy force
    BaseTemp<R> bt;  // temperature of the thermal reference state
    // anti-bounce-back on a Dirichlet face: h_i = abb - h_opp with
    // abb = abb_a - abb_b T_b, i.e. omega (T_w - T_b) off the reference
    // axis and 0 on its faces (the reference state meets the rule exactly)
    R abb_a[6], abb_b[6];
    // heat entering through one link of a face of the reference axis in the
    // reference state, FP64 (0 on the other faces)
    double flux_c[6];
    // 3D only: each row's relaxation factor and forcing factor divided by
    // |M_k|^2, with the integer factor its relaxed term carries in
    // collide_store_d3 folded in (indices K3)
    R k3[kK3Count];
};

static_assert(kinds_share_norm<Flow<2>>() && kinds_share_norm<Heat<2>>() && !kinds_share_norm<Flow<3>>(),
              "2D rates carry 1/|M_k|^2, 3D ones do not");

template <class St> struct StepArgs {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    typename St::TF* fdst;
    typename St::TG* gdst;
    double* flux[6];  // per-node wall heat flux of this step, per face
    Geometry geo;
    Coef<typename St::R> c;
};

// logical block id: blocks are dealt to the XCDs round-robin, so give each
// XCD a contiguous run of the domain (its L2 then holds the lines shared
// between neighbouring blocks)
__device__ __forceinline__ uint32_t logical_block(uint32_t per_xcd) {
    const uint32_t b = blockIdx.x;
    return (b % kXcd) * per_xcd + b / kXcd;
}

__device__ __forceinline__ void coords(const Geometry& g, uint32_t idx, uint32_t& x,
                                       uint32_t& y, uint32_t& z) {
    const uint32_t r = g.divx.div(idx);
    x = idx - r * g.nx;
    z = g.divy.div(r);
    y = r - z * g.ny;
}

// -------------------------------------------------------------- arithmetic
// compile-time loop: f(std::integral_constant<int, B>), ..., up to E - 1
template <int B, int E, class F> __device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Element i of array p.  With O32 the byte offset is formed in 32 bits
// (valid for arrays under 4 GiB), which lets the load or store take the
// array base from scalar registers and the offset from one vector register.
template <bool O32, class T> __device__ __forceinline__ T* elem(T* p, uint32_t i) {
    if constexpr (O32) return (T*)((char*)p + i * (uint32_t)sizeof(T));
    else return p + i;
}
template <bool O32, class T> __device__ __forceinline__ const T* elem(const T* p, uint32_t i) {
    if constexpr (O32) return (const T*)((const char*)p + i * (uint32_t)sizeof(T));
    else return p + i;
}

// Destinations of the post-collision populations of one node: the tiled
// arrays in global memory.
// NT: non-temporal stores (a one-pass kernel whose waves end after their
// stores); plain stores for kernels that keep loading after storing.
template <class St, int QF, int QG, bool O32 = false, bool NT = true> struct GlobalDst {
    typename St::TF* f;
    typename St::TG* g;
    uint32_t base_f, base_g;
    __device__ GlobalDst(typename St::TF* f_, typename St::TG* g_, uint32_t idx)
        : f(f_), g(g_), base_f(pop_at<QF>(idx, 0)), base_g(pop_at<QG>(idx, 0)) {}
    __device__ void sf(int i, typename St::TF v) const {
        if constexpr (NT) __builtin_nontemporal_store(v, elem<O32>(f, base_f + i * kTile));
        else *elem<O32>(f, base_f + i * kTile) = v;
    }
    __device__ void sg(int i, typename St::TG v) const {
        if constexpr (NT) __builtin_nontemporal_store(v, elem<O32>(g, base_g + i * kTile));
        else *elem<O32>(g, base_g + i * kTile) = v;
    }
};


// i heads a pair of opposite velocities (i < opp i)
template <class L> constexpr bool pair_head(int i) { return i != 0 && i < L::opp[i]; }

// +1: row k is even under e -> -e (M_k,opp i = M_k,i); -1: odd
// (M_k,opp i = -M_k,i, M_k,0 = 0).  Every row of these bases is one or the
// other.
template <class L> constexpr int row_parity(int k) {
    bool even = true, odd = L::M(k, 0) == 0;
    for (int i = 1; i < L::Q; ++i) {
        if (L::M(k, i) != L::M(k, L::opp[i])) even = false;
        if (L::M(k, i) != -L::M(k, L::opp[i])) odd = false;
    }
    return even ? 1 : odd ? -1 : 0;
}
template <class L> constexpr bool rows_have_parity() {
    for (int k = 0; k < L::Q; ++k)
        if (row_parity<L>(k) == 0) return false;
    return true;
}
static_assert(rows_have_parity<Flow<2>>() && rows_have_parity<Flow<3>>() && rows_have_parity<Heat<2>>() &&
                  rows_have_parity<Heat<3>>(),
              "every moment row must be even or odd");

// 1/x: the hardware reciprocal in FP32 (1 ulp), exact division in FP64
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }

// a * b + c, rounded once
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The 2D collision (D2Q9 flow, D2Q5 heat) written out: the moments of the
// basis in lattice.hpp, their second-order equilibria (m_eq(rho, u) -
// m_eq(1, 0) in deviation form), the Guo forcing moments of Eq. (6a) and
// the inverse transform, with the terms that several rows share formed
// once.  Velocities: 1 +x, 2 +y, 3 -x, 4 -y, 5 (+x,+y), 6 (-x,+y), 7
// (-x,-y), 8 (+x,-y); flow rows rho, e, eps, jx, qx, jy, qy, pxx, pxy;
// heat rows T, jx, jy, e, pxx.  Rates come divided by their rows' |M_k|^2.
// Buoyancy acts along y only, so every F_x term is dropped.
template <class St, class Dst>
__device__ __forceinline__ bool collide_store_d2(typename St::R* h, typename St::R* g,
                                                 const Coef<typename St::R>& c, typename St::R tb,
                                                 const Dst& dst) {
    using R = typename St::R;
    // flow moments from the sums S and differences D of opposite pairs
    const R S1 = h[1] + h[3], D1 = h[1] - h[3];
    const R S2 = h[2] + h[4], D2 = h[2] - h[4];
    const R S5 = h[5] + h[7], D5 = h[5] - h[7];
    const R S6 = h[6] + h[8], D6 = h[6] - h[8];
    const R A = S1 + S2, B = S5 + S6;       // axis and diagonal sums
    const R drho = (h[0] + A) + B;
    const R m_e = fmar(R(-4), h[0], fmar(R(2), B, -A));    // -4 h0 - A + 2 B
    const R m_eps = fmar(R(4), h[0], fmar(R(-2), A, B));   // 4 h0 - 2 A + B
    const R m_pxx = S1 - S2, m_pxy = S5 - S6;
    const R P = D5 - D6, Qd = D5 + D6;      // diagonal x and y momenta
    const R jx = D1 + P, jy = D2 + Qd;
    const R m_qx = fmar(R(-2), D1, P), m_qy = fmar(R(-2), D2, Qd);
    // heat moments
    const R Sg1 = g[1] + g[3], Dg1 = g[1] - g[3];
    const R Sg2 = g[2] + g[4], Dg2 = g[2] - g[4];
    const R Cg = Sg1 + Sg2;
    const R dT = g[0] + Cg;
    const R n_e = fmar(R(-4), g[0], Cg);
    const R n_pxx = Sg1 - Sg2;
    // macroscopic fields and the buoyancy force F = (0, Fy)
    const R rho = R(1) + drho;
    const R T = tb + dT;
    const R Fy = rho * c.gbeta * (dT + (tb - c.t0));
    const R inv_rho = recip(rho);
    const R ux = jx * inv_rho;
    const R uy = fmar(R(0.5), Fy, jy) * inv_rho;
    const R ux2 = ux * ux, uy2 = uy * uy;
    const R ruu = rho * (ux2 + uy2);
    const R uF = uy * Fy;
    // relaxed increments dm_k (already divided by |M_k|^2): -s (m - m_eq)
    // + b (M F~)_k, with (M F~) = (6 uF, -6 uF, -Fx, -Fy, 2 (u Fx - v Fy),
    // u Fy + v Fx) on rows e, eps, qx, qy, pxx, pxy, and F / |M_j|^2 on the
    // momentum rows (they gain exactly F)
    const R dm_e = fmar(R(6) * c.b[kE], uF, -c.s[kE] * fmar(R(-3), ruu, fmar(R(2), drho, m_e)));
    const R dm_eps = fmar(R(-6) * c.b[kEps], uF, -c.s[kEps] * fmar(R(3), ruu, m_eps - drho));
    const R dm_qx = -c.s[kQ] * fmar(rho, ux, m_qx);
    const R dm_qy = fmar(-c.b[kQ], Fy, -c.s[kQ] * fmar(rho, uy, m_qy));
    const R dm_pxx = fmar(R(-2) * c.b[kNu], uF, -c.s[kNu] * fmar(-rho, ux2 - uy2, m_pxx));
    const R dm_pxy = fmar(c.b[kNu], ux * Fy, -c.s[kNu] * fmar(-rho, ux * uy, m_pxy));
    const R dm_jy = Fy * R(1.0 / 6.0);
    // inverse transform: h_i += sum_k M_ki dm_k, as even (e) and odd (o)
    // parts of each opposite pair
    h[0] = fmar(R(4), dm_eps - dm_e, h[0]);
    {
        const R a = fmar(R(-2), dm_eps, -dm_e);  // shared by the axis pairs
        const R e1 = a + dm_pxx, e2 = a - dm_pxx;
        const R o2 = fmar(R(-2), dm_qy, dm_jy);
        const R b = fmar(R(2), dm_e, dm_eps);    // shared by the diagonal pairs
        const R e5 = b + dm_pxy, e6 = b - dm_pxy;
        const R q = dm_jy + dm_qy;
        const R o5 = q + dm_qx, o6 = q - dm_qx;
        h[1] = fmar(R(-2), dm_qx, h[1] + e1);
        h[3] = fmar(R(2), dm_qx, h[3] + e1);
        h[2] = (h[2] + e2) + o2;
        h[4] = (h[4] + e2) - o2;
        h[5] = (h[5] + e5) + o5;
        h[7] = (h[7] + e5) - o5;
        h[6] = (h[6] + e6) + o6;
        h[8] = (h[8] + e6) - o6;
    }
    // heat: n_eq = (T, u T, v T, a_T dT, 0) in deviation form
    const R dn_x = -c.q[kJx] * fmar(-ux, T, Dg1);
    const R dn_y = -c.q[kJy] * fmar(-uy, T, Dg2);
    const R dn_e = -c.q[kE] * fmar(-c.a_t, dT, n_e);
    const R dn_p = -c.q[kNu] * n_pxx;
    g[0] = fmar(R(-4), dn_e, g[0]);
    {
        const R e1 = dn_e + dn_p, e2 = dn_e - dn_p;
        g[1] = (g[1] + e1) + dn_x;
        g[3] = (g[3] + e1) - dn_x;
        g[2] = (g[2] + e2) + dn_y;
        g[4] = (g[4] + e2) - dn_y;
    }
    static_for<0, 9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.sf(i, St::EF::enc(h[i]));
    });
    static_for<0, 5>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.sg(i, St::EG::enc(g[i]));
    });
    return isfinite(drho + dT) && ux2 + uy2 <= R(1.0 / 3.0);
}

// The 3D collision (D3Q19 flow, D3Q7 heat) written out: the moments of
// the basis in lattice.hpp (rows rho, e, eps, jx, qx, jy, qy, jz, qz,
// 3p_xx, 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z; heat rows
// T, jx, jy, jz, e, 3p_xx, p_ww), their equilibria and Guo forcing moments
// (Eq. 6b) with buoyancy along z only, and the inverse transform, with the
// terms that several rows share formed once.  Velocities: 1/2 +-x, 3/4
// +-y, 5/6 +-z, then the edge pairs 7/8 (1,1,0), 9/10 (1,-1,0), 11/12
// (1,0,1), 13/14 (1,0,-1), 15/16 (0,1,1), 17/18 (0,1,-1).  Each relaxed
// increment dm_k = d_k / |M_k|^2 uses the factors of Coef::k3, and the
// equilibrium parts use rho u = J = j + F/2: rho u_a u_b = J_a u_b.
template <class St, class Dst>
__device__ __forceinline__ bool collide_store_d3(typename St::R* h, typename St::R* g,
                                                 const Coef<typename St::R>& c, typename St::R tb,
                                                 const Dst& dst) {
    using R = typename St::R;
    const R* k = c.k3;
    // flow moments from the sums S and differences D of opposite pairs
    const R Sx = h[1] + h[2], Dx = h[1] - h[2];
    const R Sy = h[3] + h[4], Dy = h[3] - h[4];
    const R Sz = h[5] + h[6], Dz = h[5] - h[6];
    const R S7 = h[7] + h[8], D7 = h[7] - h[8];
    const R S9 = h[9] + h[10], D9 = h[9] - h[10];
    const R S11 = h[11] + h[12], D11 = h[11] - h[12];
    const R S13 = h[13] + h[14], D13 = h[13] - h[14];
    const R S15 = h[15] + h[16], D15 = h[15] - h[16];
    const R S17 = h[17] + h[18], D17 = h[17] - h[18];
    const R Syz = Sy + Sz, A = Sx + Syz;                   // axis sum
    const R Exy = S7 + S9, Exz = S11 + S13, Eyz = S15 + S17;  // edge sums per plane
    const R Exyz = Exy + Exz, B = Exyz + Eyz;              // edge sum
    const R drho = (h[0] + A) + B;
    // 3p_xx, 3pi_xx = (Pa + Pe, -2 Pa + Pe); p_ww, pi_ww = (Wa + We, -2 Wa + We)
    const R Pa = fmar(R(2), Sx, -Syz), Pe = fmar(R(-2), Eyz, Exyz);
    const R Wa = Sy - Sz, We = Exy - Exz;
    const R m_p = Pa + Pe, m_pi = fmar(R(-2), Pa, Pe);
    const R m_w = Wa + We, m_wi = fmar(R(-2), Wa, We);
    const R m_xy = S7 - S9, m_xz = S11 - S13, m_yz = S15 - S17;
    // odd rows: j_a = D_a + E_a and q_a = -4 D_a + E_a per axis, E_a the
    // edge part; m from the same pair combinations
    const R a7 = D7 + D9, b7 = D7 - D9, a11 = D11 + D13, b11 = D11 - D13, a15 = D15 + D17, b15 = D15 - D17;
    const R Ex = a7 + a11, Ey = b7 + a15, Ez = b11 + b15;
    const R jx = Dx + Ex, jy = Dy + Ey, jz = Dz + Ez;
    const R m_x = a7 - a11, m_y = a15 - b7, m_z = b11 - b15;
    // heat moments
    const R Sgx = g[1] + g[2], Dgx = g[1] - g[2];
    const R Sgy = g[3] + g[4], Dgy = g[3] - g[4];
    const R Sgz = g[5] + g[6], Dgz = g[5] - g[6];
    const R Sgyz = Sgy + Sgz, Cg = Sgx + Sgyz;
    const R dT = g[0] + Cg;
    const R n_e = fmar(R(-6), g[0], Cg);
    const R n_p = fmar(R(2), Sgx, -Sgyz), n_w = Sgy - Sgz;
    // macroscopic fields, the buoyancy force F = (0, 0, Fz), u = J / rho
    const R rho = R(1) + drho;
    const R T = tb + dT;
    const R Fz = rho * c.gbeta * (dT + (tb - c.t0));
    const R inv_rho = recip(rho);
    const R Jz = fmar(R(0.5), Fz, jz);
    const R ux = jx * inv_rho, uy = jy * inv_rho, uz = Jz * inv_rho;
    const R px = jx * ux, py = jy * uy, pz = Jz * uz;  // rho u_a^2
    const R pyz = py + pz, ruu = px + pyz;             // rho |u|^2
    const R pxx = fmar(R(2), px, -pyz), pww = py - pz;  // rho (3 ux^2 - |u|^2), rho (uy^2 - uz^2)
    const R uF = uz * Fz;
    // relaxed increments: -s (m - m_eq) + b (M F~) over |M_k|^2, where
    // m_e - m_e,eq = 19 (B - h0 - rho |u|^2), m_eps - m_eps,eq = 9 h0 - 7 A
    // - 2 B + 11/2 rho |u|^2, q_a - q_a,eq = 5/3 (E_a - 2 D_a) (+ Fz / 3 on
    // z); (M F~) = 38 uF and -11 uF on e and eps, -2 uF on 3p_xx and p_ww,
    // uF on 3pi_xx and pi_ww, -2/3 Fz on q_z, uy Fz and ux Fz on p_yz and
    // p_xz; the momentum rows gain exactly F
    const R dm_e = fmar(k[k3BE], uF, k[k3SE] * ((B - h[0]) - ruu));
    const R dm_eps = fmar(k[k3BEps], uF, k[k3SEps] * fmar(R(5.5), ruu, fmar(R(9), h[0], -fmar(R(7), A, R(2) * B))));
    const R dm_qx = k[k3SQ] * fmar(R(-2), Dx, Ex);
    const R dm_qy = k[k3SQ] * fmar(R(-2), Dy, Ey);
    const R dm_qz = fmar(k[k3BQ], Fz, k[k3SQ] * fmar(R(-2), Dz, Ez));
    const R dm_jz = Fz * R(1.0 / row_norm<Flow<3>>(7));
    const R dm_p = fmar(k[k3BP], uF, k[k3SP] * (m_p - pxx));
    const R dm_pi = fmar(k[k3BPi], uF, k[k3SPi] * fmar(R(0.5), pxx, m_pi));
    const R dm_w = fmar(k[k3BW], uF, k[k3SW] * (m_w - pww));
    const R dm_wi = fmar(k[k3BWi], uF, k[k3SWi] * fmar(R(0.5), pww, m_wi));
    const R dm_xy = k[k3SO] * fmar(-jx, uy, m_xy);
    const R dm_yz = fmar(k[k3BO], uy * Fz, k[k3SO] * fmar(-jy, uz, m_yz));
    const R dm_xz = fmar(k[k3BO], ux * Fz, k[k3SO] * fmar(-jx, uz, m_xz));
    const R dm_mx = k[k3SM] * m_x, dm_my = k[k3SM] * m_y, dm_mz = k[k3SM] * m_z;
    // inverse transform: h_i += sum_k M_ki dm_k, as even and odd parts of
    // each opposite pair
    h[0] = fmar(R(-30), dm_e, fmar(R(12), dm_eps, h[0]));
    {
        const R C = fmar(R(-11), dm_e, R(-4) * dm_eps);  // shared by the axis pairs
        const R P = fmar(R(-2), dm_pi, dm_p), W = fmar(R(-2), dm_wi, dm_w);
        const R e_x = fmar(R(2), P, C), CmP = C - P;
        const R e_y = CmP + W, e_z = CmP - W;
        const R o_z = fmar(R(-4), dm_qz, dm_jz);
        h[1] = fmar(R(-4), dm_qx, h[1] + e_x);
        h[2] = fmar(R(4), dm_qx, h[2] + e_x);
        h[3] = fmar(R(-4), dm_qy, h[3] + e_y);
        h[4] = fmar(R(4), dm_qy, h[4] + e_y);
        h[5] = (h[5] + e_z) + o_z;
        h[6] = (h[6] + e_z) - o_z;
    }
    {
        const R G = fmar(R(8), dm_e, dm_eps);  // shared by the edge pairs
        const R Pp = dm_p + dm_pi, Wp = dm_w + dm_wi;
        const R GP = G + Pp;
        const R e_xy = GP + Wp, e_xz = GP - Wp, e_yz = fmar(R(-2), Pp, G);
        const R X = dm_qx, Y = dm_qy, Z = dm_jz + dm_qz;
        const R e7 = e_xy + dm_xy, e9 = e_xy - dm_xy;
        const R e11 = e_xz + dm_xz, e13 = e_xz - dm_xz;
        const R e15 = e_yz + dm_yz, e17 = e_yz - dm_yz;
        const R o7 = (X + Y) + (dm_mx - dm_my), o9 = (X - Y) + (dm_mx + dm_my);
        const R o11 = (X + Z) + (dm_mz - dm_mx), o13 = (X - Z) - (dm_mx + dm_mz);
        const R o15 = (Y + Z) + (dm_my - dm_mz), o17 = (Y - Z) + (dm_my + dm_mz);
        h[7] = (h[7] + e7) + o7;
        h[8] = (h[8] + e7) - o7;
        h[9] = (h[9] + e9) + o9;
        h[10] = (h[10] + e9) - o9;
        h[11] = (h[11] + e11) + o11;
        h[12] = (h[12] + e11) - o11;
        h[13] = (h[13] + e13) + o13;
        h[14] = (h[14] + e13) - o13;
        h[15] = (h[15] + e15) + o15;
        h[16] = (h[16] + e15) - o15;
        h[17] = (h[17] + e17) + o17;
        h[18] = (h[18] + e17) - o17;
    }
    // heat: n_eq = (T, u T, a_T dT, 0, 0) in deviation form
    const R dn_x = k[k3QJ] * fmar(-ux, T, Dgx);
    const R dn_y = k[k3QJ] * fmar(-uy, T, Dgy);
    const R dn_z = k[k3QJ] * fmar(-uz, T, Dgz);
    const R dn_e = k[k3QE] * fmar(-c.a_t, dT, n_e);
    const R dn_p = k[k3QP] * n_p, dn_w = k[k3QW] * n_w;
    g[0] = fmar(R(-6), dn_e, g[0]);
    {
        const R e_x = fmar(R(2), dn_p, dn_e), EmP = dn_e - dn_p;
        const R e_y = EmP + dn_w, e_z = EmP - dn_w;
        g[1] = (g[1] + e_x) + dn_x;
        g[2] = (g[2] + e_x) - dn_x;
        g[3] = (g[3] + e_y) + dn_y;
        g[4] = (g[4] + e_y) - dn_y;
        g[5] = (g[5] + e_z) + dn_z;
        g[6] = (g[6] + e_z) - dn_z;
    }
    static_for<0, 19>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.sf(i, St::EF::enc(h[i]));
    });
    static_for<0, 7>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.sg(i, St::EG::enc(g[i]));
    });
    // unstable: a non-finite density or temperature, or a speed above the
    // lattice sound speed c_s = 1/sqrt(3)
    return isfinite(drho + dT) && ruu * inv_rho <= R(1.0 / 3.0);
}

// the basis entries written into collide_store_d3
static_assert(Flow<3>::M(1, 0) == -30 && Flow<3>::M(2, 0) == 12 && Flow<3>::M(1, 1) == -11 &&
                  Flow<3>::M(2, 1) == -4 && Flow<3>::M(1, 7) == 8 && Flow<3>::M(2, 7) == 1 &&
                  Flow<3>::M(4, 1) == -4 && Flow<3>::M(4, 7) == 1 && Flow<3>::M(9, 1) == 2 &&
                  Flow<3>::M(10, 1) == -4 && Flow<3>::M(9, 3) == -1 && Flow<3>::M(10, 3) == 2 &&
                  Flow<3>::M(9, 7) == 1 && Flow<3>::M(10, 7) == 1 && Flow<3>::M(9, 15) == -2 &&
                  Flow<3>::M(10, 15) == -2 && Flow<3>::M(11, 3) == 1 && Flow<3>::M(12, 3) == -2 &&
                  Flow<3>::M(11, 7) == 1 && Flow<3>::M(12, 7) == 1 && Flow<3>::M(11, 11) == -1 &&
                  Flow<3>::M(13, 9) == -1 && Flow<3>::M(15, 13) == -1 && Flow<3>::M(14, 17) == -1 &&
                  Flow<3>::M(16, 7) == 1 && Flow<3>::M(17, 7) == -1 && Flow<3>::M(16, 11) == -1 &&
                  Flow<3>::M(18, 11) == 1 && Flow<3>::M(17, 15) == 1 && Flow<3>::M(18, 15) == -1 &&
                  Heat<3>::M(4, 0) == -6 && Heat<3>::M(4, 1) == 1 && Heat<3>::M(5, 1) == 2 &&
                  Heat<3>::M(5, 3) == -1 && Heat<3>::M(6, 3) == 1 && Heat<3>::M(6, 5) == -1,
              "D3Q19 / D3Q7 basis entries of the written-out collision");
static_assert(row_norm<Flow<3>>(4) == row_norm<Flow<3>>(6) && row_norm<Flow<3>>(4) == row_norm<Flow<3>>(8) &&
                  row_norm<Flow<3>>(13) == row_norm<Flow<3>>(14) && row_norm<Flow<3>>(13) == row_norm<Flow<3>>(15) &&
                  row_norm<Flow<3>>(16) == row_norm<Flow<3>>(17) && row_norm<Flow<3>>(16) == row_norm<Flow<3>>(18) &&
                  row_norm<Heat<3>>(1) == row_norm<Heat<3>>(2) && row_norm<Heat<3>>(1) == row_norm<Heat<3>>(3),
              "rows that share a factor of Coef::k3 share their norm");

// Moments, both collisions and the store of one node (hf/hg: the
// pre-collision deviations).  Returns false if the node's density or
// temperature is not finite or its speed exceeds the lattice sound speed.
template <int DIM, class St, class Dst>
__device__ __forceinline__ bool collide_store(typename St::R* hf, typename St::R* hg,
                                              const Coef<typename St::R>& c, typename St::R tb, const Dst& dst) {
    if constexpr (DIM == 2) return collide_store_d2<St>(hf, hg, c, tb, dst);
    else return collide_store_d3<St>(hf, hg, c, tb, dst);
}

// --------------------------------------------------------- store helpers
// Raw buffer stores.  A lane whose byte offset is at or beyond the buffer
// size stores nothing (the hardware drops out-of-range buffer writes), so a
// store masked this way needs no branch: every lane executes it.  Offsets
// stay below 2^32 for buffers under 4 GiB - 4 KiB, with any immediate offset
// the compiler folds in.
constexpr uint32_t kBufferWord3 = 0x00020000u;  // gfx9 raw buffer, 32-bit data format

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, (int)kBufferWord3);
}

template <class T>
__device__ __forceinline__ void buffer_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t offset) {
    if constexpr (sizeof(T) == 2) {
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(short, v), r, (int)offset, 0, 0);
    } else if constexpr (sizeof(T) == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, v), r, (int)offset, 0, 0);
    } else {
        using I2 = int __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(I2, v), r, (int)offset, 0, 0);
    }
}

// Raw buffer load of an in-range offset: the constant part of the offset
// goes into the instruction (a 32-bit global address offset cannot take it:
// the sum might wrap).
template <class T> __device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, uint32_t offset) {
    if constexpr (sizeof(T) == 2) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(r, (int)offset, 0, 0));
    } else if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)offset, 0, 0));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)offset, 0, 0));
    }
}

// Wall heat flux sinks: put<face>(g, local, value, wall) records the value
// of a link that crosses a Dirichlet wall (wall true) at index `local` of
// that face.
struct PtrFlux {  // per-face arrays
    double* const* flux;
    bool on;
    template <int face> __device__ void put(const Geometry&, uint32_t local, double v, bool wall) const {
        if (on && wall) flux[face][local] = v;
    }
};


// ----------------------------------------------------------------- the step
// Sources of the pull.  pull_f<i, ex, ey, ez, o>(out) returns the decoded
// population f_i arriving at the node along e_i = (ex, ey, ez): from the
// neighbour at -e_i, or, when that link crosses a wall (out), the opposite
// population o at the node itself (bounce-back); pull_g likewise for g.
//
// GlobalSrc: the tiled arrays in global memory.  at(sx, sy, sz) is the index of the node displaced by
// (sx, sy, sz) in {-1, 0, 1}^3 from the current one; lf/lg read a
// population plane there.  In global memory a displacement across a
// periodic face wraps (the offsets are prepared per node); in an LDS tile
// the halo already holds the wrapped neighbours.
// Pull sources in global memory; U24: every node index is below 2^30.
template <class St, int QF, int QG, bool O32 = false, bool U24 = false> struct GlobalSrc {
    const typename St::TF* f;
    const typename St::TG* g;
    uint32_t idx;
    int32_t oxm, oxp, oym, oyp, ozm, ozp;
    __device__ uint32_t at(int sx, int sy, int sz) const {
        return (uint32_t)((int32_t)idx + (sx < 0 ? oxm : sx > 0 ? oxp : 0) + (sy < 0 ? oym : sy > 0 ? oyp : 0) +
                          (sz < 0 ? ozm : sz > 0 ? ozp : 0));
    }
    __device__ typename St::TF lf(int i, uint32_t node) const {
        return *elem<O32>(f, U24 ? pop_at24<QF>(node, i) : pop_at<QF>(node, i));
    }
    __device__ typename St::TG lg(int i, uint32_t node) const {
        return *elem<O32>(g, U24 ? pop_at24<QG>(node, i) : pop_at<QG>(node, i));
    }
    // both cases from one node index and one plane: a single load serves either
    template <int i, int ex, int ey, int ez, int o> __device__ typename St::R pull_f(bool out) const {
        return St::EF::dec(lf(out ? o : i, out ? at(0, 0, 0) : at(-ex, -ey, -ez)));
    }
    template <int i, int ex, int ey, int ez, int o> __device__ typename St::R pull_g(bool out) const {
        return St::EG::dec(lg(out ? o : i, out ? at(0, 0, 0) : at(-ex, -ey, -ez)));
    }
};


// Where a node's axis neighbours are: in the domain, across a periodic face
// (wrapped), or beyond a wall.
struct Neighbours {
    bool okxm, okxp, okym, okyp, okzm, okzp;  // a neighbour exists on that side
    bool inxm, inxp, inym, inyp, inzm, inzp;  // it is inside without wrapping
};

__device__ __forceinline__ Neighbours neighbours(const Geometry& g, uint32_t x, uint32_t y, uint32_t z) {
    Neighbours n;
    n.inxm = x > 0, n.inxp = x + 1 < g.nx;
    n.inym = y > 0, n.inyp = y + 1 < g.ny;
    n.inzm = z > 0, n.inzp = z + 1 < g.nz;
    n.okxm = n.inxm || g.periodic[0], n.okxp = n.inxp || g.periodic[0];
    n.okym = n.inym || g.periodic[1], n.okyp = n.inyp || g.periodic[1];
    n.okzm = n.inzm || g.periodic[2], n.okzp = n.inzp || g.periodic[2];
    return n;
}

template <class St, int QF, int QG, bool O32 = false, bool U24 = false>
__device__ __forceinline__ GlobalSrc<St, QF, QG, O32, U24> global_src(const Geometry& g, const Neighbours& n,
                                                                      const typename St::TF* f,
                                                                      const typename St::TG* gp, uint32_t idx) {
    const int32_t nx = (int32_t)g.nx, sy = nx, sz = nx * (int32_t)g.ny;
    GlobalSrc<St, QF, QG, O32, U24> s;
    s.f = f;
    s.g = gp;
    s.idx = idx;
    s.oxm = n.inxm ? -1 : nx - 1;
    s.oxp = n.inxp ? 1 : 1 - nx;
    s.oym = n.inym ? -sy : ((int32_t)g.ny - 1) * sy;
    s.oyp = n.inyp ? sy : -((int32_t)g.ny - 1) * sy;
    s.ozm = n.inzm ? -sz : ((int32_t)g.nz - 1) * sz;
    s.ozp = n.inzp ? sz : -((int32_t)g.nz - 1) * sz;
    return s;
}

// One fused update of the node at (x, y, z): pull from `src` with the wall
// rules, moments, both collisions, store to `dst`; the wall heat flux of
// the node's Dirichlet links goes to the flux sink `fx`.  Walls = false is
// for nodes known to have every link inside the domain (or across a
// periodic face): it drops the wall rules and the flux at compile time.
// Returns false if the new rho or T is not finite.
template <int DIM, class St, bool Walls = true, class Src, class Dst, class Flux>
__device__ __forceinline__ bool step_node(const Geometry& g, const Coef<typename St::R>& c, const Neighbours& nb,
                                          uint32_t x, uint32_t y, uint32_t z, const Src& src, const Dst& dst,
                                          const Flux& fx) {
    using R = typename St::R;
    using L = Flow<DIM>;
    using H = Heat<DIM>;
    R hf[L::Q], hg[H::Q];
    const R tb = base_temp(c.bt, x, y, z);
    // The gather is free of branches: a link that crosses a wall reads the
    // opposite plane at the node itself (bounce-back) through the same
    // single load, so every load is issued before any result is waited
    // for; the wall heat fluxes are stored after the gather.
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
        const bool out = Walls && ((ex > 0 && !nb.okxm) || (ex < 0 && !nb.okxp) || (ey > 0 && !nb.okym) ||
                                   (ey < 0 && !nb.okyp) || (ez > 0 && !nb.okzm) || (ez < 0 && !nb.okzp));
        hf[i] = src.template pull_f<i, ex, ey, ez, L::opp[i]>(out);
    });
    R wall_v[H::Q];
    bool wall_abb[H::Q];
    static_for<0, H::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ex = H::ex[i], ey = H::ey[i], ez = H::ez[i];
        // the wall a crossing link meets: axis of e_i, the side it comes from
        constexpr int axis = ex != 0 ? 0 : ey != 0 ? 1 : 2;
        constexpr int face = 2 * axis + ((ex + ey + ez) > 0 ? 0 : 1);
        const bool out = Walls && ((ex > 0 && !nb.okxm) || (ex < 0 && !nb.okxp) || (ey > 0 && !nb.okym) ||
                                   (ey < 0 && !nb.okyp) || (ez > 0 && !nb.okzm) || (ez < 0 && !nb.okzp));
        const R v = src.template pull_g<i, ex, ey, ez, H::opp[i]>(out);
        // anti-bounce-back on a Dirichlet wall, plain bounce-back (adiabatic)
        // otherwise
        wall_abb[i] = i != 0 && out && g.dirichlet[face];
        wall_v[i] = v;
        hg[i] = wall_abb[i] ? (c.abb_a[face] - c.abb_b[face] * tb) - v : v;
    });
    if constexpr (Walls)
        static_for<1, H::Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int ex = H::ex[i], ey = H::ey[i], ez = H::ez[i];
            constexpr int axis = ex != 0 ? 0 : ey != 0 ? 1 : 2;
            constexpr int face = 2 * axis + ((ex + ey + ez) > 0 ? 0 : 1);
            const uint32_t local = axis == 0 ? y + g.ny * z : axis == 1 ? x + g.nx * z : x + g.nx * y;
            // omega T_w - 2 g+_out in deviation form, from the constant the
            // rule applied (widened) and the reference state's own flux
            const double abb = (double)(c.abb_a[face] - c.abb_b[face] * tb);
            fx.template put<face>(g, local, abb + c.flux_c[face] - 2.0 * (double)wall_v[i], wall_abb[i]);
        });
    return collide_store<DIM, St>(hf, hg, c, tb, dst);
}

// the update of node idx of the arrays fsrc/gsrc into fdst/gdst
template <int DIM, class St>
__device__ __forceinline__ bool step_node_global(const Geometry& g, const Coef<typename St::R>& c,
                                                 const typename St::TF* fsrc, const typename St::TG* gsrc,
                                                 typename St::TF* fdst, typename St::TG* gdst,
                                                 double* const* flux, uint32_t idx) {
    constexpr int QF = Flow<DIM>::Q, QG = Heat<DIM>::Q;
    uint32_t x, y, z;
    coords(g, idx, x, y, z);
    const Neighbours nb = neighbours(g, x, y, z);
    const auto src = global_src<St, QF, QG>(g, nb, fsrc, gsrc, idx);
    const GlobalDst<St, QF, QG> dst(fdst, gdst, idx);
    return step_node<DIM, St>(g, c, nb, x, y, z, src, dst, PtrFlux{flux, true});
}

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs<St> a) {
    const uint32_t idx = logical_block(a.geo.blocks_per_xcd) * kBlock + threadIdx.x;
    if (idx >= a.geo.N) return;
    step_node_global<DIM, St>(a.geo, a.c, a.fsrc, a.gsrc, a.fdst, a.gdst, a.flux, idx);
}

// coordinate v along an axis of n nodes -> domain coordinate: wrapped on a
// periodic axis (any number of times: a region can be wider than the
// domain), -1 beyond a wall
__device__ __forceinline__ int32_t region_coord(int32_t v, uint32_t n, int32_t periodic) {
    if (v >= 0 && v < (int32_t)n) return v;
    if (!periodic) return -1;
    const int32_t r = v % (int32_t)n;
    return r < 0 ? r + (int32_t)n : r;
}

// ----------------------------- several steps per launch, register rows (2D)
// A wavefront walks down a strip of 64 - 2 NS columns, one row per
// iteration, and advances them NS steps (NS = 2 .. 5).  Lane l holds column
// x0 - NS + l.  The last rows of the input state and of every intermediate
// step stay in registers as decoded values (rounded through the storage
// type, so exactly what a single step would store and reload); the
// x-neighbours of a lane come from its neighbour lanes by DPP wave shifts.
// Step j is valid on lanes j .. 63 - j, so step NS covers the strip's own
// columns (lanes NS .. 63 - NS).  Row iteration k loads input row
// y0 - NS + k; step 1 runs D + 1 rows behind it (the loads of a row are
// issued D iterations before their first use) and every further step two
// rows behind the one before, computed in the order NS, ..., 2, 1 so that
// each step reads the rows of the step before it from earlier iterations.
template <int NS> constexpr int strip_cols() { return 64 - 2 * NS; }

// the value of v held by lane l - 1 (FromLeft) or lane l + 1 (otherwise);
// lane 0 (63) has no source and reads 0 (bound_ctrl), so no old value has
// to be set up first
template <bool FromLeft> __device__ __forceinline__ float lane_shift(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v),
                                                               FromLeft ? 0x138 : 0x130, 0xf, 0xf, true));
}
template <bool FromLeft> __device__ __forceinline__ double lane_shift(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, FromLeft ? 0x138 : 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), FromLeft ? 0x138 : 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// pull source: three register rows (y - 1, y, y + 1) of decoded populations
template <class St, int QF, int QG> struct RegSrc {
    using R = typename St::R;
    const R (&fm)[QF];
    const R (&fz)[QF];
    const R (&fp)[QF];
    const R (&gm)[QG];
    const R (&gz)[QG];
    const R (&gp)[QG];
    template <int ex, int ey, class A> __device__ static R from(const A& m, const A& z, const A& p, int i) {
        R v = ey > 0 ? m[i] : ey < 0 ? p[i] : z[i];
        if constexpr (ex > 0) v = lane_shift<true>(v);
        else if constexpr (ex < 0) v = lane_shift<false>(v);
        return v;
    }
    template <int i, int ex, int ey, int ez, int o> __device__ R pull_f(bool out) const {
        const R v = from<ex, ey>(fm, fz, fp, i);
        return out ? fz[o] : v;
    }
    template <int i, int ex, int ey, int ez, int o> __device__ R pull_g(bool out) const {
        const R v = from<ex, ey>(gm, gz, gp, i);
        return out ? gz[o] : v;
    }
};

// store into a register row, decoded (the value the next step reads)
template <class St, int QF, int QG> struct RegDst {
    typename St::R (&f)[QF];
    typename St::R (&g)[QG];
    __device__ void sf(int i, typename St::TF v) const { f[i] = St::EF::dec(v); }
    __device__ void sg(int i, typename St::TG v) const { g[i] = St::EG::dec(v); }
};

// the encoded values of a node's update, kept for stores issued later
template <class St, int QF, int QG> struct EncDst {
    typename St::TF (&f)[QF];
    typename St::TG (&g)[QG];
    __device__ void sf(int i, typename St::TF v) const { f[i] = v; }
    __device__ void sg(int i, typename St::TG v) const { g[i] = v; }
};

// Global stores for the lanes that own their node.  Stores and loads
// retire through one in-order counter, and a store under a branch leaves
// the compiler unsure it was issued, so it then waits for more of the
// memory operations after a load than the load needs; the buffer form
// drops the other lanes' stores instead and keeps the code straight-line.
template <class St, int QF, int QG, bool U24 = false> struct OwnedBufDst {
    __amdgpu_buffer_rsrc_t rf, rg;
    uint32_t of, og;  // byte offset of the node's first plane, or beyond the buffer
    // idx: the node's index from the first node of the buffers (below 2^30
    // with U24)
    __device__ OwnedBufDst(__amdgpu_buffer_rsrc_t rf_, __amdgpu_buffer_rsrc_t rg_, uint32_t f_bytes,
                           uint32_t g_bytes, uint32_t idx, bool own)
        : rf(rf_), rg(rg_),
          of(own ? (U24 ? pop_at24<QF>(idx, 0) : pop_at<QF>(idx, 0)) * (uint32_t)sizeof(typename St::TF) : f_bytes),
          og(own ? (U24 ? pop_at24<QG>(idx, 0) : pop_at<QG>(idx, 0)) * (uint32_t)sizeof(typename St::TG) : g_bytes) {}
    __device__ void sf(int i, typename St::TF v) const {
        buffer_store(v, rf, of + (uint32_t)(i * kTile * sizeof(typename St::TF)));
    }
    __device__ void sg(int i, typename St::TG v) const {
        buffer_store(v, rg, og + (uint32_t)(i * kTile * sizeof(typename St::TG)));
    }
};

// One flux slot in one array, the faces back to back (face f starts after
// the node counts of faces 0 .. f-1; 2D).  Buffer stores like the
// populations: a lane not on a Dirichlet wall link stores to the dropped
// offset, so no code of the streaming kernels runs under a lane-divergent
// branch.  (Under such a branch the register allocator may place the spill
// of a value that every lane needs later, and a spill store executes for
// the active lanes only: the other lanes would reload a stale value.)  The
// store is issued only when some lane of the wavefront is on such a link
// (a wavefront-uniform branch on the ballot), which happens in the rows
// and columns next to a Dirichlet wall.
struct BufFlux2 {
    __amdgpu_buffer_rsrc_t r;
    uint32_t slot;   // first element of the slot
    uint32_t bytes;  // size of the flux area: the dropped offset
    bool on;
    template <int face> __device__ void put(const Geometry& g, uint32_t local, double v, bool wall) const {
        const uint32_t start = face == 0 ? 0u : face == 1 ? g.ny : face == 2 ? 2u * g.ny : 2u * g.ny + g.nx;
        const bool mine = on && wall;
        if (__builtin_amdgcn_ballot_w64(mine))
            buffer_store(v, r, mine ? (slot + start + local) * (uint32_t)sizeof(double) : bytes);
    }
};

template <class St> struct StreamArgs {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    typename St::TF* fdst;
    typename St::TG* gdst;
    double* flux;                     // wall heat flux area: two slots, faces back to back
    uint32_t flux_bytes;              // its size
    uint32_t f_bytes, g_bytes;        // sizes of fdst, gdst (buffer stores; 0 for arrays of 4 GiB or more)
    uint32_t slot[2];                 // first element of flux slot 0 and slot 1
    int32_t t_parity;                 // (t of the input state) mod 2: step j writes slot (t + j) mod 2
    Geometry geo;
    Coef<typename St::R> c;
    uint32_t strips;          // strips across x
    uint32_t seg_rows;        // rows per strip segment
    uint32_t units;           // strips x segments, one per wavefront
    uint32_t blocks_per_xcd;
};

// Register budget (measured): three wavefronts per SIMD (168 registers) for
// two steps, and for three steps when f and g are both 16-bit; two (256
// registers) for four and five steps (FP32 at five: 249), for three steps
// with FP32 populations, and for FP64 arithmetic.
#ifndef LBM_STREAM_WAVES_PER_SIMD
#define LBM_STREAM_WAVES_PER_SIMD 3
#endif
template <class St, int NS> constexpr int stream_waves_per_simd() {
    constexpr bool half = sizeof(typename St::TF) == 2 && sizeof(typename St::TG) == 2;
    if constexpr (sizeof(typename St::R) == 8 || NS > 3) return 2;
    else if constexpr (NS == 3) return half ? LBM_STREAM_WAVES_PER_SIMD : 2;
    else return LBM_STREAM_WAVES_PER_SIMD;
}

// One wavefront's work unit (strip unit % strips, row segment unit /
// strips) of a, advancing NS steps from the state of parity tp.  With
// Report, returns false on a lane that computed, at any of the NS steps, a
// real node whose new rho or T is not finite or whose speed exceeds the
// lattice sound speed.
template <class St, bool O32, int NS, int D, bool Report>
__device__ __forceinline__ bool stream_unit(const StreamArgs<St>& a, uint32_t unit, int32_t tp) {
    using R = typename St::R;
    constexpr int QF = Flow<2>::Q, QG = Heat<2>::Q;
    constexpr int W = strip_cols<NS>();
    static_assert(NS >= 2 && NS <= 5, "two to five steps per launch");
    const Geometry& g = a.geo;
    const int lane = (int)(threadIdx.x & 63);
    bool bad = false;
    const int32_t x0 = (int32_t)((unit % a.strips) * W);
    const int32_t y0 = (int32_t)((unit / a.strips) * a.seg_rows);
    const int32_t rows = min((int32_t)a.seg_rows, (int32_t)g.ny - y0);
    const int32_t cx = x0 - NS + lane;                          // this lane's column, unwrapped
    const int32_t col = region_coord(cx, g.nx, g.periodic[0]);  // -1 beyond a wall
    const uint32_t ucol = col < 0 ? 0u : (uint32_t)col;         // any in-domain column for dead lanes
    const bool own_col = lane >= NS && lane < NS + W && cx < (int32_t)g.nx;

    // Rings: NI input rows, R rows of each intermediate step; the loop is
    // unrolled over U = NI iterations so that every ring index is a
    // compile-time constant.
    constexpr int NI = D + 3, RS = NI % 3 == 0 ? 3 : NI, U = NI;
    // rows a step never fills (beyond a wall) are only ever discarded by the
    // bounce-back selects; start them at zero so no value is indeterminate
    R fin[NI][QF] = {}, gin[NI][QG] = {};          // input rows
    R fs[NS - 1][RS][QF] = {}, gs[NS - 1][RS][QG] = {};  // rows of steps 1 .. NS-1

    // The loop body is straight-line: every iteration loads a row and
    // computes every step; rows outside the segment or beyond a wall use an
    // in-domain stand-in row and are never stored.  (Branches around the
    // loads would leave paths on which a load is not waited for, after which
    // the compiler drains every outstanding load before the next row.)
    const int32_t last = (int32_t)g.ny - 1;
    const __amdgpu_buffer_rsrc_t rflux = buffer_rsrc(a.flux, a.flux_bytes);
    // Destinations of step NS in row yy: buffer resources over the whole
    // arrays when byte offsets fit 32 bits (O32), else based at the first
    // tile of the row (a wavefront-uniform base; a row and its halo span at
    // most nx + 64 nodes), so both forms store without a branch.
    const __amdgpu_buffer_rsrc_t rf = buffer_rsrc(a.fdst, a.f_bytes), rg = buffer_rsrc(a.gdst, a.g_bytes);
    // the sources have the sizes of the destinations (the two buffers of a
    // ping-pong pair)
    const __amdgpu_buffer_rsrc_t rfs = buffer_rsrc(a.fsrc, a.f_bytes), rgs = buffer_rsrc(a.gsrc, a.g_bytes);
    auto row_dst = [&](uint32_t x, uint32_t yy, bool own) {
        if constexpr (O32) {
            return OwnedBufDst<St, QF, QG>(rf, rg, a.f_bytes, a.g_bytes, x + g.nx * yy, own);
        } else {
            const uint32_t row0 = g.nx * yy;
            const uint32_t t0 = row0 / kTile, tiles = (row0 + g.nx - 1) / kTile + 1 - t0;
            const uint32_t fb = tiles * (uint32_t)(QF * kTile * sizeof(typename St::TF));
            const uint32_t gb = tiles * (uint32_t)(QG * kTile * sizeof(typename St::TG));
            return OwnedBufDst<St, QF, QG>(buffer_rsrc(a.fdst + (size_t)t0 * (QF * kTile), fb),
                                           buffer_rsrc(a.gdst + (size_t)t0 * (QG * kTile), gb), fb, gb,
                                           x + row0 - t0 * kTile, own);
        }
    };
    // Row y of step j feeds a stored result only inside the dependency cone
    // of the segment, rows y0 - (NS - j) .. y0 + rows - 1 + (NS - j) (for
    // j = NS the segment itself); elsewhere (while the step pipeline fills
    // and drains) the update is skipped by a wavefront-uniform branch, and
    // nothing needed reads the ring slot it would have written.  The stores
    // of step NS stay outside any branch: a branch around them would make
    // the compiler wait for them before later loads.
    // (FP64 arithmetic keeps every step: the branches cost it registers.)
    auto needed = [&](int j, int32_t y) {
        const int32_t rel = y - y0;
        return sizeof(R) == 8 || (rel >= -(NS - j) && rel <= rows - 1 + (NS - j));
    };
    auto iteration = [&](auto slot, auto walls, int32_t k) {
        constexpr int S = decltype(slot)::value;  // k mod U
        constexpr bool Wl = decltype(walls)::value;
        // ring slot of what iteration k - j loaded (input) or computed (a step)
        constexpr auto in = [](int j) { return ((S - j) % NI + NI) % NI; };
        constexpr auto st = [](int j) { return ((S - j) % RS + RS) % RS; };
        const int32_t yin = y0 - NS + k;
        // 1. issue the loads of input row yin (its slot held row yin - NI).
        //    Past the last row the segment needs (y0 + rows - 1 + NS, while
        //    the pipeline drains) the loads repeat that row, which the cache
        //    still holds: what they feed is never stored.
        {
            const int32_t yl = min(yin, y0 + rows - 1 + NS);
            const int32_t rin = region_coord(yl, g.ny, g.periodic[1]);
            const uint32_t row_in = (uint32_t)(rin >= 0 ? rin : min(max(yl, 0), last));
            const uint32_t node = ucol + g.nx * row_in;
            const uint32_t bf = pop_at<QF>(node, 0), bg = pop_at<QG>(node, 0);
            using TF = typename St::TF;
            using TG = typename St::TG;
            static_for<0, QF>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (O32)
                    fin[in(0)][i] = St::EF::dec(buffer_load<TF>(rfs, (bf + i * kTile) * (uint32_t)sizeof(TF)));
                else
                    fin[in(0)][i] = St::EF::dec(a.fsrc[bf + i * kTile]);
            });
            static_for<0, QG>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (O32)
                    gin[in(0)][i] = St::EG::dec(buffer_load<TG>(rgs, (bg + i * kTile) * (uint32_t)sizeof(TG)));
                else
                    gin[in(0)][i] = St::EG::dec(a.gsrc[bg + i * kTile]);
            });
        }
        const int32_t y1 = yin - 1 - D;  // row of step 1; step j runs on row y1 - 2 (j - 1)
        // 2. steps NS, ..., 2: step j on row yj from the rows yj - 1, yj,
        //    yj + 1 of step j - 1 (computed in iterations k-3, k-2, k-1),
        //    into the ring slot of step j that step j + 1 has just read
        static_for<0, NS - 1>([&](auto jc) {
            constexpr int j = NS - decltype(jc)::value;  // NS, NS-1, ..., 2
            const int32_t yj = y1 - 2 * (j - 1);
            const bool own = own_col && yj >= y0 && yj < y0 + rows;
            const uint32_t yy = (uint32_t)min(max(yj, 0), last);
            const uint32_t x = own_col ? (uint32_t)cx : ucol;
            const Neighbours nb = neighbours(g, x, yy, 0);
            const RegSrc<St, QF, QG> src{fs[j - 2][st(3)], fs[j - 2][st(2)], fs[j - 2][st(1)],
                                         gs[j - 2][st(3)], gs[j - 2][st(2)], gs[j - 2][st(1)]};
            const BufFlux2 fx{rflux, a.slot[(tp + j) & 1], a.flux_bytes, own};
            if constexpr (j == NS) {
                // The update runs only on the segment's rows (needed(NS, y)
                // is exactly them); the stores always issue, to the dropped
                // offset elsewhere.
                typename St::TF ef[QF];
                typename St::TG eg[QG];
                if (needed(NS, yj)) {
                    const bool ok = step_node<2, St, Wl>(g, a.c, nb, x, yy, 0u, src, EncDst<St, QF, QG>{ef, eg}, fx);
                    if constexpr (Report) bad = bad || (own && !ok);
                } else {
                    // stored to the dropped offset: any value will do, so
                    // take whatever the registers hold (an empty asm that
                    // defines them; a constant would cost a move each)
#pragma unroll
                    for (int i = 0; i < QF; ++i) asm volatile("" : "=v"(ef[i]));
#pragma unroll
                    for (int i = 0; i < QG; ++i) asm volatile("" : "=v"(eg[i]));
                }
                const OwnedBufDst<St, QF, QG> dst = row_dst(x, yy, own);
                static_for<0, QF>([&](auto ic) { dst.sf(decltype(ic)::value, ef[decltype(ic)::value]); });
                static_for<0, QG>([&](auto ic) { dst.sg(decltype(ic)::value, eg[decltype(ic)::value]); });
            } else if (needed(j, yj)) {
                const RegDst<St, QF, QG> dst{fs[j - 1][st(0)], gs[j - 1][st(0)]};
                const bool ok = step_node<2, St, Wl>(g, a.c, nb, x, yy, 0u, src, dst, fx);
                // an intermediate state is checked too where it is a real
                // node's: a valid lane of step j inside the domain
                if constexpr (Report)
                    bad = bad || (!ok && lane >= j && lane <= 63 - j && col >= 0 &&
                                  (g.periodic[1] || (yj >= 0 && yj <= last)));
            }
        });
        // 3. step 1 on row y1 from the input rows y1 - 1, y1, y1 + 1 (loaded in
        //    iterations k-2-D, k-1-D, k-D), into the slot step 2 has just read
        if (needed(1, y1)) {
            const int32_t r1 = region_coord(y1, g.ny, g.periodic[1]);
            const uint32_t yy = (uint32_t)(r1 >= 0 ? r1 : min(max(y1, 0), last));
            const Neighbours nb = neighbours(g, ucol, yy, 0);
            const RegSrc<St, QF, QG> src{fin[in(2 + D)], fin[in(1 + D)], fin[in(D)],
                                         gin[in(2 + D)], gin[in(1 + D)], gin[in(D)]};
            const RegDst<St, QF, QG> dst{fs[0][st(0)], gs[0][st(0)]};
            const bool own = own_col && y1 >= y0 && y1 < y0 + rows;
            const bool ok = step_node<2, St, Wl>(g, a.c, nb, ucol, yy, 0u, src, dst,
                                                 BufFlux2{rflux, a.slot[(tp + 1) & 1], a.flux_bytes, own});
            if constexpr (Report) bad = bad || (!ok && lane >= 1 && lane <= 62 && col >= 0 && r1 >= 0);
        }
    };
    // step NS reaches row y0 + rows - 1 at k = rows + 3 NS - 2 + D; the
    // count is rounded up to whole groups of U (the extra ones store nothing)
    auto sweep = [&](auto walls) {
        for (int32_t k = 0; k < rows + 3 * NS - 1 + D; k += U) {
            static_for<0, U>([&](auto sc) { iteration(sc, walls, k + decltype(sc)::value); });
        }
    };
    // Every update that feeds a stored result lies on lanes 1 .. 62 of step
    // 1 (columns x0 - NS + 1 .. x0 - NS + 62) and in its rows y0 - (NS - 1)
    // .. y0 + rows - 1 + (NS - 1).  When all of those nodes are at least one
    // node from every non-periodic wall, no link of theirs crosses a wall,
    // and the wavefront runs the sweep without wall rules and wall flux.
    const bool inner_x = g.periodic[0] || (x0 - NS + 1 >= 1 && x0 - NS + 62 <= (int32_t)g.nx - 2);
    const bool inner_y = g.periodic[1] || (y0 - (NS - 1) >= 1 && y0 + rows - 1 + (NS - 1) <= (int32_t)g.ny - 2);
    if (inner_x && inner_y)
        sweep(std::false_type{});
    else
        sweep(std::true_type{});
    return !bad;
}

template <class St, int NWB, bool O32, int NS, int D>
__global__ __launch_bounds__(64 * NWB) __attribute__((amdgpu_waves_per_eu(stream_waves_per_simd<St, NS>())))
void stream_kernel(StreamArgs<St> a) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t unit = logical_block(a.blocks_per_xcd) * NWB + wave;
    if (unit >= a.units) return;  // whole wavefront
    stream_unit<St, O32, NS, D, false>(a, unit, a.t_parity);
}

// Many 2D cavities, several steps per launch: wavefront w takes work unit w
// of the concatenated units of all cavities; unit_cavity maps it to its
// cavity, whose arguments (for either source buffer) sit in desc.
template <class St> struct BatchStreamArgs {
    const StreamArgs<St>* desc;   // [2][count]: the cavities' arguments with buffer A, B as source
    const uint16_t* unit_cavity;  // [units]
    const uint32_t* unit0;        // [count] first unit of each cavity
    uint32_t units, count, blocks_per_xcd;
    int32_t src;                  // source buffer of this launch
    int32_t t_parity;             // (t of the input state) mod 2
    int32_t* unstable;            // per-cavity flag, set on a non-finite node
};

// NWB bounds the wavefronts per block; a launch may use fewer (any block
// of blockDim.x / 64 wavefronts).
template <class St, int NWB, bool O32, int NS, int D>
__global__ __launch_bounds__(64 * NWB) __attribute__((amdgpu_waves_per_eu(stream_waves_per_simd<St, NS>())))
void batch_stream_kernel(BatchStreamArgs<St> b) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t unit = logical_block(b.blocks_per_xcd) * nw + wave;
    if (unit >= b.units) return;  // whole wavefront
    const uint32_t k = b.unit_cavity[unit];
    // the cavity's arguments, read through the constant address space
    // (scalar loads that the kernel's stores cannot invalidate: the tables
    // do not change during a launch)
    using CArgs = const __attribute__((address_space(4))) StreamArgs<St>;
    const StreamArgs<St>& a = *(const StreamArgs<St>*)((CArgs*)b.desc + ((uint32_t)b.src * b.count + k));
    if (!stream_unit<St, O32, NS, D, true>(a, unit - b.unit0[k], b.t_parity)) b.unstable[k] = 1;
}

// --------------------------------------------------------- batched cavities
// Many independent cavities of any size advance in one launch.  The work is
// cut into units of BS nodes of one cavity; unit_cavity maps a unit to its
// cavity, whose descriptor carries geometry, coefficients and buffers.  With
// a grid smaller than the unit count the blocks loop over units
// (persistent launch).
template <class St> struct BatchCavity {
    Geometry geo;
    Coef<typename St::R> c;
    typename St::TF* f[2];   // population buffers A, B
    typename St::TG* g[2];
    double* flux[2][6];      // wall heat flux, per slot and face
    uint32_t unit0;          // first work unit of this cavity
};

template <class St> struct BatchArgs {
    const BatchCavity<St>* cav;
    const uint16_t* unit_cavity;  // [total_units]
    uint32_t total_units;
    int32_t src;                  // buffer holding the current state (0: A, 1: B)
    int32_t slot;                 // flux slot of this step
    int32_t* unstable;            // per-cavity flag, set on a non-finite node
};

template <int DIM, class St, int BS>
__global__ __launch_bounds__(BS) void batch_step_kernel(BatchArgs<St> a) {
    for (uint32_t unit = blockIdx.x; unit < a.total_units; unit += gridDim.x) {
        const uint32_t k = a.unit_cavity[unit];
        const BatchCavity<St>& cv = a.cav[k];
        const uint32_t idx = (unit - cv.unit0) * BS + threadIdx.x;
        if (idx < cv.geo.N) {
            const bool ok = step_node_global<DIM, St>(cv.geo, cv.c, cv.f[a.src], cv.g[a.src], cv.f[1 - a.src],
                                                      cv.g[1 - a.src], cv.flux[a.slot], idx);
            if (!ok) a.unstable[k] = 1;
        }
    }
}

// -------------------------------------------------------------- init kernel
template <class St> struct InitArgs {
    typename St::TF* fdst;
    typename St::TG* gdst;
    Geometry geo;
    Coef<typename St::R> c;
    uint32_t n0, cnt;  // node range of this launch
    int32_t mode;      // 0: profile + noise, 1: fields from device arrays
    int32_t axis;      // conduction axis (-1: uniform T0)
    double t_lo, t_hi, t0;
    double amp;
    uint64_t seed;
    const double* rho;  // mode 1: [cnt] or null
    const double* u;    // mode 1: [DIM][cnt]
    const double* T;    // mode 1: [cnt]
    double w_rest, w_move;  // thermal rest-state weights
    double delta;           // odd part of the reference state's pre-collision g along its axis
};

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void init_kernel(InitArgs<St> a) {
    using R = typename St::R;
    using L = Flow<DIM>;
    using H = Heat<DIM>;
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.cnt) return;
    const uint32_t idx = a.n0 + k;
    uint32_t x, y, z;
    coords(a.geo, idx, x, y, z);
    double rho = 1.0, T, u[3] = {0.0, 0.0, 0.0};
    if (a.mode == 0) {
        const uint32_t cx[3] = {x, y, z};
        const double na = a.axis == 0 ? a.geo.nx : a.axis == 1 ? a.geo.ny : a.geo.nz;
        T = a.axis >= 0 ? a.t_lo + ((double)cx[a.axis] + 0.5) * (a.t_hi - a.t_lo) / na : a.t0;
        const uint64_t r = splitmix64(a.seed ^ splitmix64((uint64_t)idx));
        T += a.amp * (2.0 * ((double)(r >> 11) * 0x1.0p-53) - 1.0);
    } else {
        if (a.rho) rho = a.rho[k];
        for (int d = 0; d < DIM; ++d) u[d] = a.u[(size_t)d * a.cnt + k];
        T = a.T[k];
    }
    // equilibria as deviations: f_eq - w = w (drho + rho (3 eu + 4.5 eu^2 - 1.5 uu)),
    // g_eq - G = w^T (T - T_b) + (e.u) T / 2 - e_a delta (G: the reference
    // state's pre-collision populations, odd part delta along its axis a)
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    R hf[L::Q], hg[H::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double eu = L::ex[i] * u[0] + L::ey[i] * u[1] + L::ez[i] * u[2];
        hf[i] = (R)(L::w[i] * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
    }
    const R tbr = base_temp(a.c.bt, x, y, z);
    const double tb = (double)tbr;
#pragma unroll
    for (int i = 0; i < H::Q; ++i) {
        const double eu = H::ex[i] * u[0] + H::ey[i] * u[1] + H::ez[i] * u[2];
        const int ea = a.c.bt.axis == 0 ? H::ex[i] : a.c.bt.axis == 1 ? H::ey[i] : H::ez[i];
        const double wt = i == 0 ? a.w_rest : a.w_move;
        hg[i] = (R)(wt * (T - tb) + 0.5 * eu * T - ea * a.delta);
    }
    collide_store<DIM, St>(hf, hg, a.c, tbr, GlobalDst<St, L::Q, H::Q>(a.fdst, a.gdst, idx));
}

// ----------------------------------------------------- moments of one node
// FP64 moments of the stored post-collision populations at node idx:
// rho = sum f+, T = sum g+, j+ = sum e f+ = j + F, so u = (j+ - F/2)/rho.
template <int DIM, class St> struct NodeMoments {
    double rho, T, u[3];
    int nonfinite;
};

template <int DIM, class St>
__device__ __forceinline__ NodeMoments<DIM, St> node_moments(const typename St::TF* fsrc,
                                                             const typename St::TG* gsrc,
                                                             const Geometry& geo, uint32_t idx,
                                                             double gbeta, const BaseTemp<typename St::R>& bt,
                                                             double t0) {
    using L = Flow<DIM>;
    using H = Heat<DIM>;
    NodeMoments<DIM, St> m;
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0}, dT = 0.0;
    int bad = 0;
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double v = (double)St::EF::dec(fsrc[pop_at<L::Q>(idx, i)]);
        const double h = v;
        bad += !isfinite(h);
        drho += h;
        j[0] += L::ex[i] * h;
        j[1] += L::ey[i] * h;
        j[2] += L::ez[i] * h;
    }
#pragma unroll
    for (int i = 0; i < H::Q; ++i) {
        const double h = (double)St::EG::dec(gsrc[pop_at<H::Q>(idx, i)]);
        bad += !isfinite(h);
        dT += h;
    }
    uint32_t x, y, z;
    coords(geo, idx, x, y, z);
    m.rho = 1.0 + drho;
    m.T = (double)base_temp(bt, x, y, z) + dT;
    double F[3] = {0.0, 0.0, 0.0};
    F[DIM - 1] = m.rho * gbeta * (m.T - t0);
    for (int a = 0; a < 3; ++a) m.u[a] = (j[a] - 0.5 * F[a]) / m.rho;
    m.nonfinite = bad;
    return m;
}

template <class St> struct FieldArgs {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    Geometry geo;
    uint32_t n0, cnt;
    double gbeta, t0;
    BaseTemp<typename St::R> bt;
    double* rho;  // [cnt] or null
    double* u;    // [DIM][cnt] or null
    double* T;    // [cnt] or null
    unsigned long long* nonfinite;  // atomic counters: [0] non-finite populations,
                                    // [1] nodes faster than c_s = 1/sqrt(3)
};

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void fields_kernel(FieldArgs<St> a) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.cnt) return;
    const auto m = node_moments<DIM, St>(a.fsrc, a.gsrc, a.geo, a.n0 + k, a.gbeta, a.bt, a.t0);
    if (a.rho) a.rho[k] = m.rho;
    if (a.T) a.T[k] = m.T;
    if (a.u)
        for (int d = 0; d < DIM; ++d) a.u[(size_t)d * a.cnt + k] = m.u[d];
    if (m.nonfinite) atomicAdd(a.nonfinite, (unsigned long long)m.nonfinite);
    if (m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2] > 1.0 / 3.0) atomicAdd(a.nonfinite + 1, 1ull);
}

// ---------------------------------------------------------------- reductions
// 64-wide wavefront shuffle, then LDS across the block's waves.
template <class Op> __device__ __forceinline__ double wave_reduce(double v, Op op) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_down(v, o, 64));
    return v;
}

template <int NT, class Op>
__device__ __forceinline__ double block_reduce(double v, Op op, double* lds) {
    constexpr int W = NT / 64;
    v = wave_reduce(v, op);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();  // lds may still be read by a previous call
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double r = lds[0];
    for (int w = 1; w < W; ++w) r = op(r, lds[w]);
    return r;  // every thread holds the block result
}

struct AddOp { __device__ double operator()(double a, double b) const { return a + b; } };
struct MaxOp { __device__ double operator()(double a, double b) const { return fmax(a, b); } };

constexpr int kDiagVals = 6;  // mass, energy, sum |u|^2, sum u_g (T - T0), max |u|, nonfinite

template <class St> struct DiagArgs {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    Geometry geo;
    double gbeta, t0;
    BaseTemp<typename St::R> bt;
    double* partial;  // [gridDim.x][kDiagVals]
};

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void diag_kernel(DiagArgs<St> a) {
    __shared__ double lds[kBlock / 64];
    double acc[kDiagVals] = {0, 0, 0, 0, 0, 0};
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < a.geo.N; idx += gridDim.x * kBlock) {
        const auto m = node_moments<DIM, St>(a.fsrc, a.gsrc, a.geo, idx, a.gbeta, a.bt, a.t0);
        const double uu = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
        acc[0] += m.rho;
        acc[1] += m.T;
        acc[2] += uu;
        acc[3] += m.u[DIM - 1] * (m.T - a.t0);
        acc[4] = fmax(acc[4], sqrt(uu));
        acc[5] += m.nonfinite;
    }
    for (int v = 0; v < kDiagVals; ++v) {
        const double r = v == 4 ? block_reduce<kBlock>(acc[v], MaxOp{}, lds)
                                : block_reduce<kBlock>(acc[v], AddOp{}, lds);
        if (threadIdx.x == 0) a.partial[(size_t)blockIdx.x * kDiagVals + v] = r;
    }
}

// one block: reduce nblk partial rows in block order
__global__ __launch_bounds__(1024) void diag_final_kernel(const double* partial, int nblk, double* out) {
    __shared__ double lds[1024 / 64];
    for (int v = 0; v < kDiagVals; ++v) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < nblk; b += 1024) {
            const double x = partial[(size_t)b * kDiagVals + v];
            acc = v == 4 ? fmax(acc, x) : acc + x;
        }
        const double r = v == 4 ? block_reduce<1024>(acc, MaxOp{}, lds) : block_reduce<1024>(acc, AddOp{}, lds);
        if (threadIdx.x == 0) out[v] = r;
    }
}

// The values of lbm_diag from the reduced sums (mass, energy, sum |u|^2,
// sum u_g (T - T0), max |u|, nonfinite), in the field order of lbm_diag:
// t, mass, energy, umax, nu_vol, re, nonfinite.  The same FP64 operations,
// in the same order, as the host computes them for lbm_diagnostics.
struct DiagScale {
    double t, N, H, alpha, nu, dT;
};
__global__ __launch_bounds__(64) void diag_values_kernel(const double* sums, DiagScale s, double* out) {
    if (threadIdx.x != 0) return;
    out[0] = s.t;
    out[1] = sums[0];
    out[2] = sums[1];
    out[3] = sums[4];
    out[4] = 1.0 + s.H * (sums[3] / s.N) / (s.alpha * s.dT);
    out[5] = sqrt(sums[2] / s.N) * s.H / s.nu;
    out[6] = sums[5];
}

// per-face wall heat flux sums: block b reduces buffer b (face, slot) in FP64
struct FaceSumArgs {
    const double* buf[12];
    uint32_t count[12];
    double* out;  // [12]
};

__global__ __launch_bounds__(1024) void face_sum_kernel(FaceSumArgs a) {
    __shared__ double lds[1024 / 64];
    const int b = blockIdx.x;
    double acc = 0.0;
    if (a.buf[b])
        for (uint32_t i = threadIdx.x; i < a.count[b]; i += 1024) acc += a.buf[b][i];
    const double r = block_reduce<1024>(acc, AddOp{}, lds);
    if (threadIdx.x == 0) a.out[b] = r;
}

// Zeroes the unused lanes (nodes N .. end of tile) of the last storage tile
// of a population array of Q planes of `elem`-byte values, so that a
// checkpoint of the buffers depends on the state only.  One block.
__global__ __launch_bounds__(kBlock) void clear_tail_kernel(unsigned char* p, uint32_t N, uint32_t Q,
                                                            uint32_t elem) {
    const uint32_t tile = N / kTile, first = N % kTile, plane_bytes = kTile * elem;
    for (uint32_t k = threadIdx.x; k < Q * plane_bytes; k += kBlock) {
        const uint32_t plane = k / plane_bytes, rem = k % plane_bytes;
        if (rem / elem >= first) p[((size_t)tile * Q + plane) * plane_bytes + rem] = 0;
    }
}

__global__ __launch_bounds__(kBlock) void zero_bytes_kernel(unsigned char* p, uint32_t n) {
    for (uint32_t k = threadIdx.x; k < n; k += kBlock) p[k] = 0;
}

__global__ __launch_bounds__(kBlock) void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        p[i] = v;
}

__global__ __launch_bounds__(kBlock) void fill_kernel(double* p, size_t n, double v) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        p[i] = v;
}

// per-cavity wall heat flux sums: block (k, b) reduces buffer b of cavity k,
// in the order of face_sum_kernel, so that a batch member's sums equal those
// of the same cavity run alone bit for bit
struct BatchFaceArgs {
    const double* const* buf;  // [count][12]
    const uint32_t* len;       // [count][12]
    double* out;               // [count][12]
};

__global__ __launch_bounds__(1024) void batch_face_sum_kernel(BatchFaceArgs a) {
    __shared__ double lds[1024 / 64];
    const size_t b = blockIdx.x;
    const double* p = a.buf[b];
    double acc = 0.0;
    if (p)
        for (uint32_t i = threadIdx.x; i < a.len[b]; i += 1024) acc += p[i];
    const double r = block_reduce<1024>(acc, AddOp{}, lds);
    if (threadIdx.x == 0) a.out[b] = r;
}

}  // namespace lbm

#include "stream3d.hpp"
