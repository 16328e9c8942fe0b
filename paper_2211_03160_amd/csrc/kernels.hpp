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
// Every storage mode keeps deviations from the rest state, h_i = f_i - w_i
// (flow) and h^g_i = g_i - w^T_i T_b (thermal, T_b = T0), and all arithmetic
// runs on them, so the order-one rest populations never swamp the small
// non-equilibrium parts: stored as f itself, an FP32 population near w
// rounds away any deviation below half an ulp of w (~1.5e-8) every step.
// With orthogonal bases the collision is applied as an increment:
//   h+_i = h_i + sum_k M_ki dm_k / |M_k|^2.
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
struct E16 {
    using T = _Float16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v) { return (T)v; }
};
struct EB16 {  // bfloat16 kept as raw bits
    using T = uint16_t;
    __device__ static float dec(T v) { return __uint_as_float((uint32_t)v << 16); }
    __device__ static T enc(float v) {
        const uint32_t u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return (T)((u >> 16) | 0x40u);  // quiet NaN
        return (T)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
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

template <class R> struct Coef {
    R s[19];     // flow rate per moment row (0 on conserved rows)
    R b[19];     // 1 - s/2 per row
    R q[7];      // thermal rate per row
    R a_t;       // thermal equilibrium constant a_T
    R gbeta;     // g beta
    R t_base;    // T_b
    R tb_m_t0;   // T_b - T0
    R abb[6];    // omega (T_w - T_b) on Dirichlet faces
    double abb_d[6];  // the same in FP64, for the wall heat flux
};

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

// acc += C v for a compile-time integer coefficient C
template <int C, class R> __device__ __forceinline__ void cmac(R& acc, R v) {
    if constexpr (C == 1) acc += v;
    else if constexpr (C == -1) acc -= v;
    else if constexpr (C != 0) acc += R(C) * v;
}

// m_eq(rho, u) - m_eq(1, 0) for the non-conserved rows (second-order
// equilibrium with local rho)
template <int DIM, class R>
__device__ __forceinline__ R eq_dev(int k, R rho, R drho, const R* u) {
    const R uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if constexpr (DIM == 2) {
        switch (k) {
        case 1: return R(-2) * drho + R(3) * rho * uu;
        case 2: return drho - R(3) * rho * uu;
        case 4: return -rho * u[0];
        case 6: return -rho * u[1];
        case 7: return rho * (u[0] * u[0] - u[1] * u[1]);
        case 8: return rho * u[0] * u[1];
        default: return R(0);
        }
    } else {
        const R pxx = R(3) * u[0] * u[0] - uu, pww = u[1] * u[1] - u[2] * u[2];
        switch (k) {
        case 1: return R(-11) * drho + R(19) * rho * uu;
        case 2: return R(3) * drho - R(5.5) * rho * uu;
        case 4: return R(-2.0 / 3.0) * rho * u[0];
        case 6: return R(-2.0 / 3.0) * rho * u[1];
        case 8: return R(-2.0 / 3.0) * rho * u[2];
        case 9: return rho * pxx;
        case 10: return R(-0.5) * rho * pxx;
        case 11: return rho * pww;
        case 12: return R(-0.5) * rho * pww;
        case 13: return rho * u[0] * u[1];
        case 14: return rho * u[1] * u[2];
        case 15: return rho * u[0] * u[2];
        default: return R(0);
        }
    }
}

// forcing moments M F~ of Eq. (6a) / Eq. (6b); the xy entry of Eq. (6a)
// is u F_y + v F_x
template <int DIM, class R>
__device__ __forceinline__ R force_mom(int k, const R* u, const R* F) {
    const R uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    if constexpr (DIM == 2) {
        switch (k) {
        case 1: return R(6) * uF;
        case 2: return R(-6) * uF;
        case 4: return -F[0];
        case 6: return -F[1];
        case 7: return R(2) * u[0] * F[0] - R(2) * u[1] * F[1];
        case 8: return u[0] * F[1] + u[1] * F[0];
        default: return R(0);
        }
    } else {
        switch (k) {
        case 1: return R(38) * uF;
        case 2: return R(-11) * uF;
        case 4: return R(-2.0 / 3.0) * F[0];
        case 6: return R(-2.0 / 3.0) * F[1];
        case 8: return R(-2.0 / 3.0) * F[2];
        case 9: return R(4) * u[0] * F[0] - R(2) * u[1] * F[1] - R(2) * u[2] * F[2];
        case 10: return R(-2) * u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
        case 11: return R(2) * u[1] * F[1] - R(2) * u[2] * F[2];
        case 12: return -u[1] * F[1] + u[2] * F[2];
        case 13: return u[0] * F[1] + u[1] * F[0];
        case 14: return u[1] * F[2] + u[2] * F[1];
        case 15: return u[0] * F[2] + u[2] * F[0];
        default: return R(0);
        }
    }
}

// Moments, both collisions and the store of one node.  hf/hg hold the
// pre-collision deviations on entry.
// Destinations of the post-collision populations of one node: the tiled
// arrays in global memory (non-temporal stores) or a tile in LDS.
template <class St, int QF, int QG> struct GlobalDst {
    typename St::TF* f;
    typename St::TG* g;
    uint32_t base_f, base_g;
    __device__ GlobalDst(typename St::TF* f_, typename St::TG* g_, uint32_t idx)
        : f(f_), g(g_), base_f(pop_at<QF>(idx, 0)), base_g(pop_at<QG>(idx, 0)) {}
    __device__ void sf(int i, typename St::TF v) const { __builtin_nontemporal_store(v, f + base_f + i * kTile); }
    __device__ void sg(int i, typename St::TG v) const { __builtin_nontemporal_store(v, g + base_g + i * kTile); }
};

template <class St> struct LdsDst {
    typename St::TF* f;
    typename St::TG* g;
    uint32_t n, at;  // plane stride, local node index
    __device__ void sf(int i, typename St::TF v) const { f[i * n + at] = v; }
    __device__ void sg(int i, typename St::TG v) const { g[i * n + at] = v; }
};

// Returns false if the node's density or temperature is not finite.
template <int DIM, class St, class Dst>
__device__ __forceinline__ bool collide_store(typename St::R* hf, typename St::R* hg,
                                              const Coef<typename St::R>& c, const Dst& dst) {
    using R = typename St::R;
    using L = Flow<DIM>;
    using H = Heat<DIM>;
    constexpr int QF = L::Q, QG = H::Q;

    R drho = R(0), j[3] = {R(0), R(0), R(0)}, dT = R(0);
    static_for<0, QF>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        drho += hf[i];
        cmac<L::ex[i]>(j[0], hf[i]);
        cmac<L::ey[i]>(j[1], hf[i]);
        cmac<L::ez[i]>(j[2], hf[i]);
    });
    static_for<0, QG>([&](auto ic) { dT += hg[decltype(ic)::value]; });
    const R rho = R(1) + drho;
    const R T = c.t_base + dT;
    R F[3] = {R(0), R(0), R(0)};
    F[DIM - 1] = rho * c.gbeta * (dT + c.tb_m_t0);  // buoyancy, upward
    const R inv_rho = R(1) / rho;
    R u[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + R(0.5) * F[a]) * inv_rho;

    // flow: dm_k for every row, scaled by 1/|M_k|^2
    R dm[QF];
    static_for<0, QF>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int kind = L::kind[k];
        R d;
        if constexpr (kind == kRho) {
            d = R(0);
        } else if constexpr (kind == kJx || kind == kJy || kind == kJz) {
            d = F[kind - kJx];  // momentum gains exactly F for any rate
        } else {
            R mk = R(0);
            static_for<0, QF>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                cmac<L::M(k, i)>(mk, hf[i]);
            });
            d = -c.s[k] * (mk - eq_dev<DIM>(k, rho, drho, u)) + c.b[k] * force_mom<DIM>(k, u, F);
        }
        dm[k] = d * R(1.0 / row_norm<L>(k));
    });
    static_for<0, QF>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        R acc = hf[i];
        static_for<1, QF>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            cmac<L::M(k, i)>(acc, dm[k]);
        });
        hf[i] = acc;
    });

    // thermal: n_eq = (T, u T, a_T T, 0...) in deviation form
    R dn[QG];
    static_for<0, QG>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int kind = H::kind[k];
        R nk = R(0);
        static_for<0, QG>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            cmac<H::M(k, i)>(nk, hg[i]);
        });
        R d;
        if constexpr (kind == kRho) d = R(0);
        else if constexpr (kind == kJx || kind == kJy || kind == kJz) d = -c.q[k] * (nk - u[kind - kJx] * T);
        else if constexpr (kind == kE) d = -c.q[k] * (nk - c.a_t * dT);
        else d = -c.q[k] * nk;
        dn[k] = d * R(1.0 / row_norm<H>(k));
    });
    static_for<0, QG>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        R acc = hg[i];
        static_for<1, QG>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            cmac<H::M(k, i)>(acc, dn[k]);
        });
        hg[i] = acc;
    });

    // store post-collision populations at the node
    static_for<0, QF>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.sf(i, St::EF::enc(hf[i]));
    });
    static_for<0, QG>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        dst.sg(i, St::EG::enc(hg[i]));
    });
    return isfinite(drho + dT);
}

// ----------------------------------------------------------------- the step
// Sources of the pull.  at(sx, sy, sz) is the index of the node displaced by
// (sx, sy, sz) in {-1, 0, 1}^3 from the current one; lf/lg read a
// population plane there.  In global memory a displacement across a
// periodic face wraps (the offsets are prepared per node); in an LDS tile
// the halo already holds the wrapped neighbours.
template <class St, int QF, int QG> struct GlobalSrc {
    const typename St::TF* f;
    const typename St::TG* g;
    uint32_t idx;
    int32_t oxm, oxp, oym, oyp, ozm, ozp;
    __device__ uint32_t at(int sx, int sy, int sz) const {
        return (uint32_t)((int32_t)idx + (sx < 0 ? oxm : sx > 0 ? oxp : 0) + (sy < 0 ? oym : sy > 0 ? oyp : 0) +
                          (sz < 0 ? ozm : sz > 0 ? ozp : 0));
    }
    __device__ typename St::TF lf(int i, uint32_t node) const { return f[pop_at<QF>(node, i)]; }
    __device__ typename St::TG lg(int i, uint32_t node) const { return g[pop_at<QG>(node, i)]; }
};

template <class St> struct LdsSrc {
    const typename St::TF* f;
    const typename St::TG* g;
    uint32_t n;              // plane stride
    int32_t at0, sy_stride;  // local node index, row stride
    __device__ uint32_t at(int sx, int sy, int) const { return (uint32_t)(at0 + sx + sy * sy_stride); }
    __device__ typename St::TF lf(int i, uint32_t node) const { return f[i * n + node]; }
    __device__ typename St::TG lg(int i, uint32_t node) const { return g[i * n + node]; }
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

template <class St, int QF, int QG>
__device__ __forceinline__ GlobalSrc<St, QF, QG> global_src(const Geometry& g, const Neighbours& n,
                                                            const typename St::TF* f, const typename St::TG* gp,
                                                            uint32_t idx) {
    const int32_t nx = (int32_t)g.nx, sy = nx, sz = nx * (int32_t)g.ny;
    GlobalSrc<St, QF, QG> s;
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
// the node's Dirichlet links goes to `flux` when write_flux is set.
// Returns false if the new rho or T is not finite.
template <int DIM, class St, class Src, class Dst>
__device__ __forceinline__ bool step_node(const Geometry& g, const Coef<typename St::R>& c, const Neighbours& nb,
                                          uint32_t x, uint32_t y, uint32_t z, const Src& src, const Dst& dst,
                                          double* const* flux, bool write_flux) {
    using R = typename St::R;
    using TF = typename St::TF;
    using L = Flow<DIM>;
    using H = Heat<DIM>;
    const uint32_t self = src.at(0, 0, 0);
    R hf[L::Q], hg[H::Q];
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
        const bool out = (ex > 0 && !nb.okxm) || (ex < 0 && !nb.okxp) || (ey > 0 && !nb.okym) ||
                         (ey < 0 && !nb.okyp) || (ez > 0 && !nb.okzm) || (ez < 0 && !nb.okzp);
        TF v = src.lf(i, out ? self : src.at(-ex, -ey, -ez));
        if (out) v = src.lf(L::opp[i], self);  // half-way bounce-back
        hf[i] = St::EF::dec(v);
    });
    static_for<0, H::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int ex = H::ex[i], ey = H::ey[i], ez = H::ez[i];
        const bool out = (ex > 0 && !nb.okxm) || (ex < 0 && !nb.okxp) || (ey > 0 && !nb.okym) ||
                         (ey < 0 && !nb.okyp) || (ez > 0 && !nb.okzm) || (ez < 0 && !nb.okzp);
        R r = St::EG::dec(src.lg(i, out ? self : src.at(-ex, -ey, -ez)));
        if (out) {
            // the wall this link crosses: axis of e_i, the side it comes from
            constexpr int axis = ex != 0 ? 0 : ey != 0 ? 1 : 2;
            constexpr int face = 2 * axis + ((ex + ey + ez) > 0 ? 0 : 1);
            const R back = St::EG::dec(src.lg(H::opp[i], self));
            if (g.dirichlet[face]) {
                r = c.abb[face] - back;  // anti-bounce-back
                if (write_flux) {
                    const uint32_t local = axis == 0 ? y + g.ny * z : axis == 1 ? x + g.nx * z : x + g.nx * y;
                    flux[face][local] = c.abb_d[face] - 2.0 * (double)back;
                }
            } else {
                r = back;  // adiabatic bounce-back
            }
        }
        hg[i] = r;
    });
    return collide_store<DIM, St>(hf, hg, c, dst);
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
    return step_node<DIM, St>(g, c, nb, x, y, z, src, dst, flux, true);
}

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void step_kernel(StepArgs<St> a) {
    const uint32_t idx = logical_block(a.geo.blocks_per_xcd) * kBlock + threadIdx.x;
    if (idx >= a.geo.N) return;
    step_node_global<DIM, St>(a.geo, a.c, a.fsrc, a.gsrc, a.fdst, a.gdst, a.flux, idx);
}

// ------------------------------------------------- two steps per launch (2D)
// Temporal blocking: one block owns an output tile of kTile x TY nodes.
// Step t+1 is computed for the tile and a ring of one node around it (the
// region, RX x RY) from global memory into LDS, in the storage type, so the
// values are exactly those a single step would have written; step t+2 is
// then computed for the tile from LDS and written to global memory.  Global
// traffic per node and two steps is one read and one write of the
// populations instead of two of each.  Region nodes beyond a wall are
// skipped (no tile node pulls from them: their links bounce back), region
// nodes across a periodic face hold the wrapped node.
template <class St> struct Step2Args {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    typename St::TF* fdst;
    typename St::TG* gdst;
    double* flux1[6];  // wall heat flux of step t+1, per face
    double* flux2[6];  // of step t+2
    Geometry geo;
    Coef<typename St::R> c;
    uint32_t tiles_x, tiles;  // tiles per row, in all
    uint32_t tiles_per_xcd;
};

// region coordinate -> domain coordinate, or -1 beyond a wall
__device__ __forceinline__ int32_t region_coord(int32_t v, uint32_t n, int32_t periodic) {
    if (v < 0) v = periodic ? v + (int32_t)n : -1;
    else if (v >= (int32_t)n) v = periodic ? v - (int32_t)n : -1;
    return v < (int32_t)n ? v : -1;
}

template <class St, int TY, int NW>
__global__ __launch_bounds__(64 * NW) void step2_kernel(Step2Args<St> a) {
    using TF = typename St::TF;
    using TG = typename St::TG;
    constexpr int QF = Flow<2>::Q, QG = Heat<2>::Q;
    constexpr int TX = kTile, RX = TX + 2, RY = TY + 2, RN = RX * RY;
    static_assert(2 * RY <= 64, "the halo columns must fit one wavefront");
    __shared__ TF sf[QF * RN];
    __shared__ TG sg[QG * RN];
    const Geometry& g = a.geo;
    const uint32_t tile = logical_block(a.tiles_per_xcd);
    if (tile >= a.tiles) return;  // whole block
    const int32_t x0 = (int32_t)((tile % a.tiles_x) * TX), y0 = (int32_t)((tile / a.tiles_x) * TY);
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);

    // step t+1 on the region: RY rows of the kTile inner columns, then one
    // unit of the two halo columns
    for (int unit = wave; unit <= RY; unit += NW) {
        int lx, ly;
        if (unit < RY) {
            lx = lane + 1, ly = unit;
        } else {
            if (lane >= 2 * RY) continue;
            lx = (lane & 1) ? RX - 1 : 0, ly = lane >> 1;
        }
        const int32_t gx = region_coord(x0 - 1 + lx, g.nx, g.periodic[0]);
        const int32_t gy = region_coord(y0 - 1 + ly, g.ny, g.periodic[1]);
        if (gx < 0 || gy < 0) continue;
        const uint32_t idx = (uint32_t)gx + g.nx * (uint32_t)gy;
        const bool own = lx >= 1 && lx <= TX && ly >= 1 && ly <= TY && x0 - 1 + lx < (int32_t)g.nx &&
                         y0 - 1 + ly < (int32_t)g.ny;
        const Neighbours nb = neighbours(g, (uint32_t)gx, (uint32_t)gy, 0);
        const auto src = global_src<St, QF, QG>(g, nb, a.fsrc, a.gsrc, idx);
        const LdsDst<St> dst{sf, sg, (uint32_t)RN, (uint32_t)(ly * RX + lx)};
        step_node<2, St>(g, a.c, nb, (uint32_t)gx, (uint32_t)gy, 0u, src, dst, a.flux1, own);
    }
    __syncthreads();

    // step t+2 on the tile
    for (int row = wave; row < TY; row += NW) {
        const uint32_t x = (uint32_t)(x0 + lane), y = (uint32_t)(y0 + row);
        if (x >= g.nx || y >= g.ny) continue;
        const uint32_t idx = x + g.nx * y;
        const Neighbours nb = neighbours(g, x, y, 0);
        const LdsSrc<St> src{sf, sg, (uint32_t)RN, (row + 1) * RX + lane + 1, RX};
        const GlobalDst<St, QF, QG> dst(a.fdst, a.gdst, idx);
        step_node<2, St>(g, a.c, nb, x, y, 0u, src, dst, a.flux2, true);
    }
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
    // g_eq - w^T T_b = w^T (T - T_b) + (e.u) T / 2
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    R hf[L::Q], hg[H::Q];
#pragma unroll
    for (int i = 0; i < L::Q; ++i) {
        const double eu = L::ex[i] * u[0] + L::ey[i] * u[1] + L::ez[i] * u[2];
        hf[i] = (R)(L::w[i] * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu)));
    }
    const double tb = (double)a.c.t_base;
#pragma unroll
    for (int i = 0; i < H::Q; ++i) {
        const double eu = H::ex[i] * u[0] + H::ey[i] * u[1] + H::ez[i] * u[2];
        const double wt = i == 0 ? a.w_rest : a.w_move;
        hg[i] = (R)(wt * (T - tb) + 0.5 * eu * T);
    }
    collide_store<DIM, St>(hf, hg, a.c, GlobalDst<St, L::Q, H::Q>(a.fdst, a.gdst, idx));
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
                                                             uint32_t N, uint32_t idx,
                                                             double gbeta, double t_base,
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
    m.rho = 1.0 + drho;
    m.T = t_base + dT;
    double F[3] = {0.0, 0.0, 0.0};
    F[DIM - 1] = m.rho * gbeta * (m.T - t0);
    for (int a = 0; a < 3; ++a) m.u[a] = (j[a] - 0.5 * F[a]) / m.rho;
    m.nonfinite = bad;
    return m;
}

template <class St> struct FieldArgs {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    uint32_t N, n0, cnt;
    double gbeta, t_base, t0;
    double* rho;  // [cnt] or null
    double* u;    // [DIM][cnt] or null
    double* T;    // [cnt] or null
    unsigned long long* nonfinite;  // atomic counter
};

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void fields_kernel(FieldArgs<St> a) {
    const uint32_t k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.cnt) return;
    const auto m = node_moments<DIM, St>(a.fsrc, a.gsrc, a.N, a.n0 + k, a.gbeta, a.t_base, a.t0);
    if (a.rho) a.rho[k] = m.rho;
    if (a.T) a.T[k] = m.T;
    if (a.u)
        for (int d = 0; d < DIM; ++d) a.u[(size_t)d * a.cnt + k] = m.u[d];
    if (m.nonfinite) atomicAdd(a.nonfinite, (unsigned long long)m.nonfinite);
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
    uint32_t N;
    double gbeta, t_base, t0;
    double* partial;  // [gridDim.x][kDiagVals]
};

template <int DIM, class St>
__global__ __launch_bounds__(kBlock) void diag_kernel(DiagArgs<St> a) {
    __shared__ double lds[kBlock / 64];
    double acc[kDiagVals] = {0, 0, 0, 0, 0, 0};
    for (uint32_t idx = blockIdx.x * kBlock + threadIdx.x; idx < a.N; idx += gridDim.x * kBlock) {
        const auto m = node_moments<DIM, St>(a.fsrc, a.gsrc, a.N, idx, a.gbeta, a.t_base, a.t0);
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

__global__ __launch_bounds__(kBlock) void fill_kernel(double* p, size_t n, double v) {
    for (size_t i = blockIdx.x * (size_t)kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        p[i] = v;
}

// per-cavity wall heat flux sums: block (k, b) reduces buffer b of cavity k
struct BatchFaceArgs {
    const double* const* buf;  // [count][12]
    const uint32_t* len;       // [count][12]
    double* out;               // [count][12]
};

__global__ __launch_bounds__(256) void batch_face_sum_kernel(BatchFaceArgs a) {
    __shared__ double lds[256 / 64];
    const size_t b = blockIdx.x;
    const double* p = a.buf[b];
    double acc = 0.0;
    if (p)
        for (uint32_t i = threadIdx.x; i < a.len[b]; i += 256) acc += p[i];
    const double r = block_reduce<256>(acc, AddOp{}, lds);
    if (threadIdx.x == 0) a.out[b] = r;
}

}  // namespace lbm
