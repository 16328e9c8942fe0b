// stream3d.hpp -- two time steps per launch in 3D (D3Q19 + D3Q7).
//
// A one-step launch reads and writes every population once per step, so
// at 208 B per FP32 lattice update it is pinned to the HBM ceiling.  Here a
// block of 512 threads owns a 32 x 16 tile of (x, y) columns, one node per
// thread, and walks along z through a segment of planes, advancing each
// node two steps:
//   step 1 at plane q: the pull gather from global memory (the one-step
//     kernel's sources and wall rules), both collisions; the populations
//     that the second step pulls across the tile (those with a nonzero x
//     or y velocity: 16 of D3Q19, 4 of D3Q7) go to a ring of three LDS
//     planes, the others (rest and +/-z) to a ring of three register planes
//     of the thread's own column;
//   step 2 at plane p: the pull from the rings (planes p - 1, p, p + 1 of
//     step 1, x/y neighbours from LDS), both collisions, the store to global
//     memory.
// Step 1 is valid on the whole tile (its sources are in global memory),
// step 2 on the 30 x 14 interior, which the block stores; tiles overlap by
// two columns and two rows.  Every node update is step_node on the same
// (storage-rounded) values as a one-step launch, so results are bitwise
// those of single steps.  The loads of step 1 for the next plane are
// issued right after step 1 of this one and are in flight through the next
// plane's step 2.  The register ring rotates by moves and the LDS ring by a
// uniform slot counter, so the plane loop holds one instance of each step;
// blocks whose tile and z segment keep one node clear of every wall run a
// copy of the loop without wall rules.
#pragma once

namespace lbm {

constexpr int kT3X = 32, kT3Y = 16;               // tile of a block, one node per thread
constexpr int kT3Threads = kT3X * kT3Y;           // 512 threads, 8 wavefronts
constexpr int kT3OutX = kT3X - 2, kT3OutY = kT3Y - 2;  // nodes a tile stores

// populations that move in x or y (pulled from another column of the tile)
template <class L> constexpr bool crosses_xy(int i) { return L::ex[i] != 0 || L::ey[i] != 0; }
template <class L> constexpr int cross_count() {
    int n = 0;
    for (int k = 0; k < L::Q; ++k) n += crosses_xy<L>(k);
    return n;
}
// index of population i among those of its kind (crossing or own-column)
template <class L> constexpr int ring_index(int i) {
    int n = 0;
    for (int k = 0; k < i; ++k) n += crosses_xy<L>(k) == crosses_xy<L>(i);
    return n;
}
static_assert(cross_count<Flow<3>>() == 16 && cross_count<Heat<3>>() == 4, "D3Q19 / D3Q7 crossing populations");
constexpr int kT3Cross = 16 + 4;  // per node and plane in LDS
constexpr int kT3Own = 3 + 3;     // per node and plane in registers

template <class St> struct Stream3Args {
    const typename St::TF* fsrc;
    const typename St::TG* gsrc;
    typename St::TF* fdst;
    typename St::TG* gdst;
    double* flux;              // wall heat flux area: two slots, per-face arrays back to back
    uint32_t slot1, slot2;     // first element of the slot of the first and of the second step
    uint32_t flux_bytes;       // size of the flux area
    Geometry geo;
    Coef<typename St::R> c;
    uint32_t tiles_x, tiles_y, segs, seg_planes;
    uint32_t blocks_per_xcd;
};

// Wall heat flux of one node into its face's array of one slot (faces back
// to back, each of the node count of its plane), through a buffer store
// issued when some lane of the wavefront is on a Dirichlet link (a
// wavefront-uniform branch; the other lanes store to the dropped offset).
struct BufFlux3 {
    __amdgpu_buffer_rsrc_t r;
    uint32_t slot, bytes;
    bool on;
    template <int face> __device__ void put(const Geometry& g, uint32_t local, double v, bool wall) const {
        const uint32_t ax = g.ny * g.nz, ay = g.nx * g.nz, az = g.nx * g.ny;
        const uint32_t start = face == 0 ? 0u : face == 1 ? ax : face == 2 ? 2 * ax : face == 3 ? 2 * ax + ay
                             : face == 4 ? 2 * ax + 2 * ay : 2 * ax + 2 * ay + az;
        const bool mine = on && wall;
        if (__builtin_amdgcn_ballot_w64(mine))
            buffer_store(v, r, mine ? (slot + start + local) * (uint32_t)sizeof(double) : bytes);
    }
};

// Step-1 sources gathered ahead: f[i], g[i] already hold what the pull
// reads (the neighbour's population, or the node's own opposite one across
// a wall).
template <class St, int QF, int QG> struct PreSrc {
    using R = typename St::R;
    const R (&f)[QF];
    const R (&g)[QG];
    template <int i, int ex, int ey, int ez, int o> __device__ R pull_f(bool) const { return f[i]; }
    template <int i, int ex, int ey, int ez, int o> __device__ R pull_g(bool) const { return g[i]; }
};

// direction index of an in-plane displacement (dx, dy) in {-1, 0, 1}^2
constexpr int dir9(int dx, int dy) { return (dx + 1) * 3 + (dy + 1); }

// Step-2 sources: planes p - 1, p, p + 1 of step 1 (LDS ring offsets om, oz,
// op in elements) in LDS (crossing populations, at the tile position of
// the source node: nbr[dir9(-ex, -ey)], clamped into the tile for halo
// lanes, whose results are never stored) and in registers (own-column
// populations).
template <class St> struct RingSrc {
    using R = typename St::R;
    const R* lds;
    const R (&own_m)[kT3Own];
    const R (&own_z)[kT3Own];
    const R (&own_p)[kT3Own];
    const int (&nbr)[9];
    int om, oz, op;
    template <class L, int base, int i, int ex, int ey, int ez, int o> __device__ R pull(bool out) const {
        // across a wall: the node's own opposite population at plane p
        if (out) {
            if constexpr (crosses_xy<L>(o)) return lds[oz + (base + ring_index<L>(o)) * kT3Threads + nbr[dir9(0, 0)]];
            else return own_z[(base == 0 ? 0 : 3) + ring_index<L>(o)];
        }
        if constexpr (crosses_xy<L>(i)) {
            const int off = ez > 0 ? om : ez < 0 ? op : oz;
            return lds[off + (base + ring_index<L>(i)) * kT3Threads + nbr[dir9(-ex, -ey)]];
        } else {
            const R(&r)[kT3Own] = ez > 0 ? own_m : ez < 0 ? own_p : own_z;
            return r[(base == 0 ? 0 : 3) + ring_index<L>(i)];
        }
    }
    template <int i, int ex, int ey, int ez, int o> __device__ R pull_f(bool out) const {
        return pull<Flow<3>, 0, i, ex, ey, ez, o>(out);
    }
    template <int i, int ex, int ey, int ez, int o> __device__ R pull_g(bool out) const {
        return pull<Heat<3>, 16, i, ex, ey, ez, o>(out);
    }
};

// Step-1 results of one node into the rings (decoded after rounding through
// the storage type: what a single step would store and reload).
template <class St> struct RingDst {
    using R = typename St::R;
    R* lds;  // slot base + the node's tile position
    R (&own)[kT3Own];
    __device__ void sf(int i, typename St::TF v) const {
        const R d = St::EF::dec(v);
        if (crosses_xy<Flow<3>>(i)) lds[ring_index<Flow<3>>(i) * kT3Threads] = d;
        else own[ring_index<Flow<3>>(i)] = d;
    }
    __device__ void sg(int i, typename St::TG v) const {
        const R d = St::EG::dec(v);
        if (crosses_xy<Heat<3>>(i)) lds[(16 + ring_index<Heat<3>>(i)) * kT3Threads] = d;
        else own[3 + ring_index<Heat<3>>(i)] = d;
    }
};

// One block's z segment, with (Walls) or without wall rules.
template <class St, bool Walls>
__device__ __forceinline__ void stream3_segment(const Stream3Args<St>& a, typename St::R* lds, uint32_t bx,
                                                uint32_t by, int32_t z0, int32_t z1) {
    using R = typename St::R;
    using L = Flow<3>;
    using H = Heat<3>;
    constexpr int QF = L::Q, QG = H::Q;
    const Geometry& g = a.geo;
    const int tx = (int)(threadIdx.x % kT3X), ty = (int)(threadIdx.x / kT3X);
    // this thread's column, unwrapped, and its domain coordinates (a
    // stand-in inside the domain for columns beyond a wall)
    const int32_t cx = (int32_t)(bx * kT3OutX) - 1 + tx, cy = (int32_t)(by * kT3OutY) - 1 + ty;
    const int32_t rx = region_coord(cx, g.nx, g.periodic[0]), ry = region_coord(cy, g.ny, g.periodic[1]);
    const uint32_t x = (uint32_t)(rx >= 0 ? rx : min(max(cx, 0), (int32_t)g.nx - 1));
    const uint32_t y = (uint32_t)(ry >= 0 ? ry : min(max(cy, 0), (int32_t)g.ny - 1));
    const bool own_xy = tx >= 1 && tx <= kT3X - 2 && ty >= 1 && ty <= kT3Y - 2 && cx < (int32_t)g.nx &&
                        cy < (int32_t)g.ny;
    // tile positions of the in-plane neighbours, clamped into the tile
    int nbr[9];
    static_for<0, 9>([&](auto dc) {
        constexpr int d = decltype(dc)::value, dx = d / 3 - 1, dy = d % 3 - 1;
        nbr[d] = min(max(ty + dy, 0), kT3Y - 1) * kT3X + min(max(tx + dx, 0), kT3X - 1);
    });
    // the wavefront's first row (y of lane 0) for the row-based store resources
    const int wy = (int)__builtin_amdgcn_readfirstlane(ty);
    const int32_t wcy = (int32_t)(by * kT3OutY) - 1 + wy;
    const uint32_t wrow = (uint32_t)min(max(wcy, 0), (int32_t)g.ny - 1);
    const __amdgpu_buffer_rsrc_t rflux = buffer_rsrc(a.flux, a.flux_bytes);
    constexpr int kSlot = kT3Cross * kT3Threads;  // elements of one LDS ring slot

    R rm[kT3Own] = {}, rz[kT3Own] = {}, rp[kT3Own] = {}, rn[kT3Own];  // register ring: planes p-1, p, p+1, new
    R pf[QF], pg[QG];  // step-1 sources of the next plane, gathered ahead

    // the plane of step 1 for ring position q (relative to z0 - 1), wrapped
    // on a periodic z axis, -1 if it lies beyond a wall or is not needed.
    // Without wall rules every plane the segment needs exists (inside the
    // domain, or wrapped), and positions past the last one it needs repeat
    // that plane: the loop then has no branch around its loads (which would
    // make the compiler wait for every load in flight at the join), and
    // what those repeats compute is never read.
    auto step1_plane = [&](int32_t q) __attribute__((always_inline)) {
        const int32_t zq = z0 - 1 + q;
        if constexpr (!Walls) return region_coord(min(zq, z1), g.nz, g.periodic[2]);
        if (zq > z1) return -1;
        return region_coord(zq, g.nz, g.periodic[2]);
    };
    // gather the step-1 sources of plane zq (the pull with the wall rules)
    // into df, dg
    auto gather = [&](int32_t zq, R(&df)[QF], R(&dg)[QG]) __attribute__((always_inline)) {
        const Neighbours nb = neighbours(g, x, y, (uint32_t)zq);
        const uint32_t idx = x + g.nx * (y + g.ny * (uint32_t)zq);
        const auto src = global_src<St, QF, QG, false, true>(g, nb, a.fsrc, a.gsrc, idx);
        static_for<0, QF>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int ex = L::ex[i], ey = L::ey[i], ez = L::ez[i];
            const bool out = Walls && ((ex > 0 && !nb.okxm) || (ex < 0 && !nb.okxp) || (ey > 0 && !nb.okym) ||
                                       (ey < 0 && !nb.okyp) || (ez > 0 && !nb.okzm) || (ez < 0 && !nb.okzp));
            df[i] = src.template pull_f<i, ex, ey, ez, L::opp[i]>(out);
        });
        static_for<0, QG>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int ex = H::ex[i], ey = H::ey[i], ez = H::ez[i];
            const bool out = Walls && ((ex > 0 && !nb.okxm) || (ex < 0 && !nb.okxp) || (ey > 0 && !nb.okym) ||
                                       (ey < 0 && !nb.okyp) || (ez > 0 && !nb.okzm) || (ez < 0 && !nb.okzp));
            dg[i] = src.template pull_g<i, ex, ey, ez, H::opp[i]>(out);
        });
    };
    // step 1 of plane zq from the gathered sources pf, pg into LDS slot s and rn
    auto step1 = [&](int32_t zq, int s, const R (&pf)[QF], const R (&pg)[QG]) __attribute__((always_inline)) {
        const Neighbours nb = neighbours(g, x, y, (uint32_t)zq);
        const bool own = own_xy && zq >= z0 && zq < z1;
        step_node<3, St, Walls>(g, a.c, nb, x, y, (uint32_t)zq, PreSrc<St, QF, QG>{pf, pg},
                                RingDst<St>{lds + s * kSlot + nbr[dir9(0, 0)], rn},
                                BufFlux3{rflux, a.slot1, a.flux_bytes, own});
    };
    auto rotate = [&]() __attribute__((always_inline)) {
        static_for<0, kT3Own>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            rm[i] = rz[i];
            rz[i] = rp[i];
            rp[i] = rn[i];
        });
    };
    // step 2 of plane p from LDS slots sm, sz, sp (planes p - 1, p, p + 1)
    // into registers (ef, eg, encoded); store2 writes them to global memory
    // for the nodes the tile owns.
    typename St::TF ef[QF];
    typename St::TG eg[QG];
    auto step2 = [&](int32_t p, int sm, int sz, int sp, typename St::TF (&ef)[QF],
                     typename St::TG (&eg)[QG]) __attribute__((always_inline)) {
        const Neighbours nb = neighbours(g, x, y, (uint32_t)p);
        const RingSrc<St> src{lds, rm, rz, rp, nbr, sm * kSlot, sz * kSlot, sp * kSlot};
        step_node<3, St, Walls>(g, a.c, nb, x, y, (uint32_t)p, src, EncDst<St, QF, QG>{ef, eg},
                                BufFlux3{rflux, a.slot2, a.flux_bytes, own_xy});
    };
    auto store2 = [&](int32_t p, const typename St::TF (&ef)[QF], const typename St::TG (&eg)[QG])
                      __attribute__((always_inline)) {
        // through a buffer resource based at the first storage tile of the
        // wavefront's rows (a wavefront-uniform base; its two rows and
        // their halo span at most 2 nx + 64 nodes)
        const uint32_t row0 = g.nx * (wrow + g.ny * (uint32_t)p);
        const uint32_t t0 = row0 / kTile, tiles = (2 * g.nx + kTile - 1) / kTile + 2;
        const uint32_t fb = tiles * (uint32_t)(QF * kTile * sizeof(typename St::TF));
        const uint32_t gb = tiles * (uint32_t)(QG * kTile * sizeof(typename St::TG));
        const uint32_t idx = x + g.nx * (y + g.ny * (uint32_t)p);
        const OwnedBufDst<St, QF, QG, true> dst(buffer_rsrc(a.fdst + (size_t)t0 * (QF * kTile), fb),
                                                buffer_rsrc(a.gdst + (size_t)t0 * (QG * kTile), gb), fb, gb,
                                                idx - t0 * kTile, own_xy);
        static_for<0, QF>([&](auto ic) { dst.sf(decltype(ic)::value, ef[decltype(ic)::value]); });
        static_for<0, QG>([&](auto ic) { dst.sg(decltype(ic)::value, eg[decltype(ic)::value]); });
    };

    // prologue: step 1 of ring positions 0, 1, 2 (planes z0 - 1, z0, z0 + 1)
    // into LDS slots 0, 1, 2; afterwards rm, rz, rp hold them, and the
    // sources of position 3 are on their way
    for (int q = 0; q < 3; ++q) {
        const int32_t zq = step1_plane(q);
        if (!Walls || zq >= 0) {
            gather(zq, pf, pg);
            step1(zq, q, pf, pg);
        }
        rotate();
    }
    int32_t zn = step1_plane(3);
    if (!Walls || zn >= 0) gather(zn, pf, pg);
    __syncthreads();
    // Plane p = z0 + r needs ring positions r, r + 1, r + 2 (LDS slots s0,
    // s0 + 1, s0 + 2 mod 3 with s0 = r mod 3); then step 1 of position
    // r + 3 (plane p + 2, its sources gathered one iteration earlier) goes
    // into slot s0, which step 2 has just read, and the sources of position
    // r + 4 are loaded, to be used after the next plane's step 2.  Step 2's
    // stores are issued after the barrier, in front of step 1's arithmetic
    // (measured: 5 % faster than before the barrier, 7 % faster than after
    // step 1).  (Keeping a second register set so that the loads could be
    // issued before step 1 measured 7 % slower: more registers, no gain in
    // latency.)
    int s0 = 0;
    const int32_t planes = z1 - z0;
    for (int32_t r = 0; r < planes; ++r) {
        const int s1 = s0 == 2 ? 0 : s0 + 1, s2 = s1 == 2 ? 0 : s1 + 1;
        step2(z0 + r, s0, s1, s2, ef, eg);
        __syncthreads();
        store2(z0 + r, ef, eg);
        if (!Walls || zn >= 0) step1(zn, s0, pf, pg);
        const int32_t zn2 = step1_plane(r + 4);
        if (!Walls || zn2 >= 0) gather(zn2, pf, pg);
        rotate();
        zn = zn2;
        __syncthreads();
        s0 = s1;
    }
}

template <class St>
__global__ __launch_bounds__(kT3Threads) __attribute__((amdgpu_waves_per_eu(2)))
void stream3_kernel(Stream3Args<St> a) {
    __shared__ typename St::R lds[3 * kT3Cross * kT3Threads];
    const Geometry& g = a.geo;
    const uint32_t blk = logical_block(a.blocks_per_xcd);
    if (blk >= a.tiles_x * a.tiles_y * a.segs) return;  // whole block
    const uint32_t bx = blk % a.tiles_x, by = (blk / a.tiles_x) % a.tiles_y, seg = blk / (a.tiles_x * a.tiles_y);
    const int32_t z0 = (int32_t)(seg * a.seg_planes);
    const int32_t z1 = min(z0 + (int32_t)a.seg_planes, (int32_t)g.nz);
    // Every update that feeds a stored result lies in the tile's columns
    // bx*30 - 1 .. bx*30 + 30 and rows by*14 - 1 .. by*14 + 14 (step 1; step
    // 2 inside them) and in planes z0 - 1 .. z1.  When all of those nodes
    // are at least one node from every non-periodic wall, no link of theirs
    // crosses a wall and the segment runs without wall rules.
    const int32_t xa = (int32_t)(bx * kT3OutX) - 1, ya = (int32_t)(by * kT3OutY) - 1;
    const bool inner_x = g.periodic[0] || (xa >= 1 && xa + kT3X - 1 <= (int32_t)g.nx - 2);
    const bool inner_y = g.periodic[1] || (ya >= 1 && ya + kT3Y - 1 <= (int32_t)g.ny - 2);
    const bool inner_z = g.periodic[2] || (z0 - 1 >= 1 && z1 <= (int32_t)g.nz - 2);
    if (inner_x && inner_y && inner_z)
        stream3_segment<St, false>(a, lds, bx, by, z0, z1);
    else
        stream3_segment<St, true>(a, lds, bx, by, z0, z1);
}

}  // namespace lbm
