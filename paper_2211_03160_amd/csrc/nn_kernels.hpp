// nn_kernels.hpp -- BF16 MFMA kernels of the warm-start network (gfx950).
//
// Activations and gradients are BF16 tensors in NHWC order with a channel
// count that is a multiple of 16; products accumulate in FP32 on the matrix
// cores with gfx950's double-depth instruction v_mfma_f32_16x16x32_bf16.  A
// 3x3 convolution is an implicit GEMM: M = output pixels, N = output
// channels, K = 9 taps x input channels (tap-major), taken 32 at a time.
// Operand layout of the 16x16x32 instruction (lane l of a wavefront):
//   A (16 x 32, rows = M): lane l holds A[l % 16][8 (l / 16) + j], j < 8
//   B (32 x 16, rows = K): lane l holds B[8 (l / 16) + j][l % 16]
//   D (16 x 16 FP32):      lane l holds D[4 (l / 16) + j][l % 16]
// Eight consecutive K values of one lane lie in one tap (channel counts
// are multiples of 8), so each A and B fragment is one 16-byte load; K
// values past 9 x cin (cin = 16: 144 = 4.5 x 32) are zero.  Weights are
// kept as [tap][Cout][Cin].
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lbm {
namespace nn {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // 16 bytes = 8 BF16 values

__device__ __forceinline__ v4f mfma32(v4u a, v4u b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // nearest even
}

struct ConvArgs {
    const uint16_t* x;   // [P][cin], P = n h w
    const uint16_t* wt;  // [9][cout][cin]
    const float* bias;   // [cout] or null
    uint16_t* y;         // [P][cout]
    int32_t n, h, w, cin, cout, relu;
    uint32_t P, ptiles;  // pixels, 16-pixel tiles
};

// One wavefront computes 16 MT pixels x (16 NT) output channels: each K
// step loads MT activation fragments and NT weight fragments and issues
// MT x NT MFMAs (the weight fragments are shared by the MT pixel tiles).
template <int NT, int MT = 1>
__global__ __launch_bounds__(256) void conv3x3_kernel(ConvArgs a) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gw = blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t groups = (uint32_t)a.cout / (16 * NT);
    const uint32_t pgroups = (a.ptiles + MT - 1) / MT;
    if (gw >= pgroups * groups) return;
    const uint32_t pg = gw % pgroups, cg = gw / pgroups;
    const uint32_t m = lane & 15, kg = lane >> 4;
    bool pin[MT];
    int32_t pj[MT], pi[MT], pn[MT];
#pragma unroll
    for (int u = 0; u < MT; ++u) {
        const uint32_t p = (pg * MT + u) * 16 + m;
        pin[u] = p < a.P;
        pj[u] = pin[u] ? (int32_t)(p % a.w) : 0;
        pi[u] = pin[u] ? (int32_t)((p / a.w) % a.h) : 0;
        pn[u] = pin[u] ? (int32_t)(p / ((uint32_t)a.w * a.h)) : 0;
    }
    v4f acc[MT][NT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[u][t] = v4f{0.f, 0.f, 0.f, 0.f};
    const uint32_t K = 9u * (uint32_t)a.cin;
    for (uint32_t k0 = 0; k0 < K; k0 += 32) {
        // this lane's eight K values: tap, first input channel
        const uint32_t k = k0 + 8 * kg;
        const bool kin = k < K;
        const uint32_t tap = kin ? k / (uint32_t)a.cin : 0, ci0 = kin ? k % (uint32_t)a.cin : 0;
        const int32_t dy = (int32_t)tap / 3 - 1, dx = (int32_t)tap % 3 - 1;
        v4u av[MT];
#pragma unroll
        for (int u = 0; u < MT; ++u) {
            const int32_t si = pi[u] + dy, sj = pj[u] + dx;
            const bool ok = kin && pin[u] && si >= 0 && si < a.h && sj >= 0 && sj < a.w;
            av[u] = v4u{0u, 0u, 0u, 0u};
            if (ok) av[u] = *(const v4u*)(a.x + ((size_t)((size_t)pn[u] * a.h + si) * a.w + sj) * a.cin + ci0);
        }
        const uint16_t* wtap = a.wt + (size_t)tap * a.cout * a.cin + ci0;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint32_t co = (cg * NT + t) * 16 + m;
            v4u bv = v4u{0u, 0u, 0u, 0u};
            if (kin) bv = *(const v4u*)(wtap + (size_t)co * a.cin);
#pragma unroll
            for (int u = 0; u < MT; ++u) acc[u][t] = mfma32(av[u], bv, acc[u][t]);
        }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const uint32_t co = (cg * NT + t) * 16 + m;
        const float bb = a.bias ? a.bias[co] : 0.0f;
#pragma unroll
        for (int u = 0; u < MT; ++u)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t q = (pg * MT + u) * 16 + 4 * kg + j;
                if (q < a.P) {
                    float v = acc[u][t][j] + bb;
                    if (a.relu) v = fmaxf(v, 0.0f);
                    a.y[(size_t)q * a.cout + co] = f2bf(v);
                }
            }
    }
}

// flipped, transposed weights for the data gradient:
// wf[tap'][ci][co] = wt[8 - tap'][co][ci]
__global__ void wflip_kernel(const uint16_t* wt, uint16_t* wf, int32_t cin, int32_t cout) {
    const size_t total = (size_t)9 * cin * cout;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int32_t co = (int32_t)(e % cout);
        const int32_t ci = (int32_t)((e / cout) % cin);
        const int32_t tap = (int32_t)(e / ((size_t)cout * cin));
        wf[e] = wt[((size_t)(8 - tap) * cout + co) * cin + ci];
    }
}

struct WGradArgs {
    const uint16_t* x;   // [P][cin]
    const uint16_t* dz;  // [P][cout]
    float* partial;      // [chunks][9][cout][cin]
    int32_t n, h, w, cin, cout;
    uint32_t P, chunk;   // pixels per chunk (multiple of 32)
    uint32_t chunks;
};

// dW[tap][co][ci] = sum_p dz[p][co] x[p shifted by tap][ci]: M = co,
// N = ci (4 tiles per wave), K = pixels of one chunk, 32 per instruction.
// Both operands are stored pixel-major, so a lane's eight consecutive
// pixels of one channel are 2 cout (2 cin) bytes apart: every K step loads
// the 32-pixel tiles with 16-byte loads (8 channels of one pixel per lane)
// and writes them transposed into the wavefront's own LDS area, from which
// each operand fragment is one 16-byte read.  (A wavefront's LDS accesses
// execute in order, so no barrier is needed: the wavefronts of a block
// share nothing.)
constexpr int kWgPad = 40;  // LDS row of 32 pixels plus 8 (spreads the banks of the fragment reads)
struct WgradLds {
    uint16_t a[16][kWgPad];  // dz tile, [co][pixel]
    uint16_t b[64][kWgPad];  // x tile, [ci][pixel]
};
__global__ __launch_bounds__(256) void wgrad_kernel(WGradArgs a) {
    __shared__ WgradLds lds[4];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t gw = blockIdx.x * 4 + wv;
    // input channels in groups of up to four 16-wide tiles per wavefront
    const uint32_t cot = (uint32_t)a.cout / 16, cit = ((uint32_t)a.cin + 63) / 64;
    const uint32_t per_chunk = 9 * cot * cit;
    if (gw >= per_chunk * a.chunks) return;  // whole wavefront
    WgradLds& L = lds[wv];
    const uint32_t chunk = gw / per_chunk, r = gw % per_chunk;
    const uint32_t tap = r / (cot * cit), cb = (r / cit) % cot, ib = r % cit;
    const int rest = a.cin / 16 - (int)ib * 4;
    const int NTc = rest < 4 ? rest : 4;
    const int32_t di = (int32_t)tap / 3 - 1, dj = (int32_t)tap % 3 - 1;
    const uint32_t m = lane & 15, kg = lane >> 4;
    // this lane's share of the tile loads: pixel pl of the step, channels ch8 .. ch8 + 7
    const uint32_t pl = lane >> 1, ch8 = (lane & 1) * 8;
    v4f acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    const uint32_t p_begin = chunk * a.chunk;
    const uint32_t p_end = p_begin + a.chunk < a.P ? p_begin + a.chunk : a.P;
    for (uint32_t p0 = p_begin; p0 < p_end; p0 += 32) {
        const uint32_t p = p0 + pl;
        v4u dv = v4u{0u, 0u, 0u, 0u};
        v4u xv[4] = {v4u{0u, 0u, 0u, 0u}, v4u{0u, 0u, 0u, 0u}, v4u{0u, 0u, 0u, 0u}, v4u{0u, 0u, 0u, 0u}};
        if (p < p_end) {
            dv = *(const v4u*)(a.dz + (size_t)p * a.cout + cb * 16 + ch8);
            const int32_t pj = (int32_t)(p % a.w), pi = (int32_t)((p / a.w) % a.h);
            const int32_t pn = (int32_t)(p / ((uint32_t)a.w * a.h));
            const int32_t si = pi + di, sj = pj + dj;
            if (si >= 0 && si < a.h && sj >= 0 && sj < a.w) {
                const uint16_t* xs = a.x + (size_t)((pn * a.h + si) * a.w + sj) * a.cin + ib * 64 + ch8;
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (t < NTc) xv[t] = *(const v4u*)(xs + t * 16);
            }
        }
        // transposed into LDS: channel-major rows of 32 pixels
        {
            const uint16_t* d = (const uint16_t*)&dv;
#pragma unroll
            for (int j = 0; j < 8; ++j) L.a[ch8 + j][pl] = d[j];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t < NTc) {
                const uint16_t* xx = (const uint16_t*)&xv[t];
#pragma unroll
                for (int j = 0; j < 8; ++j) L.b[t * 16 + ch8 + j][pl] = xx[j];
            }
        }
        const v4u a8 = *(const v4u*)&L.a[m][8 * kg];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (t < NTc) acc[t] = mfma32(a8, *(const v4u*)&L.b[t * 16 + m][8 * kg], acc[t]);
    }
    float* out = a.partial + ((size_t)chunk * 9 + tap) * a.cout * a.cin;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t < NTc) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t co = cb * 16 + 4 * kg + j;
                const uint32_t ci = (ib * 4 + t) * 16 + m;
                out[(size_t)co * a.cin + ci] = acc[t][j];
            }
        }
    }
}

// sum the chunk partials in chunk order: dw[e] = sum_c partial[c][e]
__global__ void sum_chunks_kernel(const float* partial, uint32_t chunks, size_t count, float* dw) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
        float s = 0.0f;
        for (uint32_t c = 0; c < chunks; ++c) s += partial[(size_t)c * count + e];
        dw[e] = s;
    }
}

// db[co] = sum_p dz[p][co] in two passes with a fixed reduction order.
// Pass 1: block c sums pixels [c per, (c + 1) per) of every channel into
// partial[c][co]: thread t takes channels 8 (t % G) .. + 7 (G = cout / 8
// groups, one 16-byte load) of every R-th pixel (R = 256 / G rows side by
// side, so a row is one contiguous read), then the R row sums are added in
// order.  Pass 2 is bias_sum_kernel over the blocks.
__global__ __launch_bounds__(256) void bias_partial_kernel(const uint16_t* dz, uint32_t P, int32_t cout,
                                                           uint32_t per, float* partial) {
    __shared__ float lds[256 * 8];
    const uint32_t G = (uint32_t)cout / 8, R = 256u / G;
    const uint32_t t = threadIdx.x, grp = t % G, row = t / G;
    const uint32_t p0 = blockIdx.x * per, p1 = p0 + per < P ? p0 + per : P;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (row < R) {
        for (uint32_t p = p0 + row; p < p1; p += R) {
            const v4u v = *(const v4u*)(dz + (size_t)p * cout + grp * 8);
            const uint16_t* h = (const uint16_t*)&v;
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j] += bf2f(h[j]);
        }
    }
    if (row < R) {  // (256 % G threads beyond the last row hold nothing)
#pragma unroll
        for (int j = 0; j < 8; ++j) lds[row * (uint32_t)cout + grp * 8 + j] = s[j];
    }
    __syncthreads();
    if (t < (uint32_t)cout) {
        float v = 0.0f;
        for (uint32_t k = 0; k < R; ++k) v += lds[k * (uint32_t)cout + t];
        partial[(size_t)blockIdx.x * cout + t] = v;
    }
}

// Pass 2 of the bias gradient: db[co] = sum over the nb partial sums of
// channel co, one block per channel: thread t adds partials t, t + 256, ...
// in order, then the 256 sums are added pairwise in a fixed tree.
__global__ __launch_bounds__(256) void bias_sum_kernel(const float* partial, uint32_t nb, int32_t cout, float* db) {
    __shared__ float lds[256];
    const uint32_t co = blockIdx.x, t = threadIdx.x;
    float s = 0.0f;
    for (uint32_t b = t; b < nb; b += 256) s += partial[(size_t)b * cout + co];
    lds[t] = s;
    __syncthreads();
    for (uint32_t o = 128; o > 0; o >>= 1) {
        if (t < o) lds[t] += lds[t + o];
        __syncthreads();
    }
    if (t == 0) db[co] = lds[0];
}

__global__ void relu_backward_kernel(const uint16_t* y, const uint16_t* dy, uint16_t* dz, size_t count) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        dz[e] = bf2f(y[e]) > 0.0f ? dy[e] : (uint16_t)0;
}

// x [n][h][w][c] -> y [n][h/2][w/2][c], 2x2 means
__global__ void avgpool2_kernel(const uint16_t* x, uint16_t* y, int32_t n, int32_t h, int32_t w, int32_t c) {
    const size_t total = (size_t)n * (h / 2) * (w / 2) * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int32_t ch = (int32_t)(e % c);
        const size_t q = e / c;
        const int32_t j = (int32_t)(q % (w / 2)), i = (int32_t)((q / (w / 2)) % (h / 2));
        const int32_t b = (int32_t)(q / ((size_t)(w / 2) * (h / 2)));
        const size_t base = (((size_t)b * h + 2 * i) * w + 2 * j) * c + ch;
        const float s = bf2f(x[base]) + bf2f(x[base + c]) + bf2f(x[base + (size_t)w * c]) +
                        bf2f(x[base + (size_t)w * c + c]);
        y[e] = f2bf(0.25f * s);
    }
}

// gradient of avgpool2: dx[n][h][w][c] = dy[n][h/2][w/2][c] / 4
__global__ void avgpool2_backward_kernel(const uint16_t* dy, uint16_t* dx, int32_t n, int32_t h, int32_t w, int32_t c) {
    const size_t total = (size_t)n * h * w * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int32_t ch = (int32_t)(e % c);
        const size_t q = e / c;
        const int32_t j = (int32_t)(q % w), i = (int32_t)((q / w) % h), b = (int32_t)(q / ((size_t)w * h));
        dx[e] = f2bf(0.25f * bf2f(dy[(((size_t)b * (h / 2) + i / 2) * (w / 2) + j / 2) * c + ch]));
    }
}

// nearest upsampling x [n][h][w][c] -> y [n][2h][2w][c]
__global__ void upsample2_kernel(const uint16_t* x, uint16_t* y, int32_t n, int32_t h, int32_t w, int32_t c) {
    const size_t total = (size_t)n * 4 * h * w * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int32_t ch = (int32_t)(e % c);
        const size_t q = e / c;
        const int32_t j = (int32_t)(q % (2 * w)), i = (int32_t)((q / (2 * w)) % (2 * h));
        const int32_t b = (int32_t)(q / ((size_t)4 * w * h));
        y[e] = x[(((size_t)b * h + i / 2) * w + j / 2) * c + ch];
    }
}

// gradient of upsample2: dx[n][h][w][c] = sum of the 2x2 block of dy
__global__ void upsample2_backward_kernel(const uint16_t* dy, uint16_t* dx, int32_t n, int32_t h, int32_t w, int32_t c) {
    const size_t total = (size_t)n * h * w * c;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int32_t ch = (int32_t)(e % c);
        const size_t q = e / c;
        const int32_t j = (int32_t)(q % w), i = (int32_t)((q / w) % h), b = (int32_t)(q / ((size_t)w * h));
        const size_t base = (((size_t)b * 2 * h + 2 * i) * 2 * w + 2 * j) * c + ch;
        const float s = bf2f(dy[base]) + bf2f(dy[base + c]) + bf2f(dy[base + (size_t)2 * w * c]) +
                        bf2f(dy[base + (size_t)2 * w * c + c]);
        dx[e] = f2bf(s);
    }
}

// dst[p][doff + k] (+)= src[p][soff + k] for k < cc
__global__ void copy_channels_kernel(const uint16_t* src, int32_t cs, int32_t soff, uint16_t* dst, int32_t cd,
                                     int32_t doff, int32_t cc, size_t pixels, int32_t accumulate) {
    const size_t total = pixels * cc;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / cc;
        const int32_t k = (int32_t)(e % cc);
        const uint16_t v = src[p * cs + soff + k];
        uint16_t& d = dst[p * cd + doff + k];
        d = accumulate ? f2bf(bf2f(d) + bf2f(v)) : v;
    }
}

// masked MSE over the first `used` channels: per-block partial sums of
// mask (y - t)^2, and dy = 2 mask (y - t) / count (BF16)
__global__ __launch_bounds__(256) void mse_kernel(const uint16_t* y, int32_t cy, const float* target,
                                                  const float* mask, size_t pixels, int32_t used, float inv_count,
                                                  uint16_t* dy, float* partial) {
    __shared__ float lds[256];
    float s = 0.0f;
    const size_t total = pixels * cy;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t p = e / cy;
        const int32_t k = (int32_t)(e % cy);
        float g = 0.0f;
        if (k < used) {
            const float mk = mask[p * used + k];
            const float d = (bf2f(y[e]) - target[p * used + k]) * mk;
            s += d * d;
            g = 2.0f * d * inv_count;
        }
        if (dy) dy[e] = f2bf(g);
    }
    lds[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = lds[0];
}

__global__ void sum_partials_kernel(const float* partial, int32_t n, float scale, float* out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float s = 0.0f;
        for (int32_t i = 0; i < n; ++i) s += partial[i];
        out[0] = s * scale;
    }
}

// Adam (Kingma & Ba, 2015) on FP32 master weights; also refreshes the
// BF16 copy used by the kernels
__global__ void adam_kernel(float* w, const float* g, float* m, float* v, size_t count, float lr, float b1, float b2,
                            float eps, float c1, float c2, uint16_t* wbf) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[e];
        const float mi = b1 * m[e] + (1.0f - b1) * gi;
        const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[e] = wi;
        if (wbf) wbf[e] = f2bf(wi);
    }
}

__global__ void f32_to_bf16_kernel(const float* src, uint16_t* dst, size_t count) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        dst[e] = f2bf(src[e]);
}

__global__ void bf16_to_f32_kernel(const uint16_t* src, float* dst, size_t count) {
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        dst[e] = bf2f(src[e]);
}

}  // namespace nn
}  // namespace lbm
