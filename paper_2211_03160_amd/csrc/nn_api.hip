// nn_api.hip -- host side of include/lbm_nn.h: shape checks and launches of
// the BF16 MFMA network kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "../../include/lbm_nn.h"
#include "nn_kernels.hpp"

using namespace lbm::nn;

namespace {

thread_local char g_nn_err[512] = "";

lbm_status nn_fail(lbm_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_nn_err, sizeof(g_nn_err), fmt, ap);
    va_end(ap);
    return st;
}

lbm_status launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return nn_fail(LBM_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return LBM_OK;
}

unsigned grid1(size_t n, unsigned bs = 256, unsigned cap = 65536) {
    const size_t g = (n + bs - 1) / bs;
    return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

bool pos(int32_t v) { return v > 0; }

}  // namespace

extern "C" {

const char* lbm_nn_last_error(void) { return g_nn_err; }

lbm_status lbm_nn_conv3x3(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t cin, const uint16_t* wt,
                          const float* bias, int32_t cout, int32_t relu, uint16_t* y, void* stream) {
    if (!x || !wt || !y) return nn_fail(LBM_E_INVALID, "conv3x3: null tensor");
    if (!pos(n) || !pos(h) || !pos(w) || !pos(cin) || !pos(cout) || cin % 16 || cout % 16)
        return nn_fail(LBM_E_INVALID, "conv3x3: bad shape n=%d h=%d w=%d cin=%d cout=%d", n, h, w, cin, cout);
    const double P = (double)n * h * w;
    if (P * (cin > cout ? cin : cout) > 4.0e9) return nn_fail(LBM_E_INVALID, "conv3x3: tensor too large");
    ConvArgs a{x, wt, bias, y, n, h, w, cin, cout, relu, (uint32_t)P, (uint32_t)((P + 15) / 16)};
    const int NT = cout % 64 == 0 ? 4 : cout % 32 == 0 ? 2 : 1;
    // pixel tiles per wavefront: as many as keep at least 4096 wavefronts
    // (16 per compute unit) in the launch
    const size_t waves1 = (size_t)a.ptiles * (cout / (16 * NT));
    const int MT = waves1 >= 4 * 4096 ? 4 : waves1 >= 2 * 4096 ? 2 : 1;
    const size_t waves = ((size_t)a.ptiles + MT - 1) / MT * (cout / (16 * NT));
    const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
    hipStream_t s = (hipStream_t)stream;
    auto go = [&](auto ntc, auto mtc) {
        hipLaunchKernelGGL((conv3x3_kernel<decltype(ntc)::value, decltype(mtc)::value>), grid, block, 0, s, a);
    };
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I4 = std::integral_constant<int, 4>;
    auto by_mt = [&](auto ntc) {
        if (MT == 4) go(ntc, I4{});
        else if (MT == 2) go(ntc, I2{});
        else go(ntc, I1{});
    };
    if (NT == 4) by_mt(I4{});
    else if (NT == 2) by_mt(I2{});
    else by_mt(I1{});
    return launched("conv3x3");
}

lbm_status lbm_nn_conv3x3_flip(const uint16_t* wt, int32_t cin, int32_t cout, uint16_t* wf, void* stream) {
    if (!wt || !wf || !pos(cin) || !pos(cout)) return nn_fail(LBM_E_INVALID, "conv3x3_flip: bad arguments");
    const size_t total = (size_t)9 * cin * cout;
    hipLaunchKernelGGL(wflip_kernel, dim3(grid1(total)), dim3(256), 0, (hipStream_t)stream, wt, wf, cin, cout);
    return launched("conv3x3_flip");
}

lbm_status lbm_nn_conv3x3_wgrad(const uint16_t* x, const uint16_t* dz, int32_t n, int32_t h, int32_t w,
                                int32_t cin, int32_t cout, float* partial, int32_t chunks, float* dw, float* db,
                                void* stream) {
    if (!x || !dz || !partial || !dw) return nn_fail(LBM_E_INVALID, "conv3x3_wgrad: null tensor");
    if (!pos(n) || !pos(h) || !pos(w) || !pos(cin) || !pos(cout) || cin % 16 || cout % 16 || chunks < 1 ||
        chunks > 4096)
        return nn_fail(LBM_E_INVALID, "conv3x3_wgrad: bad shape");
    const uint32_t P = (uint32_t)n * h * w;
    uint32_t per = (P + chunks - 1) / chunks;
    per = (per + 31) / 32 * 32;  // whole 32-pixel steps of the MFMA
    const uint32_t used = (P + per - 1) / per;  // chunks that hold pixels
    WGradArgs a{x, dz, partial, n, h, w, cin, cout, P, per, used};
    const size_t waves = (size_t)used * 9 * (cout / 16) * ((cin + 63) / 64);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(wgrad_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, a);
    lbm_status st = launched("conv3x3_wgrad");
    if (st) return st;
    const size_t count = (size_t)9 * cout * cin;
    hipLaunchKernelGGL(sum_chunks_kernel, dim3(grid1(count)), dim3(256), 0, s, (const float*)partial, used, count, dw);
    if ((st = launched("conv3x3_wgrad sum"))) return st;
    if (db) {
        // the partial buffer is free again (stream order): bias sums of the
        // same pixel chunks, then added in chunk order
        // ranges of about 512 pixels (enough blocks to fill the GPU), at most
        // as many partial sums as the scratch holds (9 cin >= 144 per chunk)
        if (cout > 256) return nn_fail(LBM_E_INVALID, "conv3x3_wgrad: bias gradient needs cout <= 256");
        const uint32_t nb_want = std::min<uint32_t>((P + 511) / 512, 144u * used);
        const uint32_t per_b = (P + nb_want - 1) / nb_want, nb = (P + per_b - 1) / per_b;
        hipLaunchKernelGGL(bias_partial_kernel, dim3(nb), dim3(256), 0, s, dz, P, cout, per_b, partial);
        if ((st = launched("conv3x3_wgrad bias"))) return st;
        hipLaunchKernelGGL(bias_sum_kernel, dim3((unsigned)cout), dim3(256), 0, s, (const float*)partial, nb, cout, db);
        if ((st = launched("conv3x3_wgrad bias sum"))) return st;
    }
    return LBM_OK;
}

lbm_status lbm_nn_relu_backward(const uint16_t* y, const uint16_t* dy, uint16_t* dz, int64_t count, void* stream) {
    if (!y || !dy || !dz || count < 0) return nn_fail(LBM_E_INVALID, "relu_backward: bad arguments");
    hipLaunchKernelGGL(relu_backward_kernel, dim3(grid1(count)), dim3(256), 0, (hipStream_t)stream, y, dy, dz,
                       (size_t)count);
    return launched("relu_backward");
}

lbm_status lbm_nn_avgpool2(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t c, uint16_t* y,
                           void* stream) {
    if (!x || !y || !pos(n) || !pos(h) || !pos(w) || !pos(c) || h % 2 || w % 2)
        return nn_fail(LBM_E_INVALID, "avgpool2: bad arguments");
    hipLaunchKernelGGL(avgpool2_kernel, dim3(grid1((size_t)n * h * w * c / 4)), dim3(256), 0, (hipStream_t)stream,
                       x, y, n, h, w, c);
    return launched("avgpool2");
}

lbm_status lbm_nn_avgpool2_backward(const uint16_t* dy, int32_t n, int32_t h, int32_t w, int32_t c, uint16_t* dx,
                                    void* stream) {
    if (!dy || !dx || !pos(n) || !pos(h) || !pos(w) || !pos(c) || h % 2 || w % 2)
        return nn_fail(LBM_E_INVALID, "avgpool2_backward: bad arguments");
    hipLaunchKernelGGL(avgpool2_backward_kernel, dim3(grid1((size_t)n * h * w * c)), dim3(256), 0,
                       (hipStream_t)stream, dy, dx, n, h, w, c);
    return launched("avgpool2_backward");
}

lbm_status lbm_nn_upsample2(const uint16_t* x, int32_t n, int32_t h, int32_t w, int32_t c, uint16_t* y,
                            void* stream) {
    if (!x || !y || !pos(n) || !pos(h) || !pos(w) || !pos(c)) return nn_fail(LBM_E_INVALID, "upsample2: bad arguments");
    hipLaunchKernelGGL(upsample2_kernel, dim3(grid1((size_t)n * 4 * h * w * c)), dim3(256), 0, (hipStream_t)stream,
                       x, y, n, h, w, c);
    return launched("upsample2");
}

lbm_status lbm_nn_upsample2_backward(const uint16_t* dy, int32_t n, int32_t h, int32_t w, int32_t c, uint16_t* dx,
                                     void* stream) {
    if (!dy || !dx || !pos(n) || !pos(h) || !pos(w) || !pos(c))
        return nn_fail(LBM_E_INVALID, "upsample2_backward: bad arguments");
    hipLaunchKernelGGL(upsample2_backward_kernel, dim3(grid1((size_t)n * h * w * c)), dim3(256), 0,
                       (hipStream_t)stream, dy, dx, n, h, w, c);
    return launched("upsample2_backward");
}

lbm_status lbm_nn_copy_channels(const uint16_t* src, int32_t cs, int32_t soff, uint16_t* dst, int32_t cd,
                                int32_t doff, int32_t cc, int64_t pixels, int32_t accumulate, void* stream) {
    if (!src || !dst || !pos(cs) || !pos(cd) || !pos(cc) || soff < 0 || doff < 0 || soff + cc > cs ||
        doff + cc > cd || pixels < 0)
        return nn_fail(LBM_E_INVALID, "copy_channels: bad arguments");
    hipLaunchKernelGGL(copy_channels_kernel, dim3(grid1((size_t)pixels * cc)), dim3(256), 0, (hipStream_t)stream,
                       src, cs, soff, dst, cd, doff, cc, (size_t)pixels, accumulate);
    return launched("copy_channels");
}

lbm_status lbm_nn_mse(const uint16_t* y, int32_t cy, const float* target, const float* mask, int64_t pixels,
                      int32_t used, double count, uint16_t* dy, float* loss, float* scratch, void* stream) {
    if (!y || !target || !mask || !loss || !scratch || !pos(cy) || !pos(used) || used > cy || pixels < 0 ||
        !(count > 0))
        return nn_fail(LBM_E_INVALID, "mse: bad arguments");
    const unsigned grid = grid1((size_t)pixels * cy, 256, 1024);
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(mse_kernel, dim3(grid), dim3(256), 0, s, y, cy, target, mask, (size_t)pixels, used,
                       (float)(1.0 / count), dy, scratch);
    lbm_status st = launched("mse");
    if (st) return st;
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, s, (const float*)scratch, (int32_t)grid,
                       (float)(1.0 / count), loss);
    return launched("mse sum");
}

lbm_status lbm_nn_adam(float* w, const float* g, float* m, float* v, int64_t count, float lr, float beta1,
                       float beta2, float eps, int32_t step, uint16_t* w_bf16, void* stream) {
    if (!w || !g || !m || !v || count < 0 || step < 1) return nn_fail(LBM_E_INVALID, "adam: bad arguments");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3(grid1((size_t)count)), dim3(256), 0, (hipStream_t)stream, w, g, m, v,
                       (size_t)count, lr, beta1, beta2, eps, c1, c2, w_bf16);
    return launched("adam");
}

lbm_status lbm_nn_to_bf16(const float* src, uint16_t* dst, int64_t count, void* stream) {
    if (!src || !dst || count < 0) return nn_fail(LBM_E_INVALID, "to_bf16: bad arguments");
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(grid1((size_t)count)), dim3(256), 0, (hipStream_t)stream, src, dst,
                       (size_t)count);
    return launched("to_bf16");
}

lbm_status lbm_nn_to_f32(const uint16_t* src, float* dst, int64_t count, void* stream) {
    if (!src || !dst || count < 0) return nn_fail(LBM_E_INVALID, "to_f32: bad arguments");
    hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(grid1((size_t)count)), dim3(256), 0, (hipStream_t)stream, src, dst,
                       (size_t)count);
    return launched("to_f32");
}

}  // extern "C"
