// probe.hip -- HBM bandwidth probes: the ceiling against which the
// streaming kernels of this library are measured.
//
// A one-pass kernel in which every thread moves `K` 16-byte vectors, the
// vectors of a block contiguous (256 threads x K), so a wavefront issues
// 1 KiB per load instruction and the whole grid touches each byte once:
//   kind 0  copy  dst[i] = src[i]   (one read and one write per byte pair)
//   kind 1  read  src only; the XOR of everything loaded is stored to dst[0]
//                 only if it equals a fixed pattern, which keeps the loads
//   kind 2  write dst only (a fill)
// Non-temporal access (flag 1) marks the lines as streaming so they do not
// displace other data in the caches; both forms are offered because which
// one is faster is a property of the memory system, measured, not assumed.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/lbm.h"

namespace {

constexpr int kProbeBlock = 256;
typedef uint32_t v4u __attribute__((ext_vector_type(4)));  // one 16-byte vector
constexpr uint32_t kReadPattern = 0x9e3779b9u;

template <int K, int KIND, bool NT>
__global__ __launch_bounds__(kProbeBlock) void probe_kernel(const v4u* __restrict__ src,
                                                            v4u* __restrict__ dst, size_t n) {
    const size_t base = (size_t)blockIdx.x * (kProbeBlock * K) + threadIdx.x;
    v4u v[K];
    if constexpr (KIND != 2) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t i = base + (size_t)k * kProbeBlock;
            if (i < n) v[k] = NT ? __builtin_nontemporal_load(src + i) : src[i];
            else v[k] = v4u{0u, 0u, 0u, 0u};
        }
    }
    if constexpr (KIND == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t i = base + (size_t)k * kProbeBlock;
            if (i < n) {
                if (NT) __builtin_nontemporal_store(v[k], dst + i);
                else dst[i] = v[k];
            }
        }
    } else if constexpr (KIND == 1) {
        uint32_t acc = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
        if (acc == kReadPattern) dst[0] = v4u{acc, acc, acc, acc};
    } else {
        const v4u w{(uint32_t)base, 1u, 2u, 3u};
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const size_t i = base + (size_t)k * kProbeBlock;
            if (i < n) {
                if (NT) __builtin_nontemporal_store(w, dst + i);
                else dst[i] = w;
            }
        }
    }
}

template <int K, int KIND>
void launch_k(bool nt, const v4u* src, v4u* dst, size_t n, hipStream_t s) {
    const size_t per_block = (size_t)kProbeBlock * K;
    const dim3 grid((unsigned)((n + per_block - 1) / per_block));
    if (nt) hipLaunchKernelGGL((probe_kernel<K, KIND, true>), grid, dim3(kProbeBlock), 0, s, src, dst, n);
    else hipLaunchKernelGGL((probe_kernel<K, KIND, false>), grid, dim3(kProbeBlock), 0, s, src, dst, n);
}

template <int KIND>
void launch_kind(int per_thread, bool nt, const v4u* src, v4u* dst, size_t n, hipStream_t s) {
    switch (per_thread) {
    case 1: launch_k<1, KIND>(nt, src, dst, n, s); break;
    case 2: launch_k<2, KIND>(nt, src, dst, n, s); break;
    case 4: launch_k<4, KIND>(nt, src, dst, n, s); break;
    default: launch_k<8, KIND>(nt, src, dst, n, s); break;
    }
}

}  // namespace

extern "C" lbm_status lbm_probe_bandwidth(int32_t kind, const void* src, void* dst, size_t bytes,
                                          int32_t per_thread, int32_t flags, void* hip_stream) {
    if (kind < 0 || kind > 2) return LBM_E_INVALID;
    if (per_thread != 1 && per_thread != 2 && per_thread != 4 && per_thread != 8) return LBM_E_INVALID;
    if (flags & ~1) return LBM_E_INVALID;
    if (bytes == 0 || bytes % 16 || (uintptr_t)src % 16 || (uintptr_t)dst % 16) return LBM_E_INVALID;
    if ((kind != 2 && !src) || !dst) return LBM_E_INVALID;
    const size_t n = bytes / 16;
    if ((n + (size_t)kProbeBlock * per_thread - 1) / ((size_t)kProbeBlock * per_thread) > 0x7fffffffu)
        return LBM_E_INVALID;
    const bool nt = flags & 1;
    const hipStream_t s = (hipStream_t)hip_stream;
    const v4u* in = (const v4u*)src;
    v4u* out = (v4u*)dst;
    if (kind == 0) launch_kind<0>(per_thread, nt, in, out, n, s);
    else if (kind == 1) launch_kind<1>(per_thread, nt, in, out, n, s);
    else launch_kind<2>(per_thread, nt, in, out, n, s);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_E_DEVICE;
}
