// Random-access rate probe (see include/hm_roofline.h).
#include <hip/hip_runtime.h>

#include "hm_kmer.h"
#include "hm_roofline.h"

namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t mix(uint64_t z) {  // SplitMix64 output function
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// kInflight independent accesses per thread per iteration
template <int KIND, int kInflight>
__global__ __launch_bounds__(kBlock) void k_random(uint64_t *buf, uint64_t mask, uint64_t n_iter, uint64_t seed,
                                                   uint64_t *sink) {
    const uint64_t tid = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint64_t acc = 0;
    for (uint64_t it = 0; it < n_iter; ++it) {
        uint64_t idx[kInflight];
#pragma unroll
        for (int j = 0; j < kInflight; ++j) {
            idx[j] = mix(seed ^ ((tid * n_iter + it) * kInflight + j)) & mask;
            if (KIND == HM_RA_LINE_RMW || KIND == HM_RA_PROBE_CAS) idx[j] &= ~7ull;  // first word of a 64-byte line
        }
        if (KIND == HM_RA_LOAD) {
            uint64_t v[kInflight];
#pragma unroll
            for (int j = 0; j < kInflight; ++j) v[j] = buf[idx[j]];
#pragma unroll
            for (int j = 0; j < kInflight; ++j) acc += v[j];
        } else if (KIND == HM_RA_LOAD_COHERENT) {
            uint64_t v[kInflight];
#pragma unroll
            for (int j = 0; j < kInflight; ++j)
                v[j] = __hip_atomic_load(buf + idx[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < kInflight; ++j) acc += v[j];
        } else if (KIND == HM_RA_ATOMIC_ADD) {
#pragma unroll
            for (int j = 0; j < kInflight; ++j)
                __hip_atomic_fetch_add(buf + idx[j], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (KIND == HM_RA_ATOMIC_OR_RET) {
            uint64_t v[kInflight];
#pragma unroll
            for (int j = 0; j < kInflight; ++j)
                v[j] = __hip_atomic_fetch_or(buf + idx[j], 1ull << (idx[j] & 63), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < kInflight; ++j) acc += v[j];
        } else if (KIND == HM_RA_PROBE_CAS) {
            uint4 v[kInflight];
#pragma unroll
            for (int j = 0; j < kInflight; ++j) v[j] = *reinterpret_cast<const uint4 *>(buf + idx[j]);
#pragma unroll
            for (int j = 0; j < kInflight; ++j) {
                uint64_t expected = (uint64_t)v[j].z | ((uint64_t)v[j].w << 32);
                __hip_atomic_compare_exchange_strong(buf + idx[j] + 1, &expected, expected + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                acc += expected;
            }
        } else if (KIND == HM_RA_LINE_RMW) {
            uint64_t v[kInflight];
#pragma unroll
            for (int j = 0; j < kInflight; ++j)
                v[j] = __hip_atomic_load(buf + idx[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
            for (int j = 0; j < kInflight; ++j) {
                uint32_t *w = reinterpret_cast<uint32_t *>(buf + idx[j]);
                __hip_atomic_fetch_add(w + 4 + (v[j] & 3), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(w + 8 + ((v[j] >> 2) & 3), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
    if (acc == 0x8BADF00Dull) *sink = acc;  // practically never; keeps the loads alive
}

__global__ __launch_bounds__(kBlock) void k_copy(uint4 *dst, const uint4 *src, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

template <int INFL>
int launch_random(int kind, uint64_t *buf, uint64_t mask, uint64_t n_ops, uint64_t seed, uint64_t *sink, int cus,
                  hipStream_t s) {
    const uint64_t threads = (uint64_t)cus * 8 * kBlock;
    const uint64_t n_iter = (n_ops + threads * INFL - 1) / (threads * INFL);
    const dim3 g(cus * 8), b(kBlock);
    switch (kind) {
    case HM_RA_LOAD: hipLaunchKernelGGL((k_random<HM_RA_LOAD, INFL>), g, b, 0, s, buf, mask, n_iter, seed, sink); break;
    case HM_RA_LOAD_COHERENT:
        hipLaunchKernelGGL((k_random<HM_RA_LOAD_COHERENT, INFL>), g, b, 0, s, buf, mask, n_iter, seed, sink);
        break;
    case HM_RA_ATOMIC_ADD:
        hipLaunchKernelGGL((k_random<HM_RA_ATOMIC_ADD, INFL>), g, b, 0, s, buf, mask, n_iter, seed, sink);
        break;
    case HM_RA_ATOMIC_OR_RET:
        hipLaunchKernelGGL((k_random<HM_RA_ATOMIC_OR_RET, INFL>), g, b, 0, s, buf, mask, n_iter, seed, sink);
        break;
    case HM_RA_PROBE_CAS:
        hipLaunchKernelGGL((k_random<HM_RA_PROBE_CAS, INFL>), g, b, 0, s, buf, mask, n_iter, seed, sink);
        break;
    default: hipLaunchKernelGGL((k_random<HM_RA_LINE_RMW, INFL>), g, b, 0, s, buf, mask, n_iter, seed, sink); break;
    }
    return hipGetLastError() == hipSuccess ? HM_OK : HM_EHIP;
}

}  // namespace

extern "C" int hm_random_access(uint64_t *buf, uint64_t n_words, int32_t kind, uint64_t n_ops, uint64_t seed,
                                uint64_t *sink, hipStream_t s) {
    if (!buf || !sink || n_words < 16 || (n_words & (n_words - 1))) return HM_EINVAL;
    const bool serial = (kind & HM_RA_SERIAL) != 0;
    kind &= ~HM_RA_SERIAL;
    if (kind < HM_RA_LOAD || kind > HM_RA_PROBE_CAS || (serial && kind == HM_RA_COPY)) return HM_EINVAL;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return HM_EHIP;
    if (kind == HM_RA_COPY) {
        const uint64_t n = n_words / 4;  // uint4 elements in half the buffer
        hipLaunchKernelGGL(k_copy, dim3(cus * 16), dim3(kBlock), 0, s, reinterpret_cast<uint4 *>(buf + n_words / 2),
                           reinterpret_cast<const uint4 *>(buf), n);
        return hipGetLastError() == hipSuccess ? HM_OK : HM_EHIP;
    }
    const uint64_t mask = n_words - 1;
    return serial ? launch_random<1>(kind, buf, mask, n_ops, seed, sink, cus, s)
                  : launch_random<4>(kind, buf, mask, n_ops, seed, sink, cus, s);
}
