// Memory-system probes for the RAMBO access patterns (include/rambo_roofline.h).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "rambo.h"
#include "rambo_roofline.h"

namespace rambo_dev {

constexpr int kPerThread = 8;   // independent accesses in flight per thread
constexpr uint32_t kImprobable = 0x9E3779B9u;

template <int G>
__global__ __launch_bounds__(kBlock) void k_gather(const uint8_t *buf, uint64_t n_slots, uint64_t n_access,
                                                   uint64_t seed, uint32_t *sink)
{
    constexpr int V = G >= 16 ? G / 16 : 1;   // uint4 loads per access
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t first = t * kPerThread;
    uint32_t acc = 0;
    uint64_t slot[kPerThread];
#pragma unroll
    for (int a = 0; a < kPerThread; ++a)
        slot[a] = __umul64hi(mix64(seed + first + a), n_slots);
    auto fold = [&](const uint8_t *p) {
        if constexpr (G == 4) {
            acc ^= *reinterpret_cast<const uint32_t *>(p);
        } else if constexpr (G == 8) {
            const uint2 v = *reinterpret_cast<const uint2 *>(p);
            acc ^= v.x ^ v.y;
        } else {
#pragma unroll
            for (int i = 0; i < V; ++i) {
                const uint4 v = reinterpret_cast<const uint4 *>(p)[i];
                acc ^= v.x ^ v.y ^ v.z ^ v.w;
            }
        }
    };
    if (first + kPerThread <= n_access) {
#pragma unroll
        for (int a = 0; a < kPerThread; ++a)
            fold(buf + slot[a] * G);
    } else {
        for (int a = 0; a < kPerThread && first + a < n_access; ++a)
            fold(buf + slot[a] * G);
    }
    if (acc == kImprobable)
        sink[0] = acc;
}

__global__ __launch_bounds__(kBlock) void k_atomic_or(uint32_t *buf, uint64_t n_words, uint64_t n_access,
                                                      uint64_t seed)
{
    const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const uint64_t first = t * kPerThread;
#pragma unroll
    for (int a = 0; a < kPerThread; ++a) {
        if (first + a >= n_access)
            break;
        const uint64_t h = mix64(seed + first + a);
        atomicOr(buf + __umul64hi(h, n_words), 1u << (h & 31u));
    }
}

// The write pattern of the partitioned insert's binning: workgroup g owns a
// chunk of every one of `streams` buckets (chunk (b, g) at (b * nwg + g) *
// cap words) and each round appends a run of `run` words to each, the lanes
// writing consecutive words; with `misaligned` each chunk starts its runs
// 0..15 words into its first 64-byte segment (mix64 of the bucket and the
// workgroup), so runs start and end inside segments, as appends at a
// running cursor do.
constexpr int kAppendBlock = 1024;

__global__ __launch_bounds__(kAppendBlock) void k_append(uint32_t *buf, uint32_t streams, uint32_t run,
                                                         uint32_t rounds, uint64_t cap, uint32_t misaligned)
{
    const uint32_t g = blockIdx.x, nwg = gridDim.x;
    const uint32_t per_round = streams * run;
    for (uint32_t r = 0; r < rounds; ++r)
        for (uint32_t i = threadIdx.x; i < per_round; i += kAppendBlock) {
            const uint32_t b = i / run, j = i % run;
            const uint32_t off = misaligned ? (uint32_t)(mix64(((uint64_t)b << 32) | g) & 15u) : 0u;
            buf[((uint64_t)b * nwg + g) * cap + off + (uint64_t)r * run + j] = i ^ r;
        }
}

__global__ __launch_bounds__(kBlock) void k_copy(const uint4 *src, uint4 *dst, uint64_t n)
{
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

}  // namespace rambo_dev

using namespace rambo_dev;

namespace {
uint32_t blocks_for(uint64_t n_access)
{
    const uint64_t threads = (n_access + kPerThread - 1) / kPerThread;
    return (uint32_t)((threads + kBlock - 1) / kBlock);
}
}  // namespace

extern "C" int rambo_roofline_gather(const void *buf, uint64_t buf_bytes, uint32_t access_bytes, uint64_t n_access,
                                     uint64_t seed, uint32_t *sink, hipStream_t stream)
{
    if (!buf || !sink || access_bytes == 0 || buf_bytes < access_bytes || buf_bytes % access_bytes)
        return RAMBO_EINVAL;
    if (n_access == 0)
        return RAMBO_OK;
    const uint64_t slots = buf_bytes / access_bytes;
    const auto *b = static_cast<const uint8_t *>(buf);
    const dim3 grid(blocks_for(n_access)), block(kBlock);
    switch (access_bytes) {
    case 4: hipLaunchKernelGGL(k_gather<4>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    case 8: hipLaunchKernelGGL(k_gather<8>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    case 16: hipLaunchKernelGGL(k_gather<16>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    case 32: hipLaunchKernelGGL(k_gather<32>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    case 64: hipLaunchKernelGGL(k_gather<64>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    case 128: hipLaunchKernelGGL(k_gather<128>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    case 256: hipLaunchKernelGGL(k_gather<256>, grid, block, 0, stream, b, slots, n_access, seed, sink); break;
    default: return RAMBO_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? RAMBO_OK : RAMBO_EHIP;
}

extern "C" int rambo_roofline_atomic_or(uint32_t *buf, uint64_t buf_words, uint64_t n_access, uint64_t seed,
                                        hipStream_t stream)
{
    if (!buf || buf_words == 0)
        return RAMBO_EINVAL;
    if (n_access == 0)
        return RAMBO_OK;
    hipLaunchKernelGGL(k_atomic_or, dim3(blocks_for(n_access)), dim3(kBlock), 0, stream, buf, buf_words, n_access,
                       seed);
    return hipGetLastError() == hipSuccess ? RAMBO_OK : RAMBO_EHIP;
}

extern "C" int rambo_roofline_copy(const void *src, void *dst, uint64_t bytes, hipStream_t stream)
{
    if (!src || !dst || bytes % 16)
        return RAMBO_EINVAL;
    if (bytes == 0)
        return RAMBO_OK;
    const uint64_t n = bytes / 16;
    hipLaunchKernelGGL(k_copy, dim3(256 * 64), dim3(kBlock), 0, stream, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), n);
    return hipGetLastError() == hipSuccess ? RAMBO_OK : RAMBO_EHIP;
}

extern "C" int rambo_roofline_append(uint32_t *buf, uint64_t buf_words, uint32_t streams, uint32_t run,
                                     uint32_t misaligned, uint32_t n_workgroups, uint64_t *written_words,
                                     hipStream_t stream)
{
    if (!buf || !written_words || streams == 0 || run == 0 || n_workgroups == 0 ||
        (uint64_t)streams * run > 0xFFFFFFFFull)   // a round's words are counted in 32 bits
        return RAMBO_EINVAL;
    // chunk of cap words per (bucket, workgroup), a multiple of 16; a run
    // starts at most 15 words in, so rounds * run + 15 <= cap
    const uint64_t cap = buf_words / ((uint64_t)streams * n_workgroups) / 16 * 16;
    if (cap < 16 + (uint64_t)run)
        return RAMBO_EINVAL;
    const uint64_t rounds = std::min<uint64_t>((cap - 15) / run, 0xFFFFFFFFull);
    *written_words = rounds * run * streams * n_workgroups;
    hipLaunchKernelGGL(k_append, dim3(n_workgroups), dim3(kAppendBlock), 0, stream, buf, streams, run,
                       (uint32_t)rounds, cap, misaligned ? 1u : 0u);
    return hipGetLastError() == hipSuccess ? RAMBO_OK : RAMBO_EHIP;
}
