// Device ceilings for the roofline of the sampling and streaming kernels:
//   k_probe_hash  the sampling loop's arithmetic alone (64 live tests per edge
//                 word, keys in scalar registers, no memory traffic): the
//                 integer-ALU ceiling of hash evaluations per second;
//   k_probe_copy  a 16-byte-per-lane streaming copy: the achievable HBM bandwidth;
//   k_probe_gather independent 4-byte reads at pseudo-random places of a buffer far
//                 larger than the caches: the rate of random reads (the access
//                 pattern of the union-find's parent lookups), and, under a byte
//                 counter, the bytes one such read moves from HBM.
#pragma once

#include "common.h"

namespace pacim {

__global__ void __launch_bounds__(256) k_probe_hash(const uint64_t *__restrict__ K, uint32_t iters, uint64_t T,
                                                    unsigned long long *__restrict__ sink) {
    uint64_t x = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * 0x100000001ull;
    uint32_t acc = 0;
    for (uint32_t it = 0; it < iters; ++it) {
        const uint64_t xp = xs30(x);
        uint64_t live = 0;
        for (uint32_t b0 = 0; b0 < 64; b0 += 8) {
            uint32_t chunk = 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) chunk |= (mix64_from_xs30(xp ^ xs30_key(K[b0 + j])) < T) ? (1u << j) : 0u;
            live |= (uint64_t)chunk << b0;
        }
        acc += (uint32_t)__popcll(live);
        x += kPhi;
    }
    if (acc == 0xFFFFFFFFu) *sink = acc;  // never true; keeps the loop alive
}

__global__ void __launch_bounds__(256) k_probe_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                    uint64_t count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

// Each thread reads `per` words at pseudo-random word offsets of buf (words
// entries); the addresses do not depend on loaded data, so every read of a thread
// can be in flight at once.
__global__ void __launch_bounds__(256) k_probe_gather(const uint32_t *__restrict__ buf, uint64_t words, uint32_t per,
                                                      unsigned long long *__restrict__ sink) {
    uint64_t h = mix64((uint64_t)blockIdx.x * blockDim.x + threadIdx.x + 1);
    uint32_t acc = 0;
    for (uint32_t i = 0; i < per; ++i) {
        h = mix64(h + kPhi);
        acc += buf[h % words];
    }
    if (acc == 0xFFFFFFFFu) *sink = acc;  // never true for the probe's fill; keeps the reads alive
}

}  // namespace pacim
