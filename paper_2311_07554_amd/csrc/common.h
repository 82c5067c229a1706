// Device-side building blocks shared by the sketch and selection kernels.
// gfx950 (CDNA4): 64-wide wavefronts; every "wave" helper below assumes all 64
// lanes of the wave execute it together.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pacim {

constexpr uint64_t kPhi = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSaltCenter = 0xC000000000000001ull;
constexpr uint64_t kSaltTriv = 0xC000000000000002ull;
constexpr uint64_t kAllLive = 0xFFFFFFFFFFFFFFFFull;
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kWave = 64;
constexpr int kFan = 64;        // winning-tree fan-out: one wave lane per child
constexpr int kFanLog = 6;
constexpr int kMaxLevels = 8;   // internal tree levels; 64^6 > 2^32 vertices

// Distance in elements between two sketches' arrays in the labelling scratch
// (parent, member counts, smallest center ranks; [B][stride]).  n is rounded up
// to 256 bytes and, from 2^16 vertices on, padded by 65 x 256 bytes: with a
// power-of-two stride the same vertex of the B sketches falls on one memory
// channel, and the hooking pass, which touches a vertex in several sketches at
// once, ran 25% slower on 2^20 vertices.  Small arrays stay in cache anyway.
__host__ __device__ constexpr size_t sketch_stride(uint32_t n) {
    return (((size_t)n + 63) & ~(size_t)63) + (n >= (1u << 16) ? 4160 : 0);
}

// SplitMix64 output function (Steele, Lea, Flood 2014).  Two 64-bit multiplies.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// K(seed, x): per-sketch (or per-salt) key of the live-edge hash.
__device__ __forceinline__ uint64_t sketch_key(uint64_t seed, uint64_t x) { return mix64(seed * kPhi + x); }

__device__ __forceinline__ uint64_t edge_word(uint32_t u, uint32_t v) {
    return u < v ? ((uint64_t)u << 32) | v : ((uint64_t)v << 32) | u;
}

// Probability model of one edge: uniform threshold, or the trivalency class.
struct ProbDev {
    int kind;          // 0 uniform, 1 trivalency
    uint64_t t0;       // uniform threshold, or the p = 0.1 threshold
    uint64_t t1, t2;   // p = 0.01, 0.001 thresholds (trivalency)
    uint64_t ktriv;    // K(0, kSaltTriv)
};

__device__ __forceinline__ uint64_t edge_threshold(const ProbDev &pm, uint64_t x) {
    if (pm.kind == 0) return pm.t0;
    uint64_t c = mix64(x ^ pm.ktriv) % 3u;
    return c == 0 ? pm.t0 : (c == 1 ? pm.t1 : pm.t2);
}

__device__ __forceinline__ bool is_live(uint64_t x, uint64_t kr, uint64_t T) {
    return T == kAllLive || mix64(x ^ kr) < T;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
    return x;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t y = __shfl_xor(x, off);
        x = y > x ? y : x;
    }
    return x;
}

// Inclusive prefix sum over the lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= (uint32_t)off) x += y;
    }
    return x;
}

// Wave-aggregated append: lanes with pred reserve consecutive slots of a
// global counter with one atomic per wave.  Returns the slot (valid if pred)
// and writes the wave's total to *total.
__device__ __forceinline__ uint32_t wave_append(uint32_t *counter, bool pred, uint32_t *total) {
    const uint32_t lane = lane_id();
    const uint64_t m = __ballot(pred);
    const uint32_t cnt = (uint32_t)__popcll(m);
    uint32_t base = 0;
    if (cnt) {
        if (lane == 0) base = atomicAdd(counter, cnt);
        base = __shfl(base, 0);
    }
    *total = cnt;
    return base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Global wave index / count for kernels that hand one item to each wave.
__device__ __forceinline__ uint32_t wave_index() { return (blockIdx.x * blockDim.x + threadIdx.x) / kWave; }
__device__ __forceinline__ uint32_t wave_count() { return (gridDim.x * blockDim.x) / kWave; }

// Key of the winning tree: larger gain first, smaller id on equal gains; 0 =
// removed.  ((gain + 1) << kb) | (2^kb - 1 - v).
__device__ __forceinline__ uint64_t pack_key(uint64_t gain, uint32_t v, uint32_t kb) {
    const uint64_t mask = (1ull << kb) - 1ull;
    return ((gain + 1ull) << kb) | (mask - (uint64_t)v);
}
__device__ __forceinline__ uint64_t key_gain(uint64_t key, uint32_t kb) { return (key >> kb) - 1ull; }

}  // namespace pacim
