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
constexpr uint64_t kSaltRange = 0xC000000000000003ull;
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
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// mix64(x ^ k) for many keys k of one word x: its first step, z ^= z >> 30, is
// linear over xor, so (x ^ k) ^ ((x ^ k) >> 30) = xs30(x) ^ xs30(k).  A sampling
// loop takes xs30(x) once per edge and xs30(k) once per sketch key (wave-uniform:
// scalar instructions), and each hash starts at the multiply.
__host__ __device__ __forceinline__ uint64_t xs30(uint64_t z) { return z ^ (z >> 30); }
// xs30 of a wave-uniform key, kept in scalar registers and hidden from the
// compiler's algebra (it would otherwise fold xs30(x) ^ xs30(k) back into
// xs30(x ^ k), one vector shift per hash again).
__device__ __forceinline__ uint64_t xs30_key(uint64_t k) {
    uint64_t z = xs30(k);
    asm volatile("" : "+s"(z));
    return z;
}
__host__ __device__ __forceinline__ uint64_t mix64_from_xs30(uint64_t z) {
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A loaded value made opaque to the compiler, so that a load issued
// unconditionally (inactive lanes reading a harmless entry) stays unconditional:
// otherwise the compiler turns "load, then select" back into a branch around the
// load and waits for each load inside its branch.
__device__ __forceinline__ uint32_t pin_vgpr(uint32_t x) {
    asm volatile("" : "+v"(x));
    return x;
}

// K(seed, x): per-sketch (or per-salt) key of the live-edge hash.
__host__ __device__ __forceinline__ uint64_t sketch_key(uint64_t seed, uint64_t x) { return mix64(seed * kPhi + x); }

__device__ __forceinline__ uint64_t edge_word(uint32_t u, uint32_t v) {
    return u < v ? ((uint64_t)u << 32) | v : ((uint64_t)v << 32) | u;
}

// Edge-probability models (the kind values of im_prob_kind) as integer
// thresholds: an edge is live in a sketch iff its hash is below T_e.
enum : int { kProbConstant = 0, kProbTrivalency = 1, kProbRange = 2, kProbWic = 3, kProbPerEdge = 4 };

struct ProbDev {
    int kind;
    uint64_t t0;             // constant: T(p); trivalency: T(0.1); range: T(lo)
    uint64_t t1, t2;         // trivalency: T(0.01), T(0.001); range: t1 = T(hi) - T(lo)
    uint64_t ktriv;          // trivalency: K(0, kSaltTriv); range: K(0, kSaltRange)
    const uint64_t *off;     // WIC: the graph's CSR offsets (degrees)
    const uint64_t *csr_thr; // the threshold of every CSR entry j (or null): WIC with CompactSketch, so
                             // that GetCenter's scans need neither the neighbour's degree nor a division,
                             // and the per-edge model
    const uint64_t *edge_thr;  // per-edge model: the threshold of every undirected edge, edge-list order
};

// floor(2^65 / s) = floor(2 / s * 2^64), the WIC threshold of an edge whose end
// degrees sum to s (s <= 2: p = 1, always live).  64-bit operations only:
// 2^64 - 1 = q s + r gives 2^64 = q1 s + m1, and 2^65 = 2 q1 s + 2 m1 with
// 2 m1 < 2 s.
__host__ __device__ __forceinline__ uint64_t wic_threshold(uint64_t s) {
    if (s <= 2) return kAllLive;
    const uint64_t q = ~0ull / s, r = ~0ull - q * s;
    const bool wrap = r + 1 == s;
    const uint64_t q1 = q + (wrap ? 1u : 0u), m1 = wrap ? 0u : r + 1;
    return 2 * q1 + (2 * m1 >= s ? 1u : 0u);
}

// Threshold of edge {u, v} (canonical word x, index e in the edge list, used by the
// per-edge model only) under model KIND.
template <int KIND>
__device__ __forceinline__ uint64_t edge_threshold_of(const ProbDev &pm, uint32_t u, uint32_t v, uint64_t x,
                                                      uint64_t e = 0) {
    if (KIND == kProbPerEdge) return pm.edge_thr[e];
    if (KIND == kProbConstant) return pm.t0;
    if (KIND == kProbTrivalency) {
        const uint64_t c = mix64(x ^ pm.ktriv) % 3u;
        return c == 0 ? pm.t0 : (c == 1 ? pm.t1 : pm.t2);
    }
    if (KIND == kProbRange) return pm.t0 + __umul64hi(pm.t1, mix64(x ^ pm.ktriv));
    return wic_threshold((pm.off[u + 1] - pm.off[u]) + (pm.off[v + 1] - pm.off[v]));
}

// Threshold of edge {u, v} where only its end points are known (not the per-edge
// model, whose searches read csr_thr and whose edge passes know the index).
__device__ __forceinline__ uint64_t edge_threshold(const ProbDev &pm, uint32_t u, uint32_t v, uint64_t x) {
    switch (pm.kind) {
    case kProbConstant: return edge_threshold_of<kProbConstant>(pm, u, v, x);
    case kProbTrivalency: return edge_threshold_of<kProbTrivalency>(pm, u, v, x);
    case kProbRange: return edge_threshold_of<kProbRange>(pm, u, v, x);
    case kProbWic: return edge_threshold_of<kProbWic>(pm, u, v, x);
    default: return 0;
    }
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

// Sum over the 64 lanes of a 32-bit value whose total fits in 32 bits, returned
// wave-uniform: two quad permutations and two row rotations (DPP, no LDS) leave
// every lane of a 16-lane row holding the row's sum, then the four row sums are
// read out.  All 64 lanes must be active.
__device__ __forceinline__ uint32_t wave_sum_u32_rows(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);   // quad_perm 1,0,3,2
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);   // quad_perm 2,3,0,1
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x124, 0xF, 0xF, false);  // row_ror 4
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);  // row_ror 8
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 0) + (uint32_t)__builtin_amdgcn_readlane((int)x, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)x, 32) + (uint32_t)__builtin_amdgcn_readlane((int)x, 48);
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
