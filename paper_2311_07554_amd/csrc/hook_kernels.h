// The sampling pass of the sketch construction (Sec. 3, Sketch(r), with the
// fusion of sampling and labelling: a sampled graph is never stored): one thread
// per undirected edge tests the edge in each of the pass's sketches and unites
// its endpoints in every sketch where it is live, in union-find forests whose
// roots are the smallest numbers of their components.  The forest operations are
// shared with the batched path, whose forests are vertex-major too.
#pragma once

#include "common.h"

namespace pacim {

// Relaxed loads of the union-find forest.  A value read here may be older than
// the newest one (another XCD's L2, this CU's L1), but parent pointers only ever
// move to smaller ids that stay ancestors, so an old value is still an ancestor.
__device__ __forceinline__ uint32_t uf_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One sketch's forest: entry of number x at P[x * vs].
__device__ __forceinline__ uint32_t uf_find(uint32_t *P, uint32_t vs, uint32_t x) {
    for (;;) {
        uint32_t p = uf_load(P + (size_t)x * vs);
        if (p == x) return x;
        uint32_t gp = uf_load(P + (size_t)p * vs);
        if (gp == p) return p;
        // path halving; any ancestor is a valid parent
        __hip_atomic_store(P + (size_t)x * vs, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

// uf_find continuing from x whose parent p the caller already loaded.
__device__ __forceinline__ uint32_t uf_find_from(uint32_t *P, uint32_t vs, uint32_t x, uint32_t p) {
    for (;;) {
        if (p == x) return x;
        const uint32_t gp = uf_load(P + (size_t)p * vs);
        if (gp == p) return p;
        __hip_atomic_store(P + (size_t)x * vs, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
        p = uf_load(P + (size_t)x * vs);
    }
}

// Union by hooking the larger root under the smaller, so the last root of every
// component is its smallest number whatever the schedule.  A failed CAS
// returns the root's fresh parent, strictly smaller, so a+b strictly decreases
// on every retry: the loop ends even when uf_find read old values.  pa / pb:
// the parents of a and b, already loaded.
__device__ __forceinline__ void uf_unite_from(uint32_t *P, uint32_t vs, uint32_t a, uint32_t pa, uint32_t b,
                                              uint32_t pb) {
    a = uf_find_from(P, vs, a, pa);
    b = uf_find_from(P, vs, b, pb);
    for (;;) {
        if (a == b) return;
        if (a < b) { uint32_t t = a; a = b; b = t; }
        uint32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(P + (size_t)a * vs, &expected, b, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = uf_find(P, vs, expected);
        b = uf_find(P, vs, b);
    }
}

// Live mask of one edge word x over sketches [0, B): bit b set iff the edge is
// live in sketch b.  K must hold round_up(B, 8) keys.
template <int KIND>
__device__ __forceinline__ uint64_t live_mask(uint32_t u, uint32_t v, uint64_t x, uint64_t e,
                                              const uint64_t *__restrict__ K, uint32_t B, const ProbDev &pm) {
    const uint64_t T = edge_threshold_of<KIND>(pm, u, v, x, e);
    const uint64_t all = B >= 64 ? ~0ull : ((1ull << B) - 1ull);
    if (T == kAllLive) return all;
    const uint64_t xp = xs30(x);
    uint64_t live = 0;
    for (uint32_t b0 = 0; b0 < B; b0 += 8) {
        uint32_t chunk = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j) chunk |= (mix64_from_xs30(xp ^ xs30_key(K[b0 + j])) < T) ? (1u << j) : 0u;
        live |= (uint64_t)chunk << b0;
    }
    return live & all;
}

constexpr uint32_t kHookBlock = 256;
constexpr int kHookIlp = 4;  // live sketches of an edge whose first parent loads are issued together

// Unions of edge (u, v) in every sketch whose bit is set in live (sketch b's
// entry of number x at parent[b + x * vs]: vs = the pass's scratch width for the
// single-query scratch; vs = the query's R for the batched path, whose rows hold
// all of a query's sketches and whose caller offsets parent to the pass's first
// sketch).  The parents of both endpoints in up to kHookIlp sketches are loaded
// before any of those unions walks on, so a thread keeps several independent
// memory accesses in flight instead of one chain.
__device__ __forceinline__ void unite_live(uint32_t *parent, uint32_t vs, uint64_t live, uint32_t u, uint32_t v) {
    while (live) {
        uint32_t bs[kHookIlp], pu[kHookIlp], pv[kHookIlp];
        int c = 0;
#pragma unroll
        for (int i = 0; i < kHookIlp; ++i) {
            bs[i] = 0;
            if (live) {
                bs[i] = (uint32_t)__builtin_ctzll(live);
                live &= live - 1ull;
                ++c;
            }
        }
#pragma unroll
        for (int i = 0; i < kHookIlp; ++i)
            if (i < c) {
                const uint32_t *P = parent + bs[i];
                pu[i] = uf_load(P + (size_t)u * vs);
                pv[i] = uf_load(P + (size_t)v * vs);
            }
#pragma unroll
        for (int i = 0; i < kHookIlp; ++i)
            if (i < c) uf_unite_from(parent + bs[i], vs, u, pu[i], v, pv[i]);
    }
}

// One thread per undirected edge: its live mask over the pass's sketches (from
// the endpoints' ids, edges[e]), then one union per live sketch (between the
// endpoints' labelling-order numbers, iedges[e]) in the vertex-major forests of
// width vs.
template <int KIND>
__global__ void __launch_bounds__(kHookBlock) k_sample_hook(const uint2 *__restrict__ edges,
                                                            const uint2 *__restrict__ iedges, uint64_t m,
                                                            const uint64_t *__restrict__ K, uint32_t B, ProbDev pm,
                                                            uint32_t *__restrict__ parent, uint32_t vs) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const uint2 uv = edges[e], iuv = iedges[e];
        unite_live(parent, vs, live_mask<KIND>(uv.x, uv.y, ((uint64_t)uv.x << 32) | uv.y, e, K, B, pm), iuv.x,
                   iuv.y);
    }
}

}  // namespace pacim
