// Sketch construction (Sec. 3, Sketch(r); Algorithm 1, step 1) for a batch of
// B sketches per pass over the edge list.
//
//   k_sketch_keys     K(seed, r) for every sketch
//   k_batch_init      parent[b][x] = x, cnt = 0, minc = x's center rank (or a given value)
//   k_sample_hook     one thread per undirected edge: B live tests (Sample(e, r),
//                     fused: sampled graphs are never stored), then union by
//                     hooking the larger root under the smaller one
//   k_compress        every vertex points at its root (the smallest number in its
//                     CC); non-root members counted at the root; centers'
//                     smallest rank recorded at the root (CompactSketch)
//   k_emit_full       (label, size) per (v, r) into E[n][R] and the initial gains
//   k_giant_sample    per sketch, the largest component among sampled vertices'
//   k_gain0_emit      CompactSketch: the triple label_c / size_c [rho][R], the
//                     initial gains and that component's membership bitmap, in
//                     one pass over the vertices
//   k_center_*        hashed Bernoulli(alpha) centers, ranked by id
//
// The forests of a pass number the vertices in the graph's labelling order
// (x = newid[v] for vertex v, v = iperm[x]): the highest-degree vertices first,
// so that the parents that most unions touch share a few cache lines.  The
// hashes still take the vertices' own ids.  Readers translate with newid; a
// label written out is a vertex id again (iperm of the root).
#pragma once

#include "common.h"

namespace pacim {

__global__ void k_sketch_keys(uint64_t seed, uint32_t R, uint64_t *__restrict__ K) {
    uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) K[r] = sketch_key(seed, r);
}

// K(seed, first + i) for i < count: the keys of a range of simulated worlds.
__global__ void k_world_keys(uint64_t seed, uint32_t first, uint32_t count, uint64_t *__restrict__ K) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) K[i] = sketch_key(seed, (uint64_t)first + i);
}

// Influence by simulation: for each of the pass's B worlds (labelled, compressed),
// the seeds' distinct components, each counted once through flag[b][root], their
// sizes (1 + members counted at the root) summed into *total.  grid (x, B).
__global__ void __launch_bounds__(256) k_influence_accum(const uint32_t *__restrict__ parent,
                                                         const uint32_t *__restrict__ cnt, uint32_t *__restrict__ flag,
                                                         const uint32_t *__restrict__ newid, uint32_t n,
                                                         const uint32_t *__restrict__ seeds, uint32_t k,
                                                         unsigned long long *__restrict__ total) {
    const size_t base = (size_t)blockIdx.y * sketch_stride(n);
    uint64_t sum = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const uint32_t root = parent[base + newid[seeds[i]]];
        if (atomicExch(&flag[base + root], 1u) == 0u) sum += 1u + cnt[base + root];
    }
    sum = wave_sum_u64(sum);
    if (lane_id() == 0 && sum) atomicAdd(total, (unsigned long long)sum);
}

// thr[j] = WIC threshold of CSR entry j (row u, column cols[j]); one wave per row.
__global__ void __launch_bounds__(256) k_csr_wic_thr(const uint64_t *__restrict__ off,
                                                     const uint32_t *__restrict__ cols, uint32_t n,
                                                     uint64_t *__restrict__ thr) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t waves = gridDim.x * (blockDim.x / kWave);
    for (uint32_t u = (blockIdx.x * blockDim.x + threadIdx.x) / kWave; u < n; u += waves) {
        const uint64_t o0 = off[u], o1 = off[u + 1];
        for (uint64_t j = o0 + lane; j < o1; j += kWave) {
            const uint32_t w = cols[j];
            thr[j] = wic_threshold((o1 - o0) + (off[w + 1] - off[w]));
        }
    }
}

// out[x] = in[iperm[x]]: a per-vertex array in labelling order.
__global__ void k_to_label_order(const uint32_t *__restrict__ in, const uint32_t *__restrict__ iperm, uint32_t n,
                                 uint32_t *__restrict__ out) {
    const uint32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) out[x] = in[iperm[x]];
}

// minc starts at each vertex's own center rank when center_rank is given (so a
// root's own rank needs no atomic), else at minc_init.  Numbers [0, n_init):
// isolated vertices (numbered last) keep their entries from an earlier pass of
// the same build, as no pass writes them.
__global__ void k_batch_init(uint32_t *__restrict__ parent, uint32_t *__restrict__ cnt, uint32_t *__restrict__ minc,
                             uint32_t n, uint32_t n_init, uint32_t minc_init,
                             const uint32_t *__restrict__ center_rank) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t at = (size_t)blockIdx.y * sketch_stride(n) + v;
    if (v < n_init) {
        parent[at] = v;
        cnt[at] = 0;
        if (minc) minc[at] = center_rank ? center_rank[v] : minc_init;
    }
}

// Relaxed loads of the union-find forest.  A value read here may be older than
// the newest one (another XCD's L2, this CU's L1), but parent pointers only ever
// move to smaller ids that stay ancestors, so an old value is still an ancestor.
__device__ __forceinline__ uint32_t uf_load(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t uf_find(uint32_t *P, uint32_t x) {
    for (;;) {
        uint32_t p = uf_load(P + x);
        if (p == x) return x;
        uint32_t gp = uf_load(P + p);
        if (gp == p) return p;
        // path halving; any ancestor is a valid parent
        __hip_atomic_store(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

// uf_find continuing from x whose parent p the caller already loaded.
__device__ __forceinline__ uint32_t uf_find_from(uint32_t *P, uint32_t x, uint32_t p) {
    for (;;) {
        if (p == x) return x;
        const uint32_t gp = uf_load(P + p);
        if (gp == p) return p;
        __hip_atomic_store(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
        p = uf_load(P + x);
    }
}

// Union by hooking the larger root under the smaller, so the last root of every
// component is its smallest number whatever the schedule.  A failed CAS
// returns the root's fresh parent, strictly smaller, so a+b strictly decreases
// on every retry: the loop ends even when uf_find read old values.  pa / pb:
// the parents of a and b, already loaded.
__device__ __forceinline__ void uf_unite_from(uint32_t *P, uint32_t a, uint32_t pa, uint32_t b, uint32_t pb) {
    a = uf_find_from(P, a, pa);
    b = uf_find_from(P, b, pb);
    for (;;) {
        if (a == b) return;
        if (a < b) { uint32_t t = a; a = b; b = t; }
        uint32_t expected = a;
        if (__hip_atomic_compare_exchange_strong(P + a, &expected, b, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT))
            return;
        a = uf_find(P, expected);
        b = uf_find(P, b);
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
// forest at parent + b * stride).  The parents of both endpoints in up to
// kHookIlp sketches are loaded before any of those unions walks on, so a thread
// keeps several independent memory accesses in flight instead of one chain.
__device__ __forceinline__ void unite_live(uint32_t *parent, size_t stride, uint64_t live, uint32_t u, uint32_t v) {
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
                const uint32_t *P = parent + (size_t)bs[i] * stride;
                pu[i] = uf_load(P + u);
                pv[i] = uf_load(P + v);
            }
#pragma unroll
        for (int i = 0; i < kHookIlp; ++i)
            if (i < c) uf_unite_from(parent + (size_t)bs[i] * stride, u, pu[i], v, pv[i]);
    }
}

// One thread per undirected edge: its live mask over the pass's sketches (from
// the endpoints' ids, edges[e]), then one union per live sketch (between the
// endpoints' labelling-order numbers, iedges[e]).
template <int KIND>
__global__ void __launch_bounds__(kHookBlock) k_sample_hook(const uint2 *__restrict__ edges,
                                                            const uint2 *__restrict__ iedges, uint64_t m,
                                                            const uint64_t *__restrict__ K, uint32_t B, ProbDev pm,
                                                            uint32_t *__restrict__ parent, uint32_t n) {
    const size_t ns = sketch_stride(n);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const uint2 uv = edges[e], iuv = iedges[e];
        unite_live(parent, ns, live_mask<KIND>(uv.x, uv.y, ((uint64_t)uv.x << 32) | uv.y, e, K, B, pm), iuv.x, iuv.y);
    }
}

// grid: (G, B), block 256: the blocks of sketch blockIdx.y stride over its
// first n_act numbers (the vertices with an edge; an isolated vertex stays its
// own root with no members and its own center rank).  A wave takes 4 x 64
// consecutive numbers per step, issuing the four parent loads (and root walks)
// together before counting.  In social-like graphs almost every non-root vertex
// of a sketch lies in one giant component, so per-vertex atomics on its root
// counter serialise.  Each wave therefore keeps the first root it meets as a
// "hot" root whose member count and smallest center rank it accumulates in
// registers and flushes once at the end; members of other roots are combined per
// distinct root in the wave and added with one atomic per root.
constexpr uint32_t kCompressIlp = 4;
__global__ void __launch_bounds__(256) k_compress(uint32_t *__restrict__ parent, uint32_t *__restrict__ cnt,
                                                  uint32_t n, uint32_t n_act,
                                                  const uint32_t *__restrict__ center_rank,
                                                  uint32_t *__restrict__ minc) {
    const uint32_t lane = lane_id();
    const size_t base = (size_t)blockIdx.y * sketch_stride(n);
    uint32_t *P = parent + base;
    uint32_t hot = kNone, hot_cnt = 0, hot_min = kNone;  // wave-uniform
    const uint32_t stride = gridDim.x * blockDim.x * kCompressIlp;
    const uint32_t wbase = (blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1))) * kCompressIlp;
    for (uint32_t v0 = wbase; v0 < n_act; v0 += stride) {
        uint32_t rr[kCompressIlp], pp[kCompressIlp], cc[kCompressIlp];
#pragma unroll
        for (uint32_t j = 0; j < kCompressIlp; ++j) {
            const uint32_t v = v0 + j * kWave + lane;
            rr[j] = v;
            pp[j] = v < n_act ? P[v] : v;
            if (center_rank) cc[j] = center_rank[v < n_act ? v : 0];
        }
#pragma unroll
        for (uint32_t j = 0; j < kCompressIlp; ++j) {
            const uint32_t v = v0 + j * kWave + lane;
            uint32_t r = rr[j], p = pp[j];
            while (p != r) { r = p; p = P[r]; }
            if (r != v && v < n_act) P[v] = r;
            rr[j] = r;
        }
#pragma unroll
        for (uint32_t j = 0; j < kCompressIlp; ++j) {
            const uint32_t v = v0 + j * kWave + lane;
            const bool valid = v < n_act;
            const uint32_t r = rr[j];
            bool need = valid && r != v;
            if (hot == kNone) {
                const uint64_t m = __ballot(need);
                if (m) hot = __shfl(r, (int)__builtin_ctzll(m));
            }
            const bool in_hot = need && r == hot;
            hot_cnt += (uint32_t)__popcll(__ballot(in_hot));
            if (in_hot) need = false;
            for (uint64_t m = __ballot(need); m; m = __ballot(need)) {
                const uint32_t lr = __shfl(r, (int)__builtin_ctzll(m));
                const bool same = need && r == lr;
                const uint64_t sm = __ballot(same);
                if (lane == (uint32_t)__builtin_ctzll(m)) atomicAdd(cnt + base + lr, (uint32_t)__popcll(sm));
                if (same) need = false;
            }
            if (center_rank) {
                const uint32_t cr = valid ? pin_vgpr(cc[j]) : kNone;
                bool cneed = cr != kNone && r != v;  // a root's own rank is already in minc
                uint32_t hm = (cneed && r == hot) ? cr : kNone;
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) hm = min(hm, (uint32_t)__shfl_xor(hm, off));
                hot_min = min(hot_min, hm);
                if (r == hot) cneed = false;
                for (uint64_t m = __ballot(cneed); m; m = __ballot(cneed)) {
                    const uint32_t lr = __shfl(r, (int)__builtin_ctzll(m));
                    const bool same = cneed && r == lr;
                    uint32_t mn = same ? cr : kNone;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) mn = min(mn, (uint32_t)__shfl_xor(mn, off));
                    if (lane == (uint32_t)__builtin_ctzll(m)) atomicMin(minc + base + lr, mn);
                    if (same) cneed = false;
                }
            }
        }
    }
    if (lane == 0 && hot != kNone) {
        if (hot_cnt) atomicAdd(cnt + base + hot, hot_cnt);
        if (center_rank && hot_min != kNone) atomicMin(minc + base + hot, hot_min);
    }
}

// One block of 256 threads per tile of 32 vertices; B <= 64.  The (label, size)
// entries of the tile are staged in LDS (17 KB, so that many blocks share a CU)
// and each E row segment E[v][r0 .. r0+B) is written by consecutive lanes.
// Thread t reads the entries of vertex t % 32 in sketches t / 32, t / 32 + 8, ...
// and keeps their sizes' sum for the initial gains.
constexpr int kEmitTile = 32;
constexpr int kEmitGroups = 256 / kEmitTile;
__global__ void __launch_bounds__(256) k_emit_full(const uint32_t *__restrict__ parent,
                                                   const uint32_t *__restrict__ cnt,
                                                   const uint32_t *__restrict__ newid,
                                                   const uint32_t *__restrict__ iperm, uint32_t n,
                                                   uint32_t n_linked, uint32_t B, uint32_t R, uint32_t r0,
                                                   uint2 *__restrict__ E, uint64_t *__restrict__ gain0) {
    __shared__ uint2 tile[kEmitTile][65];
    __shared__ uint64_t part[kEmitGroups][kEmitTile];
    const uint32_t v0 = blockIdx.x * kEmitTile;
    const uint32_t vi = threadIdx.x % kEmitTile, grp = threadIdx.x / kEmitTile, v = v0 + vi;
    const size_t ns = sketch_stride(n);
    uint64_t acc = 0;
    const uint32_t iv = v < n ? newid[v] : 0u;
    if (v < n && iv >= n_linked) {  // isolated: its own singleton in every sketch
        for (uint32_t b = grp; b < B; b += kEmitGroups) {
            tile[vi][b] = make_uint2(v, 1u);
            acc += 1u;
        }
    } else if (v < n) {
#pragma unroll 4
        for (uint32_t b = grp; b < B; b += kEmitGroups) {
            const size_t base = (size_t)b * ns;
            const uint32_t root = parent[base + iv];
            const uint32_t sz = 1u + cnt[base + root];
            // the label is the root's vertex id; its own entry carries the size
            tile[vi][b] = root == iv ? make_uint2(v, sz) : make_uint2(iperm[root], 0u);
            acc += sz;
        }
    }
    part[grp][vi] = acc;
    __syncthreads();
    for (uint32_t idx = threadIdx.x; idx < kEmitTile * B; idx += blockDim.x) {
        const uint32_t ti = idx / B, b = idx % B, tv = v0 + ti;
        if (tv < n) E[(size_t)tv * R + r0 + b] = tile[ti][b];
    }
    if (threadIdx.x < kEmitTile && v0 + threadIdx.x < n) {
        uint64_t s = 0;
#pragma unroll
        for (int g = 0; g < kEmitGroups; ++g) s += part[g][threadIdx.x];
        gain0[v0 + threadIdx.x] += s;
    }
}

// The largest component packed as (size << 32) | (2^32 - 1 - root).
__device__ __forceinline__ uint32_t giant_root_of(uint64_t gbest) { return 0xFFFFFFFFu - (uint32_t)gbest; }
__device__ __forceinline__ uint32_t giant_size_of(uint64_t gbest) { return (uint32_t)(gbest >> 32); }

// Per sketch (one workgroup each), the largest of the components of kGiantSamples
// evenly spaced vertices: when a sketch has a giant component (the case the
// bitmaps serve), one of the samples lies in it.  Any component is correct for
// the bulk rounds that use it; a small one only makes them search more.
constexpr uint32_t kGiantSamples = 1024;
__global__ void __launch_bounds__(256) k_giant_sample(const uint32_t *__restrict__ parent,
                                                      const uint32_t *__restrict__ cnt, uint32_t n,
                                                      unsigned long long *__restrict__ gbest) {
    __shared__ unsigned long long best_w[256 / kWave];
    const size_t base = (size_t)blockIdx.x * sketch_stride(n);
    unsigned long long best = 0;
    for (uint32_t j = threadIdx.x; j < kGiantSamples; j += blockDim.x) {
        const uint32_t v = (uint32_t)((uint64_t)j * n / kGiantSamples);
        const uint32_t root = parent[base + v];
        const unsigned long long c = ((unsigned long long)(1u + cnt[base + root]) << 32) | (0xFFFFFFFFull - root);
        best = c > best ? c : best;
    }
    best = wave_max_u64(best);
    if (lane_id() == 0) best_w[threadIdx.x / kWave] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (uint32_t w = 1; w < blockDim.x / kWave; ++w) best = best_w[w] > best ? best_w[w] : best;
        gbest[blockIdx.x] = best;
    }
}

// One pass over every vertex of the pass's B sketches (compressed: parent[b][v] is
// v's root) for CompactSketch:
//   - the initial gains, sum over sketches of |CC_b(v)|;
//   - gbits non-null: bit v % 64 of gbits[(v / 64) * R + r0 + b] = [v lies in the
//     component of giant_root_of(gbest[b])] (word-major: a vertex word's R
//     sketches are contiguous), and gsum[v] += the sizes of those components over
//     the pass's sketches (the bulk rounds' sum over covered largest components
//     starts from it);
//   - for a center v of rank cr, its triple entries label_c[cr][r0 + b] = the
//     smallest center rank in its component (minc at the root) and size_c = the
//     component size if that rank is cr's own, else 0 (center-major [rho][R]).
// A workgroup takes 64 consecutive vertices (one per lane) and its four waves
// split the sketches (wave w: b = w, w + 4, ...), so a lane issues the root loads
// of up to 16 sketches before the first size gather; the waves' gain sums meet
// in LDS.  The block's centers have consecutive ranks, so their triple entries
// of the pass are runs of B words, one per center: up to 16 centers are staged in
// LDS and written out with one lane per sketch (a block with more centers, rare
// for alpha < 1/4, writes them directly); the largest-component bitmap words of
// the block (B contiguous words) are staged the same way.  B <= 64.
constexpr uint32_t kG0Waves = 4;
constexpr uint32_t kG0PerWave = 64 / kG0Waves;
constexpr uint32_t kG0StageCenters = 16;
__global__ void __launch_bounds__(256) k_gain0_emit(const uint32_t *__restrict__ parent,
                                                    const uint32_t *__restrict__ cnt,
                                                    const uint32_t *__restrict__ minc,
                                                    const uint32_t *__restrict__ center_rank, uint32_t rho,
                                                    uint32_t n, uint32_t B, uint32_t r0, uint32_t R,
                                                    uint32_t *__restrict__ label_c, uint32_t *__restrict__ size_c,
                                                    uint64_t *__restrict__ gain0,
                                                    const unsigned long long *__restrict__ gbest,
                                                    uint64_t *__restrict__ gbits, uint32_t nw,
                                                    uint64_t *__restrict__ gsum,
                                                    const uint32_t *__restrict__ newid, uint32_t n_linked) {
    __shared__ unsigned long long part[kG0Waves][kWave], gpart[kG0Waves][kWave], gword[kWave];
    __shared__ uint32_t tl[kG0StageCenters][kWave + 1], ts[kG0StageCenters][kWave + 1];
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t v = blockIdx.x * kWave + lane;
    const bool valid = v < n;
    const uint32_t cr = valid ? center_rank[v] : kNone;
    const uint64_t cmask = __ballot(cr != kNone);  // the same in every wave of the block
    const uint32_t nc = (uint32_t)__popcll(cmask);
    const bool stage = nc <= kG0StageCenters;
    const uint32_t cr0 = nc ? (uint32_t)__builtin_amdgcn_readlane((int)cr, (int)__builtin_ctzll(cmask)) : 0u;
    const uint32_t iv = valid ? newid[v] : 0u;
    const bool alone = valid && iv >= n_linked;  // isolated: root itself, size 1, its own rank
    const size_t ns = sketch_stride(n);
    // Each group of loads is issued unconditionally (inactive lanes read entry 0)
    // and back to back, then waited for once.
    uint32_t root[kG0PerWave], sz[kG0PerWave], l[kG0PerWave], t[kG0PerWave];
#pragma unroll
    for (uint32_t i = 0; i < kG0PerWave; ++i) {
        const uint32_t b = wv + kG0Waves * i;
        const bool act = valid && b < B && !alone;
        t[i] = parent[act ? b * ns + iv : 0];
    }
#pragma unroll
    for (uint32_t i = 0; i < kG0PerWave; ++i) {
        const uint32_t b = wv + kG0Waves * i;
        const bool act = valid && b < B && !alone;
        root[i] = act ? pin_vgpr(t[i]) : ((valid && b < B) ? iv : kNone);
    }
#pragma unroll
    for (uint32_t i = 0; i < kG0PerWave; ++i) {
        const uint32_t b = wv + kG0Waves * i;
        const bool act = valid && b < B && !alone;
        t[i] = cnt[act ? b * ns + root[i] : 0];
    }
#pragma unroll
    for (uint32_t i = 0; i < kG0PerWave; ++i) {
        const uint32_t c = pin_vgpr(t[i]);
        sz[i] = root[i] == kNone ? 0u : (alone ? 1u : 1u + c);
    }
    if (cr != kNone) {
#pragma unroll
        for (uint32_t i = 0; i < kG0PerWave; ++i) {
            const uint32_t b = wv + kG0Waves * i;
            const bool act = b < B && !alone;
            t[i] = minc[act ? b * ns + root[i] : 0];
        }
#pragma unroll
        for (uint32_t i = 0; i < kG0PerWave; ++i) {
            const uint32_t m = pin_vgpr(t[i]);
            l[i] = root[i] == kNone ? kNone : (alone ? cr : m);
        }
    }
    uint64_t s = 0, gs = 0;
#pragma unroll
    for (uint32_t i = 0; i < kG0PerWave; ++i) {
        const uint32_t b = wv + kG0Waves * i;
        if (b >= B) break;  // wave-uniform
        s += sz[i];
        if (cr != kNone) {
            const uint32_t lv = l[i], sv = (l[i] == cr) ? sz[i] : 0u;
            if (stage) {
                tl[cr - cr0][b] = lv;
                ts[cr - cr0][b] = sv;
            } else {
                const size_t at = (size_t)cr * R + r0 + b;
                label_c[at] = lv;
                size_c[at] = sv;
            }
        }
        if (gbits) {
            const unsigned long long gb = gbest[b];
            const bool in_giant = valid && root[i] == giant_root_of(gb);
            const uint64_t m = __ballot(in_giant);
            if (lane == 0) gword[b] = m;
            gs += in_giant ? giant_size_of(gb) : 0u;
        }
    }
    part[wv][lane] = s;
    gpart[wv][lane] = gs;
    __syncthreads();
    if (stage) {
        for (uint32_t j = wv; j < nc; j += kG0Waves)
            if (lane < B) {
                const size_t at = (size_t)(cr0 + j) * R + r0 + lane;
                label_c[at] = tl[j][lane];
                size_c[at] = ts[j][lane];
            }
    }
    if (gbits && wv == 1 && lane < B && blockIdx.x < nw) gbits[(size_t)blockIdx.x * R + r0 + lane] = gword[lane];
    if (wv == 0 && valid) {
        uint64_t t = 0, tg = 0;
#pragma unroll
        for (uint32_t w = 0; w < kG0Waves; ++w) t += part[w][lane], tg += gpart[w][lane];
        gain0[v] += t;
        if (gbits) gsum[v] += tg;
    }
}

// ---- centers: flag, per-chunk counts, scan, ranks --------------------------
constexpr uint32_t kCenterChunk = 1024;  // vertices per block (256 threads x 4)

__device__ __forceinline__ bool center_flag(uint32_t v, uint64_t kc, uint64_t Ta) {
    return Ta == kAllLive || mix64((uint64_t)v ^ kc) < Ta;
}

__global__ void __launch_bounds__(256) k_center_count(uint32_t n, uint64_t seed, uint64_t Ta,
                                                      uint32_t *__restrict__ chunk_cnt) {
    __shared__ uint32_t s;
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    const uint64_t kc = sketch_key(seed, kSaltCenter);
    uint32_t c = 0;
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t v = blockIdx.x * kCenterChunk + j * 256 + threadIdx.x;
        if (v < n && center_flag(v, kc, Ta)) ++c;
    }
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) chunk_cnt[blockIdx.x] = s;
}

// single block: exclusive scan of chunk counts in place, total into *rho
__global__ void __launch_bounds__(1024) k_center_scan(uint32_t nchunks, uint32_t *__restrict__ chunk_cnt,
                                                      uint32_t *__restrict__ rho) {
    __shared__ uint32_t part[1024];
    const uint32_t per = (nchunks + 1023) / 1024;
    const uint32_t lo = threadIdx.x * per, hi = min(nchunks, lo + per);
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += chunk_cnt[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    uint32_t run = part[threadIdx.x] - s;
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t c = chunk_cnt[i];
        chunk_cnt[i] = run;
        run += c;
    }
    if (threadIdx.x == 1023) *rho = part[1023];
}

__global__ void __launch_bounds__(256) k_center_write(uint32_t n, uint64_t seed, uint64_t Ta,
                                                      const uint32_t *__restrict__ chunk_off,
                                                      uint32_t *__restrict__ center_rank,
                                                      uint32_t *__restrict__ centers) {
    __shared__ uint32_t flags[kCenterChunk];
    __shared__ uint32_t pre[kCenterChunk];
    const uint64_t kc = sketch_key(seed, kSaltCenter);
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t i = j * 256 + threadIdx.x, v = blockIdx.x * kCenterChunk + i;
        flags[i] = (v < n && center_flag(v, kc, Ta)) ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // serial scan of 1024 flags: negligible next to the hash
        uint32_t run = chunk_off[blockIdx.x];
        for (uint32_t i = 0; i < kCenterChunk; ++i) { pre[i] = run; run += flags[i]; }
    }
    __syncthreads();
    for (uint32_t j = 0; j < 4; ++j) {
        const uint32_t i = j * 256 + threadIdx.x, v = blockIdx.x * kCenterChunk + i;
        if (v < n) {
            if (flags[i]) {
                center_rank[v] = pre[i];
                centers[pre[i]] = v;
            } else {
                center_rank[v] = kNone;
            }
        }
    }
}

}  // namespace pacim
