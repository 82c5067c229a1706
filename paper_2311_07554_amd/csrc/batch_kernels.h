// Batched selection: many independent queries (graph, model, R, k) built and
// selected by five persistent kernels that a single hipGraph launches.
//
//   k_bat_init      parent[b][x] = x, cnt = 0 over every query's R x n scratch
//   k_bat_hook      sample + union-find hooking over every (query, 64-sketch pass, edge)
//   k_bat_compress  roots and member counts over every (query, sketch, number)
//   k_bat_emit      E[n][R] rows and initial gains over every (query, 64-vertex tile)
// The forests number vertices in each graph's labelling order (hubs first; the
// hashes take vertex ids), like the single-query build; E holds vertex ids.
//   k_bat_select    one workgroup per query (work-stealing counter): winning tree
//                   built from the initial gains, then k rounds of Algorithm 5
//                   with the frontier levels separated by workgroup barriers
//   k_bat_plan / k_bat_prepare / k_bat_tree_level
//                   whole-GPU work a selection workgroup would do slowly alone:
//                   initial keys and trees of new queries, and, for a query
//                   whose next round is predicted to re-evaluate nearly every
//                   vertex (the previous seed covered a large share of every
//                   sketch), the marginal of every vertex and a rebuilt tree;
//                   the next k_bat_select launch then finishes that round
//
// Work items of the flattened kernels are located by a binary search over the
// per-query prefix sums.  E is never modified during selection: the CCs already
// covered by a seed are kept in a per-query hash set of (sketch, label) pairs,
// which lets several selections share one sketch set (the server does so).
#pragma once

#include "common.h"
#include "select_kernels.h"
#include "sketch_kernels.h"

namespace pacim {

struct BatchQuery {
    uint32_t n, R, k, kb;
    uint64_t m;                      // undirected edges
    const uint2 *edges;              // [m], u < v (vertex ids: the hash input)
    const uint2 *iedges;             // [m], the same edges' endpoints in the graph's labelling order
    const uint32_t *newid, *iperm;   // [n] labelling order: number of vertex v, vertex of number x
    ProbDev pm;
    const uint64_t *K;               // sketch keys, round_up(R, 8) + 8 entries
    uint2 *E;                        // [n][R]: (CC label, CC size if v is the label else 0)
    uint64_t *gain0;                 // [n]
    uint32_t *parent, *cnt;          // [R][n] scratch of the build, indexed by labelling-order number
    uint64_t *key;                   // [n]
    uint8_t *in_s;                   // [n]
    uint32_t *ids, *fr;              // winning tree levels / frontiers
    uint32_t *evl;                   // [n] re-evaluation list
    unsigned long long *cov;         // covered (sketch, label) pairs, cov_mask + 1 slots
    uint32_t cov_mask;
    uint32_t *seeds;                 // [k]
    unsigned long long *gains;       // [k]
    uint32_t *evals;                 // [k]
    TreeDesc td;
    uint32_t rounds_done;
    uint32_t tree_ready;             // keys, covered set and tree initialised
    uint32_t bulk_pending;           // 1: the next round evaluates every vertex
    uint32_t prep;                   // this phase: 1 initialise, 2 bulk evaluation, 0 none
    uint32_t err;
};

constexpr unsigned long long kCovEmpty = ~0ull;

// Largest q with pre[q] <= i (pre: nq + 1 non-decreasing prefix sums, i < pre[nq]).
__device__ __forceinline__ uint32_t find_query(const uint64_t *__restrict__ pre, uint32_t nq, uint64_t i) {
    uint32_t lo = 0, hi = nq;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ uint32_t cov_slot(uint32_t r, uint32_t label, uint32_t mask) {
    return ((label * 0x9E3779B1u) ^ (r * 0x85EBCA77u)) & mask;
}

// The set of one query is written and read by one workgroup only (inserts by
// atomic CAS, reads after a workgroup barrier), so workgroup-scope loads, which
// may be served by the CU's caches, see every insert.
__device__ __forceinline__ bool cov_has(const unsigned long long *cov, uint32_t mask, uint32_t r, uint32_t label) {
    const unsigned long long want = ((unsigned long long)r << 32) | label;
    for (uint32_t h = cov_slot(r, label, mask);; h = (h + 1) & mask) {
        const unsigned long long c = __hip_atomic_load(cov + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (c == want) return true;
        if (c == kCovEmpty) return false;
    }
}

__device__ __forceinline__ void cov_insert(unsigned long long *cov, uint32_t mask, uint32_t r, uint32_t label) {
    const unsigned long long want = ((unsigned long long)r << 32) | label;
    for (uint32_t h = cov_slot(r, label, mask);; h = (h + 1) & mask) {
        const unsigned long long old = atomicCAS(cov + h, kCovEmpty, want);
        if (old == kCovEmpty || old == want) return;
    }
}

// Uncovered size of entry e = E[v][r] (e.x: label, e.y: size if v is the label).
__device__ __forceinline__ uint32_t uncovered_size(const uint2 *__restrict__ E, uint32_t R, uint32_t v, uint32_t r,
                                                   uint2 e, const unsigned long long *cov, uint32_t mask) {
    uint32_t sz = (e.x == v) ? e.y : E[(size_t)e.x * R + r].y;
    if (sz > 1 && cov_has(cov, mask, r, e.x)) sz = 0;
    return sz;
}

// Marginal of up to kEvalUnroll vertices by one wave, their loads issued
// together: one evaluation is a short chain of dependent loads (row entry,
// label's size, covered-set probe), so a wave keeps several chains in flight.
constexpr int kEvalUnroll = 4;
__device__ __forceinline__ void marginal_cov_multi(const uint2 *__restrict__ E, uint32_t R, const uint32_t *vs,
                                                   const unsigned long long *cov, uint32_t mask, uint64_t *out) {
    uint64_t s[kEvalUnroll];
#pragma unroll
    for (int u = 0; u < kEvalUnroll; ++u) s[u] = 0;
    for (uint32_t r = lane_id(); r < R; r += kWave) {
        uint2 e[kEvalUnroll];
#pragma unroll
        for (int u = 0; u < kEvalUnroll; ++u)
            e[u] = vs[u] != kNone ? E[(size_t)vs[u] * R + r] : make_uint2(0u, 0u);
#pragma unroll
        for (int u = 0; u < kEvalUnroll; ++u)
            if (vs[u] != kNone) s[u] += uncovered_size(E, R, vs[u], r, e[u], cov, mask);
    }
#pragma unroll
    for (int u = 0; u < kEvalUnroll; ++u) out[u] = wave_sum_u64(s[u]);
}

// Marginal(S, v) on immutable full labels: uncovered CC sizes over the R sketches
// (one wave).  A singleton CC {v} is never covered while v is not a seed.
__device__ __forceinline__ uint64_t marginal_cov(const uint2 *__restrict__ E, uint32_t R, uint32_t v,
                                                 const unsigned long long *cov, uint32_t mask) {
    const uint2 *row = E + (size_t)v * R;
    uint64_t s = 0;
    for (uint32_t r = lane_id(); r < R; r += kWave) {
        const uint2 e = row[r];
        uint32_t sz = (e.x == v) ? e.y : E[(size_t)e.x * R + r].y;
        if (sz > 1 && cov_has(cov, mask, r, e.x)) sz = 0;
        s += sz;
    }
    return wave_sum_u64(s);
}

// (sketch, vertex) items: each query's R rows of n vertices are padded to whole
// waves (npad = n rounded up to 64), so a wave never straddles two rows and finds
// its query and sketch once.
__device__ __forceinline__ uint32_t row_pad(uint32_t n) { return (n + 63u) & ~63u; }

__global__ void __launch_bounds__(256) k_bat_init(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                  const uint64_t *__restrict__ pre_vn,
                                                  uint32_t *__restrict__ next_q) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_q = 0;
    const uint64_t total = pre_vn[nq], stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint64_t i0 = i & ~63ull;
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre_vn, nq, i0));
        const BatchQuery &Q = qs[q];
        const uint32_t npad = row_pad(Q.n);
        const uint64_t wl = i0 - pre_vn[q];
        const uint32_t b = (uint32_t)(wl / npad);
        const uint32_t v = (uint32_t)(wl - (uint64_t)b * npad) + lane_id();
        if (v < Q.n) {
            Q.parent[(size_t)b * Q.n + v] = v;
            Q.cnt[(size_t)b * Q.n + v] = 0;
        }
    }
}

// pre_hook: per-query item counts rounded up to whole waves, so every wave lies in
// one query and reads its descriptor through scalar loads.  blockDim must be a
// multiple of 64.
__global__ void __launch_bounds__(1024) k_bat_hook(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                   const uint64_t *__restrict__ pre_hook) {
    const uint64_t total = pre_hook[nq], stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre_hook, nq, i & ~63ull));
        const BatchQuery &Q = qs[q];
        const uint64_t local = i - pre_hook[q];
        if (local >= (uint64_t)((Q.R + 63) / 64) * Q.m) continue;
        const uint32_t pass = (uint32_t)(local / Q.m);
        const uint64_t e = local - (uint64_t)pass * Q.m;
        const uint32_t b0 = pass * 64, nb = min(64u, Q.R - b0);
        const uint2 uv = Q.edges[e], iuv = Q.iedges[e];
        const uint64_t x = ((uint64_t)uv.x << 32) | uv.y;
        const uint64_t T = edge_threshold(Q.pm, uv.x, uv.y, x);
        uint64_t live;
        if (T == kAllLive) {
            live = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
        } else {
            live = 0;
            const uint64_t *K = Q.K + b0;
            for (uint32_t c0 = 0; c0 < nb; c0 += 8) {
                uint32_t chunk = 0;
#pragma unroll
                for (int j = 0; j < 8; ++j) chunk |= (mix64(x ^ K[c0 + j]) < T) ? (1u << j) : 0u;
                live |= (uint64_t)chunk << c0;
            }
            live &= nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
        }
        unite_live(Q.parent + (size_t)b0 * Q.n, Q.n, 1u, live, iuv.x, iuv.y);
    }
}

// Roots and member counts, one wave per 64 vertices of one (query, sketch) row.
// Each wave keeps one hot counter (in practice a giant component's root) in a
// register, across rows (it is an address); members of other roots are
// combined per distinct root in the wave and added with one atomic per root.
__global__ void __launch_bounds__(256) k_bat_compress(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                      const uint64_t *__restrict__ pre_vn) {
    const uint32_t lane = lane_id();
    const uint64_t total = pre_vn[nq], stride = (uint64_t)gridDim.x * blockDim.x;
    unsigned long long hot = 0;
    uint32_t hot_cnt = 0;
    for (uint64_t wb = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) & ~63ull; wb < total; wb += stride) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre_vn, nq, wb));
        const BatchQuery &Q = qs[q];
        const uint32_t n = Q.n, npad = row_pad(n);
        const uint64_t wl = wb - pre_vn[q];
        const uint32_t b = (uint32_t)(wl / npad);
        const uint32_t v = (uint32_t)(wl - (uint64_t)b * npad) + lane;
        uint32_t *P = Q.parent + (size_t)b * n;
        unsigned long long target = 0;
        if (v < n) {
            uint32_t r = v, p = P[v];
            while (p != r) { r = p; p = P[r]; }
            if (r != v) {
                P[v] = r;
                target = (unsigned long long)(Q.cnt + (size_t)b * n + r);
            }
        }
        bool need = target != 0;
        if (hot == 0) {
            const uint64_t m = __ballot(need);
            if (m) hot = __shfl(target, (int)__builtin_ctzll(m));
        }
        const bool in_hot = need && target == hot;
        hot_cnt += (uint32_t)__popcll(__ballot(in_hot));
        if (in_hot) need = false;
        for (uint64_t m = __ballot(need); m; m = __ballot(need)) {
            const unsigned long long lt = __shfl(target, (int)__builtin_ctzll(m));
            const bool same = need && target == lt;
            const uint64_t sm = __ballot(same);
            if (lane == (uint32_t)__builtin_ctzll(m)) atomicAdd(reinterpret_cast<uint32_t *>(lt), (uint32_t)__popcll(sm));
            if (same) need = false;
        }
    }
    if (lane == 0 && hot && hot_cnt) atomicAdd(reinterpret_cast<uint32_t *>(hot), hot_cnt);
}

// One block of 256 threads per (query, kEmitTile-vertex tile); the R sketches are
// staged 64 at a time in LDS so E row segments are written by consecutive lanes.
__global__ void __launch_bounds__(256) k_bat_emit(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                  const uint64_t *__restrict__ pre_tiles) {
    __shared__ uint2 tile[kEmitTile][65];
    __shared__ uint32_t gsz[kEmitTile][65];
    const uint64_t total = pre_tiles[nq];
    for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
        const uint32_t q = find_query(pre_tiles, nq, it);
        const BatchQuery &Q = qs[q];
        const uint32_t n = Q.n, R = Q.R;
        const uint32_t v0 = (uint32_t)(it - pre_tiles[q]) * kEmitTile;
        uint64_t gsum = 0;
        for (uint32_t b0 = 0; b0 < R; b0 += 64) {
            const uint32_t nb = min(64u, R - b0);
            for (uint32_t idx = threadIdx.x; idx < kEmitTile * nb; idx += blockDim.x) {
                const uint32_t b = idx / kEmitTile, vi = idx % kEmitTile, v = v0 + vi;
                if (v < n) {
                    const size_t base = (size_t)(b0 + b) * n;
                    const uint32_t x = Q.newid[v];
                    const uint32_t root = Q.parent[base + x];
                    const uint32_t s = 1u + Q.cnt[base + root];
                    // the label is the root's vertex id; its own entry carries the size
                    tile[vi][b] = root == x ? make_uint2(v, s) : make_uint2(Q.iperm[root], 0u);
                    gsz[vi][b] = s;
                }
            }
            __syncthreads();
            for (uint32_t idx = threadIdx.x; idx < kEmitTile * nb; idx += blockDim.x) {
                const uint32_t vi = idx / nb, b = idx % nb, v = v0 + vi;
                if (v < n) Q.E[(size_t)v * R + b0 + b] = tile[vi][b];
            }
            if (threadIdx.x < kEmitTile)
                for (uint32_t b = 0; b < nb; ++b) gsum += gsz[threadIdx.x][b];
            __syncthreads();
        }
        if (threadIdx.x < kEmitTile && v0 + threadIdx.x < n) Q.gain0[v0 + threadIdx.x] = gsum;
    }
}

// Selection, one workgroup per query (blockDim a multiple of 64, at most 1024).
// Runs up to round_budget rounds of each query it takes; rounds_done persists so
// a later launch continues where this one stopped.
// order: the queries in the order workgroups take them (largest first).
// stop_on_heavy: leave a query (bulk_pending = 1) before a round that follows a
// seed of gain >= R*n/64, for the next preparation to evaluate all its vertices.
__global__ void __launch_bounds__(1024) k_bat_select(BatchQuery *__restrict__ qs, uint32_t nq,
                                                     const uint32_t *__restrict__ order,
                                                     uint32_t *__restrict__ next_q, uint32_t round_budget,
                                                     uint32_t stop_on_heavy) {
    __shared__ uint32_t sh_q, sh_prep;
    __shared__ unsigned long long sh_delta;
    __shared__ uint32_t sh_fr[kMaxLevels + 1], sh_ev[kMaxLevels + 1];
    const uint32_t lane = lane_id(), wave = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t j = atomicAdd(next_q, 1u);
            sh_q = j < nq ? order[j] : nq;
        }
        __syncthreads();
        const uint32_t qi = sh_q;
        __syncthreads();
        if (qi >= nq) break;
        BatchQuery &Q = qs[qi];
        const uint32_t n = Q.n, R = Q.R, kb = Q.kb, k = Q.k, cmask = Q.cov_mask;
        const TreeDesc &td = Q.td;
        const uint2 *E = Q.E;
        uint64_t *key = Q.key;
        uint32_t *ids = Q.ids, *fr = Q.fr, *evl = Q.evl;
        uint32_t rd = Q.rounds_done;
        // this phase's preparation, read once by thread 0 and shared: every wave must
        // take the same path through the barrier-separated steps below
        if (threadIdx.x == 0) {
            const uint32_t prep = Q.prep;
            sh_prep = prep;
            if (prep == 1) Q.tree_ready = 1;
            if (prep == 2) {
                for (int l = 0; l <= kMaxLevels; ++l) sh_ev[l] = 0;
                sh_ev[0] = n - rd;
                Q.bulk_pending = 0;
            }
            Q.prep = 0;
        }
        __syncthreads();
        const bool bulk = sh_prep == 2;  // keys fresh, tree rebuilt: this round's seed is the root
        for (uint32_t budget = 0; rd < k && budget < round_budget; ++budget, ++rd) {
            if (!(bulk && budget == 0) && stop_on_heavy && rd > 0 &&
                Q.gains[rd - 1] * 64ull >= (unsigned long long)R * n) {
                if (threadIdx.x == 0) Q.bulk_pending = 1;
                break;
            }
            if (bulk && budget == 0) goto round_end;
            // the root is always stale: evaluate it
            if (wave == 0) {
                const uint32_t rid = ids[td.lvl_off[0]];
                const uint64_t g = marginal_cov(E, R, rid, Q.cov, cmask);
                const uint64_t nk = Q.in_s[rid] ? 0ull : pack_key(g, rid, kb);
                if (lane == 0) {
                    key[rid] = nk;
                    sh_delta = nk;
                    for (int l = 0; l <= kMaxLevels; ++l) { sh_fr[l] = 0; sh_ev[l] = 0; }
                    sh_fr[0] = 1;
                    sh_ev[0] = 1;
                    fr[td.lvl_off[0]] = 0;
                }
            }
            __syncthreads();
            for (uint32_t l = 0; l < td.D; ++l) {
                const uint64_t delta = sh_delta;
                const bool leaf_children = (l + 1 == td.D);
                for (uint32_t i = wave; i < sh_fr[l]; i += nwaves) {
                    const uint32_t t = fr[td.lvl_off[l] + i];
                    const uint32_t pid = ids[td.lvl_off[l] + t];
                    const uint32_t c = t * kFan + lane;
                    const bool valid = c < td.lvl_n[l + 1];
                    uint32_t cid = 0;
                    bool stale = false, need_eval = false;
                    if (valid) {
                        cid = leaf_children ? c : ids[td.lvl_off[l + 1] + c];
                        stale = cid != pid;
                        need_eval = stale && key[cid] >= delta;
                    }
                    const bool explore = valid && !leaf_children && (!stale || need_eval);
                    uint32_t tot;
                    const uint32_t ep = wave_append(&sh_ev[l + 1], need_eval, &tot);
                    if (need_eval) evl[ep] = cid;
                    const uint32_t fp = wave_append(&sh_fr[l + 1], explore, &tot);
                    if (explore) fr[td.lvl_off[l + 1] + fp] = c;
                }
                __syncthreads();
                const uint32_t ne = sh_ev[l + 1];
                for (uint32_t i0 = wave * kEvalUnroll; i0 < ne; i0 += nwaves * kEvalUnroll) {
                    uint32_t vs[kEvalUnroll];
                    uint64_t g[kEvalUnroll];
#pragma unroll
                    for (int u = 0; u < kEvalUnroll; ++u) vs[u] = i0 + u < ne ? evl[i0 + u] : kNone;
                    marginal_cov_multi(E, R, vs, Q.cov, cmask, g);
                    if (lane == 0) {
                        uint64_t best = 0;
#pragma unroll
                        for (int u = 0; u < kEvalUnroll; ++u) {
                            if (vs[u] == kNone) continue;
                            const uint64_t nk = Q.in_s[vs[u]] ? 0ull : pack_key(g[u], vs[u], kb);
                            key[vs[u]] = nk;
                            best = nk > best ? nk : best;
                        }
                        atomicMax(&sh_delta, (unsigned long long)best);
                    }
                }
                __syncthreads();
            }
            for (int l = (int)td.D - 1; l >= 0; --l) {
                for (uint32_t i = wave; i < sh_fr[l]; i += nwaves) {
                    const uint32_t t = fr[td.lvl_off[l] + i];
                    const uint32_t w = relink_node(td, ids, key, (uint32_t)l, t, 0, 0, 0, false);
                    if (lane == 0) ids[td.lvl_off[l] + t] = w;
                }
                __syncthreads();
            }
        round_end:
            if (wave == 0) {
                const uint32_t s = ids[td.lvl_off[0]];
                const uint64_t ks = key[s];
                if (lane == 0) {
                    if (ks == 0 || Q.in_s[s]) Q.err = 1;
                    uint32_t evs = 0;
                    for (int l = 0; l <= kMaxLevels; ++l) evs += sh_ev[l];
                    Q.seeds[rd] = s;
                    Q.gains[rd] = key_gain(ks, kb);
                    Q.evals[rd] = evs;
                    Q.in_s[s] = 1;
                    key[s] = 0;
                }
                uint32_t child = s, child_id = s;
                uint64_t child_key = 0;
                for (int l = (int)td.D - 1; l >= 0; --l) {
                    const uint32_t t = child >> kFanLog;
                    const uint32_t w = relink_node(td, ids, key, (uint32_t)l, t, child, child_id, child_key, true);
                    const uint64_t wk = (w == s) ? 0ull : key[w];
                    if (lane == 0) ids[td.lvl_off[l] + t] = w;
                    child = t;
                    child_id = w;
                    child_key = wk;
                }
                for (uint32_t r = lane; r < R; r += kWave) cov_insert(Q.cov, cmask, r, E[(size_t)s * R + r].x);
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) Q.rounds_done = rd;
        __syncthreads();
    }
}

// Decides each query's work for this phase and rearms the selection counter.
__global__ void k_bat_plan(BatchQuery *__restrict__ qs, uint32_t nq, uint32_t *__restrict__ next_q) {
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) *next_q = 0;
    if (q < nq) qs[q].prep = !qs[q].tree_ready ? 1u : (qs[q].bulk_pending == 1 ? 2u : 0u);
}

// Items of 64 vertices (or 64 covered-set slots); pre counts max(ceil(n/64),
// ceil(slots/64)) per query (wave-uniform).  prep 1: initial keys, no seeds, empty
// covered set; prep 2: every vertex's marginal.
__global__ void __launch_bounds__(256) k_bat_prepare(BatchQuery *__restrict__ qs, uint32_t nq,
                                                     const uint64_t *__restrict__ pre) {
    const uint64_t total = pre[nq];
    const uint32_t lane = lane_id();
    for (uint64_t i = wave_index(); i < total; i += wave_count()) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre, nq, i));
        BatchQuery &Q = qs[q];
        const uint32_t prep = Q.prep;
        if (prep == 0) continue;
        const uint32_t v0 = (uint32_t)(i - pre[q]) * kWave;
        if (prep == 1) {
            const uint32_t v = v0 + lane;
            if (v < Q.n) {
                Q.key[v] = pack_key(Q.gain0[v], v, Q.kb);
                Q.in_s[v] = 0;
            }
            if (v <= Q.cov_mask) Q.cov[v] = kCovEmpty;
        } else {
            for (uint32_t j = 0; j < kWave && v0 + j < Q.n; j += kEvalUnroll) {
                uint32_t vs[kEvalUnroll];
                uint64_t g[kEvalUnroll];
#pragma unroll
                for (int u = 0; u < kEvalUnroll; ++u) {
                    const uint32_t v = v0 + j + u;
                    vs[u] = (j + u < kWave && v < Q.n) ? v : kNone;
                }
                marginal_cov_multi(Q.E, Q.R, vs, Q.cov, Q.cov_mask, g);
                if (lane < kEvalUnroll && vs[lane] != kNone) {
                    uint64_t gl = g[0];
#pragma unroll
                    for (int u = 1; u < kEvalUnroll; ++u) gl = lane == (uint32_t)u ? g[u] : gl;
                    Q.key[vs[lane]] = Q.in_s[vs[lane]] ? 0ull : pack_key(gl, vs[lane], Q.kb);
                }
            }
        }
    }
}

// One level of the winning trees of the queries with prep != 0, j levels above
// the deepest internal level (pre: per-query node counts of that level; one wave
// per node).  Launched for j = 0, 1, ... so each level sees its children final.
__global__ void __launch_bounds__(256) k_bat_tree_level(BatchQuery *__restrict__ qs, uint32_t nq,
                                                        const uint64_t *__restrict__ pre, uint32_t j) {
    const uint64_t total = pre[nq];
    for (uint64_t i = wave_index(); i < total; i += wave_count()) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre, nq, i));
        BatchQuery &Q = qs[q];
        if (Q.prep == 0 || j >= Q.td.D) continue;
        const uint32_t l = Q.td.D - 1 - j;
        const uint32_t t = (uint32_t)(i - pre[q]);
        if (t >= Q.td.lvl_n[l]) continue;
        const uint32_t w = relink_node(Q.td, Q.ids, Q.key, l, t, 0, 0, 0, false);
        if (lane_id() == 0) Q.ids[Q.td.lvl_off[l] + t] = w;
    }
}

}  // namespace pacim
