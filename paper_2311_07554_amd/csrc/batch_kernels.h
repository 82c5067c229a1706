// Batched selection: many independent queries (graph, model, R, k) built and
// selected by five persistent kernels that a single hipGraph launches.
//
//   k_bat_init      every query's forests to identity and counters to 0
//   k_bat_hook      sample + union-find hooking over every (query, 64-sketch pass, edge)
//   k_bat_compress  roots and member counts over every (query, 64-number tile)
//   k_bat_emit      E[n][R] rows and initial gains over every (query, 64-vertex tile)
// The forests number vertices in each graph's labelling order (hubs first; the
// hashes take vertex ids), like the single-query build, and are vertex-major: the
// entry of number x in sketch b at x * R + b, so a vertex's entries in all R
// sketches are one contiguous row; E holds vertex ids.
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
    uint32_t *parent, *cnt;          // [n][R] scratch of the build, indexed by labelling-order number
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

// Set-up of the forests and counters, four entries per thread: item i of a query
// covers its entries 4i .. 4i + 3 of n x R, entry (x, b) at x * R + b.  pre_vn
// counts items per query, ceil(n R / 4) rounded up to a multiple of 64 so that a
// wave never straddles two queries.  Four entries that all exist are written with
// one 16-byte store per array (the arrays start 256-byte aligned), the last few
// of a query entry by entry.
__global__ void __launch_bounds__(256) k_bat_init(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                  const uint64_t *__restrict__ pre_vn,
                                                  uint32_t *__restrict__ next_q) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *next_q = 0;
    const uint64_t total = pre_vn[nq], stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre_vn, nq, i & ~63ull));
        const BatchQuery &Q = qs[q];
        const uint64_t w0 = (i - pre_vn[q]) * 4u, end = (uint64_t)Q.n * Q.R;
        if (w0 >= end) continue;
        const uint32_t x0 = (uint32_t)(w0 / Q.R), r0 = (uint32_t)(w0 - (uint64_t)x0 * Q.R);
        uint32_t x[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) x[k] = x0 + (r0 + k) / Q.R;
        if (w0 + 4u <= end) {
            *reinterpret_cast<uint4 *>(Q.parent + w0) = make_uint4(x[0], x[1], x[2], x[3]);
            *reinterpret_cast<uint4 *>(Q.cnt + w0) = make_uint4(0u, 0u, 0u, 0u);
        } else {
            for (uint32_t k = 0; w0 + k < end; ++k) {
                Q.parent[w0 + k] = x[k];
                Q.cnt[w0 + k] = 0;
            }
        }
    }
}

// The sampling pass over every (query, 64-sketch pass, chunk of kBatHookChunk
// edges) item, one workgroup per item: the workgroup reads its query once, and
// every thread of it samples the same 64 sketches.  pre_hook: items per query,
// passes x chunks.  The batched path takes the four models whose threshold the end
// points give (a per-edge model is rejected before the launch).
constexpr uint32_t kBatHookChunk = 1024;
__global__ void __launch_bounds__(1024) k_bat_hook(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                   const uint64_t *__restrict__ pre_hook) {
    __shared__ uint32_t sh_q;
    const uint64_t total = pre_hook[nq];
    for (uint64_t it = blockIdx.x; it < total; it += gridDim.x) {
        __syncthreads();  // the previous item's readers of sh_q are done
        if (threadIdx.x == 0) sh_q = find_query(pre_hook, nq, it);
        __syncthreads();
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)sh_q);  // uniform: scalar loads
        const BatchQuery &Q = qs[q];
        const uint64_t chunks = (Q.m + kBatHookChunk - 1) / kBatHookChunk;
        const uint64_t local = it - pre_hook[q];
        const uint32_t pass = (uint32_t)(local / chunks);
        const uint64_t e0 = (local - (uint64_t)pass * chunks) * kBatHookChunk;
        const uint64_t e1 = min(e0 + kBatHookChunk, Q.m);
        const uint32_t b0 = pass * 64, nb = min(64u, Q.R - b0);
        const uint64_t *K = Q.K + b0;
        const uint64_t all = nb >= 64 ? ~0ull : ((1ull << nb) - 1ull);
        for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
            const uint2 uv = Q.edges[e], iuv = Q.iedges[e];
            const uint64_t x = ((uint64_t)uv.x << 32) | uv.y;
            const uint64_t T = edge_threshold(Q.pm, uv.x, uv.y, x);
            uint64_t live = all;
            if (T != kAllLive) {
                live = 0;
                for (uint32_t c0 = 0; c0 < nb; c0 += 8) {
                    uint32_t chunk = 0;
#pragma unroll
                    for (int j = 0; j < 8; ++j) chunk |= (mix64(x ^ K[c0 + j]) < T) ? (1u << j) : 0u;
                    live |= (uint64_t)chunk << c0;
                }
                live &= all;
            }
            unite_live(Q.parent + b0, Q.R, live, iuv.x, iuv.y);
        }
    }
}

// Tiles of the per-vertex passes: 64 consecutive numbers (compress) or vertices
// (emit) of one query, one wave each; lane b of a wave is sketch p0 + b of the
// 64-sketch group p0 the wave is on, the groups taken one after another.
constexpr uint32_t kBatTile = 64;
constexpr uint32_t kBatIlp = 8;

// Roots and member counts: each lane walks every number of the tile to its root in
// its sketch (kBatIlp numbers' walks in lock step), points the number at it and
// counts it there.  A lane keeps one "hot" root per group in a register (the first
// root it meets, replaced while it has at most one member), since most members of
// a sketch often share one giant component's root.
__global__ void __launch_bounds__(256) k_bat_compress(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                      const uint64_t *__restrict__ pre_tiles) {
    const uint32_t lane = lane_id();
    const uint64_t total = pre_tiles[nq];
    for (uint64_t t = wave_index(); t < total; t += wave_count()) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre_tiles, nq, t));
        const BatchQuery &Q = qs[q];
        const uint32_t n = Q.n, R = Q.R;
        uint32_t *P = Q.parent;
        uint32_t *C = Q.cnt;
        const uint32_t x0 = (uint32_t)(t - pre_tiles[q]) * kBatTile, x1 = min(x0 + kBatTile, n);
        for (uint32_t p0 = 0; p0 < R; p0 += kWave) {
            const uint32_t b = p0 + lane;
            const bool act = b < R;
            uint32_t hot = kNone, hot_cnt = 0;
            for (uint32_t xb = x0; xb < x1; xb += kBatIlp) {
                uint32_t pp[kBatIlp], rt[kBatIlp];
#pragma unroll
                for (uint32_t j = 0; j < kBatIlp; ++j) {
                    const bool ok = act && xb + j < x1;
                    pp[j] = P[ok ? (size_t)(xb + j) * R + b : 0];
                }
#pragma unroll
                for (uint32_t j = 0; j < kBatIlp; ++j) {
                    rt[j] = xb + j;
                    if (act && xb + j < x1) pp[j] = pin_vgpr(pp[j]);
                    else pp[j] = rt[j];
                }
                for (;;) {
                    bool more = false;
#pragma unroll
                    for (uint32_t j = 0; j < kBatIlp; ++j) more |= pp[j] != rt[j];
                    if (!more) break;
                    uint32_t nx[kBatIlp];
#pragma unroll
                    for (uint32_t j = 0; j < kBatIlp; ++j) nx[j] = P[pp[j] != rt[j] ? (size_t)pp[j] * R + b : 0];
#pragma unroll
                    for (uint32_t j = 0; j < kBatIlp; ++j)
                        if (pp[j] != rt[j]) {
                            rt[j] = pp[j];
                            pp[j] = pin_vgpr(nx[j]);
                        }
                }
#pragma unroll
                for (uint32_t j = 0; j < kBatIlp; ++j) {
                    const uint32_t x = xb + j;
                    if (!act || x >= x1) continue;
                    const uint32_t r = rt[j];
                    if (r == x) continue;
                    P[(size_t)x * R + b] = r;
                    if (r != hot && hot_cnt <= 1) {
                        if (hot != kNone && hot_cnt) atomicAdd(C + (size_t)hot * R + b, hot_cnt);
                        hot = r;
                        hot_cnt = 0;
                    }
                    if (r == hot) ++hot_cnt;
                    else atomicAdd(C + (size_t)r * R + b, 1u);
                }
            }
            if (act && hot != kNone && hot_cnt) atomicAdd(C + (size_t)hot * R + b, hot_cnt);
        }
    }
}

// E rows and initial gains: per vertex v of the tile the wave reads the row of its
// number newid[v] (lane b: sketch p0 + b), gathers the root counts and the roots'
// vertex ids, and writes E[v][p0 + b] = (v, size) at a root, (the root's vertex id,
// 0) elsewhere; the vertex's sizes are summed across lanes (DPP) and groups, lane j
// keeping vertex v0 + j's sum.
__global__ void __launch_bounds__(256) k_bat_emit(const BatchQuery *__restrict__ qs, uint32_t nq,
                                                  const uint64_t *__restrict__ pre_tiles) {
    constexpr uint32_t kIlp = 4;
    const uint32_t lane = lane_id();
    const uint64_t total = pre_tiles[nq];
    for (uint64_t t = wave_index(); t < total; t += wave_count()) {
        const uint32_t q = (uint32_t)__builtin_amdgcn_readfirstlane((int)find_query(pre_tiles, nq, t));
        const BatchQuery &Q = qs[q];
        const uint32_t n = Q.n, R = Q.R;
        const uint32_t *P = Q.parent;
        const uint32_t *C = Q.cnt;
        const uint32_t v0 = (uint32_t)(t - pre_tiles[q]) * kBatTile;
        const uint32_t vl = v0 + lane;
        const uint32_t my_iv = vl < n ? Q.newid[vl] : 0u;
        const bool small = (uint64_t)n * kWave < (1ull << 32);  // a group's sum of one vertex fits 32 bits
        uint64_t g_sum = 0;
        for (uint32_t p0 = 0; p0 < R; p0 += kWave) {
            const uint32_t b = p0 + lane;
            const bool act = b < R;
            for (uint32_t j0 = 0; j0 < kBatTile; j0 += kIlp) {
                uint32_t iv[kIlp], tt[kIlp], root[kIlp], c[kIlp], lab[kIlp];
#pragma unroll
                for (uint32_t u = 0; u < kIlp; ++u) {
                    iv[u] = (uint32_t)__builtin_amdgcn_readlane((int)my_iv, (int)(j0 + u));
                    const bool rd = act && v0 + j0 + u < n;
                    tt[u] = P[rd ? (size_t)iv[u] * R + b : 0];
                }
#pragma unroll
                for (uint32_t u = 0; u < kIlp; ++u) {
                    const bool rd = act && v0 + j0 + u < n;
                    root[u] = rd ? pin_vgpr(tt[u]) : iv[u];
                    c[u] = C[rd ? (size_t)root[u] * R + b : 0];
                    lab[u] = Q.iperm[rd ? root[u] : 0];
                }
#pragma unroll
                for (uint32_t u = 0; u < kIlp; ++u) {
                    const uint32_t v = v0 + j0 + u;
                    if (v >= n) break;  // wave-uniform
                    const uint32_t sz = act ? 1u + pin_vgpr(c[u]) : 0u;
                    if (act)
                        Q.E[(size_t)v * R + b] = root[u] == iv[u] ? make_uint2(v, sz) : make_uint2(pin_vgpr(lab[u]), 0u);
                    const uint64_t g = small ? (uint64_t)wave_sum_u32_rows(sz) : wave_sum_u64(sz);
                    if (lane == j0 + u) g_sum += g;
                }
            }
        }
        if (vl < n) Q.gain0[vl] = g_sum;
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
