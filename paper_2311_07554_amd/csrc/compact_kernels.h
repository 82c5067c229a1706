// CompactSketch evaluation (Sec. 3): Marginal(S, v) = sum_r delta_r with
// <delta_r, l> = GetCenter(Phi_r, v, S), and MarkSeed zeroing size_c of (r, l).
//
// GetCenter is a BFS from v over the live edges of sketch r that stops at the
// first center it reaches (delta = size_c[label_c[center]], the CC's size or 0
// once a seed covered it); if the CC holds no center the BFS exhausts it and
// delta = |CC|, or 0 if a seed was met.  Theorem 3.1 bounds the expected number
// of vertices visited by min(1/alpha, T).
//
// GPU form: one wave per (vertex, sketch) search.  The wave takes one queued
// vertex at a time and scans its adjacency 64 neighbours per step, one lane per
// neighbour (hash test, center test, ballot); newly reached vertices are
// deduplicated in an LDS hash set and appended to an LDS queue with one ballot.
// A search that would outgrow the LDS queue is handed, whole, to a slower
// global-memory version (bitmap + queue of n entries per slot), so the result is
// exact for every component size.
#pragma once

#include "common.h"
#include "select_kernels.h"
#include "sketch_kernels.h"

namespace pacim {

constexpr uint32_t kQCap = 512;    // LDS queue entries per wave
constexpr uint32_t kHCap = 1024;   // LDS hash-set slots per wave (2 x queue)
constexpr uint32_t kBfsBlock = 256;
constexpr uint32_t kBfsWaves = kBfsBlock / kWave;

struct GraphDev {
    const uint64_t *off;
    const uint32_t *cols;
};

struct CompactDev;
__device__ __forceinline__ size_t tri_at(const CompactDev &cd, uint32_t r, uint32_t i);

struct CompactDev {
    const uint32_t *center_rank;   // [n], rank or kNone
    const uint32_t *label_c;       // [rho][R] (center-major: a center's R entries are contiguous)
    uint32_t *size_c;              // [rho][R]
    uint32_t rho;
    uint64_t kc, Ta;               // center test: mix64(v ^ kc) < Ta (a hash, no memory access)
    unsigned long long *memo;      // [slots][R][2] kept GetCenter results (below), ~0 if empty
    uint32_t memo_mask;            // slots - 1 (slots a power of two)
    uint32_t R;
    unsigned long long *covmin;    // [R][nw] bit m: the component without a center whose smallest
                                   // vertex is m holds a seed (set by MarkSeed)
    uint32_t nw;                   // 64-bit words per sketch, ceil(n / 64)
};

// Entry of sketch r and center rank i in label_c / size_c.
__device__ __forceinline__ size_t tri_at(const CompactDev &cd, uint32_t r, uint32_t i) { return (size_t)i * cd.R + r; }

// What GetCenter finds from (v, r) never changes (a sketch's components are
// fixed; only their compact sizes are zeroed and seeds are added), so results are
// kept, direct-mapped by vertex, and a later search from the same vertex in the
// same sketch (a re-evaluation, or MarkSeed from the vertex just chosen) reads
// them instead:
//   word 0 = (v << 32) | label             the component holds a center: delta is
//                                           the compact size at that label;
//   word 0 = (v << 32) | 2^31 | size,      the component has no center: delta is
//   word 1 = (v << 32) | smallest vertex   its size unless a seed lies in it, which
//                                           MarkSeed records in covmin by that vertex.
// Both words carry the vertex id, and every write for (v, r) writes the same
// values, so a slot being taken over by another vertex reads as a miss whatever
// the interleaving.
constexpr uint32_t kMemoNoCenter = 0x80000000u;
__device__ __forceinline__ unsigned long long *memo_entry(const CompactDev &cd, uint32_t v, uint32_t r) {
    const uint32_t slot = (v * 0x9E3779B1u ^ (v >> 16)) & cd.memo_mask;
    return cd.memo + ((size_t)slot * cd.R + r) * 2;
}

struct BfsOut {
    uint64_t delta;
    uint32_t label;   // label_c of the reached center, or kNone
    bool overflow;
    uint32_t visits;  // vertices whose adjacency the search scanned
    uint32_t ccsize;  // no center reached (and no overflow): the component's size
    uint32_t ccmin;   //   and its smallest vertex
};

__device__ __forceinline__ bool covmin_test(const CompactDev &cd, uint32_t r, uint32_t m) {
    return (__hip_atomic_load(&cd.covmin[(size_t)r * cd.nw + (m >> 6)], __ATOMIC_RELAXED,
                              __HIP_MEMORY_SCOPE_AGENT) >> (m & 63)) & 1ull;
}

// MarkSeed's record for a search that ended without a center (one lane).
__device__ __forceinline__ void covmin_mark(const CompactDev &cd, uint32_t r, uint32_t m) {
    atomicOr(&cd.covmin[(size_t)r * cd.nw + (m >> 6)], 1ull << (m & 63));
}

__device__ __forceinline__ uint32_t hs_slot(uint32_t w) { return (w * 0x9E3779B1u) >> (32 - 10); }
static_assert(kHCap == 1024, "hs_slot assumes 2^10 slots");

// The center's label and, in the same round trip, its own size entry: when the
// center labels its component (the usual case) that is the component's size, and
// only otherwise is the label's entry read.
__device__ __forceinline__ BfsOut center_hit(const CompactDev &cd, uint32_t r, uint32_t rank) {
    const size_t at = tri_at(cd, r, rank);
    const uint32_t l = cd.label_c[at];
    const uint32_t own = pin_vgpr(cd.size_c[at]);
    return BfsOut{l == rank ? own : cd.size_c[tri_at(cd, r, l)], l, false, 0};
}

// GetCenter with the queue and visited set in LDS (q: kQCap, hs: kHCap words).
// o0v / o1v: v's adjacency range, already loaded by the caller.
__device__ BfsOut getcenter_lds(const GraphDev &g, const ProbDev &pm, uint64_t kr, const CompactDev &cd,
                                uint32_t r, const uint8_t *__restrict__ in_s, uint32_t v, uint32_t *q,
                                uint32_t *hs, uint64_t o0v, uint64_t o1v) {
    const uint32_t lane = lane_id();
    if (center_flag(v, cd.kc, cd.Ta)) return center_hit(cd, r, cd.center_rank[v]);
    for (uint32_t i = lane; i < kHCap; i += kWave) hs[i] = kNone;
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        q[0] = v;
        hs[hs_slot(v)] = v;
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t head = 0, tail = 1, found = kNone;
    // the adjacency range of the next queued vertex is loaded together with the
    // current vertex's neighbours when that vertex is already queued (pre = its
    // queue index), so a scanned vertex usually costs one round trip, not two
    uint32_t pre = 0;
    uint64_t p0 = o0v, p1 = o1v;
    while (head < tail && found == kNone) {
        const uint32_t u = q[head];
        uint64_t o0 = p0, o1 = p1;
        if (pre != head) {
            o0 = g.off[u];
            o1 = g.off[u + 1];
        }
        ++head;
        pre = kNone;
        if (head < tail) {
            const uint32_t un = q[head];
            pre = head;
            p0 = g.off[un];
            p1 = g.off[un + 1];
        }
        for (uint64_t base = o0; base < o1; base += kWave) {
            const uint64_t j = base + lane;
            bool live = false;
            uint32_t w = 0;
            if (j < o1) {
                w = g.cols[j];
                const uint64_t x = edge_word(u, w);
                live = is_live(x, kr, pm.csr_thr ? pm.csr_thr[j] : edge_threshold(pm, u, w, x));
            }
            const uint64_t cm = __ballot(live && center_flag(w, cd.kc, cd.Ta));
            if (cm) {
                found = cd.center_rank[__shfl(w, (int)__builtin_ctzll(cm))];
                break;
            }
            bool ins = false;
            if (live) {
                uint32_t h = hs_slot(w);
                for (;;) {
                    const uint32_t old = atomicCAS(&hs[h], kNone, w);
                    if (old == kNone) { ins = true; break; }
                    if (old == w) break;
                    h = (h + 1) & (kHCap - 1);
                }
            }
            const uint64_t im = __ballot(ins);
            const uint32_t ni = (uint32_t)__popcll(im);
            if (tail + ni > kQCap) return BfsOut{0, kNone, true, head};
            if (ins) q[tail + (uint32_t)__popcll(im & ((1ull << lane) - 1ull))] = w;
            tail += ni;
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (found != kNone) {
        BfsOut o = center_hit(cd, r, found);
        o.visits = head;
        return o;
    }
    // the component has no center: its smallest vertex, and whether a seed lies in
    // it (read once for the whole queue, off the search's chain of loads)
    uint32_t mn = kNone;
    bool seed = false;
    for (uint32_t i = lane; i < tail; i += kWave) {
        const uint32_t w = q[i];
        mn = min(mn, w);
        seed = seed || in_s[w] != 0;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mn = min(mn, (uint32_t)__shfl_xor(mn, off));
    const bool met = __ballot(seed) != 0;
    return BfsOut{met ? 0ull : (uint64_t)tail, kNone, false, head, tail, mn};
}

// The same search with an n-entry queue and an n-bit visited bitmap in global
// memory (one slot per wave); clears its bitmap bits before returning.
__device__ BfsOut getcenter_global(const GraphDev &g, const ProbDev &pm, uint64_t kr, const CompactDev &cd,
                                   uint32_t r, const uint8_t *__restrict__ in_s, uint32_t v, uint32_t *gq,
                                   uint32_t *gvis) {
    const uint32_t lane = lane_id();
    if (center_flag(v, cd.kc, cd.Ta)) return center_hit(cd, r, cd.center_rank[v]);
    if (lane == 0) {
        gq[0] = v;
        atomicOr(&gvis[v >> 5], 1u << (v & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    uint32_t head = 0, tail = 1, found = kNone;
    while (head < tail && found == kNone) {
        const uint32_t u = __hip_atomic_load(&gq[head], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        ++head;
        const uint64_t o1 = g.off[u + 1];
        for (uint64_t base = g.off[u]; base < o1; base += kWave) {
            const uint64_t j = base + lane;
            bool live = false;
            uint32_t w = 0;
            if (j < o1) {
                w = g.cols[j];
                const uint64_t x = edge_word(u, w);
                live = is_live(x, kr, pm.csr_thr ? pm.csr_thr[j] : edge_threshold(pm, u, w, x));
            }
            const uint64_t cm = __ballot(live && center_flag(w, cd.kc, cd.Ta));
            if (cm) {
                found = cd.center_rank[__shfl(w, (int)__builtin_ctzll(cm))];
                break;
            }
            bool ins = false;
            if (live) {
                const uint32_t bit = 1u << (w & 31);
                ins = (atomicOr(&gvis[w >> 5], bit) & bit) == 0;
            }
            const uint64_t im = __ballot(ins);
            if (ins) gq[tail + (uint32_t)__popcll(im & ((1ull << lane) - 1ull))] = w;
            tail += (uint32_t)__popcll(im);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
    // clear the visited bits; for a component without a center, its smallest vertex
    // and whether a seed lies in it
    uint32_t mn = kNone;
    bool seed = false;
    for (uint32_t i = lane; i < tail; i += kWave) {
        const uint32_t w = __hip_atomic_load(&gq[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        atomicAnd(&gvis[w >> 5], ~(1u << (w & 31)));
        mn = min(mn, w);
        if (found == kNone) seed = seed || in_s[w] != 0;
    }
    const bool met = __ballot(seed) != 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    if (found != kNone) {
        BfsOut o = center_hit(cd, r, found);
        o.visits = head;
        return o;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mn = min(mn, (uint32_t)__shfl_xor(mn, off));
    return BfsOut{met ? 0ull : (uint64_t)tail, kNone, false, head, tail, mn};
}

// A kept result for (v, r), if the slot holds one (all lanes read it).
__device__ __forceinline__ bool memo_read(const CompactDev &cd, uint32_t v, uint32_t r, BfsOut *o) {
    const unsigned long long *e = memo_entry(cd, v, r);
    const unsigned long long x = __hip_atomic_load(&e[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(x >> 32) != v) return false;
    const uint32_t p = (uint32_t)x;
    if (!(p & kMemoNoCenter)) {
        *o = BfsOut{cd.size_c[tri_at(cd, r, p)], p, false, 0, 0, 0};
        return true;
    }
    const unsigned long long y = __hip_atomic_load(&e[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((uint32_t)(y >> 32) != v) return false;
    const uint32_t size = p & ~kMemoNoCenter, m = (uint32_t)y;
    *o = BfsOut{covmin_test(cd, r, m) ? 0ull : (uint64_t)size, kNone, false, 0, size, m};
    return true;
}

// Keeps the result of a completed search from (v, r) (lane 0).
__device__ __forceinline__ void memo_write(const CompactDev &cd, uint32_t v, uint32_t r, const BfsOut &o) {
    unsigned long long *e = memo_entry(cd, v, r);
    const unsigned long long tag = (unsigned long long)v << 32;
    if (o.label != kNone) {
        __hip_atomic_store(&e[0], tag | o.label, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if (o.ccsize < kMemoNoCenter) {
        __hip_atomic_store(&e[1], tag | o.ccmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&e[0], tag | kMemoNoCenter | o.ccsize, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// GetCenter through the kept results (all lanes take part; lane 0 writes).
// v's adjacency range is loaded beside the probe of the kept results, so a search
// that misses them starts one round trip earlier.
__device__ __forceinline__ BfsOut getcenter_memo_lds(const GraphDev &g, const ProbDev &pm, uint64_t kr,
                                                     const CompactDev &cd, uint32_t r, const uint8_t *in_s, uint32_t v,
                                                     uint32_t *q, uint32_t *hs) {
    const uint64_t o0v = g.off[v], o1v = g.off[v + 1];
    BfsOut o;
    if (memo_read(cd, v, r, &o)) return o;
    o = getcenter_lds(g, pm, kr, cd, r, in_s, v, q, hs, o0v, o1v);
    if (!o.overflow && lane_id() == 0) memo_write(cd, v, r, o);
    return o;
}

__device__ __forceinline__ BfsOut getcenter_memo_global(const GraphDev &g, const ProbDev &pm, uint64_t kr,
                                                        const CompactDev &cd, uint32_t r, const uint8_t *in_s,
                                                        uint32_t v, uint32_t *gq, uint32_t *gvis) {
    BfsOut o;
    if (memo_read(cd, v, r, &o)) return o;
    o = getcenter_global(g, pm, kr, cd, r, in_s, v, gq, gvis);
    if (lane_id() == 0) memo_write(cd, v, r, o);
    return o;
}

// The overflow list holds ov_cap tasks: evaluation searches in its first half,
// MarkSeed searches in its second, so that one step may produce both.
__device__ __forceinline__ uint2 *mark_list(uint2 *ov, uint32_t ov_cap) { return ov + ov_cap / 2; }
__device__ __forceinline__ const uint2 *mark_list(const uint2 *ov, uint32_t ov_cap) { return ov + ov_cap / 2; }

// Overflow tasks of one step go to list ovl (capacity ov_cap), counted in *ocnt.
__device__ __forceinline__ void push_overflow(SelState *st, uint32_t *ocnt, uint2 *ov, uint32_t ov_cap, uint32_t a,
                                              uint32_t r) {
    const uint32_t slot = atomicAdd(ocnt, 1u);
    if (slot < ov_cap) ov[slot] = make_uint2(a, r);
    else st->err = 2;
}

// Adds one sketch's delta to a listed vertex; the last of its R searches turns the
// sum into the vertex's key and raises Delta*.  partial = (tasks left << 40) + sum.
constexpr int kPartialShift = 40;
__device__ __forceinline__ void add_delta(SelState *st, unsigned long long *partial, uint32_t e, uint64_t delta,
                                          const uint32_t *evl, uint32_t kb, const uint8_t *in_s, uint64_t *key) {
    const unsigned long long old = atomicAdd(&partial[e], (unsigned long long)(delta - (1ull << kPartialShift)));
    if ((old >> kPartialShift) == 1ull) {
        const uint64_t sum = (old & ((1ull << kPartialShift) - 1ull)) + delta;
        const uint32_t v = evl[e];
        const uint64_t nk = in_s[v] ? 0ull : pack_key(sum, v, kb);
        key[v] = nk;
        if (nk) atomicMax(&st->delta, (unsigned long long)nk);
    }
}

// eval(l) on CompactSketch: one wave per (listed vertex, sketch), sketch-major;
// searches that outgrow the LDS queue are listed for the global-memory step.
// q / hs: this wave's LDS queue (kQCap) and hash set (kHCap).
__device__ __forceinline__ void eval_compact_level(uint32_t l, SelState *st, const uint32_t *evl,
                                                   unsigned long long *partial, const GraphDev &g, const ProbDev &pm,
                                                   const uint64_t *K, uint32_t R, const CompactDev &cd, uint32_t kb,
                                                   const uint8_t *in_s, uint64_t *key, uint2 *ov, uint32_t ov_cap,
                                                   uint32_t *q, uint32_t *hs, uint32_t wi, uint32_t wc) {
    const uint32_t ne = st->ev_cnt[l];
    const uint64_t total = (uint64_t)ne * R;
    for (uint64_t task = wi; task < total; task += wc) {
        const uint32_t r = (uint32_t)(task / ne), e = (uint32_t)(task % ne);
        const uint32_t v = evl[e];
        const BfsOut o = getcenter_memo_lds(g, pm, K[r], cd, r, in_s, v, q, hs);
        if (lane_id() == 0) {
            if (o.visits) atomicAdd(&st->visits, (unsigned long long)o.visits);
            if (o.overflow) push_overflow(st, &st->ov_cnt[l], ov, ov_cap / 2, e, r);
            else add_delta(st, partial, e, o.delta, evl, kb, in_s, key);
        }
    }
}

// Global-memory searches for the tasks of one step that overflowed (count in
// st->ov_cnt[slot]); searcher `who` of `nwho` uses queue/bitmap slot `who`.
// mode 0: evaluation of level `slot` (add the delta); mode 1: MarkSeed of
// st->last_seed (zero size_c[r][label]).
__device__ __forceinline__ void overflow_level(int mode, uint32_t slot, SelState *st, const uint32_t *evl,
                                               unsigned long long *partial, const GraphDev &g, const ProbDev &pm,
                                               const uint64_t *K, const CompactDev &cd, uint32_t kb,
                                               const uint8_t *in_s, uint64_t *key, const uint2 *ov, uint32_t ov_cap,
                                               uint32_t *slot_q, uint32_t *slot_vis, uint32_t n, uint32_t who,
                                               uint32_t nwho) {
    const uint32_t cnt = min(st->ov_cnt[slot], ov_cap / 2);
    const uint2 *list = (mode == 0) ? ov : mark_list(ov, ov_cap);
    uint32_t *gq = slot_q + (size_t)who * n;
    uint32_t *gvis = slot_vis + (size_t)who * ((n + 31) / 32);
    for (uint32_t i = who; i < cnt; i += nwho) {
        const uint2 t = list[i];
        const uint32_t r = t.y;
        const uint32_t v = (mode == 0) ? evl[t.x] : st->last_seed;
        const BfsOut o = getcenter_memo_global(g, pm, K[r], cd, r, in_s, v, gq, gvis);
        if (lane_id() == 0) {
            if (o.visits) atomicAdd(&st->visits, (unsigned long long)o.visits);
            if (mode == 0) add_delta(st, partial, t.x, o.delta, evl, kb, in_s, key);
            else if (o.label != kNone) cd.size_c[tri_at(cd, r, o.label)] = 0;
            else covmin_mark(cd, r, o.ccmin);
        }
    }
}

// MarkSeed on CompactSketch: one wave per sketch, GetCenter from the new seed.
__device__ __forceinline__ void markseed_compact_level(SelState *st, const GraphDev &g, const ProbDev &pm,
                                                       const uint64_t *K, uint32_t R, const CompactDev &cd,
                                                       const uint8_t *in_s, uint2 *ov, uint32_t ov_cap, uint32_t *q,
                                                       uint32_t *hs, uint32_t wi, uint32_t wc) {
    const uint32_t s = st->last_seed;
    for (uint32_t r = wi; r < R; r += wc) {
        const BfsOut o = getcenter_memo_lds(g, pm, K[r], cd, r, in_s, s, q, hs);
        if (lane_id() == 0) {
            if (o.visits) atomicAdd(&st->visits, (unsigned long long)o.visits);
            if (o.overflow) push_overflow(st, &st->ov_cnt[kMaxLevels + 1], mark_list(ov, ov_cap), ov_cap / 2, s, r);
            else if (o.label != kNone) cd.size_c[tri_at(cd, r, o.label)] = 0;
            else covmin_mark(cd, r, o.ccmin);
        }
    }
}

// MarkSeed of the previous round's seed and the evaluation of this round's root
// (evl[0], the level-0 list) in one step: per sketch, the same wave first searches
// from the seed and zeroes its CC, then searches from the root without waiting for
// that write: the root's CC is the seed's exactly when both searches end at the
// same label (or, without a center, at the same smallest vertex), and then its
// delta is 0; any other CC is untouched by this MarkSeed.  If the MarkSeed search
// overflows, the root's search in that sketch is deferred to the evaluation
// overflow list, which runs after the MarkSeed one.
__device__ __forceinline__ void markseed_eval_root_level(SelState *st, const uint32_t *evl,
                                                         unsigned long long *partial, const GraphDev &g,
                                                         const ProbDev &pm, const uint64_t *K, uint32_t R,
                                                         const CompactDev &cd, uint32_t kb, const uint8_t *in_s,
                                                         uint64_t *key, uint2 *ov, uint32_t ov_cap, uint32_t *q,
                                                         uint32_t *hs, uint32_t wi, uint32_t wc) {
    const uint32_t s = st->last_seed;
    const uint32_t v = evl[0];
    for (uint32_t r = wi; r < R; r += wc) {
        const BfsOut m = getcenter_memo_lds(g, pm, K[r], cd, r, in_s, s, q, hs);
        if (lane_id() == 0 && m.visits) atomicAdd(&st->visits, (unsigned long long)m.visits);
        if (m.overflow) {
            if (lane_id() == 0) {
                push_overflow(st, &st->ov_cnt[kMaxLevels + 1], mark_list(ov, ov_cap), ov_cap / 2, s, r);
                push_overflow(st, &st->ov_cnt[0], ov, ov_cap / 2, 0, r);
            }
            continue;
        }
        if (lane_id() == 0) {
            if (m.label != kNone) cd.size_c[tri_at(cd, r, m.label)] = 0;
            else covmin_mark(cd, r, m.ccmin);
        }
        __builtin_amdgcn_wave_barrier();
        const BfsOut o = getcenter_memo_lds(g, pm, K[r], cd, r, in_s, v, q, hs);
        if (lane_id() == 0) {
            if (o.visits) atomicAdd(&st->visits, (unsigned long long)o.visits);
            if (o.overflow) {
                push_overflow(st, &st->ov_cnt[0], ov, ov_cap / 2, 0, r);
            } else {
                const bool same = o.label != kNone ? o.label == m.label : (m.label == kNone && o.ccmin == m.ccmin);
                add_delta(st, partial, 0, same ? 0ull : o.delta, evl, kb, in_s, key);
            }
        }
    }
}

__global__ void __launch_bounds__(kBfsBlock) k_eval_compact_bfs(uint32_t l, SelState *__restrict__ st,
                                                                const uint32_t *__restrict__ evl,
                                                                unsigned long long *__restrict__ partial,
                                                                GraphDev g, ProbDev pm, const uint64_t *__restrict__ K,
                                                                uint32_t R, CompactDev cd, uint32_t kb,
                                                                const uint8_t *__restrict__ in_s,
                                                                uint64_t *__restrict__ key,
                                                                uint2 *__restrict__ ov, uint32_t ov_cap) {
    __shared__ uint32_t lds[kBfsWaves][kQCap + kHCap];
    uint32_t *q = lds[threadIdx.x / kWave];
    eval_compact_level(l, st, evl, partial, g, pm, K, R, cd, kb, in_s, key, ov, ov_cap, q, q + kQCap, wave_index(),
                       wave_count());
}

// grid: one 64-thread block per queue/bitmap slot.
__global__ void __launch_bounds__(64) k_overflow_bfs(int mode, uint32_t slot, SelState *__restrict__ st,
                                                     const uint32_t *__restrict__ evl,
                                                     unsigned long long *__restrict__ partial, GraphDev g,
                                                     ProbDev pm, const uint64_t *__restrict__ K, CompactDev cd,
                                                     uint32_t kb, const uint8_t *__restrict__ in_s,
                                                     uint64_t *__restrict__ key, const uint2 *__restrict__ ov,
                                                     uint32_t ov_cap, uint32_t *__restrict__ slot_q,
                                                     uint32_t *__restrict__ slot_vis, uint32_t n) {
    overflow_level(mode, slot, st, evl, partial, g, pm, K, cd, kb, in_s, key, ov, ov_cap, slot_q, slot_vis, n,
                   blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBfsBlock) k_markseed_compact(SelState *__restrict__ st, GraphDev g, ProbDev pm,
                                                                const uint64_t *__restrict__ K, uint32_t R,
                                                                CompactDev cd, const uint8_t *__restrict__ in_s,
                                                                uint2 *__restrict__ ov, uint32_t ov_cap) {
    __shared__ uint32_t lds[kBfsWaves][kQCap + kHCap];
    uint32_t *q = lds[threadIdx.x / kWave];
    markseed_compact_level(st, g, pm, K, R, cd, in_s, ov, ov_cap, q, q + kQCap, wave_index(), wave_count());
}

// ---- bulk round -------------------------------------------------------------
// When the previous seed covered a large share of every sketch (a giant
// component), nearly every stale key is invalid and the lazy search ends up
// evaluating almost all vertices.  Such a round evaluates every unselected
// vertex at once instead: the R sampled graphs are re-derived from their keys
// (sketches are reproducible from r, the "fusion" of Sec. 2) with the sketch
// kernels, and Marginal(S, v) = sum_r [CC_r(v) holds no seed] * |CC_r(v)|,
// which is exactly what GetCenter returns (a CC's compact size is zeroed by
// MarkSeed iff a seed lies in it).  The tree is then rebuilt from the fresh
// keys, so its root is the plain greedy's choice.

// flag of (sketch b, root of s) = 1 for every seed chosen so far (flag zeroed by
// the set-up, k_batch_init or k_batch_init4); vertex-major forests of width vs.
__global__ void __launch_bounds__(256) k_bulk_seed_roots(const SelState *__restrict__ st,
                                                         const uint32_t *__restrict__ seeds,
                                                         const uint32_t *__restrict__ parent,
                                                         const uint32_t *__restrict__ newid, uint32_t vs,
                                                         uint32_t B, uint32_t *__restrict__ flag) {
    const uint32_t ns = st->round;
    const uint64_t total = (uint64_t)ns * B;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t b = (uint32_t)(i / ns), j = (uint32_t)(i % ns);
        flag[(size_t)parent[(size_t)newid[seeds[j]] * vs + b] * vs + b] = 1u;
    }
}

// partial[v] += sum over the batch of the uncovered CC size of v.
__global__ void __launch_bounds__(256) k_bulk_accum(const uint32_t *__restrict__ parent,
                                                    const uint32_t *__restrict__ cnt,
                                                    const uint32_t *__restrict__ flag,
                                                    const uint32_t *__restrict__ newid, uint32_t n, uint32_t vs,
                                                    uint32_t B, unsigned long long *__restrict__ partial) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint32_t iv = newid[v];
    uint64_t s = 0;
    for (uint32_t b = 0; b < B; ++b) {
        const uint32_t root = parent[(size_t)iv * vs + b];
        const size_t at = (size_t)root * vs + b;
        s += flag[at] ? 0u : 1u + cnt[at];
    }
    partial[v] += s;
}

// Fresh keys for every vertex; the round's evaluation count is every unselected vertex.
__global__ void __launch_bounds__(256) k_bulk_keys(SelState *__restrict__ st,
                                                   const unsigned long long *__restrict__ partial, uint32_t n,
                                                   uint32_t kb, const uint8_t *__restrict__ in_s,
                                                   uint64_t *__restrict__ key) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) key[v] = in_s[v] ? 0ull : pack_key(partial[v], v, kb);
    if (v == 0) {
        for (int l = 0; l <= kMaxLevels; ++l) { st->fr_cnt[l] = 0; st->ev_cnt[l] = 0; }
        for (int l = 0; l < kMaxLevels + 2; ++l) st->ov_cnt[l] = 0;
        st->ev_cnt[0] = n - st->round;
    }
}

// ---- bulk round from the largest components' bitmaps ------------------------
// The build keeps, per sketch, the largest component's size and membership
// bitmap (n bits).  Marginal(S, v) = gain0[v] - sum over sketches r whose
// component of v holds a seed of |CC_r(v)|.  A seed inside the largest
// component of r covers it (one flag per sketch, then one bitmap test per
// vertex); a seed outside it covers a smaller component, enumerated by a
// search from the seed, whose size is subtracted at each of its vertices.
// Searches are capped per sketch; past the cap the round falls back to
// re-deriving the components.

// The whole component of v in sketch kr, appended to gq from position tail
// (visited bits in gvis); returns the new tail.  Stops once tail exceeds cap
// (every vertex it marked is still queued, so the caller can clear the bits).
__device__ uint32_t component_global(const GraphDev &g, const ProbDev &pm, uint64_t kr, uint32_t v, uint32_t *gq,
                                     uint32_t *gvis, uint32_t tail, uint32_t cap) {
    const uint32_t lane = lane_id();
    if (lane == 0) {
        gq[tail] = v;
        atomicOr(&gvis[v >> 5], 1u << (v & 31));
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    uint32_t head = tail;
    ++tail;
    while (head < tail && tail <= cap) {
        const uint32_t u = __hip_atomic_load(&gq[head], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        ++head;
        const uint64_t o1 = g.off[u + 1];
        for (uint64_t base = g.off[u]; base < o1; base += kWave) {
            const uint64_t j = base + lane;
            bool ins = false;
            uint32_t w = 0;
            if (j < o1) {
                w = g.cols[j];
                const uint64_t x = edge_word(u, w);
                if (is_live(x, kr, pm.csr_thr ? pm.csr_thr[j] : edge_threshold(pm, u, w, x))) {
                    const uint32_t bit = 1u << (w & 31);
                    ins = (atomicOr(&gvis[w >> 5], bit) & bit) == 0;
                }
            }
            const uint64_t im = __ballot(ins);
            if (ins) gq[tail + (uint32_t)__popcll(im & ((1ull << lane) - 1ull))] = w;
            tail += (uint32_t)__popcll(im);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
        }
    }
    return tail;
}

// One 64-thread block per queue/bitmap slot, sketches r = slot, slot + grid, ...:
// covered[r] = [some seed lies in r's largest component]; sub[w] += |C| for every
// vertex w of every other covered component C.  *abort = 1 if a sketch's
// searches passed cap vertices.  Bitmaps are word-major: bit v of sketch r is bit
// v % 64 of gbits[(v / 64) * R + r].
__global__ void __launch_bounds__(64) k_bulk_bits_search(const SelState *__restrict__ st,
                                                         const uint32_t *__restrict__ seeds, GraphDev g, ProbDev pm,
                                                         const uint64_t *__restrict__ K, uint32_t R, uint32_t n,
                                                         const uint64_t *__restrict__ gbits, uint32_t nw,
                                                         uint8_t *__restrict__ covered,
                                                         unsigned long long *__restrict__ sub,
                                                         uint32_t *__restrict__ slot_q, uint32_t *__restrict__ slot_vis,
                                                         uint32_t cap, uint32_t *__restrict__ abort_flag) {
    const uint32_t lane = lane_id();
    const uint32_t ns = st->round;
    uint32_t *gq = slot_q + (size_t)blockIdx.x * n;
    uint32_t *gvis = slot_vis + (size_t)blockIdx.x * ((n + 31) / 32);
    for (uint32_t r = blockIdx.x; r < R; r += gridDim.x) {
        bool giant = false;
        uint32_t tail = 0;
        for (uint32_t j = 0; j < ns && tail <= cap; ++j) {
            const uint32_t s = seeds[j];
            if ((gbits[(size_t)(s >> 6) * R + r] >> (s & 63)) & 1ull) {
                giant = true;
                continue;
            }
            const uint32_t seen = __hip_atomic_load(&gvis[s >> 5], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if ((seen >> (s & 31)) & 1u) continue;  // its component is already counted
            const uint32_t start = tail;
            tail = component_global(g, pm, K[r], s, gq, gvis, tail, cap);
            if (tail > cap) break;
            const uint32_t size = tail - start;
            for (uint32_t i = start + lane; i < tail; i += kWave) {
                const uint32_t w = __hip_atomic_load(&gq[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                atomicAdd(&sub[w], (unsigned long long)size);
            }
        }
        if (tail > cap && lane == 0) atomicOr(abort_flag, 1u);
        for (uint32_t i = lane; i < tail; i += kWave) {
            const uint32_t w = __hip_atomic_load(&gq[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            atomicAnd(&gvis[w >> 5], ~(1u << (w & 31)));
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        if (lane == 0) covered[r] = giant ? 1 : 0;
    }
}

// Fresh keys of every vertex from the bitmaps (nothing if *abort_flag); the
// round's evaluation count is every unselected vertex.  c(v) = sum over sketches r
// whose largest component is covered (covered[r]) of [v in it] * its size.  One
// wave per 64-vertex bitmap word.  gsum[v] holds the same sum over every sketch,
// so when most largest components are covered the wave subtracts the uncovered
// ones from it, else it adds the covered ones: lane l loads the word of sketch
// r0 + l (the R words of one vertex word are contiguous), and the wave walks only
// the sketches of the smaller set with lane reads.
__global__ void __launch_bounds__(256) k_bulk_bits_keys(SelState *__restrict__ st, const uint64_t *__restrict__ gain0,
                                                        const unsigned long long *__restrict__ sub,
                                                        const uint64_t *__restrict__ gbits, uint32_t nw,
                                                        const uint64_t *__restrict__ gsum,
                                                        const uint8_t *__restrict__ covered,
                                                        const unsigned long long *__restrict__ gbest, uint32_t R,
                                                        uint32_t n, uint32_t kb, const uint8_t *__restrict__ in_s,
                                                        uint64_t *__restrict__ key,
                                                        const uint32_t *__restrict__ abort_flag) {
    if (*abort_flag) return;
    const uint32_t lane = lane_id();
    const uint32_t w = wave_index();
    if (w >= nw) return;
    uint32_t ncov = 0;
    for (uint32_t r0 = 0; r0 < R; r0 += kWave) {
        const uint32_t r = r0 + lane;
        ncov += (uint32_t)__popcll(__ballot(r < R && covered[r]));
    }
    const bool subtract = 2 * ncov >= R;  // wave-uniform
    const uint32_t v = w * kWave + lane;
    uint64_t c = 0;
    for (uint32_t r0 = 0; r0 < R; r0 += kWave) {
        const uint32_t r = r0 + lane;
        const bool cov = r < R && covered[r];
        const bool walk = r < R && (subtract ? !cov : cov);
        uint32_t lo = 0, hi = 0, mult = 0;
        if (walk) {
            const uint64_t word = gbits[(size_t)w * R + r];
            lo = (uint32_t)word;
            hi = (uint32_t)(word >> 32);
            mult = giant_size_of(gbest[r]);
        }
        for (uint64_t m = __ballot(walk && mult != 0); m; m &= m - 1ull) {
            const int i = (int)__builtin_ctzll(m);
            const uint32_t mu = (uint32_t)__builtin_amdgcn_readlane((int)mult, i);
            const uint32_t wlo = (uint32_t)__builtin_amdgcn_readlane((int)lo, i);
            const uint32_t whi = (uint32_t)__builtin_amdgcn_readlane((int)hi, i);
            if ((((lane < 32) ? wlo : whi) >> (lane & 31)) & 1u) c += mu;
        }
    }
    if (v < n) {
        const uint64_t cv = subtract ? gsum[v] - c : c;
        key[v] = in_s[v] ? 0ull : pack_key(gain0[v] - sub[v] - cv, v, kb);
    }
    if (v == 0) {
        for (int l = 0; l <= kMaxLevels; ++l) { st->fr_cnt[l] = 0; st->ev_cnt[l] = 0; }
        for (int l = 0; l < kMaxLevels + 2; ++l) st->ov_cnt[l] = 0;
        st->ev_cnt[0] = n - st->round;
    }
}

}  // namespace pacim
