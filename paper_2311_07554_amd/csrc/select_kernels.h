// Seed selection (Algorithm 1, step 2): NextSeed over a winning tree
// (Sec. 4, Algorithm 5), Marginal (Sec. 3) on full labels or on CompactSketch
// via GetCenter, and MarkSeed.
//
// The winning tree here has fan-out 64 instead of 2: a node is one wave and its
// children are the wave's lanes, so the depth is ceil(log64 n) (4 for 2^20
// vertices) and relinking a node is one wave-wide argmax.  Leaves are the
// vertices themselves (leaf j is vertex j); internal level l holds ids[l][t],
// the child with the largest key.  Algorithm 5's rules carry over unchanged:
//   - a node is stale iff its id differs from its parent's (the root always is);
//   - a stale node whose key is below Delta* (the best fresh key of the round)
//     is pruned with its whole subtree;
//   - a stale node at or above Delta* is re-evaluated and Delta* raised by an
//     atomic max (WriteMax);
//   - every non-pruned internal node is explored, then relinked to the child
//     with the largest key.
// The recursion of Algorithm 5 is run level by level: check(l) decides the
// children of the level-l frontier, eval(l+1) re-evaluates the ones that need
// it, and after the deepest level the frontiers are relinked bottom-up.  Keys
// are unique ((gain+1) << kb | (2^kb-1-v)), so the argmax at the root is the
// unique largest gain with the smallest id, the plain greedy's choice
// (Theorem 4.4).
#pragma once

#include "common.h"

namespace pacim {

struct TreeDesc {
    uint32_t D;                      // internal levels 0..D-1; level D = the n leaves
    uint32_t lvl_n[kMaxLevels + 1];  // nodes per level
    uint64_t lvl_off[kMaxLevels];    // offset of level l in ids / frontier buffers
};

struct SelState {
    unsigned long long delta;        // Delta*: best fresh key this round
    unsigned long long evals;        // re-evaluations over all rounds
    unsigned long long overflow;     // GetCenter searches sent to the global-memory path
    unsigned long long visits;       // vertices scanned by GetCenter searches
    uint32_t fr_cnt[kMaxLevels + 1];
    uint32_t ev_cnt[kMaxLevels + 1];
    uint32_t ov_cnt[kMaxLevels + 2]; // GetCenter searches left for the global-memory path:
                                     // per evaluation level, then MarkSeed
    uint32_t round;                  // seeds chosen so far
    uint32_t last_seed;
    uint32_t err;
    uint32_t stop_level;             // persistent rounds: level whose evaluation was left to the
                                     // per-level kernels (kNone: stopped at a round boundary)
    unsigned long long last_gain;    // gain of the last round ended
};

// ---- Marginal on full labels ------------------------------------------------
// E[v][r] = (label, size-at-label).  Uncovered size of v in sketch r is the
// size field of the label's own entry, zeroed by MarkSeed.
// Four row entries per lane are loaded before their label gathers, so a wave has
// all of them in flight at once.  Entries are read as 64-bit words (label in the
// low half) so they stay in registers: with uint2 locals the compiler turns the
// "own entry or gathered entry" choice into a load through a selected address
// and spills the row to per-lane scratch.
__device__ __forceinline__ uint64_t marginal_full(const uint2 *__restrict__ E, uint32_t R, uint32_t v) {
    constexpr int U = 4;
    const unsigned long long *row = reinterpret_cast<const unsigned long long *>(E + (size_t)v * R);
    uint64_t s = 0;
    for (uint32_t r0 = lane_id(); r0 < R; r0 += U * kWave) {
        unsigned long long e[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t r = r0 + i * kWave;
            e[i] = r < R ? row[r] : (unsigned long long)v;  // past R: own label, size 0
        }
        uint32_t y[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t lab = (uint32_t)e[i];
            y[i] = (uint32_t)(e[i] >> 32);
            if (lab != v) y[i] = E[(size_t)lab * R + r0 + i * kWave].y;
        }
#pragma unroll
        for (int i = 0; i < U; ++i) s += y[i];
    }
    return wave_sum_u64(s);
}

// ---- tree build (initial keys from Marginal(empty, v)) ------------------------
__global__ void k_keys_from_gain0(const uint64_t *__restrict__ gain0, uint32_t n, uint32_t kb,
                                  uint64_t *__restrict__ key) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < n) key[v] = pack_key(gain0[v], v, kb);
}

// argmax over the children of node t of level l (wave-wide); returns the winner id
// in every lane.  sub_child/sub_id/sub_key let the caller substitute one child's
// freshly written id and key.
__device__ __forceinline__ uint32_t relink_node(const TreeDesc &td, const uint32_t *__restrict__ ids,
                                                const uint64_t *__restrict__ key, uint32_t l, uint32_t t,
                                                uint32_t sub_child, uint32_t sub_id, uint64_t sub_key,
                                                bool use_sub) {
    const uint32_t lane = lane_id();
    const uint32_t c = t * kFan + lane;
    const bool valid = c < td.lvl_n[l + 1];
    uint32_t cid = 0;
    uint64_t ck = 0;
    if (valid) {
        cid = (l + 1 == td.D) ? c : ids[td.lvl_off[l + 1] + c];
        ck = key[cid];
        if (use_sub && c == sub_child) { cid = sub_id; ck = sub_key; }
    }
    const uint64_t best = wave_max_u64(valid ? ck : 0ull);
    const uint64_t win = __ballot(valid && ck == best);
    const uint32_t wl = (uint32_t)__builtin_ctzll(win);
    return __shfl(cid, wl);
}

__global__ void __launch_bounds__(256) k_tree_build_level(TreeDesc td, uint32_t l, uint32_t *__restrict__ ids,
                                                          const uint64_t *__restrict__ key) {
    for (uint32_t t = wave_index(); t < td.lvl_n[l]; t += wave_count()) {
        const uint32_t w = relink_node(td, ids, key, l, t, 0, 0, 0, false);
        if (lane_id() == 0) ids[td.lvl_off[l] + t] = w;
    }
}

// ---- one round ---------------------------------------------------------------
// The steps of a round are written as device functions over a range of waves
// (wave wi of wc) so that the per-level kernels below and the persistent
// selection kernel run the same code.

// round_begin (one thread): the root is always stale; it is the one level-0
// evaluation.  partial (CompactSketch only): per listed vertex, (tasks left << 40)
// + summed deltas, started at partial_init = R << 40.
__device__ __forceinline__ void round_begin_one(const TreeDesc &td, SelState *st, const uint32_t *ids,
                                                uint32_t *fr, uint32_t *evl, unsigned long long *partial,
                                                unsigned long long partial_init) {
    st->delta = 0;
    for (int l = 0; l <= kMaxLevels; ++l) { st->fr_cnt[l] = 0; st->ev_cnt[l] = 0; }
    for (int l = 0; l < kMaxLevels + 2; ++l) st->ov_cnt[l] = 0;
    st->fr_cnt[0] = 1;
    fr[td.lvl_off[0]] = 0;
    st->ev_cnt[0] = 1;
    evl[0] = ids[td.lvl_off[0]];
    if (partial) partial[0] = partial_init;
}

// check(l): one wave per frontier node t of level l, one lane per child.
__device__ __forceinline__ void check_level(const TreeDesc &td, uint32_t l, SelState *st, const uint32_t *ids,
                                            const uint64_t *key, uint32_t *fr, uint32_t *evl,
                                            unsigned long long *partial, unsigned long long partial_init,
                                            uint32_t wi, uint32_t wc) {
    const uint32_t nf = st->fr_cnt[l];
    const uint64_t delta = __hip_atomic_load(&st->delta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool leaf_children = (l + 1 == td.D);
    for (uint32_t i = wi; i < nf; i += wc) {
        const uint32_t t = fr[td.lvl_off[l] + i];
        const uint32_t pid = ids[td.lvl_off[l] + t];
        const uint32_t c = t * kFan + lane_id();
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
        const uint32_t ep = wave_append(&st->ev_cnt[l + 1], need_eval, &tot);
        if (need_eval) {
            evl[ep] = cid;
            if (partial) partial[ep] = partial_init;
        }
        const uint32_t fp = wave_append(&st->fr_cnt[l + 1], explore, &tot);
        if (explore) fr[td.lvl_off[l + 1] + fp] = c;
    }
}

// eval(l) on full labels: one wave per listed vertex.
__device__ __forceinline__ void eval_full_level(uint32_t l, SelState *st, const uint32_t *evl, const uint2 *E,
                                                uint32_t R, uint32_t kb, const uint8_t *in_s, uint64_t *key,
                                                uint32_t wi, uint32_t wc) {
    const uint32_t ne = st->ev_cnt[l];
    uint64_t best = 0;
    for (uint32_t i = wi; i < ne; i += wc) {
        const uint32_t v = evl[i];
        const uint64_t g = marginal_full(E, R, v);
        const uint64_t nk = in_s[v] ? 0ull : pack_key(g, v, kb);
        if (lane_id() == 0) key[v] = nk;
        best = nk > best ? nk : best;
    }
    if (lane_id() == 0 && best) atomicMax(&st->delta, (unsigned long long)best);
}

// relink(l): one wave per frontier node of level l (children already final).
__device__ __forceinline__ void relink_level(const TreeDesc &td, uint32_t l, const SelState *st, uint32_t *ids,
                                             const uint64_t *key, const uint32_t *fr, uint32_t wi, uint32_t wc) {
    const uint32_t nf = st->fr_cnt[l];
    for (uint32_t i = wi; i < nf; i += wc) {
        const uint32_t t = fr[td.lvl_off[l] + i];
        const uint32_t w = relink_node(td, ids, key, l, t, 0, 0, 0, false);
        if (lane_id() == 0) ids[td.lvl_off[l] + t] = w;
    }
}

// round_end (one wave): record the root as the seed, remove it (key 0) and
// relink its leaf-to-root path so the next round starts from the best stale
// key; with full labels also MarkSeed: zero the size at the seed's label in
// every sketch.
// relink false: the caller relinks the path itself (from values it holds).
__device__ __forceinline__ void round_end_wave(const TreeDesc &td, SelState *st, uint32_t *ids, uint64_t *key,
                                               uint8_t *in_s, uint32_t kb, uint32_t *seeds_out,
                                               unsigned long long *gains_out, uint32_t *evals_out, uint2 *E,
                                               uint32_t R, bool relink = true) {
    const uint32_t lane = lane_id();
    const uint32_t s = ids[td.lvl_off[0]];
    const uint64_t ks = key[s];
    const uint32_t round = st->round;
    uint32_t evs = 0, ovs = 0;
    for (int l = 0; l <= kMaxLevels; ++l) evs += st->ev_cnt[l];
    for (int l = 0; l < kMaxLevels + 2; ++l) ovs += st->ov_cnt[l];
    if (lane == 0) {
        if (ks == 0 || in_s[s]) st->err = 1;
        seeds_out[round] = s;
        gains_out[round] = key_gain(ks, kb);
        evals_out[round] = evs;
        in_s[s] = 1;
        key[s] = 0;
        st->last_seed = s;
        st->last_gain = key_gain(ks, kb);
        st->evals += evs;
        st->overflow += ovs;
    }
    // relink the path of leaf s, bottom-up, using the values this wave just wrote
    uint32_t child = s, child_id = s;
    uint64_t child_key = 0;
    for (int l = relink ? (int)td.D - 1 : -1; l >= 0; --l) {
        const uint32_t t = child >> kFanLog;
        const uint32_t w = relink_node(td, ids, key, (uint32_t)l, t, child, child_id, child_key, true);
        const uint64_t wk = (w == s) ? 0ull : key[w];
        if (lane == 0) ids[td.lvl_off[l] + t] = w;
        child = t;
        child_id = w;
        child_key = wk;
    }
    if (E) {
        const uint2 *row = E + (size_t)s * R;
        for (uint32_t r = lane; r < R; r += kWave) {
            const uint32_t lab = row[r].x;
            E[(size_t)lab * R + r].y = 0;
        }
    }
    if (lane == 0) st->round = round + 1;
}

// A round's walk while each level's frontier is one node (the usual lazy round:
// the root's fresh key still beats every other stale key, so each level explores
// only the child on the previous winner's path and evaluates nothing).
// check_level's rules on that node, with its children's ids and keys kept in LDS
// (cid_c / ck_c): it writes the frontier of the next level as check_level would
// (one node in fr, fr_cnt[l + 1] = 1; no evaluations), and stops at the first
// level whose check needs the general step (an evaluation, or more than one child
// to explore).  Returns that level (D if none); node[l] = the frontier node of
// level l for l >= 1 (level 0's is the root, 0).  delta: the round's best fresh
// key so far.  One wave.
__device__ __forceinline__ uint32_t walk_single_frontiers(const TreeDesc &td, const uint32_t *ids,
                                                          const uint64_t *key, uint64_t delta, uint32_t *fr,
                                                          uint32_t *fr_cnt, uint32_t (*cid_c)[kWave],
                                                          unsigned long long (*ck_c)[kWave], uint32_t *node) {
    const uint32_t lane = lane_id();
    uint32_t t = 0;
    uint32_t pid = ids[td.lvl_off[0]];
    for (uint32_t l = 0; l < td.D; ++l) {
        const uint32_t c = t * kFan + lane;
        const bool valid = c < td.lvl_n[l + 1];
        const bool leaf = l + 1 == td.D;
        uint32_t cid = 0;
        uint64_t ck = 0;
        if (valid) {
            cid = leaf ? c : ids[td.lvl_off[l + 1] + c];
            ck = key[cid];
        }
        const bool stale = valid && cid != pid;
        const bool need = stale && ck >= delta;
        const bool explore = valid && !leaf && (!stale || need);
        const uint64_t ex = __ballot(explore);
        if (__ballot(need) != 0ull || (!leaf && __popcll(ex) != 1)) return l;
        cid_c[l][lane] = cid;
        ck_c[l][lane] = ck;
        if (!leaf) {  // the explored child keeps the winner's id, so pid carries over
            const uint32_t nt = t * kFan + (uint32_t)__builtin_ctzll(ex);
            if (lane == 0) {
                fr[td.lvl_off[l + 1]] = nt;
                fr_cnt[l + 1] = 1;
                node[l + 1] = nt;
            }
            t = nt;
        }
    }
    return td.D;
}

// relink_level's argmax on the walked nodes of levels lstart, lstart - 1, ..., 0
// from the kept children, the path child of level l (lane sub_lane) substituted by
// the winner below it (sub_id, sub_key).  node[0] must hold 0.  One wave.
__device__ __forceinline__ void relink_kept(const TreeDesc &td, uint32_t *ids, uint32_t (*cid_c)[kWave],
                                            unsigned long long (*ck_c)[kWave], const uint32_t *node, int lstart,
                                            uint32_t sub_lane, uint32_t sub_id, uint64_t sub_key) {
    const uint32_t lane = lane_id();
    for (int l = lstart; l >= 0; --l) {
        const uint32_t t = node[l];
        const bool valid = t * kFan + lane < td.lvl_n[l + 1];
        uint32_t cid = cid_c[l][lane];
        uint64_t ck = valid ? ck_c[l][lane] : 0ull;
        if (lane == sub_lane) {
            cid = sub_id;
            ck = sub_key;
        }
        const uint64_t best = wave_max_u64(ck);
        const uint64_t win = __ballot(valid && ck == best);
        const uint32_t w = __shfl(cid, (int)__builtin_ctzll(win));
        if (lane == 0) ids[td.lvl_off[l] + t] = w;
        sub_lane = t & (kFan - 1);
        sub_id = w;
        sub_key = best;
    }
}

__global__ void k_round_begin(TreeDesc td, SelState *__restrict__ st, const uint32_t *__restrict__ ids,
                              uint32_t *__restrict__ fr, uint32_t *__restrict__ evl,
                              unsigned long long *__restrict__ partial, unsigned long long partial_init) {
    if (threadIdx.x == 0) round_begin_one(td, st, ids, fr, evl, partial, partial_init);
}

__global__ void __launch_bounds__(256) k_check(TreeDesc td, uint32_t l, SelState *__restrict__ st,
                                               const uint32_t *__restrict__ ids, const uint64_t *__restrict__ key,
                                               uint32_t *__restrict__ fr, uint32_t *__restrict__ evl,
                                               unsigned long long *__restrict__ partial,
                                               unsigned long long partial_init) {
    check_level(td, l, st, ids, key, fr, evl, partial, partial_init, wave_index(), wave_count());
}

__global__ void __launch_bounds__(256) k_eval_full(uint32_t l, SelState *__restrict__ st,
                                                   const uint32_t *__restrict__ evl, const uint2 *__restrict__ E,
                                                   uint32_t R, uint32_t kb, const uint8_t *__restrict__ in_s,
                                                   uint64_t *__restrict__ key) {
    eval_full_level(l, st, evl, E, R, kb, in_s, key, wave_index(), wave_count());
}

// Every unselected vertex evaluated on full labels, in vertex order (one wave per
// vertex): the round after a seed that covered a large share of every sketch,
// where the lazy search would re-evaluate nearly every vertex anyway.  The tree
// is rebuilt from the keys afterwards; the round's evaluation count is every
// unselected vertex.
// A lane keeps the last label it gathered for each of its sketches (E is not
// written during the round): most vertices of a sketch share one giant
// component, and re-reading that label's entry from every wave would make one
// row of E the target of most gathers.
__global__ void __launch_bounds__(256) k_bulk_full_keys(SelState *__restrict__ st, const uint2 *__restrict__ E,
                                                        uint32_t R, uint32_t n, uint32_t kb,
                                                        const uint8_t *__restrict__ in_s, uint64_t *__restrict__ key) {
    constexpr int U = 4;  // sketches per lane kept (R <= 256); larger R loops without the cache
    uint32_t last_l[U], last_y[U];
#pragma unroll
    for (int i = 0; i < U; ++i) last_l[i] = kNone, last_y[i] = 0;
    const uint32_t lane = lane_id();
    if (R <= (uint32_t)(U * kWave)) {
        // the wave's next row is loaded while the current one's gathers wait
        auto load_row = [&](uint32_t v, uint2 *e) {
            const uint2 *row = E + (size_t)v * R;
#pragma unroll
            for (int i = 0; i < U; ++i) {
                const uint32_t r = lane + i * kWave;
                e[i] = r < R ? row[r] : make_uint2(v, 0u);
            }
        };
        uint2 cur[U], nxt[U];
        uint32_t v = wave_index();
        if (v < n) load_row(v, cur);
        for (; v < n; v += wave_count()) {
            const uint32_t vn = v + wave_count();
            if (vn < n) load_row(vn, nxt);
            uint64_t g = 0;
#pragma unroll
            for (int i = 0; i < U; ++i) {
                uint32_t y = cur[i].y;
                if (cur[i].x != v) {
                    if (cur[i].x != last_l[i]) {
                        last_l[i] = cur[i].x;
                        last_y[i] = E[(size_t)cur[i].x * R + lane + i * kWave].y;
                    }
                    y = last_y[i];
                }
                g += y;
            }
            g = wave_sum_u64(g);
            if (lane == 0) key[v] = in_s[v] ? 0ull : pack_key(g, v, kb);
#pragma unroll
            for (int i = 0; i < U; ++i) cur[i] = nxt[i];
        }
    } else {
        for (uint32_t v = wave_index(); v < n; v += wave_count()) {
            const uint64_t g = marginal_full(E, R, v);
            if (lane == 0) key[v] = in_s[v] ? 0ull : pack_key(g, v, kb);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int l = 0; l <= kMaxLevels; ++l) { st->fr_cnt[l] = 0; st->ev_cnt[l] = 0; }
        for (int l = 0; l < kMaxLevels + 2; ++l) st->ov_cnt[l] = 0;
        st->ev_cnt[0] = n - st->round;
    }
}

__global__ void __launch_bounds__(256) k_relink(TreeDesc td, uint32_t l, const SelState *__restrict__ st,
                                                uint32_t *__restrict__ ids, const uint64_t *__restrict__ key,
                                                const uint32_t *__restrict__ fr) {
    relink_level(td, l, st, ids, key, fr, wave_index(), wave_count());
}

__global__ void __launch_bounds__(64) k_round_end(TreeDesc td, SelState *__restrict__ st, uint32_t *__restrict__ ids,
                                                  uint64_t *__restrict__ key, uint8_t *__restrict__ in_s,
                                                  uint32_t kb, uint32_t *__restrict__ seeds_out,
                                                  unsigned long long *__restrict__ gains_out,
                                                  uint32_t *__restrict__ evals_out, uint2 *__restrict__ E,
                                                  uint32_t R) {
    round_end_wave(td, st, ids, key, in_s, kb, seeds_out, gains_out, evals_out, E, R);
}

}  // namespace pacim
