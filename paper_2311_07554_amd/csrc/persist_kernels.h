// Lazy greedy rounds (Algorithm 5 of Sec. 4 with Marginal and MarkSeed of
// Sec. 3) in one persistent launch.
//
// With the per-level kernels a round is about a dozen launches on full labels
// and twenty on CompactSketch, most of them over a handful of tree nodes, so a
// round costs its launch latencies rather than its work.  Here one workgroup,
// the leader, runs the rounds: the steps over few items (frontiers of a few
// nodes, a few full-label evaluations, the round's end) it runs alone with
// workgroup barriers; a step with more work (the GetCenter searches of a
// CompactSketch evaluation, R per listed vertex, or a wide frontier) it
// publishes to every workgroup of the grid and waits for all of them.
//
// The leader stops early, and the host finishes with the per-level kernels,
// when an evaluation step would exceed max_step_tasks (the round is left at the
// level whose evaluation is pending, in SelState::stop_level), and after a round
// whose gain reaches bulk_gain_min (the next round is a bulk round).  On full
// labels the grid is the leader alone: its evaluations are one wave each.
//
// Requires all workgroups resident at once (cooperative launch).  Every wait has
// a time limit: a wait that runs past it sets PersistCtl::err, every workgroup
// then leaves at its next wait, and the host reports the error.
#pragma once

#include "common.h"
#include "compact_kernels.h"
#include "select_kernels.h"

namespace pacim {

constexpr uint32_t kPersistBlock = 256;
constexpr uint32_t kPersistWaves = kPersistBlock / kWave;
constexpr uint32_t kLeaderItems = 8 * kPersistWaves;  // larger steps go to the whole grid

enum : uint32_t {
    kPhExit = 0, kPhCheck, kPhRelink, kPhEvalFull, kPhEvalCompact, kPhOverflow, kPhMarkseed, kPhMarkEvalRoot
};

struct PersistCtl {
    uint32_t gen;   // generation of the published step
    uint32_t kind, arg, mode;
    uint32_t done;  // completions of non-leader workgroups over all steps
    uint32_t err;   // a wait ran past its limit
};

struct PersistArgs {
    TreeDesc td;
    SelState *st;
    uint32_t *ids;
    uint64_t *key;
    uint32_t *fr, *evl;
    unsigned long long *partial;
    unsigned long long pinit;
    uint8_t *in_s;
    uint32_t kb, R, n;
    uint32_t *seeds_out;
    unsigned long long *gains_out;
    uint32_t *evals_out;
    uint2 *E;  // full labels, or null for CompactSketch
    GraphDev g;
    ProbDev pm;
    const uint64_t *K;
    CompactDev cd;
    uint2 *ov;
    uint32_t ov_cap;
    uint32_t *slot_q, *slot_vis;
    uint32_t slots;
    uint32_t max_rounds;
    uint64_t max_step_tasks;           // larger evaluation steps go back to the host
    unsigned long long bulk_gain_min;  // 0: never stop for a bulk round
    PersistCtl *ctl;
    uint64_t spin_ticks;  // wait limit in wall_clock64() ticks
};

// Waits (one thread) until *p != v (ne) or *p >= v (!ne), then acquires.  The
// polling loads are relaxed: an acquire per poll would invalidate this CU's
// caches each time.  False if the limit passed or another workgroup gave up.
__device__ __forceinline__ bool persist_wait(const uint32_t *p, uint32_t v, bool ne, PersistCtl *ctl,
                                             uint64_t limit) {
    const uint64_t t0 = wall_clock64();
    for (;;) {
        const uint32_t x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ne ? (x != v) : (x >= v)) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            return true;
        }
        if (__hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        if (wall_clock64() - t0 > limit) {
            __hip_atomic_fetch_or(&ctl->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(2);
    }
}

// One step over waves [wi, wi + wc) of the participants.
__device__ __forceinline__ void persist_step(const PersistArgs &a, uint32_t kind, uint32_t arg, uint32_t mode,
                                             uint32_t wi, uint32_t wc, uint32_t *q, uint32_t *hs) {
    switch (kind) {
    case kPhCheck:
        check_level(a.td, arg, a.st, a.ids, a.key, a.fr, a.evl, a.E ? nullptr : a.partial, a.pinit, wi, wc);
        break;
    case kPhRelink:
        relink_level(a.td, arg, a.st, a.ids, a.key, a.fr, wi, wc);
        break;
    case kPhEvalFull:
        eval_full_level(arg, a.st, a.evl, a.E, a.R, a.kb, a.in_s, a.key, wi, wc);
        break;
    case kPhEvalCompact:
        eval_compact_level(arg, a.st, a.evl, a.partial, a.g, a.pm, a.K, a.R, a.cd, a.kb, a.in_s, a.key, a.ov,
                           a.ov_cap, q, hs, wi, wc);
        break;
    case kPhOverflow:
        if (wi < a.slots)
            overflow_level((int)mode, arg, a.st, a.evl, a.partial, a.g, a.pm, a.K, a.cd, a.kb, a.in_s, a.key, a.ov,
                           a.ov_cap, a.slot_q, a.slot_vis, a.n, wi, min(a.slots, wc));
        break;
    case kPhMarkseed:
        markseed_compact_level(a.st, a.g, a.pm, a.K, a.R, a.cd, a.in_s, a.ov, a.ov_cap, q, hs, wi, wc);
        break;
    case kPhMarkEvalRoot:
        markseed_eval_root_level(a.st, a.evl, a.partial, a.g, a.pm, a.K, a.R, a.cd, a.kb, a.in_s, a.key, a.ov,
                                 a.ov_cap, q, hs, wi, wc);
        break;
    default:
        break;
    }
}

__global__ void __launch_bounds__(kPersistBlock) k_select_persist(PersistArgs a) {
    __shared__ uint32_t lds[kPersistWaves][kQCap + kHCap];
    __shared__ uint32_t sh_kind, sh_arg, sh_mode, sh_ok, sh_val;
    __shared__ uint32_t sh_nf[kMaxLevels + 1];  // the round's frontier sizes, level by level
    // the leader's walk of single-node frontiers: children kept per level, the nodes
    __shared__ uint32_t sh_cid[kMaxLevels][kWave];
    __shared__ unsigned long long sh_ck[kMaxLevels][kWave];
    __shared__ uint32_t sh_node[kMaxLevels + 1], sh_lf;
    const uint32_t tid = threadIdx.x, w = tid / kWave;
    uint32_t *q = lds[w], *hs = q + kQCap;
    PersistCtl *ctl = a.ctl;
    const uint32_t wc_grid = gridDim.x * kPersistWaves;

    if (blockIdx.x != 0) {  // worker
        uint32_t seen = 0;
        for (;;) {
            if (tid == 0) {
                const bool ok = persist_wait(&ctl->gen, seen, true, ctl, a.spin_ticks);
                sh_kind = ok ? ctl->kind : kPhExit;
                sh_arg = ctl->arg;
                sh_mode = ctl->mode;
            }
            __syncthreads();
            const uint32_t kind = sh_kind, arg = sh_arg, mode = sh_mode;
            ++seen;
            if (kind == kPhExit) return;
            persist_step(a, kind, arg, mode, blockIdx.x * kPersistWaves + w, wc_grid, q, hs);
            __syncthreads();
            if (tid == 0) __hip_atomic_fetch_add(&ctl->done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }

    // leader
    uint32_t gen = 0, expect = 0;
    bool ok = true;
    auto grid_step = [&](uint32_t kind, uint32_t arg, uint32_t mode) {
        __syncthreads();
        if (tid == 0) {
            ctl->kind = kind;
            ctl->arg = arg;
            ctl->mode = mode;
            __hip_atomic_store(&ctl->gen, gen + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        ++gen;
        if (kind == kPhExit) return;
        persist_step(a, kind, arg, mode, w, wc_grid, q, hs);
        __syncthreads();
        expect += gridDim.x - 1;
        if (tid == 0) sh_ok = persist_wait(&ctl->done, expect, false, ctl, a.spin_ticks) ? 1u : 0u;
        __syncthreads();
        ok = ok && sh_ok;
    };
    // a value that steers the leader's control flow, read once and shared so that
    // every wave of the leader takes the same branch
    auto uniform_read = [&](const uint32_t *p) -> uint32_t {
        __syncthreads();
        if (tid == 0) sh_val = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        return sh_val;
    };
    auto local_step = [&](uint32_t kind, uint32_t arg) {
        persist_step(a, kind, arg, 0, w, kPersistWaves, q, hs);
        __syncthreads();
    };
    // items of a check/relink step: the level's frontier (sh_nf, final once the
    // level above was checked)
    auto tree_step = [&](uint32_t kind, uint32_t l) {
        if (sh_nf[l] > kLeaderItems) grid_step(kind, l, 0);
        else local_step(kind, l);
    };
    // after check(l): the frontier size of level l + 1 into sh_nf and its number of
    // evaluations returned, both read by one thread between one pair of barriers
    auto read_level = [&](uint32_t l1) -> uint32_t {
        __syncthreads();
        if (tid == 0) {
            sh_nf[l1] = __hip_atomic_load(&a.st->fr_cnt[l1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            sh_val = __hip_atomic_load(&a.st->ev_cnt[l1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
        return sh_val;
    };
    // evaluation of ne listed vertices of level l; false if it is left to the host
    auto eval_step = [&](uint32_t l, uint32_t ne) -> bool {
        if (ne == 0) return true;
        if (a.E) {
            if (ne > a.max_step_tasks) return false;
            if (ne > kLeaderItems) grid_step(kPhEvalFull, l, 0);
            else local_step(kPhEvalFull, l);
            return true;
        }
        if ((uint64_t)ne * a.R > a.max_step_tasks) return false;
        grid_step(kPhEvalCompact, l, 0);
        if (ok && uniform_read(&a.st->ov_cnt[l])) grid_step(kPhOverflow, l, 0);
        return true;
    };

    // CompactSketch: a round's MarkSeed is deferred into the next round's first
    // step (the root's evaluation) when that round runs in this launch.
    auto markseed_step = [&]() {
        grid_step(kPhMarkseed, 0, 0);
        if (ok && uniform_read(&a.st->ov_cnt[kMaxLevels + 1])) grid_step(kPhOverflow, kMaxLevels + 1, 1);
    };
    const bool fuse = !a.E && (uint64_t)a.R <= a.max_step_tasks;
    bool mark_pending = false;

    if (tid == 0) a.st->stop_level = kNone;
    __syncthreads();
    for (uint32_t r = 0; r < a.max_rounds && ok; ++r) {
        if (tid == 0) {
            round_begin_one(a.td, a.st, a.ids, a.fr, a.evl, a.E ? nullptr : a.partial, a.pinit);
            sh_nf[0] = 1;  // the root, also the one level-0 evaluation
        }
        __syncthreads();
        uint32_t pending = kNone;
        if (mark_pending) {
            mark_pending = false;
            grid_step(kPhMarkEvalRoot, 0, 0);
            if (ok && uniform_read(&a.st->ov_cnt[kMaxLevels + 1])) grid_step(kPhOverflow, kMaxLevels + 1, 1);
            if (ok && uniform_read(&a.st->ov_cnt[0])) grid_step(kPhOverflow, 0, 0);
        } else if (!eval_step(0, 1)) {
            pending = 0;
        }
        // levels [0, lf) checked by the leader's walk (single-node frontiers, no
        // evaluation), the rest by the general steps
        uint32_t lf = 0;
        if (pending == kNone && ok) {
            __syncthreads();
            if (w == 0) {
                const uint64_t delta = __hip_atomic_load(&a.st->delta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint32_t f = walk_single_frontiers(a.td, a.ids, a.key, delta, a.fr, a.st->fr_cnt, sh_cid, sh_ck,
                                                         sh_node);
                if (tid == 0) {
                    sh_node[0] = 0;
                    sh_lf = f;
                    for (uint32_t l = 1; l <= f && l <= a.td.D - 1; ++l) sh_nf[l] = 1;
                }
            }
            __syncthreads();
            lf = sh_lf;
        }
        for (uint32_t l = lf; l < a.td.D && pending == kNone && ok; ++l) {
            tree_step(kPhCheck, l);
            if (!eval_step(l + 1, read_level(l + 1))) pending = l + 1;
        }
        if (pending != kNone) {
            if (tid == 0) a.st->stop_level = pending;
            break;
        }
        for (int l = (int)a.td.D - 1; l >= (int)lf && ok; --l) tree_step(kPhRelink, (uint32_t)l);
        if (!ok) break;
        if (lf == a.td.D) {
            // every level walked: the root's winner is still the evaluated root vertex
            // and its leaf-to-root path is the walked one, so the round's relinks change
            // nothing and the seed's path is relinked from the kept children
            if (w == 0) {
                const uint32_t s = a.ids[a.td.lvl_off[0]];
                round_end_wave(a.td, a.st, a.ids, a.key, a.in_s, a.kb, a.seeds_out, a.gains_out, a.evals_out, a.E,
                               a.R, false);
                relink_kept(a.td, a.ids, sh_cid, sh_ck, sh_node, (int)a.td.D - 1, s & (kFan - 1), s, 0ull);
            }
        } else {
            if (w == 0 && lf > 0) {  // the walked levels, below them the general steps' winner
                const uint32_t tn = sh_node[lf];
                const uint32_t id = a.ids[a.td.lvl_off[lf] + tn];
                relink_kept(a.td, a.ids, sh_cid, sh_ck, sh_node, (int)lf - 1, tn & (kFan - 1), id, a.key[id]);
            }
            __syncthreads();
            if (w == 0) round_end_wave(a.td, a.st, a.ids, a.key, a.in_s, a.kb, a.seeds_out, a.gains_out, a.evals_out,
                                       a.E, a.R);
        }
        __syncthreads();
        bool stop = r + 1 >= a.max_rounds;
        if (a.bulk_gain_min) {
            __syncthreads();  // every wave has read sh_val's previous value
            if (tid == 0) {
                const uint32_t rd = a.st->round;
                sh_val = a.gains_out[rd - 1] >= a.bulk_gain_min ? 1u : 0u;
            }
            __syncthreads();
            stop = stop || sh_val != 0;
        }
        if (!a.E) {
            if (fuse && !stop) mark_pending = true;
            else markseed_step();
        }
        if (stop) break;
    }
    grid_step(kPhExit, 0, 0);
}

}  // namespace pacim
