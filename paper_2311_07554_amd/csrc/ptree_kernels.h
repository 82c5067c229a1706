// NextSeed by prefix doubling (Sec. 4, Algorithm 4) over a totally ordered
// queue of stale keys: the paper's P-tree priority queue in a GPU form.
//
// Keys are the winning tree's packed keys (larger gain first, smaller id on equal
// gains, all distinct), so "the top m entries" is one well-defined set.  The
// queue is two runs sorted in decreasing key order:
//   X  every unselected vertex, sorted once on the device when the queue is
//      built, then read from a moving head;
//   Y  the vertices re-inserted since (BatchInsert), merged into X whenever it
//      outgrows X's unread part.
// SplitAndRemove(m) takes the first m keys of merge(X, Y): a merge-path co-rank
// splits m between the two heads and each thread copies a span of the merged
// order out as vertex ids.  Max() is the larger of the two heads.  BatchInsert
// sorts the round's re-evaluated keys (bitonic tiles of 4096 keys in LDS, then
// merge passes) and merges them with Y.
//
// The paper's P-tree is a balanced BST with polylogarithmic-span batch
// operations; the sorted runs give the same extraction order with sequential,
// coalescing memory traffic instead of pointer chasing.
#pragma once

#include "common.h"
#include "select_kernels.h"

namespace pacim {

constexpr uint32_t kPtTile = 4096;  // keys sorted per workgroup in LDS (32 KB)
constexpr uint32_t kPtBlock = 256;
constexpr uint32_t kPtSpan = 8;     // merged outputs per thread

struct PtState {
    uint32_t take;  // entries the last SplitAndRemove took from X (the rest came from Y)
    uint32_t stop;  // the round's best evaluated key ranks above Max() of what is left
};

// Number of entries of a among the first d of merge(a, b); a and b are in
// decreasing order and share no key.  Requires d <= na + nb.
__device__ __forceinline__ uint32_t pt_corank(const uint64_t *a, uint32_t na, const uint64_t *b, uint32_t nb,
                                              uint32_t d) {
    uint32_t lo = d > nb ? d - nb : 0u, hi = d < na ? d : na;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] > b[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Entries [d0, d0 + cnt) of merge(a, b), handed to put(position, key) in order.
// Requires d0 + cnt <= na + nb.
template <class Put>
__device__ __forceinline__ void pt_merge_span(const uint64_t *a, uint32_t na, const uint64_t *b, uint32_t nb,
                                              uint32_t d0, uint32_t cnt, Put put) {
    uint32_t i = pt_corank(a, na, b, nb, d0), j = d0 - i;
    for (uint32_t t = 0; t < cnt; ++t) {
        const bool from_a = j >= nb || (i < na && a[i] > b[j]);
        const uint64_t kk = from_a ? a[i] : b[j];
        if (from_a) ++i;
        else ++j;
        put(d0 + t, kk);
    }
}

__device__ __forceinline__ uint64_t pt_thread_span() {
    return ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * kPtSpan;
}

// Sorts each tile of kPtTile keys of in[0, len) into decreasing order: a bitonic
// network in LDS over the smallest power of two holding the tile's keys (a short
// tail tile, or a small BatchInsert, runs a short network), padded with 0, which
// sorts last and is not written back.  A stage's compare-exchanges are disjoint,
// so each thread loads all of its pairs before writing any.
__global__ void __launch_bounds__(kPtBlock) k_pt_sort_tiles(const uint64_t *__restrict__ in, uint32_t len,
                                                            uint64_t *__restrict__ out) {
    constexpr uint32_t kPer = kPtTile / 2 / kPtBlock;  // pairs per thread at full size
    __shared__ uint64_t t[kPtTile];
    const uint32_t base = blockIdx.x * kPtTile;
    const uint32_t cnt = min(kPtTile, len - base);
    uint32_t N = 2;
    while (N < cnt) N <<= 1;
    for (uint32_t i = threadIdx.x; i < N; i += kPtBlock) t[i] = i < cnt ? in[base + i] : 0ull;
    __syncthreads();
    const uint32_t pairs = N / 2;
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            uint64_t x[kPer], y[kPer];
#pragma unroll
            for (uint32_t q = 0; q < kPer; ++q) {
                const uint32_t p = threadIdx.x + q * kPtBlock;
                const uint32_t i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                if (p < pairs) {
                    x[q] = t[i];
                    y[q] = t[i + j];
                }
            }
#pragma unroll
            for (uint32_t q = 0; q < kPer; ++q) {
                const uint32_t p = threadIdx.x + q * kPtBlock;
                const uint32_t i = ((p & ~(j - 1)) << 1) | (p & (j - 1));
                if (p < pairs) {
                    const bool dec = (i & k) == 0;
                    if (dec ? x[q] < y[q] : x[q] > y[q]) {
                        t[i] = y[q];
                        t[i + j] = x[q];
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < cnt; i += kPtBlock) out[base + i] = t[i];
}

// One merge-sort pass: sorted runs of L keys (L a multiple of 2 * kPtSpan) merged
// pairwise, in[0, len) -> out[0, len).
__global__ void __launch_bounds__(kPtBlock) k_pt_merge_pass(const uint64_t *__restrict__ in, uint32_t len,
                                                            uint32_t L, uint64_t *__restrict__ out) {
    const uint64_t d = pt_thread_span();
    if (d >= len) return;
    const uint64_t base = d / (2ull * L) * (2ull * L);
    const uint32_t rest = (uint32_t)(len - base);
    const uint32_t na = min(L, rest), nb = rest > L ? min(L, rest - L) : 0u;
    uint64_t *o = out + base;
    pt_merge_span(in + base, na, in + base + na, nb, (uint32_t)(d - base), (uint32_t)min<uint64_t>(kPtSpan, len - d),
                  [&](uint32_t p, uint64_t kk) { o[p] = kk; });
}

// out[0, na + nb) = merge(a, b).
__global__ void __launch_bounds__(kPtBlock) k_pt_merge2(const uint64_t *__restrict__ a, uint32_t na,
                                                        const uint64_t *__restrict__ b, uint32_t nb,
                                                        uint64_t *__restrict__ out) {
    const uint64_t d = pt_thread_span();
    const uint64_t tot = (uint64_t)na + nb;
    if (d >= tot) return;
    pt_merge_span(a, na, b, nb, (uint32_t)d, (uint32_t)min<uint64_t>(kPtSpan, tot - d),
                  [&](uint32_t p, uint64_t kk) { out[p] = kk; });
}

__global__ void k_pt_round_begin(SelState *__restrict__ st) {
    if (threadIdx.x != 0) return;
    st->delta = 0;
    for (int l = 0; l <= kMaxLevels; ++l) { st->fr_cnt[l] = 0; st->ev_cnt[l] = 0; }
    for (int l = 0; l < kMaxLevels + 2; ++l) st->ov_cnt[l] = 0;
}

// SplitAndRemove(m) from the unread parts X[0, nx), Y[0, ny) (m <= nx + ny): the
// vertex ids of the first m keys of merge(X, Y) into evl[0, m), the split into
// ps->take, and the batch size into the level-0 slot the evaluation kernels read.
// CompactSketch: partial[0, m) started at pinit (R searches left, sum 0).
__global__ void __launch_bounds__(kPtBlock) k_pt_extract(const uint64_t *__restrict__ X, uint32_t nx,
                                                         const uint64_t *__restrict__ Y, uint32_t ny, uint32_t m,
                                                         uint32_t kb, uint32_t *__restrict__ evl,
                                                         unsigned long long *__restrict__ partial,
                                                         unsigned long long pinit, PtState *__restrict__ ps,
                                                         SelState *__restrict__ st) {
    const uint64_t d = pt_thread_span();
    if (d == 0) {
        ps->take = pt_corank(X, nx, Y, ny, m);
        st->ev_cnt[0] = m;
        st->ov_cnt[0] = 0;
    }
    if (d >= m) return;
    const uint64_t mask = (1ull << kb) - 1ull;
    pt_merge_span(X, nx, Y, ny, (uint32_t)d, (uint32_t)min<uint64_t>(kPtSpan, m - d), [&](uint32_t p, uint64_t kk) {
        evl[p] = (uint32_t)(mask - (kk & mask));
        if (partial) partial[p] = pinit;
    });
}

// Evaluation of a large batch on full labels: like the winning tree's bulk
// round, a wave takes many listed vertices and each lane keeps the last label it
// gathered per sketch (most vertices of a sketch share its giant component, whose
// entry every wave would otherwise re-read).  Keys written and Delta* raised as
// in the per-vertex evaluation.  R <= 4 * 64.
__global__ void __launch_bounds__(256) k_pt_eval_full_list(const uint32_t *__restrict__ evl, uint32_t m,
                                                           const uint2 *__restrict__ E, uint32_t R, uint32_t kb,
                                                           const uint8_t *__restrict__ in_s,
                                                           uint64_t *__restrict__ key, SelState *__restrict__ st) {
    constexpr int U = 4;
    uint32_t last_l[U], last_y[U];
#pragma unroll
    for (int i = 0; i < U; ++i) last_l[i] = kNone, last_y[i] = 0;
    const uint32_t lane = lane_id();
    uint64_t best = 0;
    for (uint32_t e = wave_index(); e < m; e += wave_count()) {
        const uint32_t v = evl[e];
        const uint2 *row = E + (size_t)v * R;
        uint2 en[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const uint32_t r = lane + i * kWave;
            en[i] = r < R ? row[r] : make_uint2(v, 0u);
        }
        uint64_t g = 0;
#pragma unroll
        for (int i = 0; i < U; ++i) {
            uint32_t y = en[i].y;
            if (en[i].x != v) {
                if (en[i].x != last_l[i]) {
                    last_l[i] = en[i].x;
                    last_y[i] = E[(size_t)en[i].x * R + lane + i * kWave].y;
                }
                y = last_y[i];
            }
            g += y;
        }
        g = wave_sum_u64(g);
        const uint64_t nk = in_s[v] ? 0ull : pack_key(g, v, kb);
        if (lane == 0) key[v] = nk;
        best = nk > best ? nk : best;
    }
    if (lane == 0 && best) atomicMax(&st->delta, (unsigned long long)best);
}

// Evaluation of a batch whose keys are already fresh in key[] (the round
// computed every vertex's Marginal at once): Delta* raised to the batch's best.
__global__ void __launch_bounds__(256) k_pt_eval_known(const uint32_t *__restrict__ evl, uint32_t m,
                                                       const uint64_t *__restrict__ key, SelState *__restrict__ st) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t best = wave_max_u64(i < m ? key[evl[i]] : 0ull);
    if (lane_id() == 0 && best) atomicMax(&st->delta, (unsigned long long)best);
}

// The repeat-until test: does the best key evaluated this round (Delta*) rank
// above Max() of the queue left after the last SplitAndRemove?  An empty queue
// stops the round too (Max() = 0 and every key is positive).
__global__ void k_pt_check(const uint64_t *__restrict__ X, uint32_t nx, const uint64_t *__restrict__ Y, uint32_t ny,
                           uint32_t m, PtState *__restrict__ ps, SelState *__restrict__ st) {
    if (threadIdx.x != 0) return;
    const uint32_t i = ps->take, j = m - i;
    uint64_t top = 0;
    if (i < nx) top = X[i];
    if (j < ny && Y[j] > top) top = Y[j];
    ps->stop = st->delta > top ? 1u : 0u;
    st->overflow += st->ov_cnt[0];
}

// The round's end: s* (the vertex of Delta*) becomes the seed, with the round's
// evaluation count; its key is cleared so that BatchInsert's gather leaves it out
// (it sorts last).  Full labels: MarkSeed zeroes the size at s*'s label in every
// sketch.  One wave.
__device__ __forceinline__ void pt_round_end_wave(SelState *st, uint64_t *key, uint8_t *in_s, uint32_t n,
                                                  uint32_t kb, uint32_t tot, uint32_t *seeds_out,
                                                  unsigned long long *gains_out, uint32_t *evals_out, uint2 *E,
                                                  uint32_t R) {
    const uint32_t lane = lane_id();
    const uint64_t ks = st->delta;
    const uint64_t mask = (1ull << kb) - 1ull;
    const uint32_t s = (uint32_t)(mask - (ks & mask));
    if (ks == 0 || s >= n || in_s[s]) {
        if (lane == 0) st->err = 1;
        return;
    }
    const uint32_t round = st->round;
    if (lane == 0) {
        seeds_out[round] = s;
        gains_out[round] = key_gain(ks, kb);
        evals_out[round] = tot;
        in_s[s] = 1;
        key[s] = 0;
        st->last_seed = s;
        st->last_gain = key_gain(ks, kb);
        st->evals += tot;
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

__global__ void __launch_bounds__(64) k_pt_round_end(SelState *__restrict__ st, uint64_t *__restrict__ key,
                                                     uint8_t *__restrict__ in_s, uint32_t n, uint32_t kb, uint32_t tot,
                                                     uint32_t *__restrict__ seeds_out,
                                                     unsigned long long *__restrict__ gains_out,
                                                     uint32_t *__restrict__ evals_out, uint2 *__restrict__ E,
                                                     uint32_t R) {
    pt_round_end_wave(st, key, in_s, n, kb, tot, seeds_out, gains_out, evals_out, E, R);
}

// ---- whole rounds on the device (full labels) ------------------------------
// One workgroup runs round after round while everything stays small: batches of
// at most kPtDevBatch vertices (one wave per evaluation), BatchInsert sorted in
// LDS and merged with Y by the workgroup.  It stops, leaving the rest to the host
// kernels above, inside a round whose next batch is larger (state: off, batch),
// after a round whose insertion is larger, or after a round whose Y outgrew X's
// unread part (the host merges them).  Without it every batch is a host round trip.
constexpr uint32_t kPtRoundBlock = 1024;
constexpr uint32_t kPtDevBatch = 512;
constexpr uint32_t kPtDevSort = 2 * kPtDevBatch;  // keys of one round, at most
constexpr uint32_t kPtDevMerge = 1u << 18;        // largest Y merge done on the device

enum : uint32_t { kPtStopDone = 0, kPtStopMidRound = 1, kPtStopInsert = 2, kPtStopFold = 3 };

struct PtDev {
    uint64_t *buf[5];
    int32_t x, y;                // buffers of the runs X and Y
    uint32_t hx, nx, hy, ny;     // their unread parts [hx, nx), [hy, ny)
    uint32_t rounds;             // rounds completed by the launch
    uint32_t stop;               // why it returned (kPtStop*)
    uint32_t off, batch;         // mid-round: vertices evaluated in the round so far, next batch size;
                                 // insertion left to the host: the round's evaluation count
};

__global__ void __launch_bounds__(kPtRoundBlock) k_pt_rounds(PtDev *__restrict__ pd, uint32_t max_rounds,
                                                             SelState *__restrict__ st, uint64_t *__restrict__ key,
                                                             uint8_t *__restrict__ in_s, uint32_t n, uint32_t kb,
                                                             uint32_t *__restrict__ seeds_out,
                                                             unsigned long long *__restrict__ gains_out,
                                                             uint32_t *__restrict__ evals_out,
                                                             uint2 *__restrict__ E, uint32_t R,
                                                             uint32_t *__restrict__ evl) {
    constexpr uint32_t kWaves = kPtRoundBlock / kWave;
    __shared__ uint64_t srt[kPtDevSort];
    __shared__ unsigned long long sh_best[kWaves];
    __shared__ uint32_t sh_take;
    const uint32_t tid = threadIdx.x, lane = lane_id(), w = tid / kWave;
    uint64_t *b[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) b[i] = pd->buf[i];
    int32_t x = pd->x, y = pd->y;
    uint32_t hx = pd->hx, nx = pd->nx, hy = pd->hy, ny = pd->ny;
    const uint64_t mask = (1ull << kb) - 1ull;
    uint32_t rounds = 0, stop = kPtStopDone, off = 0;
    uint64_t batch = 1;
    while (rounds < max_rounds) {
        uint64_t best = 0;
        off = 0;
        batch = 1;
        bool mid = false, empty = false;
        for (;;) {
            const uint32_t nxl = nx - hx, nyl = ny - hy;
            const uint32_t m = (uint32_t)min<uint64_t>(batch, (uint64_t)nxl + nyl);
            if (m == 0) {  // no vertex left before a seed was found: cannot happen for k <= n - |S|
                empty = true;
                break;
            }
            if (m > kPtDevBatch) {
                mid = true;
                break;
            }
            const uint64_t *X = b[x] + hx, *Y = b[y] + hy;
            // SplitAndRemove(m): entry t of merge(X, Y) per thread
            if (tid < m) {
                const uint32_t i = pt_corank(X, nxl, Y, nyl, tid), j = tid - i;
                const uint64_t kk = (i < nxl && (j >= nyl || X[i] > Y[j])) ? X[i] : Y[j];
                evl[off + tid] = (uint32_t)(mask - (kk & mask));
            }
            if (tid == 0) sh_take = pt_corank(X, nxl, Y, nyl, m);
            __syncthreads();
            // Marginal of every extracted vertex, one wave each
            uint64_t wb = 0;
            for (uint32_t e = w; e < m; e += kWaves) {
                const uint32_t v = evl[off + e];
                const uint64_t g = marginal_full(E, R, v);
                const uint64_t nk = in_s[v] ? 0ull : pack_key(g, v, kb);
                if (lane == 0) key[v] = nk;
                wb = nk > wb ? nk : wb;
            }
            if (lane == 0) sh_best[w] = wb;
            __syncthreads();
            for (uint32_t i = 0; i < kWaves; ++i) best = sh_best[i] > best ? sh_best[i] : best;
            const uint32_t take = sh_take;
            uint64_t top = 0;
            if (take < nxl) top = X[take];
            if (m - take < nyl && Y[m - take] > top) top = Y[m - take];
            hx += take;
            hy += m - take;
            off += m;
            batch *= 2;
            __syncthreads();  // sh_take and sh_best are rewritten by the next batch
            if (best > top) break;
        }
        if (empty) {
            if (tid == 0) st->err = 4;
            break;
        }
        if (tid == 0) st->delta = best;
        __syncthreads();
        if (mid) {
            stop = kPtStopMidRound;
            break;
        }
        if (w == 0) pt_round_end_wave(st, key, in_s, n, kb, off, seeds_out, gains_out, evals_out, E, R);
        __syncthreads();
        ++rounds;
        // BatchInsert of the other evaluated vertices (s*'s key is now 0: it sorts last)
        const uint32_t tot = off;
        if (tot > 1) {
            const uint32_t nyl = ny - hy;
            if (tot > kPtDevSort || (uint64_t)nyl + tot - 1 > kPtDevMerge) {
                stop = kPtStopInsert;
                break;
            }
            uint32_t N = 2;
            while (N < tot) N <<= 1;
            for (uint32_t t = tid; t < N; t += kPtRoundBlock) srt[t] = t < tot ? key[evl[t]] : 0ull;
            __syncthreads();
            for (uint32_t k = 2; k <= N; k <<= 1) {
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    if (tid < N / 2) {
                        const uint32_t i = ((tid & ~(j - 1)) << 1) | (tid & (j - 1));
                        const uint64_t p0 = srt[i], p1 = srt[i + j];
                        const bool dec = (i & k) == 0;
                        if (dec ? p0 < p1 : p0 > p1) {
                            srt[i] = p1;
                            srt[i + j] = p0;
                        }
                    }
                    __syncthreads();
                }
            }
            int32_t f = 0;
            while (f == x || f == y) ++f;
            const uint32_t total = tot - 1 + nyl;
            const uint32_t per = (total + kPtRoundBlock - 1) / kPtRoundBlock;
            const uint64_t *Yl = b[y] + hy;
            uint64_t *out = b[f];
            const uint32_t d0 = tid * per;
            if (d0 < total)
                pt_merge_span(srt, tot - 1, Yl, nyl, d0, min(per, total - d0),
                              [&](uint32_t p, uint64_t kk) { out[p] = kk; });
            __syncthreads();
            y = f;
            hy = 0;
            ny = total;
        }
        if (ny - hy > nx - hx) {
            stop = kPtStopFold;
            break;
        }
    }
    if (tid == 0) {
        pd->x = x;
        pd->y = y;
        pd->hx = hx;
        pd->nx = nx;
        pd->hy = hy;
        pd->ny = ny;
        pd->rounds = rounds;
        pd->stop = stop;
        pd->off = off;
        pd->batch = (uint32_t)batch;
    }
}

// BatchInsert's input: the current keys of the round's evaluated vertices.
__global__ void __launch_bounds__(256) k_pt_gather(const uint32_t *__restrict__ evl, uint32_t cnt,
                                                   const uint64_t *__restrict__ key, uint64_t *__restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) out[i] = key[evl[i]];
}

}  // namespace pacim
