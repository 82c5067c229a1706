// Sketch construction (Sec. 3, Sketch(r); Algorithm 1, step 1) for a batch of
// B sketches per pass over the edge list.
//
//   k_sketch_keys     K(seed, r) for every sketch
//   k_batch_init(4)   entry (x, b): parent = x, cnt = 0, minc = x's center rank (or a
//                     given value); the "4" form writes 4 entries per 16-byte store
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
//
// Scratch layout (parent, cnt, minc) is vertex-major: the entry of sketch b and
// number x is at x * vs + b, vs = the scratch's sketches per pass, so a vertex's
// entries in all the pass's sketches share one or two cache lines.  The edges of
// one vertex are consecutive in the edge list, so the live sketches of one
// wave's edges mostly read the same lines for their first endpoint; the per-vertex
// passes read a vertex's sketches together.
#pragma once

#include "common.h"
#include "hook_kernels.h"

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
                                                         const uint32_t *__restrict__ newid, uint32_t vs,
                                                         const uint32_t *__restrict__ seeds, uint32_t k,
                                                         unsigned long long *__restrict__ total) {
    const uint32_t b = blockIdx.y;
    uint64_t sum = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
        const uint32_t root = parent[(size_t)newid[seeds[i]] * vs + b];
        const size_t at = (size_t)root * vs + b;
        if (atomicExch(&flag[at], 1u) == 0u) sum += 1u + cnt[at];
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
// root's own rank needs no atomic), else at minc_init.  parent null: the entries
// already hold their own numbers (an emit that reset them).  Numbers [0, n_init):
// isolated vertices (numbered last) keep their entries from an earlier pass of
// the same build, as no pass writes them.  2^lw threads per number (2^lw >= vs),
// thread t of a number writing its sketch t < vs: rows in layout order, and the
// number and sketch of a thread by shifts.
__global__ void k_batch_init(uint32_t *__restrict__ parent, uint32_t *__restrict__ cnt, uint32_t *__restrict__ minc,
                             uint32_t vs, uint32_t lw, uint32_t n_init, uint32_t minc_init,
                             const uint32_t *__restrict__ center_rank) {
    const uint64_t total = (uint64_t)n_init << lw;
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
        const uint32_t x = (uint32_t)(i >> lw), b = (uint32_t)i & ((1u << lw) - 1u);
        if (b >= vs) continue;
        const size_t at = (size_t)x * vs + b;
        if (parent) parent[at] = x;
        cnt[at] = 0;
        if (minc) minc[at] = center_rank ? center_rank[x] : minc_init;
    }
}

// k_batch_init for vs a multiple of 4 (every default pass width): the same
// values, one 16-byte store per array for 4 entries of a number's row.  A row of
// 64 entries is then 16 lanes' stores instead of 64, and the set-up, which only
// writes, runs at 6.4 TB/s instead of 3.8 (rmat24, 64 sketches per pass).
__global__ void k_batch_init4(uint32_t *__restrict__ parent, uint32_t *__restrict__ cnt, uint32_t *__restrict__ minc,
                              uint32_t vs, uint32_t n_init, uint32_t minc_init,
                              const uint32_t *__restrict__ center_rank) {
    const uint64_t total = (uint64_t)n_init * (vs / 4u);
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
        const uint32_t x = (uint32_t)((i * 4u) / vs);
        if (parent) reinterpret_cast<uint4 *>(parent)[i] = make_uint4(x, x, x, x);
        reinterpret_cast<uint4 *>(cnt)[i] = make_uint4(0u, 0u, 0u, 0u);
        if (minc) {
            const uint32_t m = center_rank ? center_rank[x] : minc_init;
            reinterpret_cast<uint4 *>(minc)[i] = make_uint4(m, m, m, m);
        }
    }
}

// Pointer jumping and counting over the first n_act numbers (the vertices with
// an edge; an isolated vertex stays its own root with no members and its own
// center rank).  One wave per run of `run` consecutive numbers (a multiple of
// kCompressIlp, at most kCompressRunMax), lane b = sketch b of the pass (b < nb):
// for each number x the wave reads x's entries of all sketches in one or two
// cache lines, each lane walks to its root, points x at it and counts x there.
// kCompressIlp numbers are loaded together.  In social-like graphs most non-root
// vertices of a sketch lie in one giant component, so per-vertex atomics on its
// root counter would serialise: each lane keeps a "hot" root whose member count
// and smallest center rank it accumulates in registers (the first root it meets,
// replaced while it has at most one member); other roots get one atomic per
// member.  At the end the workgroup's waves combine their hot roots per sketch in
// LDS, so a giant root gets one atomic per workgroup rather than per wave.
constexpr uint32_t kCompressRunMax = 128;
constexpr uint32_t kCompressIlp = 8;
constexpr uint32_t kCompressBlock = 1024;
__global__ void __launch_bounds__(kCompressBlock) k_compress(uint32_t *__restrict__ parent,
                                                             uint32_t *__restrict__ cnt, uint32_t vs, uint32_t nb,
                                                             uint32_t n_act, uint32_t run,
                                                             const uint32_t *__restrict__ center_rank,
                                                             uint32_t *__restrict__ minc) {
    constexpr uint32_t kW = kCompressBlock / kWave;
    __shared__ uint32_t sh_root[kW][kWave], sh_cnt[kW][kWave], sh_min[kW][kWave];
    const uint32_t b = lane_id(), wl = threadIdx.x / kWave;
    const bool act = b < nb;
    const uint64_t x0 = (uint64_t)wave_index() * run;
    uint32_t hot = kNone, hot_cnt = 0, hot_min = kNone;
    if (x0 < n_act) {
        const uint32_t x1 = (uint32_t)min<uint64_t>(x0 + run, n_act);
        for (uint32_t xb = (uint32_t)x0; xb < x1; xb += kCompressIlp) {
            uint32_t pp[kCompressIlp], cr[kCompressIlp], rt[kCompressIlp];
#pragma unroll
            for (uint32_t j = 0; j < kCompressIlp; ++j) {
                const uint32_t x = xb + j;
                const bool ok = act && x < x1;
                pp[j] = parent[ok ? (size_t)x * vs + b : 0];
                cr[j] = center_rank ? center_rank[x < x1 ? x : xb] : kNone;  // the same x in every lane
            }
            // the numbers' walks to their roots in lock step, one load per unfinished
            // walk per step (after the hook most entries point at their root, so one
            // step confirms all of them)
#pragma unroll
            for (uint32_t j = 0; j < kCompressIlp; ++j) {
                rt[j] = xb + j;
                if (act && xb + j < x1) pp[j] = pin_vgpr(pp[j]);
                else pp[j] = rt[j];
            }
            for (;;) {
                bool more = false;
#pragma unroll
                for (uint32_t j = 0; j < kCompressIlp; ++j) more |= pp[j] != rt[j];
                if (!more) break;
                uint32_t nx[kCompressIlp];
#pragma unroll
                for (uint32_t j = 0; j < kCompressIlp; ++j) nx[j] = parent[pp[j] != rt[j] ? (size_t)pp[j] * vs + b : 0];
#pragma unroll
                for (uint32_t j = 0; j < kCompressIlp; ++j)
                    if (pp[j] != rt[j]) {
                        rt[j] = pp[j];
                        pp[j] = pin_vgpr(nx[j]);
                    }
            }
#pragma unroll
            for (uint32_t j = 0; j < kCompressIlp; ++j) {
                const uint32_t x = xb + j;
                if (!act || x >= x1) continue;
                const uint32_t r = rt[j];
                if (r == x) continue;
                parent[(size_t)x * vs + b] = r;
                const uint32_t c = cr[j];
                if (r != hot && hot_cnt <= 1) {  // take r as the hot root, giving back a weak one
                    if (hot != kNone) {
                        if (hot_cnt) atomicAdd(cnt + (size_t)hot * vs + b, hot_cnt);
                        if (hot_min != kNone) atomicMin(minc + (size_t)hot * vs + b, hot_min);
                    }
                    hot = r;
                    hot_cnt = 0;
                    hot_min = kNone;
                }
                if (r == hot) {
                    ++hot_cnt;
                    hot_min = min(hot_min, c);  // a root's own rank is already in minc
                } else {
                    atomicAdd(cnt + (size_t)r * vs + b, 1u);
                    if (c != kNone) atomicMin(minc + (size_t)r * vs + b, c);
                }
            }
        }
    }
    sh_root[wl][b] = hot;
    sh_cnt[wl][b] = hot_cnt;
    sh_min[wl][b] = hot_min;
    __syncthreads();
    if (wl == 0 && act) {  // lane b combines the waves' hot roots of sketch b
        uint32_t r0 = kNone, c0 = 0, m0 = kNone;
        for (uint32_t k = 0; k < kW; ++k) {
            const uint32_t r = sh_root[k][b], c = sh_cnt[k][b], mn = sh_min[k][b];
            if (r == kNone) continue;
            if (r0 == kNone) r0 = r;
            if (r == r0) {
                c0 += c;
                m0 = min(m0, mn);
            } else {
                if (c) atomicAdd(cnt + (size_t)r * vs + b, c);
                if (mn != kNone) atomicMin(minc + (size_t)r * vs + b, mn);
            }
        }
        if (r0 != kNone) {
            if (c0) atomicAdd(cnt + (size_t)r0 * vs + b, c0);
            if (m0 != kNone) atomicMin(minc + (size_t)r0 * vs + b, m0);
        }
    }
}

// The vertex-major passes below take one wave per 64 consecutive vertices, lane b
// = sketch b of the pass (b < nb): per vertex the wave reads the vertex's nb
// forest entries in one or two cache lines, gathers the root sizes, and sums the
// initial gain across the lanes; kEmitIlp vertices are in flight together.  The
// per-vertex values (labelling-order number, center rank) are the same in every
// lane.  Isolated vertices (numbers >= n_linked) are their own singletons and read
// nothing.
constexpr uint32_t kEmitIlp = 4;

// Sum over the wave of x, carried in 64 bits.
__device__ __forceinline__ uint64_t wave_sum_lanes(uint64_t x) { return wave_sum_u64(x); }

// Full labels: E[v][r0 + b] = (label, size at the label's own entry) with the
// label the root's vertex id, and the initial gains.  reset: each linked entry is
// set back to its own number once read (no other vertex reads it), so the next
// pass's set-up leaves the forest alone.
__global__ void __launch_bounds__(256) k_emit_full(uint32_t *__restrict__ parent,
                                                   const uint32_t *__restrict__ cnt,
                                                   const uint32_t *__restrict__ newid,
                                                   const uint32_t *__restrict__ iperm, uint32_t n, uint32_t vs,
                                                   uint32_t n_linked, uint32_t nb, uint32_t R, uint32_t r0,
                                                   uint2 *__restrict__ E, uint64_t *__restrict__ gain0,
                                                   bool reset) {
    const uint32_t b = lane_id();
    const bool act = b < nb;
    const uint32_t v0 = wave_index() * kWave;
    if (v0 >= n) return;
    // lane j holds vertex v0 + j's number and its gain sum, written once at the end
    const uint32_t vl = v0 + b;
    const bool vok = vl < n;
    const uint32_t my_iv = vok ? newid[vl] : 0u;
    const uint64_t g_old = vok ? gain0[vl] : 0ull;
    const bool small = (uint64_t)n * kWave < (1ull << 32);  // a vertex's sum over 64 sketches fits 32 bits
    uint64_t g_add = 0;
    for (uint32_t j0 = 0; j0 < kWave; j0 += kEmitIlp) {
        uint32_t iv[kEmitIlp], t[kEmitIlp], root[kEmitIlp], c[kEmitIlp], lab[kEmitIlp];
#pragma unroll
        for (uint32_t u = 0; u < kEmitIlp; ++u) {
            const uint32_t v = v0 + j0 + u;
            iv[u] = (uint32_t)__builtin_amdgcn_readlane((int)my_iv, (int)(j0 + u));
            const bool rd = act && v < n && iv[u] < n_linked;
            t[u] = parent[rd ? (size_t)iv[u] * vs + b : 0];
        }
#pragma unroll
        for (uint32_t u = 0; u < kEmitIlp; ++u) {
            const uint32_t v = v0 + j0 + u;
            const bool rd = act && v < n && iv[u] < n_linked;
            root[u] = rd ? pin_vgpr(t[u]) : iv[u];
            if (reset && rd) parent[(size_t)iv[u] * vs + b] = iv[u];
            c[u] = cnt[rd ? (size_t)root[u] * vs + b : 0];
            lab[u] = iperm[rd ? root[u] : 0];
        }
#pragma unroll
        for (uint32_t u = 0; u < kEmitIlp; ++u) {
            const uint32_t v = v0 + j0 + u;
            if (v >= n) break;  // wave-uniform
            const bool rd = act && iv[u] < n_linked;
            const uint32_t sz = !act ? 0u : (rd ? 1u + pin_vgpr(c[u]) : 1u);
            const bool own = root[u] == iv[u];
            if (act) E[(size_t)v * R + r0 + b] = own ? make_uint2(v, sz) : make_uint2(pin_vgpr(lab[u]), 0u);
            const uint64_t g = small ? (uint64_t)wave_sum_u32_rows(sz) : wave_sum_lanes(sz);
            if (b == j0 + u) g_add = g;
        }
    }
    if (vok) gain0[vl] = g_old + g_add;
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
                                                      const uint32_t *__restrict__ cnt, uint32_t n, uint32_t vs,
                                                      uint32_t n_linked, unsigned long long *__restrict__ gbest) {
    __shared__ unsigned long long best_w[256 / kWave];
    const uint32_t b = blockIdx.x;
    unsigned long long best = 0;
    for (uint32_t j = threadIdx.x; j < kGiantSamples; j += blockDim.x) {
        const uint32_t v = (uint32_t)((uint64_t)j * n / kGiantSamples);
        const bool linked = v < n_linked;  // an isolated number is its own singleton and reads nothing
        const uint32_t root = linked ? parent[(size_t)v * vs + b] : v;
        const uint32_t members = linked ? cnt[(size_t)root * vs + b] : 0u;
        const unsigned long long c = ((unsigned long long)(1u + members) << 32) | (0xFFFFFFFFull - root);
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

// One pass over every vertex of the pass's nb sketches (compressed: every entry
// points at its root) for CompactSketch, one wave per 64-vertex word as above:
//   - the initial gains, sum over sketches of |CC_b(v)|;
//   - gbits non-null: bit v % 64 of gbits[(v / 64) * R + r0 + b] = [v lies in the
//     component of giant_root_of(gbest[b])] (word-major: a vertex word's R
//     sketches are contiguous, and here lane b writes its word once), and
//     gsum[v] += the sizes of those components over the pass's sketches (the bulk
//     rounds' sum over covered largest components starts from it);
//   - for a center v of rank cr, its triple entries label_c[cr][r0 + b] = the
//     smallest center rank in its component (minc at the root) and size_c = the
//     component size if that rank is cr's own, else 0 (center-major [rho][R], so
//     the wave writes a center's entries as one run);
//   - reset: each linked entry set back to its own number once read, as in
//     k_emit_full.
__global__ void __launch_bounds__(256) k_gain0_emit(uint32_t *__restrict__ parent,
                                                    const uint32_t *__restrict__ cnt,
                                                    const uint32_t *__restrict__ minc,
                                                    const uint32_t *__restrict__ center_rank, uint32_t rho,
                                                    uint32_t n, uint32_t vs, uint32_t nb, uint32_t r0, uint32_t R,
                                                    uint32_t *__restrict__ label_c, uint32_t *__restrict__ size_c,
                                                    uint64_t *__restrict__ gain0,
                                                    const unsigned long long *__restrict__ gbest,
                                                    uint64_t *__restrict__ gbits, uint32_t nw,
                                                    uint64_t *__restrict__ gsum,
                                                    const uint32_t *__restrict__ newid, uint32_t n_linked,
                                                    bool reset) {
    const uint32_t b = lane_id();
    const bool act = b < nb;
    const uint32_t w = wave_index();
    if (w >= nw) return;
    const uint32_t v0 = w * kWave;
    const unsigned long long gb = (act && gbits) ? gbest[b] : 0ull;
    const uint32_t groot = giant_root_of(gb), gsize = giant_size_of(gb);
    // lane j holds vertex v0 + j's number, center rank and sums, the sums written
    // once at the end
    const uint32_t vl = v0 + b;
    const bool vok = vl < n;
    const uint32_t my_iv = vok ? newid[vl] : 0u;
    const uint32_t my_cr = vok ? center_rank[vl] : kNone;
    const uint64_t g_old = vok ? gain0[vl] : 0ull;
    const uint64_t s_old = (vok && gbits) ? gsum[vl] : 0ull;
    const bool small = (uint64_t)n * kWave < (1ull << 32);  // a vertex's sums over 64 sketches fit 32 bits
    uint64_t g_add = 0, s_add = 0, gmask = 0;
    for (uint32_t j0 = 0; j0 < kWave; j0 += kEmitIlp) {
        uint32_t iv[kEmitIlp], cr[kEmitIlp], t[kEmitIlp], root[kEmitIlp], c[kEmitIlp], m[kEmitIlp];
#pragma unroll
        for (uint32_t u = 0; u < kEmitIlp; ++u) {
            const uint32_t v = v0 + j0 + u;
            iv[u] = (uint32_t)__builtin_amdgcn_readlane((int)my_iv, (int)(j0 + u));
            cr[u] = (uint32_t)__builtin_amdgcn_readlane((int)my_cr, (int)(j0 + u));
            const bool rd = act && v < n && iv[u] < n_linked;
            t[u] = parent[rd ? (size_t)iv[u] * vs + b : 0];
        }
#pragma unroll
        for (uint32_t u = 0; u < kEmitIlp; ++u) {
            const uint32_t v = v0 + j0 + u;
            const bool rd = act && v < n && iv[u] < n_linked;
            root[u] = rd ? pin_vgpr(t[u]) : iv[u];
            if (reset && rd) parent[(size_t)iv[u] * vs + b] = iv[u];
            c[u] = cnt[rd ? (size_t)root[u] * vs + b : 0];
            m[u] = minc[(rd && cr[u] != kNone) ? (size_t)root[u] * vs + b : 0];
        }
#pragma unroll
        for (uint32_t u = 0; u < kEmitIlp; ++u) {
            const uint32_t v = v0 + j0 + u;
            if (v >= n) break;  // wave-uniform
            const bool rd = act && iv[u] < n_linked;
            const uint32_t sz = !act ? 0u : (rd ? 1u + pin_vgpr(c[u]) : 1u);
            if (cr[u] != kNone && act) {  // a center: its triple entry in this sketch
                const uint32_t l = rd ? pin_vgpr(m[u]) : cr[u];
                const size_t at = (size_t)cr[u] * R + r0 + b;
                label_c[at] = l;
                size_c[at] = l == cr[u] ? sz : 0u;
            }
            const bool in_giant = act && gbits && root[u] == groot;
            gmask |= (uint64_t)in_giant << (j0 + u);
            const uint32_t gs = in_giant ? gsize : 0u;
            uint64_t g, h;
            if (small) {
                g = wave_sum_u32_rows(sz);
                h = gbits ? wave_sum_u32_rows(gs) : 0u;
            } else {
                g = wave_sum_lanes(sz);
                h = gbits ? wave_sum_lanes(gs) : 0u;
            }
            if (b == j0 + u) {
                g_add = g;
                s_add = h;
            }
        }
    }
    if (vok) {
        gain0[vl] = g_old + g_add;
        if (gbits) gsum[vl] = s_old + s_add;
    }
    if (gbits && act) gbits[(size_t)w * R + r0 + b] = gmask;
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
