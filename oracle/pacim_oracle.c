/*
 * pacim_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, single-threaded CPU statement of what the sketch-based greedy
 * influence-maximization hot path of PaC-IM (Wang, Ding, Gu, Sun, PVLDB 17(3),
 * 2023) computes under the Independent Cascade (IC) model on an undirected
 * graph.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file; the GPU library never links, calls or includes it,
 * and it includes nothing from the GPU library.
 *
 * Every function states the passage of the paper it follows.  Integer
 * arithmetic throughout; the only floating point is the one-time conversion of
 * a probability p to a 64-bit threshold.
 *
 * Readings of points the paper leaves open (listed again in the design notes):
 *   - random(e, r) (Sec. 3, function Sample) is the SplitMix64 output function
 *     mix64 applied to the canonical edge key ((min << 32) | max) xor a
 *     per-sketch key K(seed, r) = mix64(seed * phi + r), phi = 0x9E3779B97F4A7C15.
 *   - "random(e,r) <= p_e" on reals becomes the integer test h < T(p) with
 *     T(p) = floor(p * 2^64) for 0 <= p < 1; p >= 1 means every edge is live.
 *   - Trivalency edge probabilities: class = mix64(key ^ K(0, SALT_TRIV)) mod 3
 *     picks p in {0.1, 0.01, 0.001}; the class is a property of the edge, the
 *     same for every sketch and every sampling seed.
 *   - Uniform model (p_e ~ U(lo, hi) once per edge): the threshold itself is
 *     drawn, T_e = T(lo) + floor((T(hi) - T(lo)) * h_e / 2^64) with
 *     h_e = mix64(key ^ K(0, SALT_RANGE)); a property of the edge.
 *   - WIC model (p_e = 2 / (d_u + d_v)): T_e = floor(2^65 / (d_u + d_v)) exactly,
 *     degrees of the undirected graph; d_u + d_v = 2 means always live.
 *   - Per-edge model: the caller's p_e for every CSR entry (equal on both
 *     directions of an edge), T_e = T(p_e).
 *   - Ties in the greedy argmax go to the smallest vertex id (Sec. 4 only says
 *     ties are broken by vertex id).
 *   - Centers of CompactSketch: v is a center iff mix64(v ^ K(seed, SALT_CENTER))
 *     < T(alpha) (an independent Bernoulli(alpha) per vertex, the assumption of
 *     the proof of Theorem 3.1); centers are ranked by vertex id, and a CC's
 *     compact label is the smallest center rank in it (Sec. 3, sketch triple).
 *   - Marginal keeps the integer sum over the R sketches instead of dividing
 *     by R (Sec. 3, function Marginal); the division is display only.
 *
 * Pins: every function here is pinned by tests that do not reuse this code
 * (published SplitMix64 outputs, exact rational thresholds, library connected
 * components, brute-force reachability and exact IC spread on tiny graphs,
 * closed forms).  orc_celf_evaluations (Algorithm 2) keeps its queue in a total
 * order (stale score, then smaller id), so every pop and each round's evaluation
 * count are determined; the counts are pinned by rounds of Algorithm 2 worked by
 * hand, including a vertex evaluated twice in one round.
 * orc_influence is pinned by the seeds' reach summed over worlds spelled out from
 * the published mixer, by the IC cascade's exact expected spread (enumerated over
 * coin flips) within 5 standard errors, and by the p = 0 / p = 1 closed forms.
 * orc_ptree's per-round evaluation counts are unique (the queue's order is total)
 * and pinned by hand-worked rounds of Algorithm 4, by Theorem 4.1 (the plain
 * greedy's seeds, also under many ties) and by Theorem 4.2 (at most twice CELF's
 * evaluations).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_PHI 0x9E3779B97F4A7C15ULL
#define ORC_SALT_CENTER 0xC000000000000001ULL
#define ORC_SALT_TRIV 0xC000000000000002ULL
#define ORC_SALT_RANGE 0xC000000000000003ULL
#define ORC_ALL_LIVE 0xFFFFFFFFFFFFFFFFULL
#define ORC_NONE 0xFFFFFFFFu

/* SplitMix64 output function (Steele, Lea, Flood 2014; constants of Vigna's
 * public-domain splitmix64.c). */
uint64_t orc_mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

/* K(seed, x): the key of sketch x (or of a salt) under sampling seed `seed`. */
uint64_t orc_key(uint64_t seed, uint64_t x) { return orc_mix64(seed * ORC_PHI + x); }

/* p -> integer threshold.  The product p * 2^64 is exact in binary floating
 * point (a power-of-two scaling); the cast truncates toward zero. */
uint64_t orc_threshold(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return ORC_ALL_LIVE;
    return (uint64_t)ldexp(p, 64);
}

static inline uint64_t orc_edge_key(uint32_t u, uint32_t v) {
    uint32_t a = u < v ? u : v, b = u < v ? v : u;
    return ((uint64_t)a << 32) | b;
}

/* Edge probability models, as integer thresholds T_e (edge live iff h < T_e).
 *   kind 0 (Consistent, Sec. 5): the same p on every edge, T = T(p).
 *   kind 1 (trivalency): p_e drawn from {0.1, 0.01, 0.001} by the edge's hash class.
 *   kind 2 (Uniform, appendix on edge-probability distributions): p_e drawn
 *     uniformly from [p, p_hi) once per edge.  Reading: with h_e =
 *     mix64(key ^ K(0, SALT_RANGE)) a uniform 64-bit value of the edge,
 *     T_e = T(p) + floor((T(p_hi) - T(p)) * h_e / 2^64), i.e. the threshold itself
 *     is uniform over [T(p), T(p_hi)).  Requires 0 <= p <= p_hi < 1.
 *   kind 3 (WIC, same appendix): p_e = 2 / (d_u + d_v) with d the vertex degrees
 *     of the undirected graph.  T_e = floor(2^65 / (d_u + d_v)), the exact floor
 *     of p_e * 2^64; d_u + d_v = 2 (an edge whose ends have no other edge) is
 *     p_e = 1: always live.
 * du, dv are only read by kind 3, p_hi only by kind 2. */
uint64_t orc_edge_threshold(int kind, double p, double p_hi, uint32_t u, uint32_t v, uint64_t du, uint64_t dv) {
    if (kind == 0) return orc_threshold(p);
    if (kind == 1) {
        static const double tri[3] = {0.1, 0.01, 0.001};
        uint64_t c = orc_mix64(orc_edge_key(u, v) ^ orc_key(0, ORC_SALT_TRIV)) % 3;
        return orc_threshold(tri[c]);
    }
    if (kind == 2) {
        uint64_t lo = orc_threshold(p), hi = orc_threshold(p_hi);
        uint64_t h = orc_mix64(orc_edge_key(u, v) ^ orc_key(0, ORC_SALT_RANGE));
        return lo + (uint64_t)(((unsigned __int128)(hi - lo) * h) >> 64);
    }
    uint64_t s = du + dv;
    if (s <= 2) return ORC_ALL_LIVE;
    return (uint64_t)(((unsigned __int128)1 << 65) / s);
}

static inline uint64_t orc_deg(const uint64_t *offsets, uint32_t v) { return offsets[v + 1] - offsets[v]; }

/* kind 4 (per-edge probabilities given by the caller, the general p_e of Sec. 2's
 * IC definition): p_edge[j] for CSR entry j, the same value on both directions
 * of an edge; T_e = T(p_e).  Threshold of CSR entry j (row u, column w) under
 * any model. */
static inline uint64_t orc_entry_threshold(int kind, double p, double p_hi, const double *p_edge,
                                           const uint64_t *offsets, uint32_t u, uint64_t j, uint32_t w) {
    if (kind == 4) return orc_threshold(p_edge[j]);
    return orc_edge_threshold(kind, p, p_hi, u, w, orc_deg(offsets, u), orc_deg(offsets, w));
}

/* Sample(e, r) of Sec. 3: is edge {u,v} live in sketch r? */
int orc_live(uint32_t u, uint32_t v, uint32_t r, uint64_t seed, uint64_t T) {
    if (T == ORC_ALL_LIVE) return 1;
    return orc_mix64(orc_edge_key(u, v) ^ orc_key(seed, r)) < T;
}

/* Sketch(r) with full labels (the alpha = 1 memoization of Sec. 2, where a
 * vertex's influence on a sketch is its connected component in G'_r).  For
 * every vertex v: label[v] = smallest vertex id in v's CC of G'_r, size[v] =
 * |CC_r(v)|.  Computed by BFS from each not yet labelled vertex in increasing
 * id order, so the BFS source is the CC minimum.  Returns the number of CCs. */
int64_t orc_sketch(uint32_t n, const uint64_t *offsets, const uint32_t *cols, int kind, double p, double p_hi,
                   const double *p_edge, uint64_t seed, uint32_t r, uint32_t *label, uint32_t *size) {
    uint32_t *queue = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) label[v] = ORC_NONE;
    int64_t ncc = 0;
    for (uint32_t s = 0; s < n; ++s) {
        if (label[s] != ORC_NONE) continue;
        uint32_t head = 0, tail = 0;
        queue[tail++] = s;
        label[s] = s;
        while (head < tail) {
            uint32_t u = queue[head++];
            for (uint64_t j = offsets[u]; j < offsets[u + 1]; ++j) {
                uint32_t w = cols[j];
                if (label[w] != ORC_NONE) continue;
                if (!orc_live(u, w, r, seed, orc_entry_threshold(kind, p, p_hi, p_edge, offsets, u, j, w))) continue;
                label[w] = s;
                queue[tail++] = w;
            }
        }
        for (uint32_t i = 0; i < tail; ++i) size[queue[i]] = tail;
        ++ncc;
    }
    free(queue);
    return ncc;
}

/* Marginal(S, v) of the full (alpha = 1) sketch for v in [lo, hi): the sum
 * over sketches of |CC_r(v)| when that CC holds no seed yet, else 0 (Sec. 2,
 * memoized evaluation; Sec. 3, Marginal).  covered[r*n + l] != 0 marks the CC
 * with label l of sketch r as holding a seed.  Seeds get gain 0 here; the
 * greedy driver skips them. */
void orc_marginals(uint32_t n, uint32_t R, const uint32_t *label, const uint32_t *size,
                   const uint8_t *covered, uint32_t lo, uint32_t hi, uint64_t *gain) {
    for (uint32_t v = lo; v < hi; ++v) {
        uint64_t g = 0;
        for (uint32_t r = 0; r < R; ++r) {
            size_t at = (size_t)r * n + v;
            if (!covered[(size_t)r * n + label[at]]) g += size[at];
        }
        gain[v - lo] = g;
    }
}

/* MarkSeed(s) of the full sketch: the CC of s in every sketch now holds a seed. */
void orc_cover(uint32_t n, uint32_t R, const uint32_t *label, uint8_t *covered, uint32_t s) {
    for (uint32_t r = 0; r < R; ++r) covered[(size_t)r * n + label[(size_t)r * n + s]] = 1;
}

/* The plain greedy (GeneralGreedy of Sec. 2, the definition every lazy and
 * parallel variant reaches): k rounds, each evaluating every non-seed vertex
 * from scratch and taking the largest gain, smallest id on ties.  Requires
 * k <= n.  seeds[i], gains[i] are the i-th pick and its marginal gain. */
int orc_greedy(uint32_t n, uint32_t R, const uint32_t *label, const uint32_t *size, uint32_t k,
               uint32_t *seeds, uint64_t *gains) {
    if (k > n) return -1;
    uint8_t *covered = (uint8_t *)calloc((size_t)R * n + 1, 1);
    uint8_t *in_s = (uint8_t *)calloc((size_t)n + 1, 1);
    uint64_t *g = (uint64_t *)malloc((size_t)(n ? n : 1) * sizeof(uint64_t));
    for (uint32_t i = 0; i < k; ++i) {
        orc_marginals(n, R, label, size, covered, 0, n, g);
        uint32_t best = ORC_NONE;
        for (uint32_t v = 0; v < n; ++v) {
            if (in_s[v]) continue;
            if (best == ORC_NONE || g[v] > g[best]) best = v;
        }
        seeds[i] = best;
        gains[i] = g[best];
        in_s[best] = 1;
        orc_cover(n, R, label, covered, best);
    }
    free(covered); free(in_s); free(g);
    return 0;
}

/* Centers of CompactSketch (Sec. 3): vertices passing the hashed
 * Bernoulli(alpha) test, in increasing id order (center i has rank i).
 * Returns rho, the number of centers; centers may be NULL to count only. */
uint32_t orc_centers(uint32_t n, uint64_t seed, double alpha, uint32_t *centers) {
    uint64_t T = orc_threshold(alpha), K = orc_key(seed, ORC_SALT_CENTER);
    uint32_t rho = 0;
    for (uint32_t v = 0; v < n; ++v) {
        int is_c = (T == ORC_ALL_LIVE) ? 1 : (orc_mix64((uint64_t)v ^ K) < T);
        if (is_c) { if (centers) centers[rho] = v; ++rho; }
    }
    return rho;
}

/* The sketch triple <r, label[1..rho], size[1..rho]> of Sec. 3 for one sketch,
 * derived from that sketch's full labels: label_c[i] = smallest center rank j
 * with c_j in the CC of c_i; size_c[i] = |CC(c_i)| if label_c[i] = i, else 0. */
void orc_compact(uint32_t n, uint32_t rho, const uint32_t *centers, const uint32_t *label,
                 const uint32_t *size, uint32_t *label_c, uint32_t *size_c) {
    uint32_t *first = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) first[v] = ORC_NONE;
    for (uint32_t i = 0; i < rho; ++i) {          /* ranks ascend, so the first seen is the min */
        uint32_t l = label[centers[i]];
        if (first[l] == ORC_NONE) first[l] = i;
    }
    for (uint32_t i = 0; i < rho; ++i) {
        uint32_t c = centers[i];
        label_c[i] = first[label[c]];
        size_c[i] = (label_c[i] == i) ? size[c] : 0;
    }
    free(first);
}

/* GetCenter(Phi_r, v, S) of Sec. 3: BFS from v over the live edges of sketch
 * r.  If a center c_i is reached: l = label_c[i], delta = size_c[l].  Else
 * l = NONE and delta = 0 if the BFS met a seed, otherwise the number of
 * vertices it reached.  center_rank[v] is v's rank or NONE; seen is an n-byte
 * zeroed scratch array returned zeroed; queue holds n entries.  *visits gets
 * the number of vertices taken from the queue (the cost in Theorem 3.1). */
uint64_t orc_getcenter(uint32_t n, const uint64_t *offsets, const uint32_t *cols, int kind, double p,
                       double p_hi, const double *p_edge, uint64_t seed, uint32_t r, const uint32_t *center_rank, const uint32_t *label_c,
                       const uint32_t *size_c, const uint8_t *in_s, uint32_t v, uint32_t *l_out,
                       uint8_t *seen, uint32_t *queue, uint64_t *visits) {
    (void)n;
    uint32_t head = 0, tail = 0, found = ORC_NONE;
    int met_seed = 0;
    queue[tail++] = v;
    seen[v] = 1;
    while (head < tail) {
        uint32_t u = queue[head++];
        if (center_rank[u] != ORC_NONE) { found = center_rank[u]; break; }
        if (in_s[u]) met_seed = 1;
        for (uint64_t j = offsets[u]; j < offsets[u + 1]; ++j) {
            uint32_t w = cols[j];
            if (seen[w]) continue;
            if (!orc_live(u, w, r, seed, orc_entry_threshold(kind, p, p_hi, p_edge, offsets, u, j, w))) continue;
            seen[w] = 1;
            queue[tail++] = w;
        }
    }
    *visits += head;
    for (uint32_t i = 0; i < tail; ++i) seen[queue[i]] = 0;
    if (found != ORC_NONE) {
        uint32_t l = label_c[found];
        *l_out = l;
        return size_c[l];
    }
    *l_out = ORC_NONE;
    return met_seed ? 0 : (uint64_t)tail;
}

/* The greedy of Algorithm 1 run on CompactSketch with the Marginal and
 * MarkSeed functions of Sec. 3: label_c and size_c are [R][rho] (size_c is
 * updated in place by MarkSeed).  Plain (non-lazy) argmax per round, smallest
 * id on ties.  Theorem 3.1 and the alpha = 1 / alpha = 0 equivalences of
 * Sec. 3 say the result equals orc_greedy's on the same sketches.
 * *visits accumulates the vertices dequeued by every GetCenter call. */
int orc_compact_greedy(uint32_t n, const uint64_t *offsets, const uint32_t *cols, int kind, double p,
                       double p_hi, const double *p_edge, uint64_t seed, uint32_t R, uint32_t rho, const uint32_t *centers,
                       const uint32_t *label_c, uint32_t *size_c, uint32_t k, uint32_t *seeds,
                       uint64_t *gains, uint64_t *visits) {
    if (k > n) return -1;
    uint32_t *rank = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    for (uint32_t v = 0; v < n; ++v) rank[v] = ORC_NONE;
    for (uint32_t i = 0; i < rho; ++i) rank[centers[i]] = i;
    uint8_t *seen = (uint8_t *)calloc((size_t)n + 1, 1), *in_s = (uint8_t *)calloc((size_t)n + 1, 1);
    uint32_t *queue = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint64_t vis = 0;
    for (uint32_t i = 0; i < k; ++i) {
        uint32_t best = ORC_NONE;
        uint64_t bestg = 0;
        for (uint32_t v = 0; v < n; ++v) {
            if (in_s[v]) continue;
            uint64_t g = 0;
            for (uint32_t r = 0; r < R; ++r) {
                uint32_t l;
                g += orc_getcenter(n, offsets, cols, kind, p, p_hi, p_edge, seed, r, rank, label_c + (size_t)r * rho,
                                   size_c + (size_t)r * rho, in_s, v, &l, seen, queue, &vis);
            }
            if (best == ORC_NONE || g > bestg) { best = v; bestg = g; }
        }
        seeds[i] = best;
        gains[i] = bestg;
        for (uint32_t r = 0; r < R; ++r) {          /* MarkSeed */
            uint32_t l;
            orc_getcenter(n, offsets, cols, kind, p, p_hi, p_edge, seed, r, rank, label_c + (size_t)r * rho,
                          size_c + (size_t)r * rho, in_s, best, &l, seen, queue, &vis);
            if (l != ORC_NONE) size_c[(size_t)r * rho + l] = 0;
        }
        in_s[best] = 1;
    }
    if (visits) *visits = vis;
    free(rank); free(seen); free(in_s); free(queue);
    return 0;
}

/* Sequential CELF (Algorithm 2) over full labels, counting evaluations: a
 * binary max-heap keyed by (stale score, smaller id first).  Every pop is one
 * evaluation, as Algorithm 2 states (a vertex popped again in the same round is
 * evaluated again).  Seeds equal orc_greedy's; under the total order the
 * per-round counts are unique. */
static int orc_heap_less(const uint64_t *key, const uint32_t *h, uint32_t a, uint32_t b) {
    /* true if element at a ranks below element at b */
    uint64_t ka = key[h[a]], kb = key[h[b]];
    if (ka != kb) return ka < kb;
    return h[a] > h[b];
}
static void orc_sift_down(uint64_t *key, uint32_t *h, uint32_t len, uint32_t i) {
    for (;;) {
        uint32_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < len && orc_heap_less(key, h, m, l)) m = l;
        if (r < len && orc_heap_less(key, h, m, r)) m = r;
        if (m == i) return;
        uint32_t t = h[i]; h[i] = h[m]; h[m] = t;
        i = m;
    }
}
int orc_celf_evaluations(uint32_t n, uint32_t R, const uint32_t *label, const uint32_t *size, uint32_t k,
                         uint32_t *seeds, uint64_t *gains, uint64_t *evals_per_round) {
    if (k > n || n == 0) return -1;
    uint8_t *covered = (uint8_t *)calloc((size_t)R * n + 1, 1);
    uint64_t *key = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    uint32_t *h = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    orc_marginals(n, R, label, size, covered, 0, n, key);
    for (uint32_t v = 0; v < n; ++v) h[v] = v;
    uint32_t len = n;
    for (int64_t i = (int64_t)n / 2 - 1; i >= 0; --i) orc_sift_down(key, h, len, (uint32_t)i);
    for (uint32_t i = 0; i < k; ++i) {
        uint64_t ev = 0;
        for (;;) {
            uint32_t s = h[0];
            h[0] = h[--len];
            orc_sift_down(key, h, len, 0);
            uint64_t g;
            orc_marginals(n, R, label, size, covered, s, s + 1, &g);
            ++ev;
            key[s] = g;
            int wins = (len == 0) || g > key[h[0]] || (g == key[h[0]] && s < h[0]);
            if (wins) {
                seeds[i] = s;
                gains[i] = g;
                orc_cover(n, R, label, covered, s);
                break;
            }
            h[len++] = s;                        /* insert back, sift up */
            uint32_t c = len - 1;
            while (c > 0) {
                uint32_t par = (c - 1) / 2;
                if (!orc_heap_less(key, h, par, c)) break;
                uint32_t t = h[c]; h[c] = h[par]; h[par] = t;
                c = par;
            }
        }
        if (evals_per_round) evals_per_round[i] = ev;
    }
    free(covered); free(key); free(h);
    return 0;
}

/* NextSeed by prefix doubling over a parallel BST (Sec. 4, Algorithm 4 and its
 * P-tree priority queue), over full labels, single-threaded.
 *
 * T holds every unselected vertex keyed by its stale score; it is a plain array
 * kept in T's total order (larger score first, smaller id first on equal
 * scores, the greedy's tie rule), read from index `head` on:
 *   SplitAndRemove(m)  = the m entries at head..head+m-1, head advanced;
 *   Max()              = the entry at head (none once T is empty);
 *   BatchInsert(B)     = B sorted into the same order, then merged with the
 *                        entries left in T into a fresh array.
 * Each round takes batches B_0, B_1, ... of 1, 2, 4, ... entries (fewer if T
 * runs out), evaluates every vertex of a batch, keeps s*, the best (score, id)
 * evaluated in the round, and stops once s* ranks above Max() or T is empty.
 * s* is the seed; every other evaluated vertex goes back into T with its new
 * score.  Initial scores are Marginal(empty, v), exact for round 0.
 * seeds/gains are the picks; evals_per_round[i] = |B_0| + |B_1| + ...  */
typedef struct { uint64_t score; uint32_t id; } orc_pt_entry;

static int orc_pt_before(const orc_pt_entry *a, const orc_pt_entry *b) {
    if (a->score != b->score) return a->score > b->score;
    return a->id < b->id;
}
static int orc_pt_cmp(const void *pa, const void *pb) {
    const orc_pt_entry *a = (const orc_pt_entry *)pa, *b = (const orc_pt_entry *)pb;
    if (orc_pt_before(a, b)) return -1;
    if (orc_pt_before(b, a)) return 1;
    return 0;
}

int orc_ptree(uint32_t n, uint32_t R, const uint32_t *label, const uint32_t *size, uint32_t k,
              uint32_t *seeds, uint64_t *gains, uint64_t *evals_per_round) {
    if (k > n || n == 0) return -1;
    uint8_t *covered = (uint8_t *)calloc((size_t)R * n + 1, 1);
    orc_pt_entry *T = (orc_pt_entry *)malloc((size_t)n * sizeof(orc_pt_entry));
    orc_pt_entry *fresh = (orc_pt_entry *)malloc((size_t)n * sizeof(orc_pt_entry));
    orc_pt_entry *next = (orc_pt_entry *)malloc((size_t)n * sizeof(orc_pt_entry));
    uint64_t *g0 = (uint64_t *)malloc((size_t)n * sizeof(uint64_t));
    orc_marginals(n, R, label, size, covered, 0, n, g0);
    for (uint32_t v = 0; v < n; ++v) { T[v].score = g0[v]; T[v].id = v; }
    qsort(T, n, sizeof(orc_pt_entry), orc_pt_cmp);
    uint32_t head = 0, len = n;
    for (uint32_t i = 0; i < k; ++i) {
        /* the repeat-until loop of NextSeed */
        uint32_t nfresh = 0;
        orc_pt_entry best = {0, ORC_NONE};
        for (uint64_t batch = 1;; batch *= 2) {
            uint32_t m = (uint32_t)(batch < (uint64_t)(len - head) ? batch : (uint64_t)(len - head));
            for (uint32_t t = 0; t < m; ++t) {          /* B_j = SplitAndRemove(2^j) */
                uint32_t v = T[head + t].id;
                uint64_t g;
                orc_marginals(n, R, label, size, covered, v, v + 1, &g);   /* Marginal(S, v) */
                fresh[nfresh].score = g;
                fresh[nfresh].id = v;
                if (best.id == ORC_NONE || orc_pt_before(&fresh[nfresh], &best)) best = fresh[nfresh];
                ++nfresh;
            }
            head += m;
            if (head == len || orc_pt_before(&best, &T[head])) break;   /* s* beats Max() */
        }
        seeds[i] = best.id;
        gains[i] = best.score;
        if (evals_per_round) evals_per_round[i] = nfresh;
        orc_cover(n, R, label, covered, best.id);                        /* MarkSeed(s*) */
        /* BatchInsert(B_0 u B_1 u ... minus s*) */
        uint32_t nb = 0;
        for (uint32_t t = 0; t < nfresh; ++t)
            if (fresh[t].id != best.id) fresh[nb++] = fresh[t];
        qsort(fresh, nb, sizeof(orc_pt_entry), orc_pt_cmp);
        uint32_t a = head, b = 0, o = 0;
        while (a < len || b < nb) {
            if (b == nb || (a < len && orc_pt_before(&T[a], &fresh[b]))) next[o++] = T[a++];
            else next[o++] = fresh[b++];
        }
        orc_pt_entry *sw = T; T = next; next = sw;
        head = 0;
        len = o;
    }
    free(covered); free(T); free(fresh); free(next); free(g0);
    return 0;
}

/* Influence spread of a seed set by simulation (the quality measure of Sec. 5,
 * "influence evaluated by simulations"): under IC on an undirected graph one
 * cascade flips every edge's coin once, so simulation w is the live-edge world
 * of sketch key K(sim_seed, w) and the cascade from S activates every vertex
 * connected to a seed there.  Returns the sum over worlds w in [w0, w0 + sims) of
 * the number of activated vertices (a multi-source BFS per world); the estimate
 * is that sum / sims.  Duplicate seeds count once.  Model arguments as
 * orc_sketch. */
uint64_t orc_influence(uint32_t n, const uint64_t *offsets, const uint32_t *cols, int kind, double p, double p_hi,
                       const double *p_edge, const uint32_t *seeds, uint32_t k, uint64_t sim_seed, uint32_t w0, uint32_t sims) {
    uint8_t *active = (uint8_t *)calloc((size_t)n + 1, 1);
    uint32_t *queue = (uint32_t *)malloc((size_t)(n ? n : 1) * sizeof(uint32_t));
    uint64_t total = 0;
    for (uint32_t w = w0; w < w0 + sims; ++w) {
        uint32_t head = 0, tail = 0;
        for (uint32_t i = 0; i < k; ++i)
            if (!active[seeds[i]]) { active[seeds[i]] = 1; queue[tail++] = seeds[i]; }
        while (head < tail) {
            uint32_t u = queue[head++];
            for (uint64_t j = offsets[u]; j < offsets[u + 1]; ++j) {
                uint32_t x = cols[j];
                if (active[x]) continue;
                if (!orc_live(u, x, w, sim_seed, orc_entry_threshold(kind, p, p_hi, p_edge, offsets, u, j, x)))
                    continue;
                active[x] = 1;
                queue[tail++] = x;
            }
        }
        total += tail;
        for (uint32_t i = 0; i < tail; ++i) active[queue[i]] = 0;
    }
    free(active); free(queue);
    return total;
}
