/*
 * Seeded synthetic graph generators: the shared inputs of the library and of
 * the oracle.  This file holds no part of the influence-maximization method;
 * it only produces simple undirected graphs (no self-loops, no duplicate
 * pairs) in two forms:
 *
 *   - a sorted list of canonical keys  key = (min(u,v) << 32) | max(u,v);
 *   - a symmetric CSR (offsets[n+1] as uint64, cols[2m] as uint32, each row
 *     sorted ascending), built from such a key list.
 *
 * Randomness is the SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014)
 * used as a counter-based generator: draw i of stream `key` is
 * mix(key + (i+1) * 0x9E3779B97F4A7C15), which is exactly the i-th output of a
 * SplitMix64 generator whose state starts at `key`.  Because every draw is
 * addressed by its index, the parallel loops below give the same graph for any
 * thread count.
 *
 * Generators:
 *   gg_er       Erdos-Renyi G(n, M): M distinct pairs drawn uniformly.
 *   gg_rmat     R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with quadrant
 *               probabilities (a, b, c, 1-a-b-c), a seeded vertex permutation,
 *               self-loops and duplicates removed, drawn until m distinct pairs.
 *   gg_chunglu  Chung-Lu power-law graph: endpoint i drawn with probability
 *               proportional to w_i = (i+1)^(-1/(gamma-1)), weights capped at
 *               sqrt(sum w), n*d/2 endpoint pairs drawn, permuted, deduplicated.
 *
 * When a generator has more distinct pairs than asked for (gg_er, gg_rmat),
 * it keeps the m pairs with the smallest hashed priority, a uniform subset that
 * does not favour small ids.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GG_PHI 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static inline uint64_t gg_draw(uint64_t key, uint64_t i) { return gg_mix(key + (i + 1) * GG_PHI); }
static inline double gg_unit(uint64_t x) { return (double)(x >> 11) * (1.0 / 9007199254740992.0); }
static inline uint32_t gg_below(uint64_t x, uint32_t n) {
    return (uint32_t)(((unsigned __int128)x * n) >> 64);
}
static inline uint64_t gg_canon(uint32_t u, uint32_t v) {
    return u < v ? (((uint64_t)u << 32) | v) : (((uint64_t)v << 32) | u);
}

/* LSD radix sort of uint64 keys, 16-bit digits; tmp has room for n keys. */
static void gg_radix_sort(uint64_t *a, uint64_t *tmp, uint64_t n) {
    uint64_t *src = a, *dst = tmp;
    uint64_t *cnt = (uint64_t *)malloc(65536 * sizeof(uint64_t));
    for (int pass = 0; pass < 4; ++pass) {
        int shift = pass * 16;
        memset(cnt, 0, 65536 * sizeof(uint64_t));
        for (uint64_t i = 0; i < n; ++i) cnt[(src[i] >> shift) & 0xFFFF]++;
        uint64_t s = 0;
        for (int d = 0; d < 65536; ++d) { uint64_t c = cnt[d]; cnt[d] = s; s += c; }
        for (uint64_t i = 0; i < n; ++i) dst[cnt[(src[i] >> shift) & 0xFFFF]++] = src[i];
        uint64_t *t = src; src = dst; dst = t;
    }
    /* four passes: the sorted data is back in a */
    free(cnt);
}

static uint64_t gg_unique(uint64_t *a, uint64_t n) {
    if (n == 0) return 0;
    uint64_t w = 1;
    for (uint64_t i = 1; i < n; ++i)
        if (a[i] != a[w - 1]) a[w++] = a[i];
    return w;
}

/* Keep the m keys with the smallest priority mix(key ^ salt); result sorted by key. */
static uint64_t gg_keep_subset(uint64_t *keys, uint64_t *tmp, uint64_t have, uint64_t m, uint64_t salt) {
    if (have <= m) return have;
    /* pair (priority, key) sorted by priority: sort priorities, take the m-th as cut */
    for (uint64_t i = 0; i < have; ++i) tmp[i] = gg_mix(keys[i] ^ salt);
    uint64_t *t2 = (uint64_t *)malloc(have * sizeof(uint64_t));
    memcpy(t2, tmp, have * sizeof(uint64_t));
    gg_radix_sort(t2, tmp, have);
    uint64_t cut = t2[m - 1];
    free(t2);
    uint64_t w = 0;
    for (uint64_t i = 0; i < have && w < m; ++i)
        if (gg_mix(keys[i] ^ salt) <= cut) keys[w++] = keys[i];
    return w;
}

/* Draws `want` canonical pairs with draw indices [base, base+want) into out;
 * returns how many were not self-loops.  kind 0 = uniform (ER), 1 = R-MAT. */
static uint64_t gg_draw_pairs(int kind, uint64_t key, uint64_t base, uint64_t want, uint32_t n, int scale,
                              double a, double b, double c, const uint32_t *perm, uint64_t *out,
                              uint8_t *ok) {
    int64_t W = (int64_t)want;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < W; ++i) {
        uint64_t idx = base + (uint64_t)i;
        uint32_t u, v;
        if (kind == 0) {
            u = gg_below(gg_draw(key, 2 * idx), n);
            v = gg_below(gg_draw(key, 2 * idx + 1), n);
        } else {
            u = 0; v = 0;
            for (int l = 0; l < scale; ++l) {
                double x = gg_unit(gg_draw(key, idx * (uint64_t)scale + (uint64_t)l));
                uint32_t bu, bv;
                if (x < a) { bu = 0; bv = 0; }
                else if (x < a + b) { bu = 0; bv = 1; }
                else if (x < a + b + c) { bu = 1; bv = 0; }
                else { bu = 1; bv = 1; }
                u = (u << 1) | bu;
                v = (v << 1) | bv;
            }
            if (perm) { u = perm[u]; v = perm[v]; }
        }
        ok[i] = (u != v);
        out[i] = gg_canon(u, v);
    }
    uint64_t w = 0;
    for (uint64_t i = 0; i < want; ++i)
        if (ok[i]) out[w++] = out[i];
    return w;
}

static uint32_t *gg_permutation(uint32_t n, uint64_t key) {
    uint32_t *p = (uint32_t *)malloc((size_t)n * sizeof(uint32_t));
    for (uint32_t i = 0; i < n; ++i) p[i] = i;
    for (uint32_t i = n; i > 1; --i) {          /* Fisher-Yates */
        uint32_t j = gg_below(gg_draw(key, n - i), i);
        uint32_t t = p[i - 1]; p[i - 1] = p[j]; p[j] = t;
    }
    return p;
}

/* Shared driver for ER and R-MAT: draw until at least m distinct pairs exist,
 * then keep m of them.  keys_out receives exactly m sorted keys. */
static int64_t gg_pairs_until(int kind, uint32_t n, int scale, uint64_t m, double a, double b, double c,
                              uint64_t seed, int permute, uint64_t *keys_out, uint64_t cap) {
    if (n < 2 || m == 0) return 0;
    uint64_t maxpairs = (uint64_t)n * (n - 1) / 2;
    if (m > maxpairs || m > cap) return -1;
    uint64_t kdraw = gg_mix(seed ^ 0xD1B54A32D192ED03ULL);
    uint32_t *perm = (kind == 1 && permute) ? gg_permutation(n, gg_mix(seed ^ 0x8CB92BA72F3D8DD7ULL)) : NULL;
    uint64_t have = 0, drawn = 0;
    uint64_t *set = NULL, *buf = NULL, *tmp = NULL;
    uint8_t *ok = NULL;
    for (int it = 0; it < 64 && have < m; ++it) {
        uint64_t want = (m - have) + (m - have) / 4 + 1024;
        uint64_t tot_cap = have + want;
        buf = (uint64_t *)realloc(buf, tot_cap * sizeof(uint64_t));
        tmp = (uint64_t *)realloc(tmp, tot_cap * sizeof(uint64_t));
        ok = (uint8_t *)realloc(ok, want);
        if (have) memcpy(buf, set, have * sizeof(uint64_t));
        uint64_t got = gg_draw_pairs(kind, kdraw, drawn, want, n, scale, a, b, c, perm, buf + have, ok);
        drawn += want;
        uint64_t tot = have + got;
        gg_radix_sort(buf, tmp, tot);
        tot = gg_unique(buf, tot);
        uint64_t *t = set; set = buf; buf = t;      /* set now holds the distinct pairs */
        have = tot;
    }
    free(buf); free(ok); free(perm);
    int64_t ret = -2;
    if (have >= m) {
        tmp = (uint64_t *)realloc(tmp, have * sizeof(uint64_t));
        have = gg_keep_subset(set, tmp, have, m, gg_mix(seed ^ 0xA0761D6478BD642FULL));
        memcpy(keys_out, set, m * sizeof(uint64_t));
        ret = (int64_t)m;
    }
    free(set); free(tmp);
    return ret;
}

/* Erdos-Renyi G(n, M).  keys_out needs room for M keys (cap >= M). */
int64_t gg_er(uint32_t n, uint64_t M, uint64_t seed, uint64_t *keys_out, uint64_t cap) {
    return gg_pairs_until(0, n, 0, M, 0, 0, 0, seed, 0, keys_out, cap);
}

/* R-MAT on 2^scale vertices with m distinct undirected pairs. */
int64_t gg_rmat(uint32_t scale, uint64_t m, double a, double b, double c, uint64_t seed, int permute,
                uint64_t *keys_out, uint64_t cap) {
    if (scale < 1 || scale > 31) return -1;
    return gg_pairs_until(1, (uint32_t)1 << scale, (int)scale, m, a, b, c, seed, permute, keys_out, cap);
}

/* Chung-Lu power law.  Returns the number of distinct pairs written (<= n*d/2). */
int64_t gg_chunglu(uint32_t n, double avg_deg, double gamma, uint64_t seed, uint64_t *keys_out, uint64_t cap) {
    if (n < 2 || gamma <= 1.0 || avg_deg <= 0) return -1;
    uint64_t M = (uint64_t)((double)n * avg_deg / 2.0);
    if (M > cap) return -1;
    double *cdf = (double *)malloc((size_t)n * sizeof(double));
    double ex = -1.0 / (gamma - 1.0), sum = 0.0;
    for (uint32_t i = 0; i < n; ++i) { cdf[i] = pow((double)i + 1.0, ex); sum += cdf[i]; }
    double scalew = (double)n * avg_deg / sum, capw = sqrt((double)n * avg_deg), acc = 0.0;
    for (uint32_t i = 0; i < n; ++i) {
        double w = cdf[i] * scalew;
        if (w > capw) w = capw;
        acc += w;
        cdf[i] = acc;
    }
    uint32_t *perm = gg_permutation(n, gg_mix(seed ^ 0x8CB92BA72F3D8DD7ULL));
    uint64_t kdraw = gg_mix(seed ^ 0xD1B54A32D192ED03ULL);
    uint8_t *ok = (uint8_t *)malloc(M ? M : 1);
    int64_t MM = (int64_t)M;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < MM; ++i) {
        uint32_t ends[2];
        for (int e = 0; e < 2; ++e) {
            double x = gg_unit(gg_draw(kdraw, 2 * (uint64_t)i + (uint64_t)e)) * acc;
            uint32_t lo = 0, hi = n - 1;           /* first index with cdf > x */
            while (lo < hi) { uint32_t mid = lo + (hi - lo) / 2; if (cdf[mid] > x) hi = mid; else lo = mid + 1; }
            ends[e] = perm[lo];
        }
        ok[i] = ends[0] != ends[1];
        keys_out[i] = gg_canon(ends[0], ends[1]);
    }
    uint64_t w = 0;
    for (uint64_t i = 0; i < M; ++i)
        if (ok[i]) keys_out[w++] = keys_out[i];
    uint64_t *tmp = (uint64_t *)malloc((w ? w : 1) * sizeof(uint64_t));
    gg_radix_sort(keys_out, tmp, w);
    w = gg_unique(keys_out, w);
    free(tmp); free(ok); free(perm); free(cdf);
    return (int64_t)w;
}

/* Symmetric CSR from sorted unique canonical keys.  offsets has n+1 entries,
 * cols has 2m entries; each row comes out sorted ascending. */
int gg_csr_from_keys(uint32_t n, const uint64_t *keys, uint64_t m, uint64_t *offsets, uint32_t *cols) {
    memset(offsets, 0, ((size_t)n + 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < m; ++i) {
        uint32_t u = (uint32_t)(keys[i] >> 32), v = (uint32_t)keys[i];
        if (u >= n || v >= n || u == v) return -1;
        offsets[u + 1]++; offsets[v + 1]++;
    }
    for (uint32_t i = 0; i < n; ++i) offsets[i + 1] += offsets[i];
    uint64_t *pos = (uint64_t *)malloc(((size_t)n + 1) * sizeof(uint64_t));
    memcpy(pos, offsets, ((size_t)n + 1) * sizeof(uint64_t));
    /* Keys are sorted by (min, max).  Row r first receives its neighbours
     * smaller than r (keys (u, r), u ascending), then those larger than r
     * (keys (r, v), v ascending), so every row ends up sorted. */
    for (uint64_t i = 0; i < m; ++i) {           /* neighbours smaller than the row id */
        uint32_t u = (uint32_t)(keys[i] >> 32), v = (uint32_t)keys[i];
        cols[pos[v]++] = u;
    }
    for (uint64_t i = 0; i < m; ++i) {           /* neighbours larger than the row id */
        uint32_t u = (uint32_t)(keys[i] >> 32), v = (uint32_t)keys[i];
        cols[pos[u]++] = v;
    }
    free(pos);
    return 0;
}
