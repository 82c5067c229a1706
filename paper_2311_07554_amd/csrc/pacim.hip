// Host runtime and C-ABI of the MI355X influence-maximization library.
// Declarations, argument meaning and error behaviour: include/pacim.h.
//
// Device memory layout (all library-owned, one hipMalloc per array):
//   graph     offsets u64[n+1], cols u32[m_dir] (symmetric CSR, for GetCenter),
//             edges uint2[m_und] (u < v, for the sampling pass), and the union-find
//             passes' labelling order: newid u32[n], iperm u32[n], iedges uint2[m_und]
//   full      E uint2[n][R]: (CC label = one of its vertices, CC size if v is the
//             label else 0);
//             R consecutive entries per vertex so one evaluation reads 8R bytes
//             in one contiguous run, and the size lookup of a singleton CC is the
//             entry itself
//   compact   center_rank u32[n], centers u32[rho], label_c u32[rho][R], size_c u32[rho][R]
//             (center-major);
//             each sketch's largest component: gbits u64[n/64][R] membership bitmaps
//             (word-major), gsum u64[n] the sizes of those holding each vertex
//   selection key u64[n], in_s u8[n], gain0 u64[n], tree ids u32[~n/63],
//             frontier u32[~n/63], eval list u32[n], partial sums u64[n]
//   scratch   parent/cnt(/minc) u32[B][n] for B sketches per pass, freed after the build
#include "pacim.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "batch_kernels.h"
#include "compact_kernels.h"
#include "persist_kernels.h"
#include "probe_kernels.h"
#include "ptree_kernels.h"
#include "select_kernels.h"
#include "sketch_kernels.h"

using namespace pacim;

namespace {

struct KTimer {
    uint64_t launches = 0;
    double ms = 0.0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
};

}  // namespace

struct im_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t cap = 0;
    size_t used = 0;
    std::string err;
    bool profiling = false;
    std::map<std::string, KTimer> timers;
    std::vector<hipEvent_t> spare_events;
    std::mutex alloc_mu;  // device memory accounting (a server's thread allocates too)
    unsigned persist_grid = 0;  // workgroups of the persistent selection kernel (all resident)
    // Freed device blocks kept for reuse, by exact (rounded) size: hipMalloc / hipFree
    // of the build's arrays cost milliseconds per build, and hipFree synchronises the
    // device.  Callers free a block only once the work that used it has completed.
    std::multimap<size_t, void *> cache;
    size_t cached = 0;
    uint64_t clock_hz = 0;      // wall_clock64() rate
    // the batched path's instantiated graph and the signature of its launches
    void *batch_exec = nullptr;
    std::vector<uint64_t> batch_sig;
    uint64_t batch_captures = 0, batch_replays = 0;
};

struct im_graph {
    im_ctx *ctx = nullptr;
    uint32_t n = 0;
    uint64_t m_dir = 0, m_und = 0;
    uint64_t *off = nullptr;
    uint32_t *cols = nullptr;
    uint2 *edges = nullptr;
    // labelling order of the union-find passes: newid[v], its inverse iperm, and
    // the edge list's endpoints in it (iedges[e] for edges[e])
    uint32_t *newid = nullptr, *iperm = nullptr;
    uint2 *iedges = nullptr;
    uint32_t n_linked = 0;  // vertices with an edge: numbers [0, n_linked); isolated ones follow
    uint64_t *csr_thr = nullptr;  // WIC threshold per CSR entry; made by the first CompactSketch
                                  // build under WIC (GetCenter's scans read it with the column)
};

struct im_sketches {
    im_ctx *ctx = nullptr;
    const im_graph *g = nullptr;
    uint32_t n = 0, R = 0;
    uint64_t seed = 0;
    double alpha = 1.0;
    bool compact = false;
    ProbDev pm{};
    uint32_t kb = 1;
    uint32_t rho = 0;
    uint64_t kc = 0, Ta = 0;  // center test of CompactSketch: mix64(v ^ kc) < Ta
    unsigned long long *memo = nullptr;  // kept GetCenter results, [memo_mask + 1][R][2]
    unsigned long long *covmin = nullptr;  // [R][nw]: centerless components holding a seed, by smallest vertex
    uint32_t memo_mask = 0;
    uint32_t B = 1;
    // the device selection state as the last selection call left it (read once at
    // its end), so that counters need no device read; false while a call runs
    SelState st_host{};
    bool st_host_valid = true;
    // arrays
    uint64_t *K = nullptr;
    uint2 *E = nullptr;
    uint32_t *center_rank = nullptr, *centers = nullptr, *label_c = nullptr, *size_c = nullptr;
    uint32_t *size_c0 = nullptr;  // size_c as built (dump); only kept for small sketches
    uint64_t *gain0 = nullptr, *key = nullptr;
    uint64_t *gsum = nullptr;  // CompactSketch: per vertex, the sizes of the largest components holding it
    uint8_t *in_s = nullptr;
    TreeDesc td{};
    uint32_t *ids = nullptr, *fr = nullptr, *evl = nullptr;
    unsigned long long *partial = nullptr;
    SelState *st = nullptr;
    uint32_t *seeds_d = nullptr;
    unsigned long long *gains_d = nullptr;
    uint32_t *evals_d = nullptr;
    uint2 *ov = nullptr;
    uint32_t ov_cap = 0;
    uint32_t *slot_q = nullptr, *slot_vis = nullptr;
    uint32_t slots = 0;
    void *bulk_cs = nullptr;           // CCScratch of bulk rounds, allocated at the first one
    uint64_t last_gain = 0;            // gain of the latest seed (decides bulk rounds)
    uint32_t bulk_rounds = 0;
    PersistCtl *ctl = nullptr;         // step hand-off of the persistent selection kernel
    // CompactSketch: each sketch's largest component (bulk rounds without re-sampling)
    uint64_t *gbits = nullptr;         // [nw][R] membership bitmaps (word-major)
    uint32_t nw = 0;                   // 64-bit words per bitmap
    unsigned long long *gbest = nullptr;  // [R] (size << 32) | (2^32 - 1 - root) of the largest
    uint8_t *gcov = nullptr;           // [R] largest component covered by a seed
    uint32_t *bulk_abort = nullptr;
    uint32_t bulk_resampled = 0;
    bool tree_valid = true;            // the winning tree's internal nodes agree with key[]
    // NextSeed by prefix doubling (Algorithm 4): the queue's sorted runs X and Y
    // live in two of five n-key buffers (the other three are sort and merge space);
    // unread parts X[hx, nx), Y[hy, ny).
    uint64_t *pt_buf[5] = {};
    int pt_x = 0, pt_y = 1;
    uint32_t pt_hx = 0, pt_nx = 0, pt_hy = 0, pt_ny = 0;
    bool pt_valid = false;             // the runs hold the current key of every unselected vertex
    PtState *pt_state = nullptr;       // device
    PtState *pt_host = nullptr;        // pinned host copy read after each batch
    PtDev *pt_dev = nullptr;           // device rounds (full labels): runs and stop state, device
    PtDev *pt_dev_host = nullptr;      // its pinned host copy
    // bookkeeping
    std::vector<std::pair<void *, size_t>> allocs;
    uint32_t chosen = 0;
    double build_ms = 0.0, select_ms = 0.0;
    uint64_t bytes = 0;
};

// ---------------------------------------------------------------- helpers
namespace {

im_status fail(im_ctx *ctx, im_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return s;
}

#define HIP_TRY(ctx, call)                                                                 \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), IM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kCacheLimit = (size_t)48 << 30;  // device bytes the reuse cache may hold

size_t alloc_size(size_t bytes) { return ((bytes ? bytes : 8) + 4095) & ~(size_t)4095; }

void release_cache_locked(im_ctx *ctx) {
    for (auto &kv : ctx->cache) (void)hipFree(kv.second);
    ctx->cache.clear();
    ctx->cached = 0;
}

im_status dev_alloc(im_ctx *ctx, size_t bytes, void **p) {
    *p = nullptr;
    bytes = alloc_size(bytes);
    std::lock_guard<std::mutex> lk(ctx->alloc_mu);
    if (ctx->cap && ctx->used + bytes > ctx->cap)
        return fail(ctx, IM_ENOMEM, "allocation of " + std::to_string(bytes) + " bytes exceeds the context HBM cap");
    auto it = ctx->cache.find(bytes);
    // cached blocks count against the cap too: past it, they are given back first
    if (ctx->cap && it == ctx->cache.end() && ctx->used + ctx->cached + bytes > ctx->cap) release_cache_locked(ctx);
    if (it != ctx->cache.end()) {
        *p = it->second;
        ctx->cache.erase(it);
        ctx->cached -= bytes;
        ctx->used += bytes;
        return IM_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess && !ctx->cache.empty()) {
        (void)hipGetLastError();
        release_cache_locked(ctx);
        e = hipMalloc(p, bytes);
    }
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(ctx, IM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    ctx->used += bytes;
    return IM_OK;
}

void dev_free(im_ctx *ctx, void *p, size_t bytes) {
    if (!p) return;
    bytes = alloc_size(bytes);
    std::lock_guard<std::mutex> lk(ctx->alloc_mu);
    ctx->used -= std::min(ctx->used, bytes);
    if (ctx->cached + bytes <= kCacheLimit && (!ctx->cap || ctx->used + ctx->cached + bytes <= ctx->cap)) {
        ctx->cache.emplace(bytes, p);
        ctx->cached += bytes;
    } else {
        (void)hipFree(p);
    }
}

template <typename T>
im_status sk_alloc(im_sketches *s, size_t count, T **p) {
    void *q = nullptr;
    size_t bytes = count * sizeof(T);
    im_status st = dev_alloc(s->ctx, bytes, &q);
    if (st != IM_OK) return st;
    s->allocs.push_back({q, bytes ? bytes : 8});
    s->bytes += bytes;
    *p = static_cast<T *>(q);
    return IM_OK;
}

uint64_t threshold_of(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return kAllLive;
    return (uint64_t)std::ldexp(p, 64);
}

// The first problem with an edge-probability model, or null if it is valid.
const char *prob_problem(const im_prob &prob) {
    switch (prob.kind) {
    case IM_PROB_UNIFORM:
        return (prob.p >= 0.0 && prob.p <= 1.0) ? nullptr : "p must lie in [0, 1]";
    case IM_PROB_TRIVALENCY:
    case IM_PROB_WIC:
        return nullptr;
    case IM_PROB_RANGE:
        return (prob.p >= 0.0 && prob.p <= prob.p_hi && prob.p_hi < 1.0) ? nullptr
                                                                          : "range model needs 0 <= p <= p_hi < 1";
    case IM_PROB_PER_EDGE:
        return prob.p_edge ? nullptr : "per-edge model needs p_edge";
    default:
        return "unknown probability model";
    }
}

// Device form of a (valid) model on graph offsets `off` (read by WIC only).  The
// per-edge model's threshold arrays are set by the caller.
ProbDev prob_dev(const im_prob &prob, const uint64_t *off) {
    ProbDev pm{};
    pm.kind = prob.kind;
    switch (prob.kind) {
    case IM_PROB_UNIFORM:
        pm.t0 = threshold_of(prob.p);
        break;
    case IM_PROB_TRIVALENCY:
        pm.t0 = threshold_of(0.1);
        pm.t1 = threshold_of(0.01);
        pm.t2 = threshold_of(0.001);
        pm.ktriv = sketch_key(0, kSaltTriv);
        break;
    case IM_PROB_RANGE:
        pm.t0 = threshold_of(prob.p);
        pm.t1 = threshold_of(prob.p_hi) - pm.t0;
        pm.ktriv = sketch_key(0, kSaltRange);
        break;
    case IM_PROB_WIC:
        pm.off = off;
        break;
    default:
        break;
    }
    return pm;
}

uint32_t bit_length(uint64_t x) {
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

hipEvent_t take_event(im_ctx *ctx) {
    if (!ctx->spare_events.empty()) {
        hipEvent_t e = ctx->spare_events.back();
        ctx->spare_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets a launch with HIP events on the context stream when profiling is on.
struct Prof {
    im_ctx *ctx;
    const char *name;
    hipEvent_t a = nullptr;
    Prof(im_ctx *c, const char *nm, hipStream_t on = nullptr, bool enabled = true) : ctx(c), name(nm) {
        if (enabled && ctx->profiling && (!on || on == ctx->stream)) {
            a = take_event(ctx);
            if (a) (void)hipEventRecord(a, ctx->stream);
        }
    }
    ~Prof() {
        if (a) {
            hipEvent_t b = take_event(ctx);
            if (b) {
                (void)hipEventRecord(b, ctx->stream);
                ctx->timers[name].pending.push_back({a, b});
            }
        }
    }
};

void drain_timers(im_ctx *ctx) {
    for (auto &kv : ctx->timers) {
        KTimer &t = kv.second;
        for (auto &pr : t.pending) {
            (void)hipEventSynchronize(pr.second);
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) t.ms += ms;
            ++t.launches;
            ctx->spare_events.push_back(pr.first);
            ctx->spare_events.push_back(pr.second);
        }
        t.pending.clear();
    }
}

unsigned grid_for(uint64_t items, unsigned block, unsigned cap) {
    uint64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

unsigned wave_grid(uint64_t waves, unsigned cap_waves) {
    uint64_t w = std::min<uint64_t>(std::max<uint64_t>(waves, 1), cap_waves);
    return (unsigned)((w + 3) / 4);  // 4 waves per 256-thread block
}

// LSD radix sort of uint64 keys (4 x 16-bit digits).
void radix_sort_u64(std::vector<uint64_t> &a) {
    std::vector<uint64_t> tmp(a.size());
    std::vector<size_t> cnt(65536);
    for (int pass = 0; pass < 4; ++pass) {
        const int sh = pass * 16;
        std::fill(cnt.begin(), cnt.end(), 0);
        for (uint64_t x : a) cnt[(x >> sh) & 0xFFFF]++;
        size_t s = 0;
        for (auto &c : cnt) { size_t t = c; c = s; s += t; }
        for (uint64_t x : a) tmp[cnt[(x >> sh) & 0xFFFF]++] = x;
        a.swap(tmp);
    }
}

// Labelling order of the union-find passes.  A component's labels do not depend
// on how its vertices are numbered inside a pass, so the passes number them for
// locality: the `hubs` vertices of largest degree first (ties by smaller id),
// then the other vertices with an edge, then the isolated ones, each class in id
// order.  Most unions touch a hub (in an R-MAT graph of 2^20 vertices the 4,096
// largest degrees hold a third of the edge ends), and with the hubs' parents
// packed into a few lines per sketch the sampling pass at that size runs 20%
// faster.  2,048 to 8,192 hubs measured alike; 16,384 and more, or every vertex
// sorted by degree, slower; isolated vertices last alone gains a third as much.
// Within a class the order stays monotone, so per-vertex passes that translate
// v -> newid[v] read their forests in a few sequential runs.  PACIM_HUBS
// (tuning) overrides the count.
uint32_t labelling_order(uint32_t n, const std::vector<uint64_t> &off, std::vector<uint32_t> &newid,
                         std::vector<uint32_t> &iperm) {
    uint32_t hubs = 4096;
    if (const char *e = getenv("PACIM_HUBS")) hubs = (uint32_t)std::min<unsigned long>(strtoul(e, nullptr, 10), n);
    std::vector<uint8_t> cls(n);
    std::vector<uint32_t> linked;
    for (uint32_t v = 0; v < n; ++v) {
        cls[v] = off[v + 1] > off[v] ? 1 : 2;
        if (cls[v] == 1) linked.push_back(v);
    }
    auto larger = [&](uint32_t a, uint32_t b) {
        const uint64_t da = off[a + 1] - off[a], db = off[b + 1] - off[b];
        return da != db ? da > db : a < b;
    };
    if (linked.size() > hubs) std::nth_element(linked.begin(), linked.begin() + hubs, linked.end(), larger);
    for (size_t i = 0; i < std::min<size_t>(hubs, linked.size()); ++i) cls[linked[i]] = 0;
    uint32_t next[3] = {0, 0, 0};
    for (uint32_t v = 0; v < n; ++v) ++next[cls[v]];
    next[2] = next[0] + next[1];
    next[1] = next[0];
    next[0] = 0;
    newid.resize(n);
    iperm.resize(n);
    for (uint32_t v = 0; v < n; ++v) {
        newid[v] = next[cls[v]]++;
        iperm[newid[v]] = v;
    }
    return next[1];  // the vertices with an edge
}

}  // namespace

namespace {
hipError_t static_scratch_on(int device, void **ptr);
}  // namespace

// ---------------------------------------------------------------- context
extern "C" im_status im_ctx_create(int device, void *hip_stream, size_t hbm_cap, im_ctx **out) {
    if (!out) return IM_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return IM_EDEVICE;
    if (device < 0 || device >= ndev) return IM_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return IM_EDEVICE;
    im_ctx *ctx = new (std::nothrow) im_ctx();
    if (!ctx) return IM_ENOMEM;
    ctx->device = device;
    ctx->cap = hbm_cap;
    {
        // device address of the static scratch of im_influence_noalloc, resolved once
        // per device here with the device current (a failure is kept and reported by
        // that call)
        void *sp = nullptr;
        (void)static_scratch_on(device, &sp);
    }
    if (hip_stream) {
        ctx->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return IM_EDEVICE;
        }
        ctx->own_stream = true;
    }
    *out = ctx;
    return IM_OK;
}

extern "C" im_status im_ctx_destroy(im_ctx *ctx) {
    if (!ctx) return IM_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    drain_timers(ctx);
    {
        std::lock_guard<std::mutex> lk(ctx->alloc_mu);
        release_cache_locked(ctx);
    }
    for (hipEvent_t e : ctx->spare_events) (void)hipEventDestroy(e);
    if (ctx->batch_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(ctx->batch_exec));
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return IM_OK;
}

extern "C" const char *im_last_error(const im_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

extern "C" im_status im_ctx_memory(const im_ctx *ctx, size_t *used, size_t *cap) {
    if (!ctx) return IM_EINVAL;
    if (used) *used = ctx->used;
    if (cap) *cap = ctx->cap;
    return IM_OK;
}

extern "C" im_status im_ctx_set_profiling(im_ctx *ctx, int on) {
    if (!ctx) return IM_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    drain_timers(ctx);
    if (on && !ctx->profiling) ctx->timers.clear();
    ctx->profiling = on != 0;
    return IM_OK;
}

extern "C" im_status im_kernel_time(im_ctx *ctx, const char *name, uint64_t *launches, double *ms) {
    if (!ctx || !name) return IM_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    drain_timers(ctx);
    if (!strcmp(name, "batch_capture") || !strcmp(name, "batch_replay")) {
        if (launches) *launches = name[6] == 'c' ? ctx->batch_captures : ctx->batch_replays;
        if (ms) *ms = 0.0;
        return IM_OK;
    }
    auto it = ctx->timers.find(name);
    if (launches) *launches = it == ctx->timers.end() ? 0 : it->second.launches;
    if (ms) *ms = it == ctx->timers.end() ? 0.0 : it->second.ms;
    return IM_OK;
}

// ---------------------------------------------------------------- graph
extern "C" im_status im_graph_upload(im_ctx *ctx, uint32_t n, uint64_t m_dir, const uint64_t *offsets,
                                     const uint32_t *cols, int device_ptrs, im_graph **out) {
    if (!ctx || !out) return IM_EINVAL;
    *out = nullptr;
    if (n == 0) return fail(ctx, IM_EINVAL, "n must be positive");
    if (!offsets || (m_dir && !cols)) return fail(ctx, IM_EINVAL, "null CSR array");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<uint64_t> off;
    std::vector<uint32_t> col;
    if (device_ptrs) {
        off.resize((size_t)n + 1);
        col.resize(m_dir);
        // read on the context's stream, after the caller's work that wrote the arrays
        HIP_TRY(ctx, hipMemcpyAsync(off.data(), offsets, off.size() * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                    ctx->stream));
        if (m_dir)
            HIP_TRY(ctx, hipMemcpyAsync(col.data(), cols, m_dir * sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        off.assign(offsets, offsets + (size_t)n + 1);
        col.assign(cols, cols + m_dir);
    }
    if (off[0] != 0 || off[n] != m_dir) return fail(ctx, IM_EINVAL, "offsets[0] must be 0 and offsets[n] = m_dir");
    std::vector<uint32_t> mark(n, kNone);
    std::vector<uint64_t> lo, hi;
    lo.reserve(m_dir / 2);
    hi.reserve(m_dir / 2);
    for (uint32_t u = 0; u < n; ++u) {
        if (off[u + 1] < off[u]) return fail(ctx, IM_EINVAL, "offsets are not monotone");
        for (uint64_t j = off[u]; j < off[u + 1]; ++j) {
            const uint32_t w = col[j];
            if (w >= n) return fail(ctx, IM_EINVAL, "column id out of range");
            if (w == u) return fail(ctx, IM_EINVAL, "self-loop at vertex " + std::to_string(u));
            if (mark[w] == u) return fail(ctx, IM_EINVAL, "duplicate edge in row " + std::to_string(u));
            mark[w] = u;
            if (u < w) lo.push_back(((uint64_t)u << 32) | w);
            else hi.push_back(((uint64_t)w << 32) | u);
        }
    }
    if (lo.size() != hi.size()) return fail(ctx, IM_EINVAL, "CSR is not symmetric");
    radix_sort_u64(lo);
    radix_sort_u64(hi);
    if (lo != hi) return fail(ctx, IM_EINVAL, "CSR is not symmetric");
    hi.clear();
    hi.shrink_to_fit();
    const uint64_t m_und = lo.size();
    std::vector<uint2> edges(m_und);
    for (uint64_t i = 0; i < m_und; ++i) edges[i] = make_uint2((uint32_t)(lo[i] >> 32), (uint32_t)lo[i]);
    lo.clear();
    lo.shrink_to_fit();
    std::vector<uint32_t> newid, iperm;
    const uint32_t n_linked = labelling_order(n, off, newid, iperm);
    std::vector<uint2> iedges(m_und);
    for (uint64_t i = 0; i < m_und; ++i) iedges[i] = make_uint2(newid[edges[i].x], newid[edges[i].y]);

    im_graph *g = new (std::nothrow) im_graph();
    if (!g) return fail(ctx, IM_ENOMEM, "host allocation");
    g->ctx = ctx;
    g->n = n;
    g->m_dir = m_dir;
    g->m_und = m_und;
    g->n_linked = n_linked;
    im_status s;
    if ((s = dev_alloc(ctx, ((size_t)n + 1) * 8, (void **)&g->off)) != IM_OK ||
        (s = dev_alloc(ctx, m_dir * 4, (void **)&g->cols)) != IM_OK ||
        (s = dev_alloc(ctx, m_und * 8, (void **)&g->edges)) != IM_OK ||
        (s = dev_alloc(ctx, m_und * 8, (void **)&g->iedges)) != IM_OK ||
        (s = dev_alloc(ctx, (size_t)n * 4, (void **)&g->newid)) != IM_OK ||
        (s = dev_alloc(ctx, (size_t)n * 4, (void **)&g->iperm)) != IM_OK) {
        im_graph_free(g);
        return s;
    }
    hipError_t e1 = hipMemcpy(g->off, off.data(), ((size_t)n + 1) * 8, hipMemcpyHostToDevice);
    hipError_t e2 = m_dir ? hipMemcpy(g->cols, col.data(), m_dir * 4, hipMemcpyHostToDevice) : hipSuccess;
    hipError_t e3 = m_und ? hipMemcpy(g->edges, edges.data(), m_und * 8, hipMemcpyHostToDevice) : hipSuccess;
    if (e3 == hipSuccess && m_und) e3 = hipMemcpy(g->iedges, iedges.data(), m_und * 8, hipMemcpyHostToDevice);
    if (e3 == hipSuccess) e3 = hipMemcpy(g->newid, newid.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    if (e3 == hipSuccess) e3 = hipMemcpy(g->iperm, iperm.data(), (size_t)n * 4, hipMemcpyHostToDevice);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        im_graph_free(g);
        return fail(ctx, IM_EDEVICE, "graph upload copy failed");
    }
    *out = g;
    return IM_OK;
}

extern "C" im_status im_graph_free(im_graph *g) {
    if (!g) return IM_EINVAL;
    im_ctx *ctx = g->ctx;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    dev_free(ctx, g->off, ((size_t)g->n + 1) * 8);
    dev_free(ctx, g->cols, g->m_dir * 4);
    dev_free(ctx, g->edges, g->m_und * 8);
    dev_free(ctx, g->iedges, g->m_und * 8);
    dev_free(ctx, g->newid, (size_t)g->n * 4);
    dev_free(ctx, g->iperm, (size_t)g->n * 4);
    if (g->csr_thr) dev_free(ctx, g->csr_thr, g->m_dir * 8);
    delete g;
    return IM_OK;
}

// ---------------------------------------------------------------- sketches
namespace {

// Labelling scratch of one build: PACIM_SCRATCH_MB, else a quarter of the free
// device memory up to 16 GiB (64 sketches of a 2^24-vertex graph take 12.9 GB).
size_t g_scratch_budget() {
    const char *e = getenv("PACIM_SCRATCH_MB");
    if (e) return std::max<size_t>((size_t)strtoull(e, nullptr, 10), 1) << 20;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = (size_t)4 << 30;
    return std::max<size_t>(std::min<size_t>((size_t)16 << 30, free_b / 4), (size_t)256 << 20);
}

uint32_t g_batch_override() {
    const char *e = getenv("PACIM_SKETCHES_PER_PASS");
    return e ? (uint32_t)strtoul(e, nullptr, 10) : 0;
}

TreeDesc make_tree(uint32_t n) {
    TreeDesc td{};
    std::vector<uint32_t> sizes;  // internal levels from the deepest up
    uint64_t cur = n;
    do {
        cur = (cur + kFan - 1) / kFan;
        sizes.push_back((uint32_t)cur);
    } while (cur > 1);
    td.D = (uint32_t)sizes.size();
    uint64_t off = 0;
    for (uint32_t l = 0; l < td.D; ++l) {
        td.lvl_n[l] = sizes[td.D - 1 - l];
        td.lvl_off[l] = off;
        off += td.lvl_n[l];
    }
    td.lvl_n[td.D] = n;
    return td;
}

uint64_t tree_nodes(const TreeDesc &td) {
    uint64_t t = 0;
    for (uint32_t l = 0; l < td.D; ++l) t += td.lvl_n[l];
    return t;
}

uint32_t key_slots(uint32_t R) { return ((R + 7u) & ~7u) + 8u; }

// Scratch of the component-labelling passes: parent/cnt(/minc) for B sketches.
struct CCScratch {
    uint32_t B = 0;
    uint32_t *parent = nullptr, *cnt = nullptr, *minc = nullptr;
    uint32_t *crank = nullptr;  // with minc: center ranks in labelling order
    void *block = nullptr;
    size_t bytes = 0;
};

im_status cc_scratch_alloc(im_ctx *ctx, const im_graph *g, uint32_t R, bool with_minc, CCScratch *cs) {
    const uint32_t n = g->n;
    const size_t per_sketch = sketch_stride(n) * 4 * (with_minc ? 3 : 2);
    size_t budget = g_scratch_budget();
    if (ctx->cap) {
        // under a cap, leave room for the selection state a build allocates next
        // (about 48 bytes per vertex, the GetCenter queues and overflow list)
        const size_t avail = ctx->cap > ctx->used ? ctx->cap - ctx->used : 0;
        const size_t reserve = (size_t)n * 48 + ((size_t)320 << 20);
        budget = std::min(budget, avail > reserve ? avail - reserve : 0);
    }
    uint32_t B = (uint32_t)std::min<size_t>({(size_t)R, (size_t)64, std::max<size_t>(1, budget / per_sketch)});
    if (uint32_t ov = g_batch_override()) B = std::min<uint32_t>({ov, R, 64u});
    cs->B = B;
    cs->bytes = per_sketch * B + (with_minc ? sketch_stride(n) * 4 : 0);
    im_status st = dev_alloc(ctx, cs->bytes, &cs->block);
    if (st != IM_OK) return st;
    cs->parent = static_cast<uint32_t *>(cs->block);
    cs->cnt = cs->parent + (size_t)B * sketch_stride(n);
    cs->minc = with_minc ? cs->cnt + (size_t)B * sketch_stride(n) : nullptr;
    cs->crank = with_minc ? cs->minc + (size_t)B * sketch_stride(n) : nullptr;
    return IM_OK;
}

void cc_scratch_free(im_ctx *ctx, CCScratch *cs) {
    if (cs->block) dev_free(ctx, cs->block, cs->bytes);
    *cs = CCScratch();
}

// Thresholds of the per-edge model: csr[j] = T(p_edge[j]) for every CSR entry,
// edge[e] for the undirected edges in edge-list order (ascending (u, v), u < v).
// Rejects probabilities outside [0, 1] and edges whose two entries differ.
im_status per_edge_thresholds(im_ctx *ctx, const im_graph *g, const double *p_edge, std::vector<uint64_t> &csr,
                              std::vector<uint64_t> &edge) {
    const uint32_t n = g->n;
    const uint64_t md = g->m_dir;
    std::vector<uint64_t> off((size_t)n + 1);
    std::vector<uint32_t> col(md);
    HIP_TRY(ctx, hipMemcpy(off.data(), g->off, off.size() * 8, hipMemcpyDeviceToHost));
    if (md) HIP_TRY(ctx, hipMemcpy(col.data(), g->cols, md * 4, hipMemcpyDeviceToHost));
    csr.resize(md);
    for (uint64_t j = 0; j < md; ++j) {
        const double p = p_edge[j];
        if (!(p >= 0.0 && p <= 1.0)) return fail(ctx, IM_EINVAL, "per-edge probability outside [0, 1]");
        csr[j] = threshold_of(p);
    }
    // each row's entries in increasing column order (positions within the row)
    std::vector<uint32_t> ord(md);
    for (uint32_t u = 0; u < n; ++u) {
        const uint64_t o0 = off[u], d = off[u + 1] - off[u];
        for (uint64_t k = 0; k < d; ++k) ord[o0 + k] = (uint32_t)k;
        std::sort(ord.begin() + (ptrdiff_t)o0, ord.begin() + (ptrdiff_t)(o0 + d),
                  [&](uint32_t a, uint32_t b) { return col[o0 + a] < col[o0 + b]; });
    }
    edge.resize(g->m_und);
    uint64_t e = 0;
    for (uint32_t u = 0; u < n; ++u) {
        for (uint64_t k = off[u]; k < off[u + 1]; ++k) {
            const uint64_t j = off[u] + ord[k];
            const uint32_t w = col[j];
            if (w > u) {
                if (e >= edge.size()) return fail(ctx, IM_EINTERNAL, "edge count mismatch");
                edge[e++] = csr[j];
                continue;
            }
            // the entry (w, u) of the same edge, by binary search in row w
            uint64_t lo = off[w], hi = off[w + 1];
            while (lo < hi) {
                const uint64_t mid = (lo + hi) / 2;
                if (col[off[w] + ord[mid]] < u) lo = mid + 1;
                else hi = mid;
            }
            if (lo == off[w + 1] || col[off[w] + ord[lo]] != u || csr[off[w] + ord[lo]] != csr[j])
                return fail(ctx, IM_EINVAL, "per-edge probabilities differ between the two directions of an edge");
        }
    }
    if (e != g->m_und) return fail(ctx, IM_EINTERNAL, "edge count mismatch");
    return IM_OK;
}

// Workgroups of a sampling pass at most; each thread strides over the edges
// beyond that.  One edge per thread up to 2^30 edges: short-lived workgroups
// balance the uneven union work and free compute units often, so that kernels
// of another stream (a selection running beside the build) get them soon.  A
// persistent-style grid of 8,192 workgroups made the pass 7% slower at 2^24
// edges.  PACIM_HOOK_GRID_CAP (tuning) overrides.
unsigned hook_grid_cap() {
    const char *e = getenv("PACIM_HOOK_GRID_CAP");
    const unsigned long v = e ? strtoul(e, nullptr, 10) : 0ul;
    return v ? (unsigned)std::min<unsigned long>(v, 1ul << 24) : (1u << 22);
}

// One pass over the edge list for b <= cs.B sketches (keys K[0..b)): union-find
// forests in parent[n][cs.B] over the graph's labelling order (x = newid[v]; the
// root of a CC is its smallest number), member counts at the roots in cnt, and
// (if center_rank, given in labelling order) the smallest center rank of each CC
// in minc.  parent_fresh: the linked numbers' entries already hold their own
// numbers (the previous pass's emit reset them; with init_isolated false).
void enqueue_cc_pass(im_ctx *ctx, const im_graph *g, const ProbDev &pm, const uint64_t *K, uint32_t b,
                     const CCScratch &cs, uint32_t *minc, uint32_t minc_init, const uint32_t *center_rank,
                     bool init_isolated = true, hipStream_t st = nullptr, bool timed = true,
                     bool parent_fresh = false) {
    if (!st) st = ctx->stream;
    const uint32_t n = g->n;
    const unsigned hook_grid = grid_for(g->m_und, kHookBlock, hook_grid_cap());
    // isolated numbers' entries are set only for callers that read them (the
    // influence passes read the seeds'); nothing else writes them, so they keep
    // their values from an earlier pass of the same build unless a caller flags
    // seeds in minc
    const uint32_t n_init = init_isolated ? n : g->n_linked;
    {
        Prof p(ctx, "init", st, timed);
        uint32_t *const par = parent_fresh ? nullptr : cs.parent;
        const uintptr_t bases = reinterpret_cast<uintptr_t>(cs.parent) | reinterpret_cast<uintptr_t>(cs.cnt) |
                                reinterpret_cast<uintptr_t>(minc);
        if (cs.B % 4u == 0u && bases % 16u == 0u) {  // 16-byte stores: rows of whole 16-byte pieces
            k_batch_init4<<<grid_for((uint64_t)n_init * (cs.B / 4u), 256, 1u << 20), 256, 0, st>>>(
                par, cs.cnt, minc, cs.B, n_init, minc_init, center_rank);
        } else {
            uint32_t lw = 0;  // threads per number: the width rounded up to a power of two
            while ((1u << lw) < cs.B) ++lw;
            k_batch_init<<<grid_for((uint64_t)n_init << lw, 256, 1u << 20), 256, 0, st>>>(
                par, cs.cnt, minc, cs.B, lw, n_init, minc_init, center_rank);
        }
    }
    {
        Prof p(ctx, "sample_hook", st, timed);
        switch (pm.kind) {
        case kProbConstant:
            k_sample_hook<kProbConstant><<<hook_grid, kHookBlock, 0, st>>>(g->edges, g->iedges, g->m_und, K, b, pm, cs.parent, cs.B);
            break;
        case kProbTrivalency:
            k_sample_hook<kProbTrivalency><<<hook_grid, kHookBlock, 0, st>>>(g->edges, g->iedges, g->m_und, K, b, pm, cs.parent,
                                                                             cs.B);
            break;
        case kProbRange:
            k_sample_hook<kProbRange><<<hook_grid, kHookBlock, 0, st>>>(g->edges, g->iedges, g->m_und, K, b, pm, cs.parent, cs.B);
            break;
        case kProbWic:
            k_sample_hook<kProbWic><<<hook_grid, kHookBlock, 0, st>>>(g->edges, g->iedges, g->m_und, K, b, pm, cs.parent, cs.B);
            break;
        default:
            k_sample_hook<kProbPerEdge><<<hook_grid, kHookBlock, 0, st>>>(g->edges, g->iedges, g->m_und, K, b, pm, cs.parent,
                                                                          cs.B);
            break;
        }
    }
    {
        Prof p(ctx, "compress", st, timed);
        // about 16,384 runs (one wave each), fewer and longer ones keeping the
        // per-wave hot roots of a giant component few; at most 128 numbers a run
        // (R-MAT 2^24: 1.47 ms per pass at 512, 1.33 ms at 128; 2^20 takes runs of 40,
        // and 4x as many runs there doubled the time)
        const uint64_t want = ((uint64_t)g->n_linked / 16384 + kCompressIlp - 1) / kCompressIlp * kCompressIlp;
        const uint32_t run = (uint32_t)std::min<uint64_t>(kCompressRunMax, std::max<uint64_t>(kCompressIlp, want));
        const uint64_t runs = ((uint64_t)g->n_linked + run - 1) / run;  // one wave each
        const uint64_t wpb = kCompressBlock / kWave;
        k_compress<<<std::max<uint64_t>((runs + wpb - 1) / wpb, 1), kCompressBlock, 0, st>>>(
            cs.parent, cs.cnt, cs.B, b, g->n_linked, run, center_rank, minc);
    }
}

// Full-label sketches of R sketches with keys K (key_slots(R) entries already on
// the device): E[n][R] and the initial gains, B sketches per pass.
void enqueue_full_build(im_ctx *ctx, const im_graph *g, const ProbDev &pm, const uint64_t *K, uint32_t R,
                        const CCScratch &cs, uint2 *E, uint64_t *gain0, hipStream_t st) {
    const uint32_t n = g->n;
    (void)hipMemsetAsync(gain0, 0, (size_t)n * 8, st);
    for (uint32_t r0 = 0; r0 < R; r0 += cs.B) {
        const uint32_t b = std::min(cs.B, R - r0);
        const bool last = r0 + cs.B >= R;
        // the emit skips isolated numbers, and resets the forest for the next pass
        enqueue_cc_pass(ctx, g, pm, K + r0, b, cs, nullptr, kNone, nullptr, false, st, true, r0 > 0);
        Prof p(ctx, "emit", st);
        k_emit_full<<<((n + kWave - 1) / kWave + 3) / 4, 256, 0, st>>>(cs.parent, cs.cnt, g->newid, g->iperm, n, cs.B,
                                                                     g->n_linked, b, R, r0, E, gain0, !last);
    }
}

void free_sketches(im_sketches *s) {
    if (s->pt_host) {
        (void)hipHostFree(s->pt_host);
        s->pt_host = nullptr;
    }
    if (s->pt_dev_host) {
        (void)hipHostFree(s->pt_dev_host);
        s->pt_dev_host = nullptr;
    }
    if (s->bulk_cs) {
        cc_scratch_free(s->ctx, static_cast<CCScratch *>(s->bulk_cs));
        delete static_cast<CCScratch *>(s->bulk_cs);
        s->bulk_cs = nullptr;
    }
    for (auto &pr : s->allocs) dev_free(s->ctx, pr.first, pr.second);
    s->allocs.clear();
}

}  // namespace

extern "C" im_status im_sketches_free(im_sketches *s) {
    if (!s) return IM_EINVAL;
    (void)hipSetDevice(s->ctx->device);
    (void)hipStreamSynchronize(s->ctx->stream);
    free_sketches(s);
    delete s;
    return IM_OK;
}

extern "C" im_status im_build_sketches(im_ctx *ctx, const im_graph *g, im_prob prob, uint32_t R, uint64_t seed,
                                       double alpha, im_sketches **out) {
    if (!ctx || !g || !out) return IM_EINVAL;
    *out = nullptr;
    if (R == 0) return fail(ctx, IM_EINVAL, "R must be >= 1");
    if (!(alpha > 0.0) || alpha > 1.0) return fail(ctx, IM_EINVAL, "alpha must lie in (0, 1]");
    if (const char *why = prob_problem(prob)) return fail(ctx, IM_EINVAL, why);
    const uint32_t n = g->n;
    const uint32_t kb = std::max<uint32_t>(1, bit_length((uint64_t)n - 1));
    if (kb + bit_length((uint64_t)R * n + 1) > 64) return fail(ctx, IM_EINVAL, "R*n too large for 64-bit keys");
    if (alpha < 1.0 && ((uint64_t)R * n >= (1ull << kPartialShift) || R >= (1u << (64 - kPartialShift))))
        return fail(ctx, IM_EINVAL, "CompactSketch needs R*n < 2^40 and R < 2^24");
    HIP_TRY(ctx, hipSetDevice(ctx->device));

    im_sketches *s = new (std::nothrow) im_sketches();
    if (!s) return fail(ctx, IM_ENOMEM, "host allocation");
    s->ctx = ctx;
    s->g = g;
    s->n = n;
    s->R = R;
    s->seed = seed;
    s->alpha = alpha;
    s->compact = alpha < 1.0;
    s->kb = kb;
    s->pm = prob_dev(prob, g->off);
    s->kc = sketch_key(seed, kSaltCenter);
    if (prob.kind == IM_PROB_WIC && alpha < 1.0 && g->m_dir && !g->csr_thr && g->ctx != ctx) {
        // a graph of another context (a server's CompactSketch lane): the thresholds
        // live with these sketches instead of being kept on the graph
        uint64_t *thr = nullptr;
        const im_status a = sk_alloc(s, g->m_dir, &thr);
        if (a != IM_OK) {
            free_sketches(s);
            delete s;
            return a;
        }
        k_csr_wic_thr<<<wave_grid(g->n, 1u << 18), 256, 0, ctx->stream>>>(g->off, g->cols, g->n, thr);
        s->pm.csr_thr = thr;
    } else if (prob.kind == IM_PROB_WIC && alpha < 1.0 && g->m_dir) {
        if (!g->csr_thr) {
            im_graph *gm = const_cast<im_graph *>(g);
            uint64_t *thr = nullptr;
            const im_status a = dev_alloc(ctx, g->m_dir * 8, (void **)&thr);
            if (a != IM_OK) {
                delete s;
                return a;
            }
            k_csr_wic_thr<<<wave_grid(g->n, 1u << 18), 256, 0, ctx->stream>>>(g->off, g->cols, g->n, thr);
            gm->csr_thr = thr;
        }
        s->pm.csr_thr = g->csr_thr;
    }
    hipStream_t st = ctx->stream;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        delete s;
        return fail(ctx, IM_EDEVICE, "hipEventCreate failed");
    }
    CCScratch cs;
    auto bail = [&](im_status code) {
        cc_scratch_free(ctx, &cs);
        (void)hipEventDestroy(t0);
        (void)hipEventDestroy(t1);
        free_sketches(s);
        delete s;
        return code;
    };
#define SK_TRY(expr)                      \
    do {                                  \
        im_status e_ = (expr);            \
        if (e_ != IM_OK) return bail(e_); \
    } while (0)
#define SK_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            fail(ctx, IM_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));          \
            return bail(IM_EDEVICE);                                                           \
        }                                                                                      \
    } while (0)

    SK_HIP(hipEventRecord(t0, st));
    // keys of sketches 0 .. Rpad-1 (the sampling kernel reads them 8 at a time)
    const uint32_t Rpad = key_slots(R);
    SK_TRY(sk_alloc(s, (size_t)Rpad, &s->K));
    k_sketch_keys<<<grid_for(Rpad, 256, 1u << 20), 256, 0, st>>>(seed, Rpad, s->K);
    SK_HIP(hipGetLastError());
    if (prob.kind == IM_PROB_PER_EDGE) {
        // thresholds by edge (the sampling pass) and by CSR entry (GetCenter), held with the sketches
        std::vector<uint64_t> tc, te;
        SK_TRY(per_edge_thresholds(ctx, g, prob.p_edge, tc, te));
        uint64_t *dc = nullptr, *de = nullptr;
        SK_TRY(sk_alloc(s, std::max<size_t>(tc.size(), 1), &dc));
        SK_TRY(sk_alloc(s, std::max<size_t>(te.size(), 1), &de));
        if (!tc.empty()) SK_HIP(hipMemcpy(dc, tc.data(), tc.size() * 8, hipMemcpyHostToDevice));
        if (!te.empty()) SK_HIP(hipMemcpy(de, te.data(), te.size() * 8, hipMemcpyHostToDevice));
        s->pm.csr_thr = dc;
        s->pm.edge_thr = de;
    }

    // centers (CompactSketch)
    if (s->compact) {
        const uint32_t nch = (n + kCenterChunk - 1) / kCenterChunk;
        uint32_t *chunk = nullptr, *rho_d = nullptr;
        SK_TRY(sk_alloc(s, nch, &chunk));
        SK_TRY(sk_alloc(s, 1, &rho_d));
        SK_TRY(sk_alloc(s, n, &s->center_rank));
        const uint64_t Ta = threshold_of(alpha);
        s->Ta = Ta;
        k_center_count<<<nch, 256, 0, st>>>(n, seed, Ta, chunk);
        k_center_scan<<<1, 1024, 0, st>>>(nch, chunk, rho_d);
        uint32_t rho = 0;
        SK_HIP(hipMemcpyAsync(&rho, rho_d, 4, hipMemcpyDeviceToHost, st));
        SK_HIP(hipStreamSynchronize(st));
        s->rho = rho;
        SK_TRY(sk_alloc(s, std::max<uint32_t>(rho, 1), &s->centers));
        k_center_write<<<nch, 256, 0, st>>>(n, seed, Ta, chunk, s->center_rank, s->centers);
        SK_TRY(sk_alloc(s, (size_t)R * std::max<uint32_t>(rho, 1), &s->label_c));
        SK_TRY(sk_alloc(s, (size_t)R * std::max<uint32_t>(rho, 1), &s->size_c));
        s->nw = (n + 63) / 64;
        SK_TRY(sk_alloc(s, (size_t)R * s->nw, &s->gbits));
        SK_TRY(sk_alloc(s, n, &s->gsum));
        SK_HIP(hipMemsetAsync(s->gsum, 0, (size_t)n * 8, st));
        SK_TRY(sk_alloc(s, R, &s->gbest));
        SK_HIP(hipMemsetAsync(s->gbest, 0, (size_t)R * 8, st));
        SK_TRY(sk_alloc(s, R, &s->gcov));
        SK_TRY(sk_alloc(s, 1, &s->bulk_abort));
        uint32_t slots = 64;
        while (slots < n && slots < 4096) slots <<= 1;
        s->memo_mask = slots - 1;
        SK_TRY(sk_alloc(s, (size_t)slots * R * 2, &s->memo));
        SK_HIP(hipMemsetAsync(s->memo, 0xFF, (size_t)slots * R * 16, st));
        SK_TRY(sk_alloc(s, (size_t)R * s->nw, &s->covmin));
        SK_HIP(hipMemsetAsync(s->covmin, 0, (size_t)R * s->nw * 8, st));
    } else {
        s->rho = n;
        SK_TRY(sk_alloc(s, (size_t)n * R, &s->E));
    }
    SK_TRY(sk_alloc(s, n, &s->gain0));
    SK_HIP(hipMemsetAsync(s->gain0, 0, (size_t)n * 8, st));

    // component-labelling scratch: B sketches per pass over the edge list
    SK_TRY(cc_scratch_alloc(ctx, g, R, s->compact, &cs));
    s->B = cs.B;
    const uint32_t B = cs.B;
    uint32_t *parent = cs.parent, *cnt = cs.cnt, *minc = cs.minc;
    if (s->compact) k_to_label_order<<<(n + 255) / 256, 256, 0, st>>>(s->center_rank, g->iperm, n, cs.crank);
    for (uint32_t r0 = 0; r0 < R; r0 += B) {
        const uint32_t b = std::min(B, R - r0);
        // the emits and the giant sample read no entry of an isolated number; an
        // emit resets the forest for the next pass
        const bool last = r0 + B >= R;
        enqueue_cc_pass(ctx, g, s->pm, s->K + r0, b, cs, minc, kNone, s->compact ? cs.crank : nullptr, false, st, true,
                        r0 > 0);
        if (s->compact) {
            k_giant_sample<<<b, 256, 0, st>>>(parent, cnt, n, cs.B, g->n_linked, s->gbest + r0);
            Prof p(ctx, "emit");
            k_gain0_emit<<<(s->nw + 3) / 4, 256, 0, st>>>(parent, cnt, minc, s->center_rank, s->rho, n, cs.B, b, r0,
                                                          R, s->label_c, s->size_c, s->gain0, s->gbest + r0,
                                                          s->gbits, s->nw, s->gsum, g->newid,
                                                          g->n_linked, !last);
        } else {
            Prof p(ctx, "emit");
            k_emit_full<<<((n + kWave - 1) / kWave + 3) / 4, 256, 0, st>>>(parent, cnt, g->newid, g->iperm, n, cs.B,
                                                                         g->n_linked, b, R, r0, s->E, s->gain0,
                                                                         !last);
        }
        SK_HIP(hipGetLastError());
    }

    // selection state
    s->td = make_tree(n);
    const uint64_t tn = tree_nodes(s->td);
    SK_TRY(sk_alloc(s, n, &s->key));
    SK_TRY(sk_alloc(s, n, &s->in_s));
    SK_TRY(sk_alloc(s, tn, &s->ids));
    SK_TRY(sk_alloc(s, tn, &s->fr));
    SK_TRY(sk_alloc(s, n, &s->evl));
    SK_TRY(sk_alloc(s, 1, &s->st));
    SK_TRY(sk_alloc(s, 1, &s->ctl));
    SK_TRY(sk_alloc(s, n, &s->seeds_d));
    SK_TRY(sk_alloc(s, n, &s->gains_d));
    SK_TRY(sk_alloc(s, n, &s->evals_d));
    SK_HIP(hipMemsetAsync(s->in_s, 0, n, st));
    SK_HIP(hipMemsetAsync(s->st, 0, sizeof(SelState), st));
    if (s->compact) {
        SK_TRY(sk_alloc(s, n, &s->partial));
        s->ov_cap = 1u << 22;
        SK_TRY(sk_alloc(s, s->ov_cap, &s->ov));
        const size_t per_slot = (size_t)n * 4 + (size_t)((n + 31) / 32) * 4;
        s->slots = (uint32_t)std::max<size_t>(1, std::min<size_t>(64, (size_t)(256u << 20) / per_slot));
        SK_TRY(sk_alloc(s, (size_t)s->slots * n, &s->slot_q));
        SK_TRY(sk_alloc(s, (size_t)s->slots * ((n + 31) / 32), &s->slot_vis));
        SK_HIP(hipMemsetAsync(s->slot_vis, 0, (size_t)s->slots * ((n + 31) / 32) * 4, st));
    }
    k_keys_from_gain0<<<(n + 255) / 256, 256, 0, st>>>(s->gain0, n, kb, s->key);
    for (int l = (int)s->td.D - 1; l >= 0; --l)
        k_tree_build_level<<<wave_grid(s->td.lvl_n[l], 8192), 256, 0, st>>>(s->td, (uint32_t)l, s->ids, s->key);
    SK_HIP(hipGetLastError());
    SK_HIP(hipEventRecord(t1, st));
    SK_HIP(hipEventSynchronize(t1));
    cc_scratch_free(ctx, &cs);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t0, t1);
    s->build_ms = ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    *out = s;
    return IM_OK;
#undef SK_TRY
#undef SK_HIP
}

// ---------------------------------------------------------------- selection
namespace {

CompactDev compact_dev(const im_sketches *s) {
    return CompactDev{s->center_rank, s->label_c, s->size_c, s->rho,  s->kc,     s->Ta,
                      s->memo,        s->memo_mask, s->R,     s->covmin, s->nw};
}

// MarkSeed on CompactSketch for st->last_seed: one GetCenter per sketch.
void enqueue_markseed_compact(im_sketches *s) {
    hipStream_t st = s->ctx->stream;
    GraphDev gd{s->g->off, s->g->cols};
    const CompactDev cd = compact_dev(s);
    k_markseed_compact<<<wave_grid(s->R, 4096), kBfsBlock, 0, st>>>(s->st, gd, s->pm, s->K, s->R, cd, s->in_s, s->ov,
                                                                     s->ov_cap);
    k_overflow_bfs<<<s->slots, 64, 0, st>>>(1, kMaxLevels + 1, s->st, s->evl, s->partial, gd, s->pm, s->K, cd, s->kb,
                                            s->in_s, s->key, s->ov, s->ov_cap, s->slot_q, s->slot_vis, s->n);
}

// The per-level kernels of one round, from the evaluation of level l0 on
// (begin: start a new round first).  The persistent kernel hands rounds over
// at such a level.
im_status enqueue_round_part(im_sketches *s, bool begin, uint32_t l0) {
    im_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    const TreeDesc &td = s->td;
    GraphDev gd{s->g->off, s->g->cols};
    const CompactDev cd = compact_dev(s);
    const unsigned long long pinit = (unsigned long long)s->R << kPartialShift;
    auto eval = [&](uint32_t l) {
        uint64_t cap = (l == 0) ? 1 : std::min<uint64_t>((uint64_t)s->n, (uint64_t)td.lvl_n[l - 1] * kFan);
        if (!s->compact) {
            k_eval_full<<<wave_grid(cap, 8192), 256, 0, st>>>(l, s->st, s->evl, s->E, s->R, s->kb, s->in_s, s->key);
        } else {
            k_eval_compact_bfs<<<wave_grid(cap * s->R, 65536), kBfsBlock, 0, st>>>(
                l, s->st, s->evl, s->partial, gd, s->pm, s->K, s->R, cd, s->kb, s->in_s, s->key, s->ov, s->ov_cap);
            k_overflow_bfs<<<s->slots, 64, 0, st>>>(0, l, s->st, s->evl, s->partial, gd, s->pm, s->K, cd, s->kb,
                                                    s->in_s, s->key, s->ov, s->ov_cap, s->slot_q, s->slot_vis, s->n);
        }
    };
    if (begin) k_round_begin<<<1, 64, 0, st>>>(td, s->st, s->ids, s->fr, s->evl, s->partial, pinit);
    eval(l0);
    for (uint32_t l = l0; l < td.D; ++l) {
        k_check<<<wave_grid(td.lvl_n[l], 65536), 256, 0, st>>>(td, l, s->st, s->ids, s->key, s->fr, s->evl, s->partial,
                                                                pinit);
        eval(l + 1);
    }
    for (int l = (int)td.D - 1; l >= 0; --l)
        k_relink<<<wave_grid(td.lvl_n[l], 65536), 256, 0, st>>>(td, (uint32_t)l, s->st, s->ids, s->key, s->fr);
    k_round_end<<<1, 64, 0, st>>>(td, s->st, s->ids, s->key, s->in_s, s->kb, s->seeds_d, s->gains_d,
                                  s->evals_d, s->compact ? nullptr : s->E, s->R);
    if (s->compact) enqueue_markseed_compact(s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, IM_EDEVICE, std::string("select launch: ") + hipGetErrorString(e));
    return IM_OK;
}

im_status enqueue_lazy_round(im_sketches *s) { return enqueue_round_part(s, true, 0); }

// Up to max_rounds lazy rounds in one persistent launch (stops early after a
// round whose gain reaches bulk_min, if nonzero, or mid-round at a large
// evaluation step).  Waits for it; *done = rounds completed, *stop_level = the
// level whose evaluation is pending (kNone if stopped at a round boundary),
// *last_gain = gain of the last completed round.
im_status run_persistent_rounds(im_sketches *s, uint32_t max_rounds, unsigned long long bulk_min, uint32_t *done,
                                uint32_t *stop_level, uint64_t *last_gain) {
    im_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    if (!ctx->persist_grid) {
        int per_cu = 0, cus = 0, khz = 0;
        HIP_TRY(ctx, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_select_persist, kPersistBlock, 0));
        HIP_TRY(ctx, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
        HIP_TRY(ctx, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device));
        if (per_cu < 1 || cus < 1 || khz < 1) return fail(ctx, IM_EDEVICE, "persistent selection: no resident workgroup");
        ctx->persist_grid = (unsigned)cus;  // one workgroup per CU
        ctx->clock_hz = (uint64_t)khz * 1000ull;
    }
    SelState h0{};
    HIP_TRY(ctx, hipMemcpyAsync(&h0, s->st, sizeof(SelState), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipMemsetAsync(s->ctl, 0, sizeof(PersistCtl), st));
    PersistArgs a{};
    a.td = s->td;
    a.st = s->st;
    a.ids = s->ids;
    a.key = s->key;
    a.fr = s->fr;
    a.evl = s->evl;
    a.partial = s->partial;
    a.pinit = (unsigned long long)s->R << kPartialShift;
    a.in_s = s->in_s;
    a.kb = s->kb;
    a.R = s->R;
    a.n = s->n;
    a.seeds_out = s->seeds_d;
    a.gains_out = s->gains_d;
    a.evals_out = s->evals_d;
    a.E = s->compact ? nullptr : s->E;
    a.g = GraphDev{s->g->off, s->g->cols};
    a.pm = s->pm;
    a.K = s->K;
    a.cd = compact_dev(s);
    a.ov = s->ov;
    a.ov_cap = s->ov_cap;
    a.slot_q = s->slot_q;
    a.slot_vis = s->slot_vis;
    a.slots = s->slots;
    a.max_rounds = max_rounds;
    // PACIM_PERSIST_STEP (tests) lowers the limit so that rounds are handed over
    const char *ov = getenv("PACIM_PERSIST_STEP");
    a.max_step_tasks = ov ? std::max<uint64_t>(strtoull(ov, nullptr, 10), 1) : (s->compact ? (1ull << 20) : 2048ull);
    a.bulk_gain_min = bulk_min;
    a.ctl = s->ctl;
    a.spin_ticks = 120ull * ctx->clock_hz;  // two minutes
    void *args[] = {&a};
    // CompactSketch: about one wave per sketch (the GetCenter steps have R searches
    // per listed vertex); every extra workgroup costs each step a completion.
    // Under WIC a vertex expects at most sum_j 2 / (d_u + d_j) <= 2 live edges, so a search
    // from a high-degree vertex scans its whole adjacency: steps are long, and one
    // workgroup per CU runs 4x the searches at once for a small completion cost.
    unsigned grid = s->compact ? std::min<unsigned>(ctx->persist_grid, std::max<unsigned>(8u, (s->R + kPersistWaves - 1) / kPersistWaves)) : 1u;
    if (s->compact && s->pm.kind == kProbWic) grid = ctx->persist_grid;
    if (const char *pg = getenv("PACIM_PERSIST_GRID"))  // tuning: workgroups of CompactSketch launches
        if (s->compact) grid = std::max<unsigned>(1u, std::min<unsigned>(ctx->persist_grid, (unsigned)strtoul(pg, nullptr, 10)));
    const char *np = getenv("PACIM_PERSIST");  // "0" (tests): take the path below as if refused
    // A grid of one workgroup (full labels) never waits on another, so it needs no
    // cooperative launch; cooperative launches on one device run one at a time,
    // and a plain one can run beside another query's persistent selection.
    const hipError_t le = (np && !strcmp(np, "0")) ? hipErrorNotSupported
                          : grid == 1u
                              ? hipLaunchKernel(reinterpret_cast<const void *>(k_select_persist), dim3(1),
                                                dim3(kPersistBlock), args, 0, st)
                              : hipLaunchCooperativeKernel(reinterpret_cast<const void *>(k_select_persist),
                                                           dim3(grid), dim3(kPersistBlock), args, 0, st);
    if (le != hipSuccess) {
        // no cooperative launch here: one round with the per-level kernels instead
        (void)hipGetLastError();
        HIP_TRY(ctx, hipStreamSynchronize(st));  // h0 is read below
        im_status rc = enqueue_lazy_round(s);
        if (rc != IM_OK) return rc;
        unsigned long long g = 0;
        HIP_TRY(ctx, hipMemcpyAsync(&g, s->gains_d + h0.round, 8, hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        *done = 1;
        *stop_level = kNone;
        *last_gain = g;
        return IM_OK;
    }
    SelState h1{};
    PersistCtl c{};
    HIP_TRY(ctx, hipMemcpyAsync(&h1, s->st, sizeof(SelState), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipMemcpyAsync(&c, s->ctl, sizeof(PersistCtl), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    if (c.err) return fail(ctx, IM_EINTERNAL, "persistent selection: a step exceeded its time limit");
    if (h1.round < h0.round || h1.round - h0.round > max_rounds)
        return fail(ctx, IM_EINTERNAL, "persistent selection: round counter mismatch");
    *done = h1.round - h0.round;
    *stop_level = h1.stop_level;
    *last_gain = *done ? h1.last_gain : 0;
    return IM_OK;
}

// A round that evaluates every unselected vertex (compact sketches), then
// rebuilds the tree.  First from the build's largest-component bitmaps (a search
// per seed outside its sketch's largest component, capped); past the cap, by
// re-deriving the R sampled graphs' components: sum the uncovered CC sizes.
uint32_t bulk_search_cap(const im_sketches *s) {
    const char *e = getenv("PACIM_BULK_SEARCH_CAP");  // tests: force the re-deriving path
    if (e) return (uint32_t)strtoul(e, nullptr, 10);
    return std::max<uint32_t>(1024u, std::min<uint32_t>(65536u, s->n / 16));
}

im_status finish_bulk_round(im_sketches *s) {
    hipStream_t st = s->ctx->stream;
    const TreeDesc &td = s->td;
    for (int l = (int)td.D - 1; l >= 0; --l)
        k_tree_build_level<<<wave_grid(td.lvl_n[l], 8192), 256, 0, st>>>(td, (uint32_t)l, s->ids, s->key);
    k_round_end<<<1, 64, 0, st>>>(td, s->st, s->ids, s->key, s->in_s, s->kb, s->seeds_d, s->gains_d, s->evals_d,
                                  nullptr, s->R);
    enqueue_markseed_compact(s);
    ++s->bulk_rounds;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s->ctx, IM_EDEVICE, std::string("bulk round launch: ") + hipGetErrorString(e));
    return IM_OK;
}

// Fresh keys of every unselected vertex on CompactSketch (Marginal for the seeds
// chosen so far), from the largest-component bitmaps, else by re-deriving the
// sampled graphs' components.  Leaves the round open.
im_status enqueue_bulk_keys(im_sketches *s) {
    im_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    const uint32_t n = s->n;
    const uint32_t cap = bulk_search_cap(s);
    if (s->gbits && cap > 0) {
        GraphDev gd{s->g->off, s->g->cols};
        uint32_t aborted = 1;
        HIP_TRY(ctx, hipMemsetAsync(s->partial, 0, (size_t)n * 8, st));
        HIP_TRY(ctx, hipMemsetAsync(s->bulk_abort, 0, 4, st));
        k_bulk_bits_search<<<std::min(s->slots, s->R), 64, 0, st>>>(s->st, s->seeds_d, gd, s->pm, s->K, s->R, n, s->gbits,
                                                                 s->nw, s->gcov, s->partial, s->slot_q, s->slot_vis,
                                                                 cap, s->bulk_abort);
        HIP_TRY(ctx, hipMemcpyAsync(&aborted, s->bulk_abort, 4, hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        if (!aborted) {
            Prof p(ctx, "bulk_keys");
            k_bulk_bits_keys<<<(s->nw + 3) / 4, 256, 0, st>>>(s->st, s->gain0, s->partial, s->gbits, s->nw, s->gsum,
                                                              s->gcov,
                                                              s->gbest, s->R, n, s->kb, s->in_s, s->key, s->bulk_abort);
            HIP_TRY(ctx, hipGetLastError());
            return IM_OK;
        }
    }
    ++s->bulk_resampled;
    if (!s->bulk_cs) {
        CCScratch *c = new (std::nothrow) CCScratch();
        if (!c) return fail(ctx, IM_ENOMEM, "host allocation");
        im_status a = cc_scratch_alloc(ctx, s->g, s->R, true, c);
        if (a != IM_OK) { delete c; return a; }
        s->bulk_cs = c;
    }
    const CCScratch &cs = *static_cast<CCScratch *>(s->bulk_cs);
    const uint32_t B = cs.B;
    uint32_t *parent = cs.parent, *cnt = cs.cnt, *flag = cs.minc;
    hipError_t e0 = hipMemsetAsync(s->partial, 0, (size_t)n * 8, st);
    if (e0 != hipSuccess) return fail(ctx, IM_EDEVICE, std::string("bulk round: ") + hipGetErrorString(e0));
    for (uint32_t r0 = 0; r0 < s->R; r0 += B) {
        const uint32_t b = std::min(B, s->R - r0);
        enqueue_cc_pass(ctx, s->g, s->pm, s->K + r0, b, cs, flag, 0u, nullptr);
        k_bulk_seed_roots<<<grid_for((uint64_t)n * b, 256, 1024), 256, 0, st>>>(s->st, s->seeds_d, parent,
                                                                                 s->g->newid, cs.B, b, flag);
        k_bulk_accum<<<(n + 255) / 256, 256, 0, st>>>(parent, cnt, flag, s->g->newid, n, cs.B, b, s->partial);
    }
    k_bulk_keys<<<(n + 255) / 256, 256, 0, st>>>(s->st, s->partial, n, s->kb, s->in_s, s->key);
    HIP_TRY(ctx, hipGetLastError());
    return IM_OK;
}

im_status enqueue_bulk_round(im_sketches *s) {
    im_status rc = enqueue_bulk_keys(s);
    return rc != IM_OK ? rc : finish_bulk_round(s);
}

// Full labels: a round that evaluates every unselected vertex from E in vertex
// order, then rebuilds the tree and ends the round.
im_status enqueue_full_bulk_round(im_sketches *s) {
    hipStream_t st = s->ctx->stream;
    const TreeDesc &td = s->td;
    {
        Prof p(s->ctx, "bulk_keys");
        k_bulk_full_keys<<<wave_grid(s->n, 65536), 256, 0, st>>>(s->st, s->E, s->R, s->n, s->kb, s->in_s, s->key);
    }
    for (int l = (int)td.D - 1; l >= 0; --l)
        k_tree_build_level<<<wave_grid(td.lvl_n[l], 8192), 256, 0, st>>>(td, (uint32_t)l, s->ids, s->key);
    k_round_end<<<1, 64, 0, st>>>(td, s->st, s->ids, s->key, s->in_s, s->kb, s->seeds_d, s->gains_d, s->evals_d,
                                  s->E, s->R);
    ++s->bulk_rounds;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(s->ctx, IM_EDEVICE, std::string("bulk round launch: ") + hipGetErrorString(e));
    return IM_OK;
}

// Policy of bulk rounds (both label kinds): a round is run in bulk when the
// previous seed's gain shows it covered at least 1/64 of the vertices per sketch
// on average (PACIM_BULK=always|never overrides, for tests).
int bulk_policy() {
    const char *e = getenv("PACIM_BULK");
    if (!e) return 0;
    if (!strcmp(e, "always")) return 1;
    if (!strcmp(e, "never")) return -1;
    return 0;
}

}  // namespace

extern "C" im_status im_select_seeds_from(im_ctx *ctx, im_sketches *s, uint32_t k, uint32_t *seeds_out,
                                          uint64_t *gains_out) {
    if (!ctx || !s || s->ctx != ctx) return IM_EINVAL;
    if (k && (!seeds_out || !gains_out)) return fail(ctx, IM_EINVAL, "null output array");
    if ((uint64_t)k + s->chosen > s->n) return fail(ctx, IM_EINVAL, "k exceeds the number of unselected vertices");
    if (k == 0) return IM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    hipEvent_t t0, t1;
    HIP_TRY(ctx, hipEventCreate(&t0));
    HIP_TRY(ctx, hipEventCreate(&t1));
    (void)hipEventRecord(t0, st);
    im_status rc = IM_OK;
    s->st_host_valid = false;
    {
        Prof p(ctx, "select");
        if (!s->tree_valid) {  // rounds by prefix doubling moved keys: rebuild the tree from them
            for (int l = (int)s->td.D - 1; l >= 0; --l)
                k_tree_build_level<<<wave_grid(s->td.lvl_n[l], 8192), 256, 0, st>>>(s->td, (uint32_t)l, s->ids,
                                                                                  s->key);
            s->tree_valid = true;
        }
        s->pt_valid = false;
        // Lazy rounds run in persistent launches.  CompactSketch: a round follows as a
        // bulk round when the previous seed's gain reaches the bulk threshold (the
        // persistent kernel stops after such a round); gains never increase, so
        // once one is below it every later round is lazy.
        // Full labels: the same rule, the bulk round evaluating every vertex from E.
        const int pol = bulk_policy();
        const unsigned long long bmin =
            pol == 0 ? (unsigned long long)(((uint64_t)s->R * s->n + 63) / 64) : 0ull;
        uint32_t cur = s->chosen;
        uint64_t last = s->last_gain;
        for (uint32_t i = 0; i < k && rc == IM_OK;) {
            const bool bulk = cur > 0 && (pol > 0 || (pol == 0 && last >= bmin));
            if (bulk) {
                rc = s->compact ? enqueue_bulk_round(s) : enqueue_full_bulk_round(s);
                if (rc != IM_OK) break;
                unsigned long long g = 0;
                hipError_t e1 = hipMemcpyAsync(&g, s->gains_d + cur, 8, hipMemcpyDeviceToHost, st);
                hipError_t e2 = hipStreamSynchronize(st);
                if (e1 != hipSuccess || e2 != hipSuccess) {
                    rc = fail(ctx, IM_EDEVICE, "select: gain read-back failed");
                    break;
                }
                last = g;
                ++cur;
                ++i;
                continue;
            }
            const uint32_t want = pol > 0 ? 1u : k - i;
            uint32_t done = 0, stop_level = kNone;
            uint64_t g = 0;
            rc = run_persistent_rounds(s, want, bmin, &done, &stop_level, &g);
            if (rc != IM_OK) break;
            cur += done;
            i += done;
            if (done) last = g;
            if (stop_level != kNone) {
                // the persistent kernel left a large evaluation step to the per-level kernels
                rc = enqueue_round_part(s, false, stop_level);
                if (rc != IM_OK) break;
                unsigned long long g2 = 0;
                hipError_t e1 = hipMemcpyAsync(&g2, s->gains_d + cur, 8, hipMemcpyDeviceToHost, st);
                hipError_t e2 = hipStreamSynchronize(st);
                if (e1 != hipSuccess || e2 != hipSuccess) {
                    rc = fail(ctx, IM_EDEVICE, "select: gain read-back failed");
                    break;
                }
                last = g2;
                ++cur;
                ++i;
            } else if (done == 0) {
                rc = fail(ctx, IM_EINTERNAL, "persistent selection made no progress");
            }
        }
    }
    (void)hipEventRecord(t1, st);
    std::vector<uint32_t> seeds(k);
    std::vector<unsigned long long> gains(k);
    SelState hst{};
    if (rc == IM_OK) {
        hipError_t e1 = hipMemcpyAsync(seeds.data(), s->seeds_d + s->chosen, (size_t)k * 4, hipMemcpyDeviceToHost, st);
        hipError_t e2 = hipMemcpyAsync(gains.data(), s->gains_d + s->chosen, (size_t)k * 8, hipMemcpyDeviceToHost, st);
        hipError_t e3 = hipMemcpyAsync(&hst, s->st, sizeof(SelState), hipMemcpyDeviceToHost, st);
        hipError_t e4 = hipStreamSynchronize(st);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
            rc = fail(ctx, IM_EDEVICE, std::string("select: ") + hipGetErrorString(e4 != hipSuccess ? e4 : e1));
        else {
            s->st_host = hst;
            s->st_host_valid = true;
        }
    }
    float ms = 0.f;
    if (rc == IM_OK && hipEventElapsedTime(&ms, t0, t1) == hipSuccess) s->select_ms += ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc != IM_OK) return rc;
    if (hst.err) return fail(ctx, IM_EINTERNAL, "selection consistency check failed (code " + std::to_string(hst.err) + ")");
    if (hst.round != s->chosen + k) return fail(ctx, IM_EINTERNAL, "round counter mismatch");
    for (uint32_t i = 0; i < k; ++i) {
        seeds_out[i] = seeds[i];
        gains_out[i] = gains[i];
    }
    s->chosen += k;
    s->last_gain = gains[k - 1];
    return IM_OK;
}

// ---------------------------------------------------------------- NextSeed by prefix doubling
namespace {

unsigned span_grid(uint64_t items) {
    const uint64_t threads = (items + kPtSpan - 1) / kPtSpan;
    return (unsigned)std::max<uint64_t>(1, (threads + kPtBlock - 1) / kPtBlock);
}

// Sorts in[0, len) into decreasing order; a and b (n keys each, distinct from in)
// hold the passes.  Returns the one holding the result.
uint64_t *pt_sort(hipStream_t st, const uint64_t *in, uint32_t len, uint64_t *a, uint64_t *b) {
    if (len == 0) return a;
    k_pt_sort_tiles<<<(len + kPtTile - 1) / kPtTile, kPtBlock, 0, st>>>(in, len, a);
    uint64_t *src = a, *dst = b;
    for (uint64_t L = kPtTile; L < len; L *= 2) {
        k_pt_merge_pass<<<span_grid(len), kPtBlock, 0, st>>>(src, len, (uint32_t)L, dst);
        std::swap(src, dst);
    }
    return src;
}

// The three buffers holding neither X nor Y.
void pt_spare(const im_sketches *s, int f[3]) {
    int c = 0;
    for (int i = 0; i < 5; ++i)
        if (i != s->pt_x && i != s->pt_y) f[c++] = i;
}

int pt_index(const im_sketches *s, const uint64_t *p) {
    for (int i = 0; i < 5; ++i)
        if (s->pt_buf[i] == p) return i;
    return -1;
}

// Builds the queue from key[] (0 for seeds, which sort last): X = the n - chosen
// unselected vertices in decreasing key order, Y empty.
im_status pt_build(im_sketches *s) {
    im_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    if (!s->pt_buf[0]) {
        for (int i = 0; i < 5; ++i) {
            im_status a = sk_alloc(s, s->n, &s->pt_buf[i]);
            if (a != IM_OK) return a;
        }
        im_status a = sk_alloc(s, 1, &s->pt_state);
        if (a != IM_OK) return a;
        a = sk_alloc(s, 1, &s->pt_dev);
        if (a != IM_OK) return a;
        HIP_TRY(ctx, hipHostMalloc((void **)&s->pt_host, sizeof(PtState), hipHostMallocDefault));
        HIP_TRY(ctx, hipHostMalloc((void **)&s->pt_dev_host, sizeof(PtDev), hipHostMallocDefault));
    }
    s->pt_x = 0;
    s->pt_y = 1;
    int f[3];
    pt_spare(s, f);
    const uint64_t *sorted = pt_sort(st, s->key, s->n, s->pt_buf[f[0]], s->pt_buf[f[1]]);
    s->pt_x = pt_index(s, sorted);
    s->pt_y = (s->pt_x == f[0]) ? f[2] : f[0];
    s->pt_hx = 0;
    s->pt_nx = s->n - s->chosen;
    s->pt_hy = s->pt_ny = 0;
    s->pt_valid = true;
    HIP_TRY(ctx, hipGetLastError());
    return IM_OK;
}

// CompactSketch: the batch size from which a prefix-doubling round evaluates
// every vertex at once from the bitmaps (the rest of the round then reads the
// keys), instead of R GetCenter searches per listed vertex.  PACIM_PTREE_BULK
// overrides (0: never).
constexpr uint32_t kPtListEval = 1u << 14;  // full labels: batches from this size use the label-caching kernel

uint32_t pt_bulk_min(const im_sketches *s) {
    const char *e = getenv("PACIM_PTREE_BULK");
    if (e) return (uint32_t)strtoul(e, nullptr, 10);
    return std::max<uint32_t>(64u, s->n / 4096);
}

// One round of Algorithm 4: batches of 1, 2, 4, ... vertices taken from the
// queue and evaluated until the best evaluated key ranks above the queue's Max();
// that vertex is the seed (MarkSeed follows); the others are put back with their
// new keys.  The host reads the stop flag after each batch.
// Batches of one round from `off` vertices evaluated and batch size `batch` on,
// until the best evaluated key ranks above the queue's Max(); *tot = the round's
// evaluation count.  The host reads the stop flag after each batch.
im_status pt_batches(im_sketches *s, uint32_t off, uint64_t batch, uint32_t *tot) {
    im_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    GraphDev gd{s->g->off, s->g->cols};
    const CompactDev cd = compact_dev(s);
    const unsigned long long pinit = (unsigned long long)s->R << kPartialShift;
    const uint32_t bulk_min = s->compact ? pt_bulk_min(s) : 0u;
    bool all_known = false;  // key[] holds every vertex's Marginal for this round
    for (;; batch *= 2) {
        const uint32_t nxl = s->pt_nx - s->pt_hx, nyl = s->pt_ny - s->pt_hy;
        const uint32_t m = (uint32_t)std::min<uint64_t>(batch, (uint64_t)nxl + nyl);
        if (m == 0) return fail(ctx, IM_EINTERNAL, "prefix-doubling round ran out of vertices");
        const uint64_t *X = s->pt_buf[s->pt_x] + s->pt_hx, *Y = s->pt_buf[s->pt_y] + s->pt_hy;
        uint32_t *evl = s->evl + off;
        unsigned long long *part = s->compact ? s->partial + off : nullptr;
        k_pt_extract<<<span_grid(m), kPtBlock, 0, st>>>(X, nxl, Y, nyl, m, s->kb, evl, part, pinit, s->pt_state,
                                                         s->st);
        if (!all_known && bulk_min && m >= bulk_min) {
            im_status rc = enqueue_bulk_keys(s);
            if (rc != IM_OK) return rc;
            all_known = true;
            ++s->bulk_rounds;
        }
        if (all_known) {
            k_pt_eval_known<<<(m + 255) / 256, 256, 0, st>>>(evl, m, s->key, s->st);
        } else if (!s->compact && m >= kPtListEval && s->R <= 4u * kWave) {
            k_pt_eval_full_list<<<wave_grid(m / 16, 65536), 256, 0, st>>>(evl, m, s->E, s->R, s->kb, s->in_s, s->key,
                                                                          s->st);
        } else if (!s->compact) {
            k_eval_full<<<wave_grid(m, 8192), 256, 0, st>>>(0, s->st, evl, s->E, s->R, s->kb, s->in_s, s->key);
        } else {
            k_eval_compact_bfs<<<wave_grid((uint64_t)m * s->R, 65536), kBfsBlock, 0, st>>>(
                0, s->st, evl, part, gd, s->pm, s->K, s->R, cd, s->kb, s->in_s, s->key, s->ov, s->ov_cap);
            k_overflow_bfs<<<s->slots, 64, 0, st>>>(0, 0, s->st, evl, part, gd, s->pm, s->K, cd, s->kb, s->in_s,
                                                    s->key, s->ov, s->ov_cap, s->slot_q, s->slot_vis, s->n);
        }
        k_pt_check<<<1, 64, 0, st>>>(X, nxl, Y, nyl, m, s->pt_state, s->st);
        HIP_TRY(ctx, hipGetLastError());
        HIP_TRY(ctx, hipMemcpyAsync(s->pt_host, s->pt_state, sizeof(PtState), hipMemcpyDeviceToHost, st));
        HIP_TRY(ctx, hipStreamSynchronize(st));
        const uint32_t take = s->pt_host->take;
        if (take > nxl || m - take > nyl) return fail(ctx, IM_EINTERNAL, "prefix-doubling split out of range");
        s->pt_hx += take;
        s->pt_hy += m - take;
        off += m;
        if (s->pt_host->stop) break;
    }
    *tot = off;
    return IM_OK;
}

// The round's end (seed, MarkSeed) for a round of tot evaluations.
void pt_end(im_sketches *s, uint32_t tot) {
    hipStream_t st = s->ctx->stream;
    k_pt_round_end<<<1, 64, 0, st>>>(s->st, s->key, s->in_s, s->n, s->kb, tot, s->seeds_d, s->gains_d, s->evals_d,
                                     s->compact ? nullptr : s->E, s->R);
    if (s->compact) enqueue_markseed_compact(s);
}

// BatchInsert of the round's other evaluated vertices (s*'s key is now 0 and
// sorts last), merged with Y's unread part.
im_status pt_insert(im_sketches *s, uint32_t tot) {
    hipStream_t st = s->ctx->stream;
    if (tot > 1) {
        int f[3];
        pt_spare(s, f);
        k_pt_gather<<<(tot + 255) / 256, 256, 0, st>>>(s->evl, tot, s->key, s->pt_buf[f[0]]);
        const uint64_t *sorted = pt_sort(st, s->pt_buf[f[0]], tot, s->pt_buf[f[1]], s->pt_buf[f[0]]);
        const int si = pt_index(s, sorted);
        const int out = (si == f[0]) ? f[1] : f[0];
        const uint32_t nyl = s->pt_ny - s->pt_hy;
        k_pt_merge2<<<span_grid((uint64_t)tot - 1 + nyl), kPtBlock, 0, st>>>(
            sorted, tot - 1, s->pt_buf[s->pt_y] + s->pt_hy, nyl, s->pt_buf[out]);
        s->pt_y = out;
        s->pt_hy = 0;
        s->pt_ny = tot - 1 + nyl;
    }
    HIP_TRY(s->ctx, hipGetLastError());
    return IM_OK;
}

// Y is merged into X once it outgrows X's unread part, so that re-inserting stays
// proportional to what was re-inserted since.
im_status pt_fold(im_sketches *s) {
    hipStream_t st = s->ctx->stream;
    const uint32_t nxl = s->pt_nx - s->pt_hx, nyl = s->pt_ny - s->pt_hy;
    if (nyl > nxl) {
        int f[3];
        pt_spare(s, f);
        k_pt_merge2<<<span_grid((uint64_t)nxl + nyl), kPtBlock, 0, st>>>(
            s->pt_buf[s->pt_x] + s->pt_hx, nxl, s->pt_buf[s->pt_y] + s->pt_hy, nyl, s->pt_buf[f[0]]);
        s->pt_x = f[0];
        s->pt_hx = 0;
        s->pt_nx = nxl + nyl;
        s->pt_hy = s->pt_ny = 0;
    }
    HIP_TRY(s->ctx, hipGetLastError());
    return IM_OK;
}

// One round of Algorithm 4 with the host driving each batch.
im_status pt_round(im_sketches *s) {
    k_pt_round_begin<<<1, 64, 0, s->ctx->stream>>>(s->st);
    uint32_t tot = 0;
    im_status rc = pt_batches(s, 0, 1, &tot);
    if (rc != IM_OK) return rc;
    pt_end(s, tot);
    rc = pt_insert(s, tot);
    return rc != IM_OK ? rc : pt_fold(s);
}

// Up to max_rounds rounds on the device (full labels), finishing on the host the
// round or step it stopped at.  *done = rounds completed.
im_status pt_device_rounds(im_sketches *s, uint32_t max_rounds, uint32_t *done) {
    im_ctx *ctx = s->ctx;
    hipStream_t st = ctx->stream;
    PtDev &h = *s->pt_dev_host;
    for (int i = 0; i < 5; ++i) h.buf[i] = s->pt_buf[i];
    h.x = s->pt_x;
    h.y = s->pt_y;
    h.hx = s->pt_hx;
    h.nx = s->pt_nx;
    h.hy = s->pt_hy;
    h.ny = s->pt_ny;
    HIP_TRY(ctx, hipMemcpyAsync(s->pt_dev, &h, sizeof(PtDev), hipMemcpyHostToDevice, st));
    k_pt_rounds<<<1, kPtRoundBlock, 0, st>>>(s->pt_dev, max_rounds, s->st, s->key, s->in_s, s->n, s->kb, s->seeds_d,
                                             s->gains_d, s->evals_d, s->E, s->R, s->evl);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(&h, s->pt_dev, sizeof(PtDev), hipMemcpyDeviceToHost, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    s->pt_x = h.x;
    s->pt_y = h.y;
    s->pt_hx = h.hx;
    s->pt_nx = h.nx;
    s->pt_hy = h.hy;
    s->pt_ny = h.ny;
    uint32_t rounds = h.rounds;
    im_status rc = IM_OK;
    switch (h.stop) {
    case kPtStopDone:
        break;
    case kPtStopMidRound: {
        uint32_t tot = 0;
        rc = pt_batches(s, h.off, h.batch, &tot);
        if (rc != IM_OK) break;
        pt_end(s, tot);
        rc = pt_insert(s, tot);
        if (rc == IM_OK) rc = pt_fold(s);
        ++rounds;
        break;
    }
    case kPtStopInsert:
        rc = pt_insert(s, h.off);
        if (rc == IM_OK) rc = pt_fold(s);
        break;
    case kPtStopFold:
        rc = pt_fold(s);
        break;
    default:
        rc = fail(ctx, IM_EINTERNAL, "device prefix-doubling rounds: bad stop state");
    }
    if (rc == IM_OK && rounds == 0) rc = fail(ctx, IM_EINTERNAL, "device prefix-doubling rounds made no progress");
    if (rc == IM_OK && h.stop == kPtStopDone && rounds < max_rounds)
        rc = fail(ctx, IM_EINTERNAL, "device prefix-doubling rounds stopped early");
    *done = rounds;
    return rc;
}

bool pt_device_enabled() {
    const char *e = getenv("PACIM_PTREE_DEVICE");  // "0" (tests): every batch from the host
    return !(e && !strcmp(e, "0"));
}

}  // namespace

extern "C" im_status im_select_seeds_ptree(im_ctx *ctx, im_sketches *s, uint32_t k, uint32_t *seeds_out,
                                           uint64_t *gains_out) {
    if (!ctx || !s || s->ctx != ctx) return IM_EINVAL;
    if (k && (!seeds_out || !gains_out)) return fail(ctx, IM_EINVAL, "null output array");
    if ((uint64_t)k + s->chosen > s->n) return fail(ctx, IM_EINVAL, "k exceeds the number of unselected vertices");
    if (k == 0) return IM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    hipEvent_t t0, t1;
    HIP_TRY(ctx, hipEventCreate(&t0));
    HIP_TRY(ctx, hipEventCreate(&t1));
    (void)hipEventRecord(t0, st);
    im_status rc = IM_OK;
    s->st_host_valid = false;
    {
        Prof p(ctx, "select_ptree");
        if (!s->pt_valid) rc = pt_build(s);
        s->tree_valid = false;
        for (uint32_t i = 0; i < k && rc == IM_OK;) {
            if (!s->compact && pt_device_enabled()) {
                uint32_t done = 0;
                rc = pt_device_rounds(s, k - i, &done);
                i += done;
            } else {
                rc = pt_round(s);
                ++i;
            }
        }
    }
    (void)hipEventRecord(t1, st);
    std::vector<uint32_t> seeds(k);
    std::vector<unsigned long long> gains(k);
    SelState hst{};
    if (rc == IM_OK) {
        hipError_t e1 = hipMemcpyAsync(seeds.data(), s->seeds_d + s->chosen, (size_t)k * 4, hipMemcpyDeviceToHost, st);
        hipError_t e2 = hipMemcpyAsync(gains.data(), s->gains_d + s->chosen, (size_t)k * 8, hipMemcpyDeviceToHost, st);
        hipError_t e3 = hipMemcpyAsync(&hst, s->st, sizeof(SelState), hipMemcpyDeviceToHost, st);
        hipError_t e4 = hipStreamSynchronize(st);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || e4 != hipSuccess)
            rc = fail(ctx, IM_EDEVICE, std::string("select: ") + hipGetErrorString(e4 != hipSuccess ? e4 : e1));
        else {
            s->st_host = hst;
            s->st_host_valid = true;
        }
    }
    float ms = 0.f;
    if (rc == IM_OK && hipEventElapsedTime(&ms, t0, t1) == hipSuccess) s->select_ms += ms;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (rc != IM_OK) {
        s->pt_valid = false;
        return rc;
    }
    if (hst.err) return fail(ctx, IM_EINTERNAL, "selection consistency check failed (code " + std::to_string(hst.err) + ")");
    if (hst.round != s->chosen + k) return fail(ctx, IM_EINTERNAL, "round counter mismatch");
    for (uint32_t i = 0; i < k; ++i) {
        seeds_out[i] = seeds[i];
        gains_out[i] = gains[i];
    }
    s->chosen += k;
    s->last_gain = gains[k - 1];
    return IM_OK;
}

extern "C" im_status im_select_seeds(im_ctx *ctx, const im_graph *g, im_prob prob, uint32_t R, uint32_t k,
                                     uint64_t seed, uint32_t *seeds_out, uint64_t *gains_out) {
    if (!ctx || !g) return IM_EINVAL;
    if (k > g->n) return fail(ctx, IM_EINVAL, "k exceeds n");
    im_sketches *s = nullptr;
    im_status rc = im_build_sketches(ctx, g, prob, R, seed, 1.0, &s);
    if (rc != IM_OK) return rc;
    rc = im_select_seeds_from(ctx, s, k, seeds_out, gains_out);
    im_sketches_free(s);
    return rc;
}

// ---------------------------------------------------------------- influence by simulation
extern "C" im_status im_influence(im_ctx *ctx, const im_graph *g, im_prob prob, const uint32_t *seeds, uint32_t k,
                                  uint64_t sim_seed, uint32_t w0, uint32_t sims, uint64_t *total_out) {
    if (!ctx || !g || !total_out || (k && !seeds)) return IM_EINVAL;
    if (g->ctx != ctx) return fail(ctx, IM_EINVAL, "graph belongs to another context");
    if (const char *why = prob_problem(prob)) return fail(ctx, IM_EINVAL, why);
    for (uint32_t i = 0; i < k; ++i)
        if (seeds[i] >= g->n) return fail(ctx, IM_EINVAL, "seed vertex out of range");
    if ((uint64_t)w0 + sims > 0xFFFFFFFFull) return fail(ctx, IM_EINVAL, "world range exceeds 2^32");
    *total_out = 0;
    if (k == 0 || sims == 0) return IM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    ProbDev pm = prob_dev(prob, g->off);
    uint64_t *pe_dev = nullptr;  // per-edge model: thresholds by edge, for the call
    if (prob.kind == IM_PROB_PER_EDGE && g->m_und) {
        std::vector<uint64_t> tc, te;
        im_status r0 = per_edge_thresholds(ctx, g, prob.p_edge, tc, te);
        if (r0 != IM_OK) return r0;
        r0 = dev_alloc(ctx, te.size() * 8, (void **)&pe_dev);
        if (r0 != IM_OK) return r0;
        if (hipMemcpy(pe_dev, te.data(), te.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
            dev_free(ctx, pe_dev, te.size() * 8);
            return fail(ctx, IM_EDEVICE, "influence: threshold upload failed");
        }
        pm.edge_thr = pe_dev;
    }
    struct PeFree {  // the per-edge thresholds go with the call
        im_ctx *c;
        uint64_t *p;
        size_t bytes;
        ~PeFree() { if (p) dev_free(c, p, bytes); }
    } pe_free{ctx, pe_dev, (size_t)g->m_und * 8};
    const uint32_t nk = key_slots(sims);
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t small = a256((size_t)nk * 8) + a256((size_t)k * 4) + 256;
    void *blk = nullptr;
    im_status rc = dev_alloc(ctx, small, &blk);
    if (rc != IM_OK) return rc;
    uint64_t *K = static_cast<uint64_t *>(blk);
    uint32_t *sd = reinterpret_cast<uint32_t *>(static_cast<char *>(blk) + a256((size_t)nk * 8));
    unsigned long long *tot =
        reinterpret_cast<unsigned long long *>(reinterpret_cast<char *>(sd) + a256((size_t)k * 4));
    CCScratch cs;
    rc = cc_scratch_alloc(ctx, g, sims, true, &cs);
    if (rc != IM_OK) {
        dev_free(ctx, blk, small);
        return rc;
    }
    unsigned long long host_total = 0;
    hipError_t e = hipMemcpyAsync(sd, seeds, (size_t)k * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(tot, 0, 8, st);
    if (e == hipSuccess) {
        k_world_keys<<<(nk + 255) / 256, 256, 0, st>>>(sim_seed, w0, nk, K);
        for (uint32_t a = 0; a < sims; a += cs.B) {
            const uint32_t b = std::min(cs.B, sims - a);
            enqueue_cc_pass(ctx, g, pm, K + a, b, cs, cs.minc, 0u, nullptr);
            k_influence_accum<<<dim3(grid_for(k, 256, 64), b), 256, 0, st>>>(cs.parent, cs.cnt, cs.minc, g->newid,
                                                                            cs.B, sd, k, tot);
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&host_total, tot, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    cc_scratch_free(ctx, &cs);
    dev_free(ctx, blk, small);
    if (e != hipSuccess) return fail(ctx, IM_EDEVICE, std::string("influence: ") + hipGetErrorString(e));
    *total_out = host_total;
    return IM_OK;
}

// ---------------------------------------------------------------- influence without allocation
// im_influence's scratch (world keys, the seed list, the total and the labelling
// forests parent/cnt/flag of B worlds) taken from one static device array instead
// of the context's allocator.  Each device holds its own copy of the array, at its
// own address, from when the code object is loaded there until the process ends;
// the host-side name of the array is not a device address, so host code only ever
// uses the per-device address that hipGetSymbolAddress returns.
namespace {

constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kStaticScratchDevices = 64;

__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kStaticScratchDevices] = {};
hipError_t g_scratch_err[kStaticScratchDevices] = {};
bool g_scratch_done[kStaticScratchDevices] = {};

// Resolves the device address of `scratch` on `device` once (the device must be
// current); later calls return the kept result.
hipError_t static_scratch_on(int device, void **ptr) {
    *ptr = nullptr;
    if (device < 0 || device >= kStaticScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        g_scratch_err[device] = e;
        g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
        g_scratch_done[device] = true;
        if (e != hipSuccess) (void)hipGetLastError();
    }
    *ptr = g_scratch_ptr[device];
    return g_scratch_err[device];
}

__global__ void k_zero_u64(unsigned long long *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0ull;
}

}  // namespace

extern "C" im_status im_influence_static_scratch(size_t *max_bytes) {
    if (!max_bytes) return IM_EINVAL;
    *max_bytes = kStaticScratchBytes;
    return IM_OK;
}

extern "C" im_status im_influence_noalloc(im_ctx *ctx, const im_graph *g, im_prob prob, const uint32_t *seeds,
                                          uint32_t k, uint64_t sim_seed, uint32_t w0, uint32_t sims,
                                          uint64_t *total_out) {
    if (!ctx || !g || !total_out || (k && !seeds)) return IM_EINVAL;
    if (g->ctx != ctx) return fail(ctx, IM_EINVAL, "graph belongs to another context");
    if (const char *why = prob_problem(prob)) return fail(ctx, IM_EINVAL, why);
    if (prob.kind == IM_PROB_PER_EDGE)
        return fail(ctx, IM_EINVAL, "the per-edge model needs its thresholds on the device: use im_influence");
    for (uint32_t i = 0; i < k; ++i)
        if (seeds[i] >= g->n) return fail(ctx, IM_EINVAL, "seed vertex out of range");
    if ((uint64_t)w0 + sims > 0xFFFFFFFFull) return fail(ctx, IM_EINVAL, "world range exceeds 2^32");
    // layout: keys of one pass's worlds | seeds | total | parent, cnt, flag of B worlds
    auto a256 = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t head = a256((size_t)key_slots(64) * 8) + a256((size_t)k * 4) + 256;
    const size_t per_world = sketch_stride(g->n) * 4 * 3;
    if (head + per_world > kStaticScratchBytes)
        return fail(ctx, IM_EINVAL, "n = " + std::to_string(g->n) + ", k = " + std::to_string(k) +
                                        " need more than the " + std::to_string(kStaticScratchBytes >> 20) +
                                        " MiB static scratch holds (one world takes 12 bytes per vertex)");
    *total_out = 0;
    if (k == 0 || sims == 0) return IM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    void *base = nullptr;
    if (const hipError_t e = static_scratch_on(ctx->device, &base); e != hipSuccess)
        return fail(ctx, IM_EDEVICE, std::string("static scratch address: ") + hipGetErrorString(e));
    const uint32_t B = (uint32_t)std::min<size_t>({(size_t)64, (size_t)sims, (kStaticScratchBytes - head) / per_world});
    char *b8 = static_cast<char *>(base);
    uint64_t *K = reinterpret_cast<uint64_t *>(b8);
    uint32_t *sd = reinterpret_cast<uint32_t *>(b8 + a256((size_t)key_slots(64) * 8));
    unsigned long long *tot = reinterpret_cast<unsigned long long *>(b8 + a256((size_t)key_slots(64) * 8) +
                                                                     a256((size_t)k * 4));
    CCScratch cs;
    cs.B = B;
    cs.parent = reinterpret_cast<uint32_t *>(b8 + head);
    cs.cnt = cs.parent + (size_t)B * sketch_stride(g->n);
    cs.minc = cs.cnt + (size_t)B * sketch_stride(g->n);
    hipStream_t st = ctx->stream;
    const ProbDev pm = prob_dev(prob, g->off);
    unsigned long long host_total = 0;
    hipError_t e = hipMemcpyAsync(sd, seeds, (size_t)k * 4, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        k_zero_u64<<<1, 64, 0, st>>>(tot);
        for (uint32_t a = 0; a < sims; a += B) {
            const uint32_t b = std::min(B, sims - a);
            // keys of worlds w0 + a .. w0 + a + key_slots(b) - 1 (the sampling pass reads 8 at a time)
            k_world_keys<<<1, 128, 0, st>>>(sim_seed, w0 + a, key_slots(b), K);
            enqueue_cc_pass(ctx, g, pm, K, b, cs, cs.minc, 0u, nullptr, true, st, false);
            k_influence_accum<<<dim3(grid_for(k, 256, 64), b), 256, 0, st>>>(cs.parent, cs.cnt, cs.minc, g->newid,
                                                                            cs.B, sd, k, tot);
        }
        e = hipGetLastError();
        if (e == hipSuccess) e = hipMemcpyAsync(&host_total, tot, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    if (e != hipSuccess) return fail(ctx, IM_EDEVICE, std::string("influence: ") + hipGetErrorString(e));
    *total_out = host_total;
    return IM_OK;
}

// ---------------------------------------------------------------- inspection
namespace {

__global__ void k_dump_full(const uint2 *__restrict__ E, uint32_t n, uint32_t R, uint32_t r,
                            uint32_t *__restrict__ lab, uint32_t *__restrict__ siz) {
    const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const uint2 e = E[(size_t)v * R + r];
    lab[v] = e.x;
    siz[v] = E[(size_t)e.x * R + r].y;
}

// Sketch r of a CompactSketch triple (center-major) as two rho-long rows.
__global__ void k_dump_compact(const uint32_t *__restrict__ label_c, const uint32_t *__restrict__ size_c,
                               uint32_t rho, uint32_t R, uint32_t r, uint32_t *__restrict__ lab,
                               uint32_t *__restrict__ siz) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rho) return;
    lab[i] = label_c[(size_t)i * R + r];
    siz[i] = size_c[(size_t)i * R + r];
}

}  // namespace

extern "C" im_status im_sketches_dump(im_ctx *ctx, const im_sketches *s, uint32_t r, uint32_t *labels,
                                      uint32_t *sizes) {
    if (!ctx || !s || !labels || !sizes) return IM_EINVAL;
    if (r >= s->R) return fail(ctx, IM_EINVAL, "sketch index out of range");
    if (s->chosen) return fail(ctx, IM_EINVAL, "dump is only available before seeds are selected");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    if (!s->compact) {
        uint32_t *tmp = nullptr;
        im_status a = dev_alloc(ctx, (size_t)s->n * 8, (void **)&tmp);
        if (a != IM_OK) return a;
        k_dump_full<<<(s->n + 255) / 256, 256, 0, st>>>(s->E, s->n, s->R, r, tmp, tmp + s->n);
        hipError_t e1 = hipMemcpyAsync(labels, tmp, (size_t)s->n * 4, hipMemcpyDeviceToHost, st);
        hipError_t e2 = hipMemcpyAsync(sizes, tmp + s->n, (size_t)s->n * 4, hipMemcpyDeviceToHost, st);
        hipError_t e3 = hipStreamSynchronize(st);
        dev_free(ctx, tmp, (size_t)s->n * 8);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(ctx, IM_EDEVICE, "dump copy failed");
        // E labels a component by one of its vertices; the dump names it by the smallest
        std::vector<uint32_t> least(s->n, kNone);
        for (uint32_t v = 0; v < s->n; ++v) {
            if (labels[v] >= s->n) return fail(ctx, IM_EINTERNAL, "dump: label out of range");
            least[labels[v]] = std::min(least[labels[v]], v);
        }
        for (uint32_t v = 0; v < s->n; ++v) labels[v] = least[labels[v]];
        return IM_OK;
    }
    if (s->rho) {
        uint32_t *tmp = nullptr;
        im_status a = dev_alloc(ctx, (size_t)s->rho * 8, (void **)&tmp);
        if (a != IM_OK) return a;
        k_dump_compact<<<(s->rho + 255) / 256, 256, 0, st>>>(s->label_c, s->size_c, s->rho, s->R, r, tmp,
                                                              tmp + s->rho);
        hipError_t e1 = hipMemcpyAsync(labels, tmp, (size_t)s->rho * 4, hipMemcpyDeviceToHost, st);
        hipError_t e2 = hipMemcpyAsync(sizes, tmp + s->rho, (size_t)s->rho * 4, hipMemcpyDeviceToHost, st);
        hipError_t e3 = hipStreamSynchronize(st);
        dev_free(ctx, tmp, (size_t)s->rho * 8);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(ctx, IM_EDEVICE, "dump copy failed");
        return IM_OK;
    }
    HIP_TRY(ctx, hipStreamSynchronize(st));
    return IM_OK;
}

extern "C" im_status im_centers(im_ctx *ctx, const im_sketches *s, uint32_t *centers, uint32_t *rho) {
    if (!ctx || !s || !rho) return IM_EINVAL;
    *rho = s->rho;
    if (!centers) return IM_OK;
    if (!s->compact) {
        for (uint32_t v = 0; v < s->n; ++v) centers[v] = v;
        return IM_OK;
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (s->rho) HIP_TRY(ctx, hipMemcpyAsync(centers, s->centers, (size_t)s->rho * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return IM_OK;
}

extern "C" im_status im_initial_gains(im_ctx *ctx, const im_sketches *s, uint64_t *gains) {
    if (!ctx || !s || !gains) return IM_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpyAsync(gains, s->gain0, (size_t)s->n * 8, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return IM_OK;
}

extern "C" im_status im_select_trace(im_ctx *ctx, const im_sketches *s, uint32_t *evals_per_round,
                                     uint32_t count) {
    if (!ctx || !s || (count && !evals_per_round)) return IM_EINVAL;
    if (count > s->chosen) return fail(ctx, IM_EINVAL, "count exceeds the seeds chosen so far");
    if (!count) return IM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipMemcpyAsync(evals_per_round, s->evals_d, (size_t)count * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    return IM_OK;
}

extern "C" im_status im_sketches_stats(const im_sketches *s, im_sketch_stats *out) {
    if (!s || !out) return IM_EINVAL;
    SelState hst = s->st_host;
    (void)hipSetDevice(s->ctx->device);
    if (!s->st_host_valid &&
        (hipMemcpyAsync(&hst, s->st, sizeof(SelState), hipMemcpyDeviceToHost, s->ctx->stream) != hipSuccess ||
         hipStreamSynchronize(s->ctx->stream) != hipSuccess))
        return IM_EDEVICE;
    out->seeds_chosen = s->chosen;
    out->rho = s->rho;
    out->evaluations = hst.evals;
    out->bfs_overflow = hst.overflow;
    out->bfs_visits = hst.visits;
    out->build_ms = s->build_ms;
    out->select_ms = s->select_ms;
    out->sketches_per_pass = s->B;
    out->sketch_bytes = s->bytes;
    out->bulk_rounds = s->bulk_rounds;
    out->bulk_resampled = s->bulk_resampled;
    return IM_OK;
}

// ---------------------------------------------------------------- device probe
extern "C" im_status im_probe_device(im_ctx *ctx, double *hash_per_s, double *copy_bytes_per_s) {
    if (!ctx || !hash_per_s || !copy_bytes_per_s) return IM_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const size_t bytes = (size_t)1 << 30;
    void *a = nullptr, *b = nullptr, *k = nullptr;
    im_status rc = dev_alloc(ctx, bytes, &a);
    if (rc == IM_OK) rc = dev_alloc(ctx, bytes, &b);
    if (rc == IM_OK) rc = dev_alloc(ctx, 72 * 8, &k);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == IM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(ctx, IM_EDEVICE, "hipEventCreate failed");
    double best_hash = 0, best_copy = 0;
    if (rc == IM_OK) {
        k_sketch_keys<<<1, 128, 0, st>>>(1, 72, static_cast<uint64_t *>(k));
        (void)hipMemsetAsync(a, 0x5A, bytes, st);
        const unsigned blocks = 256 * 8, iters = 64;
        const uint64_t T = (uint64_t)std::ldexp(0.037, 64);
        for (int rep = 0; rep < 4; ++rep) {
            (void)hipEventRecord(e0, st);
            k_probe_hash<<<blocks, 256, 0, st>>>(static_cast<uint64_t *>(k), iters, T,
                                                 static_cast<unsigned long long *>(b));
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep && ms > 0) best_hash = std::max(best_hash, (double)blocks * 256 * iters * 64 / (ms * 1e-3));
        }
        const uint64_t cnt = bytes / 16;
        for (int rep = 0; rep < 4; ++rep) {
            (void)hipEventRecord(e0, st);
            k_probe_copy<<<256 * 16, 256, 0, st>>>(static_cast<const uint4 *>(a), static_cast<uint4 *>(b), cnt);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep && ms > 0) best_copy = std::max(best_copy, 2.0 * bytes / (ms * 1e-3));
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(ctx, IM_EDEVICE, std::string("probe: ") + hipGetErrorString(e));
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    dev_free(ctx, a, bytes);
    dev_free(ctx, b, bytes);
    dev_free(ctx, k, 72 * 8);
    if (rc != IM_OK) return rc;
    *hash_per_s = best_hash;
    *copy_bytes_per_s = best_copy;
    return IM_OK;
}

extern "C" im_status im_probe_random(im_ctx *ctx, double *reads_per_s) {
    if (!ctx || !reads_per_s) return IM_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const size_t bytes = (size_t)4 << 30;  // far beyond L2 and the 256 MB last-level cache
    void *a = nullptr, *b = nullptr;
    im_status rc = dev_alloc(ctx, bytes, &a);
    if (rc == IM_OK) rc = dev_alloc(ctx, 256, &b);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == IM_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(ctx, IM_EDEVICE, "hipEventCreate failed");
    double best = 0;
    if (rc == IM_OK) {
        (void)hipMemsetAsync(a, 0x01, bytes, st);
        const unsigned blocks = 256 * 8;
        const uint32_t per = 256;
        for (int rep = 0; rep < 4; ++rep) {
            (void)hipEventRecord(e0, st);
            k_probe_gather<<<blocks, 256, 0, st>>>(static_cast<const uint32_t *>(a), bytes / 4, per,
                                                   static_cast<unsigned long long *>(b));
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep && ms > 0) best = std::max(best, (double)blocks * 256 * per / (ms * 1e-3));
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) rc = fail(ctx, IM_EDEVICE, std::string("probe: ") + hipGetErrorString(e));
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(st);
    dev_free(ctx, a, bytes);
    dev_free(ctx, b, 256);
    if (rc != IM_OK) return rc;
    *reads_per_s = best;
    return IM_OK;
}

// ---------------------------------------------------------------- batched selection
namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }


uint32_t cov_slots(uint32_t R, uint32_t k) {
    uint64_t need = 2ull * R * std::max<uint32_t>(k, 1) + 64;
    uint32_t c = 64;
    while (c < need) c <<= 1;
    return c;
}

uint64_t prep_items(const BatchQuery &B) {
    return std::max<uint64_t>((B.n + kWave - 1) / kWave, ((uint64_t)B.cov_mask + 1 + kWave - 1) / kWave);
}

// Whole-GPU preparation before a selection launch: plan (prep per query, counter
// rearmed), initial keys / every marginal, then the trees level by level.
// pre_levels[j * stride + q] are the device prefix sums of tree level j (host copy
// in host_levels, used for the launch sizes).
void enqueue_prepare(BatchQuery *dq, uint32_t nq, const uint64_t *pre_prep, uint64_t tot_prep,
                     const uint64_t *pre_levels, const uint64_t *host_levels, uint32_t Dmax, uint32_t stride,
                     uint32_t *next_q, hipStream_t st) {
    k_bat_plan<<<(nq + 255) / 256, 256, 0, st>>>(dq, nq, next_q);
    if (tot_prep) k_bat_prepare<<<wave_grid(tot_prep, 16384), 256, 0, st>>>(dq, nq, pre_prep);
    for (uint32_t j = 0; j < Dmax; ++j) {
        const uint64_t tot = host_levels[(size_t)j * stride + nq];
        if (tot) k_bat_tree_level<<<wave_grid(tot, 16384), 256, 0, st>>>(dq, nq, pre_levels + (size_t)j * stride, j);
    }
}

}  // namespace

namespace {

// Full-label queries of a batch: one arena, the build and selection kernels in one
// hipGraph.  The instantiated graph is kept by the context together with the
// signature of its launches (arena address, grid sizes, configuration); a later
// batch whose launches have the same signature replays it without capturing
// again.  Results go to seeds[q] / gains[q]; *ms gets the launch's device time.
im_status run_full_batch(im_ctx *ctx, const std::vector<const im_query *> &queries, const im_batch_config &c,
                         std::vector<std::vector<uint32_t>> &seeds, std::vector<std::vector<uint64_t>> &gains,
                         float *ms_out) {
    const uint32_t nq = (uint32_t)queries.size();
    hipStream_t st = ctx->stream;
    im_status rc = IM_OK;

    // one arena for every query's arrays
    std::vector<BatchQuery> hq(nq);
    size_t total = 0;
    auto take = [&](size_t bytes) { size_t o = total; total += align256(bytes); return o; };
    struct Off { size_t K, E, gain0, parent, cnt, key, in_s, ids, fr, evl, cov, seeds, gains, evals; };
    std::vector<Off> off(nq);
    for (uint32_t q = 0; q < nq; ++q) {
        const im_query &Q = *queries[q];
        const uint32_t n = Q.graph->n, R = Q.R, k = std::max<uint32_t>(Q.k, 1);
        TreeDesc td = make_tree(n);
        const uint64_t tn = tree_nodes(td);
        Off &o = off[q];
        o.K = take((size_t)key_slots(R) * 8);
        o.E = take((size_t)n * R * 8);
        o.gain0 = take((size_t)n * 8);
        o.parent = take((size_t)n * R * 4);
        o.cnt = take((size_t)n * R * 4);
        o.key = take((size_t)n * 8);
        o.in_s = take(n);
        o.ids = take(tn * 4);
        o.fr = take(tn * 4);
        o.evl = take((size_t)n * 4);
        o.cov = take((size_t)cov_slots(R, Q.k) * 8);
        o.seeds = take((size_t)k * 4);
        o.gains = take((size_t)k * 8);
        o.evals = take((size_t)k * 4);
        BatchQuery &B = hq[q];
        B = BatchQuery{};
        B.n = n;
        B.R = R;
        B.k = Q.k;
        B.kb = std::max<uint32_t>(1, bit_length((uint64_t)n - 1));
        B.m = Q.graph->m_und;
        B.edges = Q.graph->edges;
        B.iedges = Q.graph->iedges;
        B.newid = Q.graph->newid;
        B.iperm = Q.graph->iperm;
        B.pm = prob_dev(Q.prob, Q.graph->off);
        B.cov_mask = cov_slots(R, Q.k) - 1;
        B.td = td;
    }
    const size_t desc_at = take(sizeof(BatchQuery) * nq);
    uint32_t Dmax = 0;
    for (uint32_t q = 0; q < nq; ++q) Dmax = std::max(Dmax, hq[q].td.D);
    const uint32_t npre = 4 + Dmax;  // (sketch, vertex), hook items, tiles, prepare items, tree levels
    const size_t pre_at = take(sizeof(uint64_t) * npre * (nq + 1));
    const size_t next_at = take(64);
    const size_t order_at = take(sizeof(uint32_t) * nq);
    char *arena = nullptr;
    rc = dev_alloc(ctx, total, (void **)&arena);
    if (rc != IM_OK) return rc;
    std::vector<uint64_t> pre((size_t)npre * (nq + 1), 0);
    for (uint32_t q = 0; q < nq; ++q) {
        BatchQuery &B = hq[q];
        const Off &o = off[q];
        B.K = reinterpret_cast<uint64_t *>(arena + o.K);
        B.E = reinterpret_cast<uint2 *>(arena + o.E);
        B.gain0 = reinterpret_cast<uint64_t *>(arena + o.gain0);
        B.parent = reinterpret_cast<uint32_t *>(arena + o.parent);
        B.cnt = reinterpret_cast<uint32_t *>(arena + o.cnt);
        B.key = reinterpret_cast<uint64_t *>(arena + o.key);
        B.in_s = reinterpret_cast<uint8_t *>(arena + o.in_s);
        B.ids = reinterpret_cast<uint32_t *>(arena + o.ids);
        B.fr = reinterpret_cast<uint32_t *>(arena + o.fr);
        B.evl = reinterpret_cast<uint32_t *>(arena + o.evl);
        B.cov = reinterpret_cast<unsigned long long *>(arena + o.cov);
        B.seeds = reinterpret_cast<uint32_t *>(arena + o.seeds);
        B.gains = reinterpret_cast<unsigned long long *>(arena + o.gains);
        B.evals = reinterpret_cast<uint32_t *>(arena + o.evals);
        pre[q + 1] = pre[q] + ((((uint64_t)B.n * B.R + 3) / 4 + 63) & ~63ull);           // 4 entries each, wave-padded
        const uint64_t hook = (uint64_t)((B.R + 63) / 64) * ((B.m + kBatHookChunk - 1) / kBatHookChunk);
        pre[(nq + 1) + q + 1] = pre[(nq + 1) + q] + hook;                                   // (pass, edge chunk)
        pre[2 * (nq + 1) + q + 1] = pre[2 * (nq + 1) + q] + (B.n + kBatTile - 1) / kBatTile;    // vertex tiles
        pre[3 * (nq + 1) + q + 1] = pre[3 * (nq + 1) + q] + prep_items(B);                       // prepare items
        for (uint32_t j = 0; j < Dmax; ++j) {                                                        // tree level j
            const uint64_t nodes = j < B.td.D ? B.td.lvl_n[B.td.D - 1 - j] : 0;
            pre[(4 + j) * (nq + 1) + q + 1] = pre[(4 + j) * (nq + 1) + q] + nodes;
        }
        k_sketch_keys<<<grid_for(key_slots(B.R), 256, 1u << 20), 256, 0, st>>>(queries[q]->seed, key_slots(B.R),
                                                                              const_cast<uint64_t *>(B.K));
    }
    BatchQuery *dq = reinterpret_cast<BatchQuery *>(arena + desc_at);
    uint64_t *dpre = reinterpret_cast<uint64_t *>(arena + pre_at);
    uint32_t *next_q = reinterpret_cast<uint32_t *>(arena + next_at);
    uint32_t *dorder = reinterpret_cast<uint32_t *>(arena + order_at);
    // selection workgroups take the queries with the most (vertex, sketch) entries first
    std::vector<uint32_t> order(nq);
    for (uint32_t q = 0; q < nq; ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return (uint64_t)hq[a].n * hq[a].R > (uint64_t)hq[b].n * hq[b].R;
    });
    (void)hipMemcpyAsync(dorder, order.data(), sizeof(uint32_t) * nq, hipMemcpyHostToDevice, st);
    hipError_t e1 = hipMemcpyAsync(dq, hq.data(), sizeof(BatchQuery) * nq, hipMemcpyHostToDevice, st);
    hipError_t e2 = hipMemcpyAsync(dpre, pre.data(), pre.size() * 8, hipMemcpyHostToDevice, st);
    hipError_t e3 = hipStreamSynchronize(st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        dev_free(ctx, arena, total);
        return fail(ctx, IM_EDEVICE, "batched setup copy failed");
    }
    const uint64_t tot_vn = pre[nq], tot_hook = pre[2 * nq + 1], tot_tiles = pre[3 * nq + 2];
    const uint64_t tot_prep = pre[4 * nq + 3];
    const unsigned g_init = grid_for(tot_vn, 256, 256 * 64);
    const unsigned g_hook = c.hook_grid ? c.hook_grid : (unsigned)std::min<uint64_t>(std::max<uint64_t>(tot_hook, 1), 16384);
    const unsigned g_comp = grid_for(tot_tiles * kWave, 256, 256 * 32);  // one wave per tile
    const unsigned g_emit = g_comp;
    const unsigned g_sel = c.select_grid ? c.select_grid : std::min<uint32_t>(nq, 256);

    // signature of every launch the graph holds: the arena address fixes every
    // pointer argument, the rest fixes the grids
    std::vector<uint64_t> sig = {(uint64_t)(uintptr_t)arena, total, nq, Dmax, g_init, g_hook, g_comp, g_emit, g_sel,
                                 c.hook_block, c.select_block, tot_prep};
    for (uint32_t j = 0; j < Dmax; ++j) sig.push_back(pre[(size_t)(4 + j) * (nq + 1) + nq]);
    hipGraphExec_t exec = nullptr;
    if (ctx->batch_exec && ctx->batch_sig == sig) {
        exec = static_cast<hipGraphExec_t>(ctx->batch_exec);
        ++ctx->batch_replays;
    } else {
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(st, hipStreamCaptureModeGlobal) != hipSuccess) {
            rc = fail(ctx, IM_EDEVICE, "hipStreamBeginCapture failed");
        } else {
            k_bat_init<<<g_init, 256, 0, st>>>(dq, nq, dpre, next_q);
            k_bat_hook<<<g_hook, c.hook_block, 0, st>>>(dq, nq, dpre + (nq + 1));
            k_bat_compress<<<g_comp, 256, 0, st>>>(dq, nq, dpre + 2 * (nq + 1));
            k_bat_emit<<<g_emit, 256, 0, st>>>(dq, nq, dpre + 2 * (nq + 1));
            // selection phases: the whole GPU prepares keys and trees (new queries; queries
            // paused before a round predicted to re-evaluate nearly every vertex), then one
            // workgroup per query runs rounds until done or until the next such round
            for (int phase = 0; phase < 3; ++phase) {
                enqueue_prepare(dq, nq, dpre + 3 * (nq + 1), tot_prep, dpre + 4 * (nq + 1),
                                pre.data() + 4 * (nq + 1), Dmax, nq + 1, next_q, st);
                k_bat_select<<<g_sel, c.select_block, 0, st>>>(dq, nq, dorder, next_q, 0xFFFFFFFFu,
                                                                phase < 2 ? 1u : 0u);
            }
            hipError_t ec = hipStreamEndCapture(st, &graph);
            if (ec != hipSuccess || !graph) rc = fail(ctx, IM_EDEVICE, std::string("capture: ") + hipGetErrorString(ec));
            else if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
                rc = fail(ctx, IM_EDEVICE, "hipGraphInstantiate failed");
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (rc == IM_OK) {
            if (ctx->batch_exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(ctx->batch_exec));
            ctx->batch_exec = exec;
            ctx->batch_sig = sig;
            ++ctx->batch_captures;
        }
    }
    hipEvent_t t0 = nullptr, t1 = nullptr;
    float ms = 0.f;
    if (rc == IM_OK) {
        (void)hipEventCreate(&t0);
        (void)hipEventCreate(&t1);
        (void)hipEventRecord(t0, st);
        hipError_t el = hipGraphLaunch(exec, st);
        (void)hipEventRecord(t1, st);
        hipError_t es = hipStreamSynchronize(st);
        if (el != hipSuccess || es != hipSuccess)
            rc = fail(ctx, IM_EDEVICE, std::string("batched launch: ") + hipGetErrorString(el != hipSuccess ? el : es));
        else (void)hipEventElapsedTime(&ms, t0, t1);
    }
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    // results
    if (rc == IM_OK) {
        std::vector<BatchQuery> back(nq);
        if (hipMemcpy(back.data(), dq, sizeof(BatchQuery) * nq, hipMemcpyDeviceToHost) != hipSuccess)
            rc = fail(ctx, IM_EDEVICE, "batched result copy failed");
        for (uint32_t q = 0; q < nq && rc == IM_OK; ++q) {
            if (back[q].err || back[q].rounds_done != queries[q]->k) {
                rc = fail(ctx, IM_EINTERNAL, "batched selection consistency check failed for query " + std::to_string(q));
                break;
            }
        }
        std::vector<unsigned long long> gtmp;
        for (uint32_t q = 0; q < nq && rc == IM_OK; ++q) {
            const uint32_t k = queries[q]->k;
            seeds[q].resize(k);
            gains[q].resize(k);
            gtmp.resize(k);
            if (!k) continue;
            if (hipMemcpy(seeds[q].data(), hq[q].seeds, (size_t)k * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(gtmp.data(), hq[q].gains, (size_t)k * 8, hipMemcpyDeviceToHost) != hipSuccess)
                rc = fail(ctx, IM_EDEVICE, "batched result copy failed");
            for (uint32_t i = 0; i < k; ++i) gains[q][i] = gtmp[i];
        }
    }
    dev_free(ctx, arena, total);
    if (rc == IM_OK && ms_out) *ms_out = ms;
    return rc;
}

bool query_is_compact(const im_query &q) { return q.alpha > 0.0 && q.alpha < 1.0; }

}  // namespace

extern "C" im_status im_select_seeds_batched(im_ctx *ctx, uint32_t nq, const im_query *queries,
                                             const im_batch_config *cfg, uint32_t *const *seeds_out,
                                             uint64_t *const *gains_out, double *device_ms) {
    if (!ctx || (nq && (!queries || !seeds_out || !gains_out))) return IM_EINVAL;
    if (nq == 0) return IM_OK;
    im_batch_config c{256, 0, 1024, 0};
    if (cfg) {
        if (cfg->hook_block) c.hook_block = cfg->hook_block;
        if (cfg->hook_grid) c.hook_grid = cfg->hook_grid;
        if (cfg->select_block) c.select_block = cfg->select_block;
        if (cfg->select_grid) c.select_grid = cfg->select_grid;
    }
    if (c.hook_block % 64 || c.hook_block > 1024 || c.select_block % 64 || c.select_block > 1024)
        return fail(ctx, IM_EINVAL, "block sizes must be multiples of 64 and at most 1024");
    std::vector<const im_query *> full, compact;
    std::vector<uint32_t> full_idx, compact_idx;
    for (uint32_t q = 0; q < nq; ++q) {
        const im_query &Q = queries[q];
        if (!Q.graph || Q.graph->ctx != ctx) return fail(ctx, IM_EINVAL, "query graph belongs to another context");
        if (Q.R == 0) return fail(ctx, IM_EINVAL, "R must be >= 1");
        if (Q.k > Q.graph->n) return fail(ctx, IM_EINVAL, "k exceeds n");
        if (!seeds_out[q] || !gains_out[q]) return fail(ctx, IM_EINVAL, "null output array");
        if (const char *why = prob_problem(Q.prob)) return fail(ctx, IM_EINVAL, why);
        if (Q.prob.kind == IM_PROB_PER_EDGE)
            return fail(ctx, IM_EINVAL, "per-edge probabilities are not supported in batched queries");
        if (!(Q.alpha >= 0.0 && Q.alpha <= 1.0)) return fail(ctx, IM_EINVAL, "alpha must lie in [0, 1]");
        const uint32_t kb = std::max<uint32_t>(1, bit_length((uint64_t)Q.graph->n - 1));
        if (kb + bit_length((uint64_t)Q.R * Q.graph->n + 1) > 64) return fail(ctx, IM_EINVAL, "R*n too large");
        if (query_is_compact(Q)) {
            if ((uint64_t)Q.R * Q.graph->n >= (1ull << kPartialShift) || Q.R >= (1u << (64 - kPartialShift)))
                return fail(ctx, IM_EINVAL, "CompactSketch needs R*n < 2^40 and R < 2^24");
            compact.push_back(&Q);
            compact_idx.push_back(q);
        } else {
            full.push_back(&Q);
            full_idx.push_back(q);
        }
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    std::vector<std::vector<uint32_t>> seeds(nq);
    std::vector<std::vector<uint64_t>> gains(nq);
    double total_ms = 0.0;
    if (!full.empty()) {
        std::vector<std::vector<uint32_t>> fs(full.size());
        std::vector<std::vector<uint64_t>> fg(full.size());
        float ms = 0.f;
        const im_status rc = run_full_batch(ctx, full, c, fs, fg, &ms);
        if (rc != IM_OK) return rc;
        for (size_t i = 0; i < full.size(); ++i) {
            seeds[full_idx[i]].swap(fs[i]);
            gains[full_idx[i]].swap(fg[i]);
        }
        total_ms += ms;
    }
    for (size_t i = 0; i < compact.size(); ++i) {
        const im_query &Q = *compact[i];
        im_sketches *sk = nullptr;
        im_status rc = im_build_sketches(ctx, Q.graph, Q.prob, Q.R, Q.seed, Q.alpha, &sk);
        if (rc != IM_OK) return rc;
        std::vector<uint32_t> &s = seeds[compact_idx[i]];
        std::vector<uint64_t> &g = gains[compact_idx[i]];
        s.resize(std::max<uint32_t>(Q.k, 1));
        g.resize(std::max<uint32_t>(Q.k, 1));
        rc = Q.k ? im_select_seeds_from(ctx, sk, Q.k, s.data(), g.data()) : IM_OK;
        total_ms += sk->build_ms + sk->select_ms;
        im_sketches_free(sk);
        if (rc != IM_OK) return rc;
    }
    for (uint32_t q = 0; q < nq; ++q)
        for (uint32_t i = 0; i < queries[q].k; ++i) {
            seeds_out[q][i] = seeds[q][i];
            gains_out[q][i] = gains[q][i];
        }
    if (device_ms) *device_ms = total_ms;
    return IM_OK;
}

// ---------------------------------------------------------------- serving
#include "server.h"
