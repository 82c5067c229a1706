// Serving: a request loop over resident graphs with continuous batching.
//
// Requests (an im_query: graph, model, R, k, sampling seed, label kind) arrive at
// any time (im_server_submit).  Two worker threads own the device work.
//
// The full-label worker:
//   - admission: a request takes a free query slot when the sketch set it needs
//     is cached or fits the HBM budget (least recently used unreferenced sets are
//     evicted first); requests wait in arrival order otherwise;
//   - sketch sets (full labels, keyed by graph, the model's device thresholds, R
//     and the sampling seed) are built on a build stream and stay resident,
//     shared by every request that uses them: selection never modifies them
//     (covered components live in each request's own set of (sketch, label)
//     pairs);
//   - steps: one launch of the batched selection kernel advances every admitted
//     request whose sketches are ready by up to rounds_per_step rounds, one
//     workgroup per request; a request whose next round would re-evaluate nearly
//     every vertex pauses, and the next step first evaluates all its vertices
//     over the whole GPU.  Requests join and leave between steps, so requests
//     that arrive while others run are admitted as slots and memory free up, and
//     builds overlap the selection steps on the device;
//   - a build that fails on the device fails every request waiting on its set
//     (IM_EDEVICE), and the set leaves the cache.
//
// The CompactSketch worker answers requests with 0 < alpha < 1 one at a time
// through the single-query build and selection on a context and stream of its
// own, capped at compact_budget, while the full-label steps go on.  Their
// selection modifies the sketch triple (MarkSeed), so their sets are built per
// request and freed after it.
//
// Each result equals what the request's im_query gets alone.
#pragma once

#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <mutex>
#include <thread>

namespace {

using srv_clock = std::chrono::steady_clock;

struct SrvSet {
    uint32_t g = 0, R = 0;
    uint64_t seed = 0;
    ProbDev pm{};           // the model as the kernels see it (thresholds), the cache key with g, R, seed
    bool failed = false;    // its build failed on the device: no longer shared, freed once unreferenced
    uint64_t *K = nullptr;
    uint2 *E = nullptr;
    uint64_t *gain0 = nullptr;
    void *block = nullptr;
    size_t bytes = 0;
    int refs = 0;
    uint64_t stamp = 0;
    hipEvent_t ready = nullptr;
};

struct SrvTicket {
    uint64_t id = 0;
    uint32_t g = 0, R = 0, k = 0;
    uint64_t seed = 0;
    double alpha = 1.0;
    bool compact = false;
    im_prob prob{};
    srv_clock::time_point t0, t1;
    bool done = false;
    im_status status = IM_OK;
    std::vector<uint32_t> seeds;
    std::vector<uint64_t> gains;
};

struct SrvSlot {
    SrvTicket *t = nullptr;
    SrvSet *set = nullptr;
    BatchQuery q{};
    // device arrays of this slot
    uint64_t *key = nullptr;
    uint8_t *in_s = nullptr;
    uint32_t *ids = nullptr, *fr = nullptr, *evl = nullptr, *seeds = nullptr, *evals = nullptr;
    unsigned long long *cov = nullptr, *gains = nullptr;
};

// First-fit sub-allocator over one device block, freed ranges coalesced.  The
// server takes all its sketch-set memory at creation: hipMalloc / hipFree in the
// request path would synchronise the device with every queued build.
struct SrvPool {
    char *base = nullptr;
    size_t size = 0;
    std::map<size_t, size_t> free_;  // offset -> length
    void init(void *b, size_t sz) {
        base = static_cast<char *>(b);
        size = sz;
        free_.clear();
        if (sz) free_[0] = sz;
    }
    void *alloc(size_t bytes) {
        bytes = align256(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > bytes) free_[off + bytes] = len - bytes;
            return base + off;
        }
        return nullptr;
    }
    void release(void *p, size_t bytes) {
        bytes = align256(bytes);
        size_t off = static_cast<char *>(p) - base;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
};

size_t set_bytes(uint32_t n, uint32_t R) {
    return align256((size_t)key_slots(R) * 8) + align256((size_t)n * R * 8) + align256((size_t)n * 8);
}

// Device bytes a CompactSketch request needs at most (im_build_sketches and its
// selection with one sketch per labelling pass), with rho taken 6 standard
// deviations above alpha * n.
size_t compact_need_bytes(uint32_t n, uint32_t R, double alpha) {
    const double mean = alpha * n;
    const size_t rho = std::min<size_t>(n, (size_t)(mean + 6.0 * std::sqrt(mean * (1.0 - alpha) + 1.0) + 64.0));
    const size_t nw = (n + 63) / 64;
    uint32_t memo = 64;
    while (memo < n && memo < 4096) memo <<= 1;
    const uint64_t tn = tree_nodes(make_tree(n));
    const size_t per_slot = (size_t)n * 4 + (size_t)((n + 31) / 32) * 4;
    const size_t slots = std::max<size_t>(1, std::min<size_t>(64, ((size_t)256 << 20) / per_slot));
    const size_t one_pass = sketch_stride(n) * 4 * 4;
    return (size_t)R * rho * 8 + (size_t)R * nw * 16 + (size_t)memo * R * 16 + (size_t)R * 16 +
           (size_t)key_slots(R) * 8 + (size_t)n * 57 + rho * 4 + tn * 8 + ((size_t)1 << 25) + slots * per_slot +
           2 * one_pass + ((size_t)1 << 20);
}

bool same_model(const ProbDev &a, const ProbDev &b) {
    return a.kind == b.kind && a.t0 == b.t0 && a.t1 == b.t1 && a.t2 == b.t2 && a.ktriv == b.ktriv;
}

// Set by the tests to make the worker treat the n-th sketch-set build as failed
// on the device (PACIM_TEST_FAIL_BUILD=n); the build itself runs normally.
uint64_t forced_build_failure() {
    const char *e = getenv("PACIM_TEST_FAIL_BUILD");
    return e ? strtoull(e, nullptr, 10) : 0;
}

}  // namespace

struct im_server {
    im_ctx *ctx = nullptr;
    std::vector<const im_graph *> graphs;
    im_server_config cfg{};
    uint32_t nmax = 0;
    hipStream_t sel = nullptr, bld = nullptr;
    CCScratch cs;
    void *slab = nullptr;
    size_t slab_bytes = 0;
    void *pool_mem = nullptr;
    SrvPool pool;
    void *dev_small = nullptr;  // descriptors, order, prefix sums, counter
    size_t small_bytes = 0;
    BatchQuery *d_desc = nullptr;
    uint32_t *d_order = nullptr, *d_next = nullptr;
    uint64_t *d_pre = nullptr;
    std::vector<SrvSlot> slots;
    std::list<SrvSet *> sets;
    size_t sets_bytes = 0, sets_budget = 0, peak = 0;
    uint64_t stamp = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<SrvTicket *> pending;
    std::map<uint64_t, SrvTicket *> tickets;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread worker;
    im_server_counters stats{};
    uint64_t fail_build = 0;   // forced failure of the n-th build (tests), 0: none
    // CompactSketch lane
    im_ctx *cctx = nullptr;
    size_t compact_budget = 0;
    std::deque<SrvTicket *> cpending;
    std::condition_variable cv_compact;
    std::thread cworker;
};

namespace {

void srv_free_set(im_server *sv, SrvSet *set) {
    if (set->ready) (void)hipEventDestroy(set->ready);
    sv->pool.release(set->block, set->bytes);
    sv->sets_bytes -= set->bytes;
    delete set;
}

// Finds or creates the sketch set of a request; nullptr if it cannot fit now.
// Called with sv->mu held.
SrvSet *srv_acquire_set(im_server *sv, const SrvTicket *t) {
    const im_graph *g = sv->graphs[t->g];
    const ProbDev pm = prob_dev(t->prob, g->off);
    for (SrvSet *s : sv->sets)
        if (!s->failed && s->g == t->g && s->R == t->R && s->seed == t->seed && same_model(s->pm, pm)) {
            ++s->refs;
            s->stamp = ++sv->stamp;
            ++sv->stats.cache_hits;
            return s;
        }
    const size_t need = set_bytes(g->n, t->R);
    void *mem = sv->pool.alloc(need);
    while (!mem) {  // evict least recently used unreferenced sets until a block fits
        SrvSet *victim = nullptr;
        for (SrvSet *s : sv->sets)
            if (s->refs == 0 && (!victim || s->stamp < victim->stamp)) victim = s;
        if (!victim) return nullptr;
        sv->sets.remove(victim);
        srv_free_set(sv, victim);
        ++sv->stats.evictions;
        mem = sv->pool.alloc(need);
    }
    SrvSet *s = new (std::nothrow) SrvSet();
    if (!s) {
        sv->pool.release(mem, need);
        return nullptr;
    }
    s->block = mem;
    s->g = t->g;
    s->R = t->R;
    s->seed = t->seed;
    s->pm = pm;
    s->bytes = need;
    char *b = static_cast<char *>(s->block);
    s->K = reinterpret_cast<uint64_t *>(b);
    s->E = reinterpret_cast<uint2 *>(b + align256((size_t)key_slots(t->R) * 8));
    s->gain0 = reinterpret_cast<uint64_t *>(b + align256((size_t)key_slots(t->R) * 8) + align256((size_t)g->n * t->R * 8));
    s->refs = 1;
    s->stamp = ++sv->stamp;
    sv->sets_bytes += need;
    sv->peak = std::max(sv->peak, sv->sets_bytes + sv->slab_bytes);
    // build on the build stream; selection steps wait for `ready`
    k_sketch_keys<<<grid_for(key_slots(t->R), 256, 1u << 20), 256, 0, sv->bld>>>(t->seed, key_slots(t->R), s->K);
    enqueue_full_build(sv->ctx, g, pm, s->K, t->R, sv->cs, s->E, s->gain0, sv->bld);
    (void)hipEventCreateWithFlags(&s->ready, hipEventDisableTiming);
    (void)hipEventRecord(s->ready, sv->bld);
    sv->sets.push_back(s);
    ++sv->stats.builds;
    if (sv->fail_build && sv->stats.builds == sv->fail_build) s->failed = true;  // checked once it is ready
    return s;
}

// Readiness of a set's build: hipSuccess when built, hipErrorNotReady while it
// runs, any other code when it failed (or the tests forced a failure).
hipError_t srv_set_state(const SrvSet *set) {
    const hipError_t e = hipEventQuery(set->ready);
    if (e == hipSuccess && set->failed) return hipErrorLaunchFailure;
    return e;
}

void srv_complete(im_server *sv, SrvSlot &sl, im_status st) {
    SrvTicket *t = sl.t;
    if (st == IM_OK && t->k) {
        t->seeds.resize(t->k);
        t->gains.resize(t->k);
        std::vector<unsigned long long> g(t->k);
        hipError_t e1 = hipMemcpyAsync(t->seeds.data(), sl.seeds, (size_t)t->k * 4, hipMemcpyDeviceToHost, sv->sel);
        hipError_t e2 = hipMemcpyAsync(g.data(), sl.gains, (size_t)t->k * 8, hipMemcpyDeviceToHost, sv->sel);
        hipError_t e3 = hipStreamSynchronize(sv->sel);
        if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) st = IM_EDEVICE;
        for (uint32_t i = 0; i < t->k; ++i) t->gains[i] = g[i];
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    t->status = st;
    t->t1 = srv_clock::now();
    t->done = true;
    ++sv->stats.completed;
    if (sl.set) {
        --sl.set->refs;
        sl.set->stamp = ++sv->stamp;
        if (sl.set->failed && sl.set->refs == 0) {
            // nothing may still write the block: wait for the build stream first
            (void)hipStreamSynchronize(sv->bld);
            sv->sets.remove(sl.set);
            srv_free_set(sv, sl.set);
        }
    }
    sl.t = nullptr;
    sl.set = nullptr;
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
}

void srv_admit(im_server *sv) {
    while (!sv->pending.empty()) {
        SrvSlot *free_slot = nullptr;
        for (auto &sl : sv->slots)
            if (!sl.t) { free_slot = &sl; break; }
        if (!free_slot) return;
        SrvTicket *t = sv->pending.front();
        SrvSet *set = srv_acquire_set(sv, t);
        if (!set) return;  // head of line waits for memory
        sv->pending.pop_front();
        const im_graph *g = sv->graphs[t->g];
        SrvSlot &sl = *free_slot;
        sl.t = t;
        sl.set = set;
        BatchQuery &B = sl.q;
        B = BatchQuery{};
        B.n = g->n;
        B.R = t->R;
        B.k = t->k;
        B.kb = std::max<uint32_t>(1, bit_length((uint64_t)g->n - 1));
        B.m = g->m_und;
        B.edges = g->edges;
        B.iedges = g->iedges;
        B.newid = g->newid;
        B.iperm = g->iperm;
        B.pm = prob_dev(t->prob, g->off);
        B.K = set->K;
        B.E = set->E;
        B.gain0 = set->gain0;
        B.key = sl.key;
        B.in_s = sl.in_s;
        B.ids = sl.ids;
        B.fr = sl.fr;
        B.evl = sl.evl;
        B.cov = sl.cov;
        B.cov_mask = cov_slots(t->R, t->k) - 1;
        B.seeds = sl.seeds;
        B.gains = sl.gains;
        B.evals = sl.evals;
        B.td = make_tree(g->n);
    }
}

double ms_since(srv_clock::time_point t) {
    return std::chrono::duration<double, std::milli>(srv_clock::now() - t).count();
}

void srv_worker(im_server *sv) {
    (void)hipSetDevice(sv->ctx->device);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    (void)hipEventCreate(&ev0);
    (void)hipEventCreate(&ev1);
    std::vector<BatchQuery> desc;
    std::vector<uint32_t> idx, order;
    std::vector<uint64_t> pre;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            const auto ta = srv_clock::now();
            srv_admit(sv);
            sv->stats.admit_ms += ms_since(ta);
            bool active = false;
            for (auto &sl : sv->slots) active |= sl.t != nullptr;
            if (!active) {
                if (sv->stop && sv->pending.empty()) {
                    (void)hipEventDestroy(ev0);
                    (void)hipEventDestroy(ev1);
                    return;
                }
                sv->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                continue;
            }
        }
        // requests of k = 0 finish at once
        for (auto &sl : sv->slots)
            if (sl.t && sl.t->k == 0) srv_complete(sv, sl, IM_OK);
        // one step over the requests whose sketch set is built
        desc.clear();
        idx.clear();
        bool failed_any = false;
        for (uint32_t i = 0; i < sv->slots.size(); ++i) {
            SrvSlot &sl = sv->slots[i];
            if (!sl.t || sl.t->k == 0) continue;
            const hipError_t e = srv_set_state(sl.set);
            if (e == hipErrorNotReady) continue;
            if (e != hipSuccess) {
                // the build failed: every request on this set fails, and the set is dropped
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    sl.set->failed = true;
                }
                (void)hipGetLastError();
                srv_complete(sv, sl, IM_EDEVICE);
                failed_any = true;
                continue;
            }
            desc.push_back(sl.q);
            idx.push_back(i);
        }
        if (failed_any) continue;
        if (desc.empty()) {
            const auto tw = srv_clock::now();
            bool any_built = false;
            for (auto &sl : sv->slots)
                if (sl.t && sl.set) {
                    // a failed build returns at once and is handled on the next pass
                    (void)hipEventSynchronize(sl.set->ready);
                    any_built = true;
                    break;
                }
            if (!any_built) std::this_thread::sleep_for(std::chrono::microseconds(50));
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stats.build_wait_ms += ms_since(tw);
            continue;
        }
        const auto ts = srv_clock::now();
        const uint32_t nq = (uint32_t)desc.size();
        order.resize(nq);
        for (uint32_t q = 0; q < nq; ++q) order[q] = q;
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
            return (uint64_t)desc[a].n * desc[a].R > (uint64_t)desc[b].n * desc[b].R;
        });
        // preparation work only for new queries and queries paused before a bulk round
        uint32_t Dmax = 0;
        for (uint32_t q = 0; q < nq; ++q) Dmax = std::max(Dmax, desc[q].td.D);
        const uint32_t stride = nq + 1;
        pre.assign((size_t)(1 + Dmax) * stride, 0);
        for (uint32_t q = 0; q < nq; ++q) {
            const BatchQuery &B = desc[q];
            const bool prep = !B.tree_ready || B.bulk_pending == 1;
            pre[q + 1] = pre[q] + (prep ? prep_items(B) : 0);
            for (uint32_t j = 0; j < Dmax; ++j) {
                const uint64_t nodes = (prep && j < B.td.D) ? B.td.lvl_n[B.td.D - 1 - j] : 0;
                pre[(1 + j) * stride + q + 1] = pre[(1 + j) * stride + q] + nodes;
            }
        }
        (void)hipMemcpyAsync(sv->d_desc, desc.data(), sizeof(BatchQuery) * nq, hipMemcpyHostToDevice, sv->sel);
        (void)hipMemcpyAsync(sv->d_order, order.data(), 4 * nq, hipMemcpyHostToDevice, sv->sel);
        (void)hipMemcpyAsync(sv->d_pre, pre.data(), 8 * pre.size(), hipMemcpyHostToDevice, sv->sel);
        (void)hipEventRecord(ev0, sv->sel);
        enqueue_prepare(sv->d_desc, nq, sv->d_pre, pre[nq], sv->d_pre + stride, pre.data() + stride, Dmax, stride,
                        sv->d_next, sv->sel);
        k_bat_select<<<std::min<uint32_t>(nq, 256), 1024, 0, sv->sel>>>(sv->d_desc, nq, sv->d_order, sv->d_next,
                                                                         sv->cfg.rounds_per_step, 1u);
        (void)hipEventRecord(ev1, sv->sel);
        hipError_t e0 = hipMemcpyAsync(desc.data(), sv->d_desc, sizeof(BatchQuery) * nq, hipMemcpyDeviceToHost, sv->sel);
        hipError_t e1 = hipStreamSynchronize(sv->sel);
        {
            float kms = 0.f;
            (void)hipEventElapsedTime(&kms, ev0, ev1);
            std::lock_guard<std::mutex> lk(sv->mu);
            ++sv->stats.steps;
            sv->stats.step_ms += ms_since(ts);
            sv->stats.busy_steps_ms += kms;
        }
        for (uint32_t q = 0; q < nq; ++q) {
            SrvSlot &sl = sv->slots[idx[q]];
            if (e0 != hipSuccess || e1 != hipSuccess) { srv_complete(sv, sl, IM_EDEVICE); continue; }
            sl.q.rounds_done = desc[q].rounds_done;
            sl.q.tree_ready = desc[q].tree_ready;
            sl.q.bulk_pending = desc[q].bulk_pending;
            sl.q.err = desc[q].err;
            if (sl.q.err) srv_complete(sv, sl, IM_EINTERNAL);
            else if (sl.q.rounds_done == sl.q.k) srv_complete(sv, sl, IM_OK);
        }
    }
}

// The CompactSketch lane: one request at a time, build + selection + free on the
// lane's own context and stream.
void srv_compact_worker(im_server *sv) {
    (void)hipSetDevice(sv->ctx->device);
    for (;;) {
        SrvTicket *t = nullptr;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            sv->cv_compact.wait(lk, [&] { return sv->stop || !sv->cpending.empty(); });
            if (sv->cpending.empty()) return;  // stopped and drained
            t = sv->cpending.front();
            sv->cpending.pop_front();
        }
        im_status st = IM_OK;
        std::vector<uint32_t> seeds(std::max<uint32_t>(t->k, 1));
        std::vector<uint64_t> gains(std::max<uint32_t>(t->k, 1));
        if (t->k) {
            im_sketches *sk = nullptr;
            st = im_build_sketches(sv->cctx, sv->graphs[t->g], t->prob, t->R, t->seed, t->alpha, &sk);
            if (st == IM_OK) {
                st = im_select_seeds_from(sv->cctx, sk, t->k, seeds.data(), gains.data());
                im_sketches_free(sk);
            }
        }
        std::lock_guard<std::mutex> lk(sv->mu);
        if (st == IM_OK) {
            t->seeds.assign(seeds.begin(), seeds.begin() + t->k);
            t->gains.assign(gains.begin(), gains.begin() + t->k);
        }
        t->status = st;
        t->t1 = srv_clock::now();
        t->done = true;
        ++sv->stats.completed;
        ++sv->stats.compact_completed;
        sv->cv_done.notify_all();
    }
}

}  // namespace

extern "C" im_status im_server_create(im_ctx *ctx, const im_graph *const *graphs, uint32_t ngraphs,
                                      const im_server_config *cfg, im_server **out) {
    if (!ctx || !out || ngraphs == 0 || !graphs) return IM_EINVAL;
    *out = nullptr;
    for (uint32_t i = 0; i < ngraphs; ++i)
        if (!graphs[i] || graphs[i]->ctx != ctx) return fail(ctx, IM_EINVAL, "graph belongs to another context");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    im_server *sv = new (std::nothrow) im_server();
    if (!sv) return fail(ctx, IM_ENOMEM, "host allocation");
    sv->ctx = ctx;
    sv->graphs.assign(graphs, graphs + ngraphs);
    im_server_config c{};
    if (cfg) c = *cfg;
    if (!c.hbm_budget) c.hbm_budget = (size_t)64 << 30;
    if (!c.max_active) c.max_active = 16;
    if (!c.rounds_per_step) c.rounds_per_step = 16;
    if (!c.max_R) c.max_R = 256;
    if (!c.max_k) c.max_k = 1000;
    if (!c.compact_budget) c.compact_budget = c.hbm_budget / 4;
    c.max_active = std::min<uint32_t>(c.max_active, 256);
    if (c.compact_budget >= c.hbm_budget) {
        delete sv;
        return fail(ctx, IM_EINVAL, "compact_budget must be smaller than hbm_budget");
    }
    sv->cfg = c;
    sv->compact_budget = c.compact_budget;
    sv->fail_build = forced_build_failure();
    for (auto *g : sv->graphs) sv->nmax = std::max(sv->nmax, g->n);
    im_status rc = IM_OK;
    auto bail = [&](im_status code) {
        if (sv->cctx) im_ctx_destroy(sv->cctx);
        if (sv->sel) (void)hipStreamDestroy(sv->sel);
        if (sv->bld) (void)hipStreamDestroy(sv->bld);
        cc_scratch_free(ctx, &sv->cs);
        if (sv->slab) dev_free(ctx, sv->slab, sv->slab_bytes);
        if (sv->pool_mem) dev_free(ctx, sv->pool_mem, sv->sets_budget);
        if (sv->dev_small) dev_free(ctx, sv->dev_small, sv->small_bytes);
        delete sv;
        return code;
    };
    if (rc != IM_OK) return bail(rc);
    if (hipStreamCreateWithFlags(&sv->sel, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&sv->bld, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(ctx, IM_EDEVICE, "stream creation failed"));
    // build scratch sized for the largest graph
    im_graph *gmax = nullptr;
    for (auto *g : sv->graphs)
        if (!gmax || g->n > gmax->n) gmax = const_cast<im_graph *>(g);
    if ((rc = cc_scratch_alloc(ctx, gmax, c.max_R, false, &sv->cs)) != IM_OK) return bail(rc);
    // query slots
    const uint64_t tn = tree_nodes(make_tree(sv->nmax));
    const size_t per_slot = align256((size_t)sv->nmax * 8) + align256(sv->nmax) + 2 * align256(tn * 4) +
                            align256((size_t)sv->nmax * 4) + align256((size_t)cov_slots(c.max_R, c.max_k) * 8) +
                            align256((size_t)c.max_k * 4) * 2 + align256((size_t)c.max_k * 8);
    sv->slab_bytes = per_slot * c.max_active;
    if (sv->slab_bytes + sv->cs.bytes + c.compact_budget >= c.hbm_budget)
        return bail(fail(ctx, IM_EINVAL, "hbm_budget is smaller than the query slots and the compact lane"));
    sv->sets_budget = c.hbm_budget - sv->slab_bytes - sv->cs.bytes - c.compact_budget;
    if (im_ctx_create(ctx->device, nullptr, c.compact_budget, &sv->cctx) != IM_OK)
        return bail(fail(ctx, IM_EDEVICE, "compact lane context creation failed"));
    if ((rc = dev_alloc(ctx, sv->slab_bytes, &sv->slab)) != IM_OK) return bail(rc);
    if ((rc = dev_alloc(ctx, sv->sets_budget, &sv->pool_mem)) != IM_OK) return bail(rc);
    sv->pool.init(sv->pool_mem, sv->sets_budget);
    sv->slots.resize(c.max_active);
    for (uint32_t i = 0; i < c.max_active; ++i) {
        char *b = static_cast<char *>(sv->slab) + per_slot * i;
        SrvSlot &sl = sv->slots[i];
        auto take_b = [&](size_t bytes) { char *p = b; b += align256(bytes); return p; };
        sl.key = reinterpret_cast<uint64_t *>(take_b((size_t)sv->nmax * 8));
        sl.in_s = reinterpret_cast<uint8_t *>(take_b(sv->nmax));
        sl.ids = reinterpret_cast<uint32_t *>(take_b(tn * 4));
        sl.fr = reinterpret_cast<uint32_t *>(take_b(tn * 4));
        sl.evl = reinterpret_cast<uint32_t *>(take_b((size_t)sv->nmax * 4));
        sl.cov = reinterpret_cast<unsigned long long *>(take_b((size_t)cov_slots(c.max_R, c.max_k) * 8));
        sl.seeds = reinterpret_cast<uint32_t *>(take_b((size_t)c.max_k * 4));
        sl.evals = reinterpret_cast<uint32_t *>(take_b((size_t)c.max_k * 4));
        sl.gains = reinterpret_cast<unsigned long long *>(take_b((size_t)c.max_k * 8));
    }
    sv->small_bytes = align256(sizeof(BatchQuery) * c.max_active) + align256(4 * c.max_active) +
                      align256(8 * (c.max_active + 1) * (1 + kMaxLevels)) + 256;
    if ((rc = dev_alloc(ctx, sv->small_bytes, &sv->dev_small)) != IM_OK) return bail(rc);
    char *b = static_cast<char *>(sv->dev_small);
    sv->d_desc = reinterpret_cast<BatchQuery *>(b);
    b += align256(sizeof(BatchQuery) * c.max_active);
    sv->d_order = reinterpret_cast<uint32_t *>(b);
    b += align256(4 * c.max_active);
    sv->d_pre = reinterpret_cast<uint64_t *>(b);
    b += align256(8 * (c.max_active + 1) * (1 + kMaxLevels));
    sv->d_next = reinterpret_cast<uint32_t *>(b);
    sv->worker = std::thread(srv_worker, sv);
    sv->cworker = std::thread(srv_compact_worker, sv);
    *out = sv;
    return IM_OK;
}

extern "C" im_status im_server_submit(im_server *sv, const im_query *q, uint64_t *ticket) {
    if (!sv || !q || !ticket) return IM_EINVAL;
    uint32_t graph = (uint32_t)sv->graphs.size();
    for (uint32_t i = 0; i < sv->graphs.size(); ++i)
        if (sv->graphs[i] == q->graph) { graph = i; break; }
    if (graph >= sv->graphs.size()) return IM_EINVAL;
    const uint32_t R = q->R, k = q->k, n = sv->graphs[graph]->n;
    if (R == 0 || R > sv->cfg.max_R || k > sv->cfg.max_k || k > n) return IM_EINVAL;
    if (prob_problem(q->prob) || q->prob.kind == IM_PROB_PER_EDGE) return IM_EINVAL;
    if (!(q->alpha >= 0.0 && q->alpha <= 1.0)) return IM_EINVAL;
    const bool compact = q->alpha > 0.0 && q->alpha < 1.0;
    const uint32_t kb = std::max<uint32_t>(1, bit_length((uint64_t)n - 1));
    if (kb + bit_length((uint64_t)R * n + 1) > 64) return IM_EINVAL;
    if (compact) {
        if ((uint64_t)R * n >= (1ull << kPartialShift)) return IM_EINVAL;
        if (compact_need_bytes(n, R, q->alpha) > sv->compact_budget) return IM_EBUSY;
    } else if (set_bytes(n, R) > sv->sets_budget) {
        return IM_EBUSY;  // can never fit the budget
    }
    SrvTicket *t = new (std::nothrow) SrvTicket();
    if (!t) return IM_ENOMEM;
    t->g = graph;
    t->R = R;
    t->k = k;
    t->seed = q->seed;
    t->alpha = compact ? q->alpha : 1.0;
    t->compact = compact;
    t->prob = q->prob;
    t->t0 = srv_clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
        delete t;
        return IM_EINVAL;
    }
    t->id = sv->next_id++;
    sv->tickets[t->id] = t;
    ++sv->stats.submitted;
    *ticket = t->id;
    if (compact) {
        sv->cpending.push_back(t);
        sv->cv_compact.notify_all();
    } else {
        sv->pending.push_back(t);
        sv->cv_work.notify_all();
    }
    return IM_OK;
}

extern "C" im_status im_server_poll(im_server *sv, uint64_t ticket, int *done) {
    if (!sv || !done) return IM_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return IM_EINVAL;
    *done = it->second->done ? 1 : 0;
    return IM_OK;
}

extern "C" im_status im_server_wait(im_server *sv, uint64_t ticket, uint32_t *seeds, uint64_t *gains,
                                    double *latency_ms) {
    if (!sv) return IM_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->tickets.find(ticket);
    if (it == sv->tickets.end()) return IM_EINVAL;
    SrvTicket *t = it->second;
    sv->cv_done.wait(lk, [&] { return t->done; });
    sv->tickets.erase(it);
    lk.unlock();
    im_status st = t->status;
    if (st == IM_OK) {
        if (t->k && (!seeds || !gains)) {
            delete t;
            return IM_EINVAL;
        }
        for (uint32_t i = 0; i < t->k; ++i) {
            seeds[i] = t->seeds[i];
            gains[i] = t->gains[i];
        }
        if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(t->t1 - t->t0).count();
    }
    delete t;
    return st;
}

extern "C" im_status im_server_stats(im_server *sv, im_server_counters *out) {
    if (!sv || !out) return IM_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    out->bytes_in_use = sv->sets_bytes + sv->slab_bytes + sv->cs.bytes;
    out->peak_bytes = sv->peak + sv->cs.bytes;
    out->cached_sets = (uint32_t)sv->sets.size();
    return IM_OK;
}

extern "C" im_status im_server_destroy(im_server *sv) {
    if (!sv) return IM_EINVAL;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        sv->cv_work.notify_all();
        sv->cv_compact.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    if (sv->cworker.joinable()) sv->cworker.join();
    if (sv->cctx) im_ctx_destroy(sv->cctx);
    im_ctx *ctx = sv->ctx;
    (void)hipStreamSynchronize(sv->bld);
    (void)hipStreamSynchronize(sv->sel);
    for (SrvSet *s : sv->sets) srv_free_set(sv, s);
    sv->sets.clear();
    for (auto &kv : sv->tickets) delete kv.second;
    cc_scratch_free(ctx, &sv->cs);
    dev_free(ctx, sv->slab, sv->slab_bytes);
    dev_free(ctx, sv->pool_mem, sv->sets_budget);
    dev_free(ctx, sv->dev_small, sv->small_bytes);
    (void)hipStreamDestroy(sv->sel);
    (void)hipStreamDestroy(sv->bld);
    delete sv;
    return IM_OK;
}
