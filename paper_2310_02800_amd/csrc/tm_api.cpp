// C ABI of the temporal motif library: contexts, graph ingest, motif
// compilation and the count / enumerate / batch entry points.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>

#include "tm_internal.h"

using tmo::GArgs;
using tmo::QArgs;

namespace {

thread_local std::string g_err;

tm_status fail(tm_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

tm_status hip_fail(hipError_t e, const char *what) {
    return fail(e == hipErrorOutOfMemory ? TM_E_OOM : TM_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                     \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) hipSetDevice(prev);
    }
};

void free_graph_buffers(tm_graph *g) {
    void *ptrs[] = {g->d_src, g->d_dst, g->d_tk, g->d_w, g->d_adj_t, g->d_adj_nbr, g->d_adj_eid, g->d_adj_w,
                    g->d_off_out, g->d_off_in, g->d_pos_out, g->d_pos_in, g->d_pr_nbr, g->d_pr_t, g->d_pr_pos,
                    g->d_nlab, g->d_el, g->d_adj_el, g->d_hub, g->d_samp, g->d_pr_samp};
    for (void *p : ptrs)
        if (p) hipFree(p);
}

template <typename T>
hipError_t dmalloc(T **p, int64_t count, int64_t *acc) {
    size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc((void **)p, bytes);
    if (e == hipSuccess && acc) *acc += (int64_t)bytes;
    return e;
}

// A per-call set of device buffers. Calls may run concurrently on several
// streams; each takes its own workspace for the duration of the call.
struct WsLease {
    tm_ctx *ctx;
    tm_ctx::Workspace *w = nullptr;
    explicit WsLease(tm_ctx *c) : ctx(c) {
        std::lock_guard<std::mutex> lk(ctx->ws_mu);
        for (auto &p : ctx->ws)
            if (!p->busy) { w = p.get(); break; }
        if (!w) {
            ctx->ws.emplace_back(new tm_ctx::Workspace());
            w = ctx->ws.back().get();
        }
        w->busy = true;
    }
    ~WsLease() {
        std::lock_guard<std::mutex> lk(ctx->ws_mu);
        w->busy = false;
    }
};

hipError_t ws_prepare(tm_ctx::Workspace *w, int64_t chunks, int nq) {
    hipError_t e = hipSuccess;
    if (!w->ctl) {
        e = hipMalloc(&w->ctl, tmo::CTL_WORDS * sizeof(uint64_t));
        if (e != hipSuccess) return e;
        e = hipHostMalloc(&w->h_ctl, 4096, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&w->ev0);
        if (e != hipSuccess) return e;
        e = hipEventCreate(&w->ev1);
        if (e != hipSuccess) return e;
    }
    if (nq > w->q_cap) {
        if (w->counts) hipFree(w->counts);
        if (w->qa) hipFree(w->qa);
        if (w->qctl) hipFree(w->qctl);
        if (w->h_qa) hipHostFree(w->h_qa);
        if (w->h_counts) hipHostFree(w->h_counts);
        w->counts = nullptr; w->qa = nullptr; w->qctl = nullptr; w->h_qa = nullptr; w->h_counts = nullptr;
        w->q_cap = 0;
        int cap = std::max(nq, 64);
        e = hipMalloc(&w->counts, 2 * cap * sizeof(uint64_t));  // counts, then step tallies
        if (e == hipSuccess) e = hipMalloc(&w->qctl, 2 * cap * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMalloc(&w->qa, cap * sizeof(QArgs));
        if (e == hipSuccess) e = hipHostMalloc(&w->h_qa, cap * sizeof(QArgs), hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc(&w->h_counts, 2 * cap * sizeof(uint64_t), hipHostMallocDefault);
        if (e != hipSuccess) return e;
        w->q_cap = cap;
    }
    if (chunks > w->chunk_cap) {
        if (w->chunk_cnt) hipFree(w->chunk_cnt);
        if (w->chunk_off) hipFree(w->chunk_off);
        w->chunk_cnt = w->chunk_off = nullptr;
        w->chunk_cap = 0;
        int64_t cap = std::max<int64_t>(chunks + 1, 1024);
        e = hipMalloc(&w->chunk_cnt, cap * sizeof(uint64_t));
        if (e == hipSuccess) e = hipMalloc(&w->chunk_off, cap * sizeof(uint64_t));
        if (e != hipSuccess) return e;
        w->chunk_cap = cap;
    }
    return hipSuccess;
}

void root_ids(const tm_graph *g, const tm_root_range *rr, int64_t *r0, int64_t *r1) {
    if (!rr) { *r0 = 0; *r1 = g->m; return; }
    *r0 = std::lower_bound(g->h_t.begin(), g->h_t.end(), rr->t_lo) - g->h_t.begin();
    *r1 = std::upper_bound(g->h_t.begin(), g->h_t.end(), rr->t_hi) - g->h_t.begin();
    if (*r1 < *r0) *r1 = *r0;
}

// Roots per chunk for a launch over `roots` roots: the configured size, cut
// down for small ranges so that there are about four chunks (each feeds one
// wavefront) per compute unit, but never below one root per lane.
int64_t chunk_for(const tm_ctx *ctx, const tmo::LaunchCfg &c, int64_t roots) {
    if (c.exact) return c.rch;
    const int64_t target = 4 * (int64_t)std::max(ctx->num_cus, 1);
    const int64_t want = std::max<int64_t>((roots + target - 1) / target, 64);
    return std::min(c.rch, want);
}

tmo::LaunchCfg default_cfg(const tm_ctx *ctx) {
    tmo::LaunchCfg c;
    c.rch = ctx->root_chunk;
    c.split = ctx->split;
    c.split_min = ctx->split_min;
    c.leaf_min = ctx->leaf_min;
    c.timed = ctx->profile != 0;
    return c;
}

// Fill one query's launch arguments. Delta is clamped to the time span (a
// larger window admits nothing more) and each gap to delta (consecutive gaps
// never exceed the whole window), so the kernel's window ends never overflow.
void fill_qargs(const tm_graph *g, const tm_motif *m, int64_t r0, int64_t r1, int64_t c0, int64_t rch, int fn,
                int64_t budget, int split, int64_t split_min, QArgs *q) {
    std::memset(q, 0, sizeof(*q));
    const int64_t span = g->m ? g->t_max - g->t_min : 0;
    q->r0 = r0;
    q->r1 = r1;
    q->delta = std::min<int64_t>(m->delta, span);
    for (int i = 0; i < 8; i++) q->gap[i] = std::min<int64_t>(m->gaps[i], q->delta);
    // anti-edge windows (in slots the motif's gaps leave free), clamped to the
    // time span like delta
    for (int j = 0; j < m->plan.n_anti; j++) q->gap[tmo::anti_slot(j)] = std::min<int64_t>(m->plan.anti_delta[j], span);
    q->c0 = c0;
    q->nchunks = (r1 - r0 + rch - 1) / rch;
    q->xns = (q->nchunks + 7) / 8;
    q->fn = fn;
    q->budget = budget;
    q->split = split;
    q->split_min = (int32_t)std::min<int64_t>(split_min, INT32_MAX);
    const tmo::Plan &p = m->plan;
    q->lab_mask = p.lab_mask;
    for (int v = 0; v < 8; v++) {
        q->nlab[v] = p.lab_val[v];
        q->nlab_hi[v] = p.lab_hi[v];
    }
    q->elab_mask = p.elab_mask;
    for (int i = 0; i < 8; i++) {
        q->elo[i] = p.elab_lo[i];
        q->ehi[i] = p.elab_hi[i];
    }
    q->npred = p.np;
    q->pred_mask = (int32_t)p.pred_mask();
    for (int j = 0; j < p.np; j++) {
        q->pth[j] = p.pred_th[j];
        q->pop[j] = (uint8_t)p.pred_op[j];
        q->plev[j] = (uint8_t)p.pred_lvl[j];
    }
    tmo::fill_plan_tables(p, q);
}

// XCD order: each query's slices start where the previous query's end in
// every XCD's chunk sequence; returns that sequence's length.
int64_t xcd_prefix(QArgs *q, int nq) {
    int64_t s = 0;
    for (int i = 0; i < nq; i++) {
        q[i].xs0 = s;
        s += q[i].xns;
    }
    return s;
}

GArgs base_args(const tm_ctx *ctx, const tm_graph *g, tm_ctx::Workspace *w, const tmo::LaunchCfg &c) {
    GArgs a;
    std::memset(&a, 0, sizeof(a));
    a.src = g->d_src;
    a.dst = g->d_dst;
    a.tk = g->d_tk;
    a.w = g->d_w;
    a.adj_t = g->d_adj_t;
    a.adj_nbr = g->d_adj_nbr;
    a.adj_eid = g->d_adj_eid;
    a.adj_w = g->d_adj_w;
    a.off_out = g->d_off_out;
    a.off_in = g->d_off_in;
    a.pos_out = g->d_pos_out;
    a.pos_in = g->d_pos_in;
    a.pr_nbr = g->d_pr_nbr;
    a.pr_t = g->d_pr_t;
    a.pr_pos = g->d_pr_pos;
    a.nlab = g->d_nlab;
    a.el = g->d_el;
    a.adj_el = g->d_adj_el;
    a.qa = (const QArgs *)w->qa;
    a.ctl = w->ctl;
    a.counts = w->counts;
    a.chunk_cnt = w->chunk_cnt;
    a.chunk_off = w->chunk_off;
    a.m_edges = g->m;
    a.split = c.split;
    a.leaf_min = (int32_t)c.leaf_min;
    a.xcd = ctx->xcd_order;
    if (ctx->samp_min > 0 && g->d_samp) {
        a.samp = g->d_samp;
        a.samp_min = (uint32_t)ctx->samp_min;
        a.samp_lg = g->samp_lg;
        a.pr_samp = g->d_pr_samp;
    }
    if (ctx->hub_lds && g->d_hub) {
        a.hub = g->d_hub;
        a.hub_words = g->hub_words;
        a.hub_dmin = g->hub_dmin;
    }
    return a;
}

int grid_for(tm_ctx *ctx, const tmo::Module *mod, uint32_t lds_bytes, int bpc) {
    if (ctx->grid > 0) return (int)ctx->grid;
    int per_cu = mod->max_blocks_per_cu > 0 ? mod->max_blocks_per_cu : 1;
    if (bpc > 0) per_cu = std::min(per_cu, bpc);
    if (lds_bytes > 0) per_cu = std::max(1, std::min(per_cu, (int)(tmo::kLdsPerCu / lds_bytes)));
    return std::max(1, per_cu * std::max(ctx->num_cus, 1));
}

// Launch sampler: while the kernel runs, copy its control words (root-chunk
// cursor, busy and waiting wavefronts, donated items waiting) every `period`
// microseconds on a side stream into pinned host memory, and keep the samples.
// The kernel is untouched; the samples show when the root queue drained and
// how many wavefronts were still busy after that (the tail the paper's
// relaunch-based redistribution targets, Sec. 5.2.2). Blocks until the kernel
// ends.
tm_status sample_launch(tm_ctx *ctx, tm_ctx::Workspace *w, int64_t chunks, hipStream_t stream) {
    HIP_TRY(hipEventRecord(w->tr_done, stream), "hipEventRecord");
    HIP_TRY(hipStreamWaitEvent(w->tr_stream, w->tr_go, 0), "hipStreamWaitEvent");
    std::vector<int64_t> rows;
    const auto t0 = std::chrono::steady_clock::now();
    for (int64_t k = 0; k < tmo::kTraceMaxSamples; k++) {
        const hipError_t q = hipEventQuery(w->tr_done);
        if (q != hipSuccess && q != hipErrorNotReady) return hip_fail(q, "hipEventQuery");
        const bool done = q == hipSuccess;
        HIP_TRY(hipMemcpyAsync(w->h_tr, w->ctl, tmo::CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost,
                               w->tr_stream), "sample copy");
        HIP_TRY(hipStreamSynchronize(w->tr_stream), "sample copy");
        const int64_t t = std::chrono::duration_cast<std::chrono::nanoseconds>(
                              std::chrono::steady_clock::now() - t0).count();
        const uint64_t *c = w->h_tr;
        const int64_t row[tmo::kTraceCols] = {t, (int64_t)c[tmo::CTL_CURSOR], chunks, (int64_t)c[tmo::CTL_BUSY],
                                              (int64_t)c[tmo::CTL_HUNGRY], (int64_t)c[tmo::CTL_AVAIL], done ? 1 : 0,
                                              (int64_t)c[tmo::CTL_HANDED]};
        rows.insert(rows.end(), row, row + tmo::kTraceCols);
        if (done) break;
        std::this_thread::sleep_for(std::chrono::microseconds(ctx->trace_us));
    }
    (void)hipGetLastError();  // a not-ready query is no error
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->trace.swap(rows);
    return TM_OK;
}

tm_status launch(tm_ctx *ctx, tm_ctx::Workspace *w, const tmo::Module *mod, int mode, GArgs *a,
                 hipStream_t stream, bool timed, int bpc) {
    hipFunction_t fn = mod->fn[mode];
    if (!fn) return fail(TM_E_DEVICE, "kernel variant missing from module");
    HIP_TRY(tmo::dev_fill_u64(w->ctl, 0, tmo::CTL_WORDS, stream), "reset counters");
    // cross-wavefront work donation: a zeroed item buffer, fresh queue
    // heads/tails and a new epoch so items of earlier launches never look ready
    // bit 1 of the split word: hand unstarted roots to waiting wavefronts
    if (a->split) a->split = 1 | (ctx->root_handoff ? 2 : 0);
    if (a->split && mode != tmo::MODE_STATS && a->nq > 0) {
        if (!w->items) {
            if (w->no_alloc) return fail(TM_E_DEVICE, "scratch view without an item region");
            const size_t bytes = tmo::kItemsTotal * tmo::kItemWords * sizeof(uint32_t);
            HIP_TRY(hipMalloc(&w->items, bytes), "work item buffer");
            // zeroed on the launch stream: a memset on the null stream is not
            // ordered before kernels on a non-blocking stream, and a late one
            // would erase items the kernel has already published
            HIP_TRY(tmo::dev_fill_u64((uint64_t *)w->items, 0, (int64_t)(bytes / sizeof(uint64_t)), stream),
                    "work item buffer");
        }
        HIP_TRY(tmo::dev_fill_u64(w->qctl, 0, 2 * (int64_t)a->nq, stream), "reset queues");
        a->items = w->items;
        a->qctl = w->qctl;
        a->item_cap = (uint32_t)(w->items_total / (uint64_t)a->nq);
        // launch number: a ready word of an earlier launch never equals it
        if (w->shared_epoch) {
            uint32_t ep = w->shared_epoch->fetch_add(1) + 1;
            if (ep == 0) ep = w->shared_epoch->fetch_add(1) + 1;  // 0 is a zeroed item's word
            a->epoch = ep;
        } else {
            a->epoch = ++w->epoch;
        }
    } else {
        a->items = nullptr;
        a->qctl = w->qctl;
        a->item_cap = 0;
        a->epoch = 0;
    }
    // the work-counter mode follows the byte model (full searches): no staging
    if (mode == tmo::MODE_STATS) { a->hub = nullptr; a->hub_words = 0; a->hub_dmin = 0; a->samp_min = 0; a->pr_samp = nullptr; }
    const uint32_t lds = a->hub_words * 4u;
    void *params[] = {a};
    const bool sampled = ctx->trace_us > 0 && !w->no_alloc;
    if (w->no_alloc) timed = false;
    if (sampled) {
        if (!w->tr_stream) HIP_TRY(hipStreamCreateWithFlags(&w->tr_stream, hipStreamNonBlocking), "sampler stream");
        if (!w->tr_go) HIP_TRY(hipEventCreateWithFlags(&w->tr_go, hipEventDisableTiming), "sampler event");
        if (!w->tr_done) HIP_TRY(hipEventCreateWithFlags(&w->tr_done, hipEventDisableTiming), "sampler event");
        if (!w->h_tr) HIP_TRY(hipHostMalloc((void **)&w->h_tr, tmo::CTL_WORDS * sizeof(uint64_t)), "sampler buffer");
        HIP_TRY(hipEventRecord(w->tr_go, stream), "hipEventRecord");  // after the control words are reset
    }
    if (timed) HIP_TRY(hipEventRecord(w->ev0, stream), "hipEventRecord");
    HIP_TRY(hipModuleLaunchKernel(fn, grid_for(ctx, mod, lds, bpc), 1, 1, ctx->block, 1, 1, lds, stream, params, nullptr),
            "hipModuleLaunchKernel");
    if (timed) HIP_TRY(hipEventRecord(w->ev1, stream), "hipEventRecord");
    if (sampled) return sample_launch(ctx, w, a->total_chunks, stream);
    return TM_OK;
}

tm_status check_pair(tm_ctx *ctx, const tm_graph *g, const tm_motif *m) {
    if (!ctx || !g || !m) return fail(TM_E_INVALID, "null context, graph or motif");
    if (g->ctx != ctx || m->ctx != ctx) return fail(TM_E_INVALID, "graph or motif belongs to another context");
    if (m->plan.np > 0 && !g->has_w) return fail(TM_E_INVALID, "motif has a weight predicate but the graph has no weights");
    if (m->plan.elab_mask && !g->has_edge_labels)
        return fail(TM_E_INVALID, "motif requires edge labels but the graph has none");
    if (m->plan.lab_mask && !g->has_labels)
        return fail(TM_E_INVALID, "motif requires vertex labels but the graph has none");
    return TM_OK;
}

// The generic (table-driven) matchers have no anti-edge checks: a motif with
// anti-edges runs its specialised matcher under either tier.
bool use_generic(int tier, const tmo::Plan &p) { return tier != 0 && p.n_anti == 0; }
bool use_generic(int tier, const tm_motif *m) { return use_generic(tier, m->plan); }

// The matchers of a batched launch: one per distinct structure, or under the
// generic tier one table-driven matcher per motif length (a module that never
// recompiles) plus the specialised matchers of motifs with anti-edges.
// fn[i] receives query i's matcher; `gplans` holds the generic plans that
// `plans` points to.
void batch_plans(const std::vector<const tmo::Plan *> &qp, int tier, std::vector<tmo::Plan> *gplans,
                 std::vector<const tmo::Plan *> *plans, std::vector<int> *fn) {
    gplans->clear();
    plans->clear();
    fn->assign(qp.size(), 0);
    if (tier) {
        gplans->reserve(TM_MAX_EDGES);
        for (int l = 1; l <= TM_MAX_EDGES; l++) gplans->push_back(tmo::generic_plan(l));
        for (auto &gp : *gplans) plans->push_back(&gp);
    }
    std::map<std::string, int> seen;
    for (size_t i = 0; i < qp.size(); i++) {
        if (use_generic(tier, *qp[i])) {
            (*fn)[i] = qp[i]->l - 1;
            continue;
        }
        auto it = seen.find(qp[i]->key());
        if (it == seen.end()) {
            it = seen.emplace(qp[i]->key(), (int)plans->size()).first;
            plans->push_back(qp[i]);
        }
        (*fn)[i] = it->second;
    }
}

// The module holding the kernel of `mode` for this motif and graph.
tm_status get_module(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, int tier, int mode,
                     std::shared_ptr<tmo::Module> *out) {
    std::string err;
    const tmo::Plan gp = tmo::generic_plan(m->plan.l);
    auto mod = ctx->compiler.get(use_generic(tier, m) ? gp : m->plan, g->key_bytes, ctx->block, &err,
                                 ctx->min_waves, tmo::mode_group(mode), ctx->step_form | (ctx->xcd_order << 1));
    if (!mod) return fail(TM_E_COMPILE, err);
    *out = mod;
    return TM_OK;
}

// One single-query pass in the given mode; leaves results in the workspace.
tm_status run_single(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range,
                     hipStream_t stream, int mode, tm_ctx::Workspace *w, tmo::Module *mod, const tmo::LaunchCfg &cfg,
                     int64_t budget, int64_t *chunks_out, int64_t *r0_out, double *ms_acc) {
    int64_t r0, r1;
    root_ids(g, range, &r0, &r1);
    const int64_t rch = chunk_for(ctx, cfg, r1 - r0);
    const int64_t chunks = (r1 - r0 + rch - 1) / rch;
    HIP_TRY(ws_prepare(w, chunks, 1), "workspace");
    fill_qargs(g, m, r0, r1, 0, rch, 0, budget, cfg.split, cfg.split_min, (QArgs *)w->h_qa);
    const int64_t xlen = xcd_prefix((QArgs *)w->h_qa, 1);
    HIP_TRY(hipMemcpyAsync(w->qa, w->h_qa, sizeof(QArgs), hipMemcpyHostToDevice, stream), "upload query");
    HIP_TRY(tmo::dev_fill_u64(w->counts, 0, 2, stream), "reset count and step tally");
    *chunks_out = chunks;
    *r0_out = r0;
    if (chunks == 0) return TM_OK;
    GArgs a = base_args(ctx, g, w, cfg);
    a.xlen = xlen;
    a.total_chunks = chunks;
    a.rch = (int32_t)rch;
    a.nq = 1;
    const bool timed = cfg.timed;
    tm_status s = launch(ctx, w, mod, mode, &a, stream, timed, cfg.bpc);
    if (s != TM_OK) return s;
    if (timed) {
        HIP_TRY(hipEventSynchronize(w->ev1), "hipEventSynchronize");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, w->ev0, w->ev1) == hipSuccess && ms_acc) *ms_acc += ms;
    }
    return TM_OK;
}

// ------------------------------------------------------------------ autotuning
//
// Launch settings change the speed of a launch, never its result. With
// TM_PARAM_AUTOTUNE on, the first count (or batch) of a key runs once under
// each candidate setting, checks that every trial gives the same counts, and
// keeps the fastest; later calls with the key reuse it. The key is the graph,
// the kernel module, and power-of-two buckets of the largest delta (clamped to
// the time span), of the root count and of the query count. The candidates
// are the knobs the paper's hyper-parameter study varies, in this design's
// terms (Appendix, impact of hyper-parameters): how much work a wavefront
// takes at once and whether busy lanes hand work to idle ones.

// Result slot of a query that ran out of its work budget.
constexpr uint64_t kCancelled = ~0ull;

int bitlen64(int64_t x) { return x > 0 ? 64 - __builtin_clzll((unsigned long long)x) : 0; }

std::string module_key(const tm_ctx *ctx, const tm_graph *g, const tmo::Plan &p) {
    return "S" + std::to_string(g->key_bytes) + "b" + std::to_string(ctx->block) +
           (ctx->min_waves ? "w" + std::to_string(ctx->min_waves) : std::string()) +
           (ctx->xcd_order ? "x" : "") + ":" + p.key();
}

std::string tune_key(const tm_graph *g, const std::string &mod, int64_t delta, int64_t roots, int q) {
    const int64_t span = g->m ? g->t_max - g->t_min : 0;
    char buf[160];
    std::snprintf(buf, sizeof(buf), "g%lld,%lld,%lld|d%d|r%d|q%d|", (long long)g->n, (long long)g->m,
                  (long long)span, bitlen64(std::min(delta, span)), bitlen64(roots), bitlen64(q));
    return std::string(buf) + mod;
}

std::vector<tmo::LaunchCfg> tune_candidates(const tm_ctx *ctx, int64_t roots) {
    std::vector<tmo::LaunchCfg> out;
    auto add = [&](int64_t rch, int split, int64_t smin) {
        tmo::LaunchCfg c;
        c.rch = rch;
        c.exact = true;
        c.split = split;
        c.split_min = smin;
        c.leaf_min = ctx->leaf_min;
        c.timed = true;
        out.push_back(c);
    };
    int64_t last_chunks = -1;
    for (int64_t rch : {16, 64, 256, 1024}) {
        const int64_t chunks = (roots + rch - 1) / rch;
        if (chunks == last_chunks) continue;  // same split of the roots as the previous size
        last_chunks = chunks;
        add(rch, 0, 32);
        add(rch, 1, 32);
        if (rch == 256 || (rch < 256 && chunks == 1)) {
            add(rch, 1, 2);
            add(rch, 1, 8);
            add(rch, 1, 128);
        }
    }
    return out;
}

// The tuned setting of `key`, if any.
bool tune_lookup(tm_ctx *ctx, const std::string &key, tmo::LaunchCfg *c) {
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    auto it = ctx->tune.find(key);
    if (it == ctx->tune.end()) return false;
    c->rch = it->second.rch;
    c->exact = true;
    c->split = it->second.split;
    c->split_min = it->second.split_min;
    c->leaf_min = it->second.leaf_min;
    c->bpc = it->second.bpc;
    return true;
}

void note_launch(tm_ctx *ctx, const tmo::LaunchCfg &c, bool tuned, double ms, int launches) {
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    ctx->last_cfg = c;
    ctx->last_tuned = tuned ? 1 : 0;
    if (c.timed) {
        ctx->last_ms = ms;
        ctx->last_launches = launches;
    }
}

// Run `once(cfg, &ms, &results)` under the setting for `key`: the tuned one,
// else (autotuning on) every candidate in turn, else the context's defaults.
// Reports the setting whose results are returned, whether it was tuned, and
// its kernel time (when timed).
template <class F>
tm_status run_tuned(tm_ctx *ctx, const std::string &key, int64_t roots, F &&once, std::vector<uint64_t> *res,
                    tmo::LaunchCfg *used, bool *tuned, double *ms_out) {
    tmo::LaunchCfg cfg = default_cfg(ctx);
    *tuned = false;
    if (ctx->autotune && roots > 0) {
        if (tune_lookup(ctx, key, &cfg)) {
            *tuned = true;
            cfg.timed = ctx->profile != 0;
        } else {
            std::vector<uint64_t> first;
            double best = 0;
            tmo::LaunchCfg best_c;
            bool have = false;
            auto trial = [&](const tmo::LaunchCfg &c) -> tm_status {
                double ms = 0;
                std::vector<uint64_t> r;
                tm_status st = once(c, &ms, &r);
                if (st != TM_OK) return st;
                if (!have) {
                    first = r;
                } else {
                    // a query over its work budget may be cancelled in some trials
                    // only; every count that two trials both finished must agree
                    for (size_t i = 0; i < r.size(); i++) {
                        if (first[i] == kCancelled) first[i] = r[i];
                        else if (r[i] != kCancelled && r[i] != first[i])
                            return fail(TM_E_DEVICE, "autotuning trials disagree on a count");
                    }
                }
                if (!have || ms < best) {
                    best = ms;
                    best_c = c;
                }
                have = true;
                return TM_OK;
            };
            // stage 1: roots per chunk and splitting; stage 2: half and twice
            // the best roots per chunk at its splitting setting; stage 3: the
            // closed-form threshold at the best of those
            for (const tmo::LaunchCfg &c : tune_candidates(ctx, roots)) {
                const tm_status st = trial(c);
                if (st != TM_OK) return st;
            }
            if (have) {
                const tmo::LaunchCfg base_c = best_c;
                const int64_t base_chunks = (roots + base_c.rch - 1) / base_c.rch;
                for (int64_t rch : {base_c.rch / 2, base_c.rch * 2}) {
                    if (rch < 1 || (roots + rch - 1) / rch == base_chunks) continue;
                    bool tried = false;
                    for (int64_t t : {16, 64, 256, 1024}) tried |= t == rch;
                    if (tried) continue;
                    tmo::LaunchCfg c = base_c;
                    c.rch = rch;
                    const tm_status st = trial(c);
                    if (st != TM_OK) return st;
                }
            }
            if (have) {
                const tmo::LaunchCfg base_c = best_c;
                for (int64_t lm : {int64_t(0), int64_t(128), int64_t(2048)}) {
                    if (lm == base_c.leaf_min) continue;
                    tmo::LaunchCfg c = base_c;
                    c.leaf_min = lm;
                    const tm_status st = trial(c);
                    if (st != TM_OK) return st;
                }
            }
            // stage 4: fewer workgroups per CU at the best setting (less
            // contention for the caches and the work queues; a launch with
            // little work to spread can run faster on fewer wavefronts)
            if (have) {
                const tmo::LaunchCfg base_c = best_c;
                for (int b : {3, 2}) {
                    tmo::LaunchCfg c = base_c;
                    c.bpc = b;
                    const tm_status st = trial(c);
                    if (st != TM_OK) return st;
                }
            }
            if (have) {
                std::lock_guard<std::mutex> lk(ctx->tune_mu);
                tmo::TuneEntry e;
                e.rch = best_c.rch;
                e.split = best_c.split;
                e.split_min = best_c.split_min;
                e.leaf_min = best_c.leaf_min;
                e.bpc = best_c.bpc;
                e.ms = best;
                ctx->tune[key] = e;
            }
            if (have) {
                *used = best_c;
                *tuned = true;
                *ms_out = best;
                *res = first;
                return TM_OK;
            }
        }
    }
    *used = cfg;
    *ms_out = 0;
    return once(cfg, ms_out, res);
}

}  // namespace

extern "C" {

const char *tm_last_error(void) { return g_err.c_str(); }

int32_t tm_version(void) { return 100; }

tm_status tm_create(int32_t device, tm_ctx **out) {
    if (!out) return fail(TM_E_INVALID, "out is null");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev), "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(TM_E_INVALID, "device ordinal out of range");
    DeviceGuard dg(device);
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    tm_ctx *ctx = new (std::nothrow) tm_ctx();
    if (!ctx) return fail(TM_E_OOM, "host allocation");
    ctx->device = device;
    ctx->num_cus = prop.multiProcessorCount;
    ctx->compiler.device = device;
    // the device's no-allocation scratch: its address on this device, looked
    // up once per device with the device current
    const hipError_t se = tmo::scratch_for_device(device, &ctx->scratch);
    if (se != hipSuccess) {
        delete ctx;
        return hip_fail(se, "hipGetSymbolAddress(scratch)");
    }
    *out = ctx;
    return TM_OK;
}

void tm_destroy(tm_ctx *ctx) {
    if (!ctx) return;
    DeviceGuard dg(ctx->device);
    hipDeviceSynchronize();
    for (auto &w : ctx->ws) {
        if (w->ctl) hipFree(w->ctl);
        if (w->h_ctl) hipHostFree(w->h_ctl);
        if (w->chunk_cnt) hipFree(w->chunk_cnt);
        if (w->chunk_off) hipFree(w->chunk_off);
        if (w->scan_tmp) hipFree(w->scan_tmp);
        if (w->counts) hipFree(w->counts);
        if (w->qa) hipFree(w->qa);
        if (w->qctl) hipFree(w->qctl);
        if (w->items) hipFree(w->items);
        if (w->h_qa) hipHostFree(w->h_qa);
        if (w->h_counts) hipHostFree(w->h_counts);
        if (w->ev0) hipEventDestroy(w->ev0);
        if (w->ev1) hipEventDestroy(w->ev1);
        if (w->tr_go) hipEventDestroy(w->tr_go);
        if (w->tr_done) hipEventDestroy(w->tr_done);
        if (w->tr_stream) hipStreamDestroy(w->tr_stream);
        if (w->h_tr) hipHostFree(w->h_tr);
    }
    for (auto &kv : ctx->compiler.cache)
        if (kv.second->mod) hipModuleUnload(kv.second->mod);
    delete ctx;
}

tm_status tm_set_param(tm_ctx *ctx, int32_t param, int64_t v) {
    if (!ctx) return fail(TM_E_INVALID, "null context");
    switch (param) {
    case TM_PARAM_BLOCK:
        if (v < 64 || v > 1024 || v % 64) return fail(TM_E_INVALID, "block must be a multiple of 64 in [64,1024]");
        ctx->block = (int)v;
        return TM_OK;
    case TM_PARAM_ROOT_CHUNK:
        if (v < 1 || v > (1 << 24)) return fail(TM_E_INVALID, "root chunk out of range");
        ctx->root_chunk = v;
        return TM_OK;
    case TM_PARAM_GRID:
        if (v < 0 || v > (1 << 20)) return fail(TM_E_INVALID, "grid out of range");
        ctx->grid = v;
        return TM_OK;
    case TM_PARAM_PROFILE:
        ctx->profile = v ? 1 : 0;
        return TM_OK;
    case TM_PARAM_SPLIT:
        ctx->split = v ? 1 : 0;
        return TM_OK;
    case TM_PARAM_SPLIT_MIN:
        if (v < 2) return fail(TM_E_INVALID, "split minimum must be >= 2");
        ctx->split_min = v;
        return TM_OK;
    case TM_PARAM_TIER:
        if (v != 0 && v != 1) return fail(TM_E_INVALID, "tier must be 0 or 1");
        ctx->tier = (int)v;
        return TM_OK;
    case TM_PARAM_AUTOTUNE:
        ctx->autotune = v ? 1 : 0;
        return TM_OK;
    case TM_PARAM_WORK_BUDGET:
        if (v < 0) return fail(TM_E_INVALID, "work budget must be >= 0");
        ctx->work_budget = v;
        return TM_OK;
    case TM_PARAM_MIN_WAVES:
        if (v < 0 || v > 8) return fail(TM_E_INVALID, "min waves per SIMD must be in [0, 8]");
        ctx->min_waves = (int)v;
        return TM_OK;
    case TM_PARAM_LEAF_MIN:
        if (v != 0 && (v < 32 || v > (1 << 24))) return fail(TM_E_INVALID, "leaf minimum must be 0 or in [32, 2^24]");
        ctx->leaf_min = v;
        return TM_OK;
    case TM_PARAM_TRACE_US:
        if (v != 0 && (v < 10 || v > 100000)) return fail(TM_E_INVALID, "sampling period must be 0 or 10..100000 us");
        ctx->trace_us = v;
        return TM_OK;
    case TM_PARAM_ROOT_HANDOFF:
        if (v != 0 && v != 1) return fail(TM_E_INVALID, "root handoff must be 0 or 1");
        ctx->root_handoff = (int)v;
        return TM_OK;
    case TM_PARAM_HUB_LDS:
        if (v != 0 && v != 1) return fail(TM_E_INVALID, "hub staging must be 0 or 1");
        ctx->hub_lds = (int)v;
        return TM_OK;
    case TM_PARAM_STEP_FORM:
        if (v != 0 && v != 1) return fail(TM_E_INVALID, "step form must be 0 or 1");
        ctx->step_form = (int)v;
        return TM_OK;
    case TM_PARAM_XCD_ORDER:
        if (v != 0 && v != 1) return fail(TM_E_INVALID, "XCD order must be 0 or 1");
        ctx->xcd_order = (int)v;
        return TM_OK;
    case TM_PARAM_LINE_SAMPLES:
        if (v != 0 && (v < 64 || v > (int64_t(1) << 30))) return fail(TM_E_INVALID, "line-sample threshold must be 0 or >= 64");
        ctx->samp_min = v;
        return TM_OK;
    default:
        return fail(TM_E_INVALID, "unknown parameter");
    }
}

tm_status tm_get_param(tm_ctx *ctx, int32_t param, int64_t *v) {
    if (!ctx || !v) return fail(TM_E_INVALID, "null argument");
    switch (param) {
    case TM_PARAM_BLOCK: *v = ctx->block; return TM_OK;
    case TM_PARAM_ROOT_CHUNK: *v = ctx->root_chunk; return TM_OK;
    case TM_PARAM_GRID: *v = ctx->grid; return TM_OK;
    case TM_PARAM_PROFILE: *v = ctx->profile; return TM_OK;
    case TM_PARAM_SPLIT: *v = ctx->split; return TM_OK;
    case TM_PARAM_SPLIT_MIN: *v = ctx->split_min; return TM_OK;
    case TM_PARAM_TIER: *v = ctx->tier; return TM_OK;
    case TM_PARAM_AUTOTUNE: *v = ctx->autotune; return TM_OK;
    case TM_PARAM_WORK_BUDGET: *v = ctx->work_budget; return TM_OK;
    case TM_PARAM_MIN_WAVES: *v = ctx->min_waves; return TM_OK;
    case TM_PARAM_LEAF_MIN: *v = ctx->leaf_min; return TM_OK;
    case TM_PARAM_TRACE_US: *v = ctx->trace_us; return TM_OK;
    case TM_PARAM_ROOT_HANDOFF: *v = ctx->root_handoff; return TM_OK;
    case TM_PARAM_HUB_LDS: *v = ctx->hub_lds; return TM_OK;
    case TM_PARAM_STEP_FORM: *v = ctx->step_form; return TM_OK;
    case TM_PARAM_LINE_SAMPLES: *v = ctx->samp_min; return TM_OK;
    case TM_PARAM_XCD_ORDER: *v = ctx->xcd_order; return TM_OK;
    default: return fail(TM_E_INVALID, "unknown parameter");
    }
}

tm_status tm_last_trace(tm_ctx *ctx, int64_t *out, int64_t cap, int64_t *n_out) {
    if (!ctx || !n_out || (cap > 0 && !out)) return fail(TM_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    const int64_t n = (int64_t)ctx->trace.size() / tmo::kTraceCols;
    *n_out = n;
    if (cap > 0) std::memcpy(out, ctx->trace.data(), (size_t)std::min(n, cap) * tmo::kTraceCols * sizeof(int64_t));
    return TM_OK;
}

tm_status tm_last_launch(tm_ctx *ctx, int64_t *root_chunk, int32_t *split, int64_t *split_min, int64_t *leaf_min,
                         int32_t *tuned) {
    if (!ctx) return fail(TM_E_INVALID, "null context");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    if (root_chunk) *root_chunk = ctx->last_cfg.rch;
    if (split) *split = ctx->last_cfg.split;
    if (split_min) *split_min = ctx->last_cfg.split_min;
    if (leaf_min) *leaf_min = ctx->last_cfg.leaf_min;
    if (tuned) *tuned = ctx->last_tuned;
    return TM_OK;
}

tm_status tm_tune_save(tm_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(TM_E_INVALID, "null argument");
    std::string text = "tmotif-tune 3\n";
    {
        std::lock_guard<std::mutex> lk(ctx->tune_mu);
        char buf[128];
        for (const auto &kv : ctx->tune) {
            std::snprintf(buf, sizeof(buf), " %lld %d %lld %lld %d %.6f\n", (long long)kv.second.rch,
                          kv.second.split, (long long)kv.second.split_min, (long long)kv.second.leaf_min,
                          kv.second.bpc, kv.second.ms);
            text += kv.first + buf;
        }
    }
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(TM_E_INVALID, std::string("cannot write ") + path);
    const bool ok = std::fwrite(text.data(), 1, text.size(), f) == text.size();
    if (std::fclose(f) != 0 || !ok) return fail(TM_E_INVALID, std::string("cannot write ") + path);
    return TM_OK;
}

tm_status tm_tune_load(tm_ctx *ctx, const char *path) {
    if (!ctx || !path) return fail(TM_E_INVALID, "null argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(TM_E_INVALID, std::string("cannot read ") + path);
    std::string text;
    char buf[65536];
    size_t got_bytes;
    while ((got_bytes = std::fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got_bytes);
    std::fclose(f);
    const std::string bad = std::string("not a tune table: ") + path;
    // version 2 tables have no workgroups-per-CU column (as many as fit)
    const std::string head = "tmotif-tune 3\n", head2 = "tmotif-tune 2\n";
    const bool v2 = text.compare(0, head2.size(), head2) == 0;
    if (!v2 && text.compare(0, head.size(), head) != 0) return fail(TM_E_INVALID, bad);
    std::map<std::string, tmo::TuneEntry> got;
    size_t pos = head.size();
    while (pos < text.size()) {
        size_t eol = text.find('\n', pos);
        if (eol == std::string::npos) return fail(TM_E_INVALID, bad);
        const std::string line = text.substr(pos, eol - pos);
        pos = eol + 1;
        const size_t sp = line.find(' ');
        if (sp == 0 || sp == std::string::npos) return fail(TM_E_INVALID, bad);
        long long rch = 0, smin = 0, lmin = 0;
        int split = 0, bpc = 0;
        double ms = 0;
        char tail = 0;
        const int want = v2 ? 5 : 6;
        const int got_n = v2 ? std::sscanf(line.c_str() + sp, " %lld %d %lld %lld %lf %c", &rch, &split, &smin, &lmin,
                                           &ms, &tail)
                             : std::sscanf(line.c_str() + sp, " %lld %d %lld %lld %d %lf %c", &rch, &split, &smin,
                                           &lmin, &bpc, &ms, &tail);
        if (got_n != want || rch < 1 || rch > (1 << 24) || (split != 0 && split != 1) || smin < 2 ||
            (lmin != 0 && (lmin < 32 || lmin > (1 << 24))) || bpc < 0 || bpc > 64)
            return fail(TM_E_INVALID, bad);
        tmo::TuneEntry e;
        e.rch = rch;
        e.split = split;
        e.split_min = smin;
        e.leaf_min = lmin;
        e.bpc = bpc;
        e.ms = ms;
        got[line.substr(0, sp)] = e;
    }
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    for (auto &kv : got) ctx->tune[kv.first] = kv.second;
    return TM_OK;
}

tm_status tm_tune_clear(tm_ctx *ctx, int64_t *n_removed) {
    if (!ctx) return fail(TM_E_INVALID, "null context");
    std::lock_guard<std::mutex> lk(ctx->tune_mu);
    if (n_removed) *n_removed = (int64_t)ctx->tune.size();
    ctx->tune.clear();
    return TM_OK;
}

tm_status tm_last_kernel_ms(tm_ctx *ctx, double *ms, int32_t *launches) {
    if (!ctx || !ms) return fail(TM_E_INVALID, "null argument");
    std::lock_guard<std::mutex> lk(ctx->prof_mu);
    *ms = ctx->last_ms;
    if (launches) *launches = ctx->last_launches;
    return TM_OK;
}

// ------------------------------------------------------------------- graph

// Hub-list sample table, staged in LDS by every workgroup of a mining kernel
// when TM_PARAM_HUB_LDS is on (a search index for the windows over the longest
// adjacency lists, Sec. 5.1.1). Words: [0] hub count H; [1, 1+H) list starts
// (positions in the unified adjacency, ascending); [1+H, 2+2H) sample offsets;
// [2+2H, 2+3H) log2 strides; samples (time keys) from word 2+3H rounded up to
// even. The lists are chosen longest first while the table fits kHubMaxWords.
static hipError_t build_hub_table(tm_graph *g, hipStream_t s, int64_t *acc) {
    const int64_t n = g->n;
    if (g->m < (int64_t)tmo::kHubMinLen) return hipSuccess;
    std::vector<uint32_t> oo(n + 1), oi(n + 1);
    hipError_t e = hipMemcpyAsync(oo.data(), g->d_off_out, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(oi.data(), g->d_off_in, (n + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    struct L { uint32_t len, start; };
    std::vector<L> cand;
    for (int64_t v = 0; v < n; v++) {
        if (oo[v + 1] - oo[v] >= tmo::kHubMinLen) cand.push_back({oo[v + 1] - oo[v], oo[v]});
        if (oi[v + 1] - oi[v] >= tmo::kHubMinLen) cand.push_back({oi[v + 1] - oi[v], oi[v]});
    }
    std::sort(cand.begin(), cand.end(), [](const L &a, const L &b) { return a.len != b.len ? a.len > b.len : a.start < b.start; });
    const uint32_t kw = (uint32_t)g->key_bytes / 4u;  // words per key
    std::vector<L> hubs;
    std::vector<uint32_t> lgs, cnts;
    uint32_t total = 0;
    for (const L &c : cand) {
        if (hubs.size() == tmo::kHubMaxLists) break;
        uint32_t lg = 5;
        while (((c.len + (1u << lg) - 1) >> lg) > tmo::kHubSamplesPerList) lg++;
        const uint32_t k = (c.len + (1u << lg) - 1) >> lg;
        const uint32_t H = (uint32_t)hubs.size() + 1;
        const uint32_t words = ((2 + 3 * H + 1) & ~1u) + (total + k) * kw;
        if (words > tmo::kHubMaxWords) break;
        hubs.push_back(c);
        lgs.push_back(lg);
        cnts.push_back(k);
        total += k;
    }
    if (hubs.empty()) return hipSuccess;
    const uint32_t H = (uint32_t)hubs.size();
    uint32_t dmin = hubs.back().len;
    // sort by start for the lookup; offsets follow that order
    std::vector<uint32_t> ord(H);
    for (uint32_t h = 0; h < H; h++) ord[h] = h;
    std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) { return hubs[a].start < hubs[b].start; });
    const uint32_t base = (2 + 3 * H + 1) & ~1u;
    const uint32_t words = base + total * kw;
    std::vector<uint32_t> tab(base, 0u);
    tab[0] = H;
    uint32_t off = 0;
    for (uint32_t j = 0; j < H; j++) {
        const uint32_t h = ord[j];
        tab[1 + j] = hubs[h].start;
        tab[1 + H + j] = off;
        tab[2 + 2 * H + j] = lgs[h];
        off += cnts[h];
    }
    tab[1 + 2 * H] = off;
    e = dmalloc(&g->d_hub, words, acc);
    if (e == hipSuccess) e = hipMemcpyAsync(g->d_hub, tab.data(), base * sizeof(uint32_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = tmo::dev_hub_samples(g->d_hub, base, total, g->d_adj_t, g->key_bytes, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // the host table is freed on return
    if (e != hipSuccess) return e;
    g->hub_words = words;
    g->hub_dmin = dmin;
    g->hub_lists = (int32_t)H;
    return hipSuccess;
}

tm_status tm_load_graph(tm_ctx *ctx, int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                        const float *w, uint32_t flags, tm_graph **out) {
    if (!ctx || !out) return fail(TM_E_INVALID, "null context or out");
    *out = nullptr;
    if (flags != 0) return fail(TM_E_INVALID, "unknown flags");
    if (n < 1 || n >= (int64_t(1) << 31) - 1) return fail(TM_E_INVALID, "n_nodes out of range");
    if (m < 0 || m >= (int64_t(1) << 31) - 1) return fail(TM_E_INVALID, "n_edges out of range");
    if (m > 0 && (!src || !dst || !t)) return fail(TM_E_INVALID, "null edge arrays");
    DeviceGuard dg(ctx->device);
    tm_graph *g = new (std::nothrow) tm_graph();
    if (!g) return fail(TM_E_OOM, "host allocation");
    g->ctx = ctx;
    g->device = ctx->device;
    g->n = n;
    g->m = m;
    g->has_w = w != nullptr;
    hipStream_t s = nullptr;
    auto cleanup = [&](tm_status st) {
        if (s) { hipStreamSynchronize(s); hipStreamDestroy(s); }
        free_graph_buffers(g);
        delete g;
        return st;
    };
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) { s = nullptr; return cleanup(hip_fail(e, "hipStreamCreate")); }

    // sortedness and time range on the host (the input is host memory)
    bool sorted = true;
    for (int64_t i = 1; i < m && sorted; i++) sorted = t[i - 1] <= t[i];
    g->was_sorted = sorted;

    int64_t *d_t = nullptr;
    int64_t acc = 0;
    e = dmalloc(&g->d_src, m, &acc);
    if (e == hipSuccess) e = dmalloc(&g->d_dst, m, &acc);
    if (e == hipSuccess && g->has_w) e = dmalloc(&g->d_w, m, &acc);
    if (e == hipSuccess) e = dmalloc(&d_t, m, nullptr);
    if (e != hipSuccess) { if (d_t) hipFree(d_t); return cleanup(hip_fail(e, "graph allocation")); }
    e = hipMemcpyAsync(d_t, t, m * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (sorted) {
        if (e == hipSuccess) e = hipMemcpyAsync(g->d_src, src, m * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(g->d_dst, dst, m * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g->has_w) e = hipMemcpyAsync(g->d_w, w, m * sizeof(float), hipMemcpyHostToDevice, s);
    } else {
        int32_t *s_in = nullptr, *d_in = nullptr;
        float *w_in = nullptr;
        int64_t *d_perm = nullptr;
        if (e == hipSuccess) e = dmalloc(&s_in, m, nullptr);
        if (e == hipSuccess) e = dmalloc(&d_in, m, nullptr);
        if (e == hipSuccess && g->has_w) e = dmalloc(&w_in, m, nullptr);
        if (e == hipSuccess) e = dmalloc(&d_perm, m, nullptr);
        if (e == hipSuccess) e = hipMemcpyAsync(s_in, src, m * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(d_in, dst, m * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess && g->has_w) e = hipMemcpyAsync(w_in, w, m * sizeof(float), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = tmo::dev_sort_by_time(m, d_t, d_perm, s);
        if (e == hipSuccess)
            e = tmo::dev_gather_edges(m, d_perm, s_in, d_in, w_in, g->d_src, g->d_dst, g->d_w, s);
        if (e == hipSuccess) {
            g->perm.resize(m);
            e = hipMemcpyAsync(g->perm.data(), d_perm, m * sizeof(int64_t), hipMemcpyDeviceToHost, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        hipFree(s_in); hipFree(d_in); if (w_in) hipFree(w_in); hipFree(d_perm);
    }
    g->h_t.resize(m);
    if (e == hipSuccess) e = hipMemcpyAsync(g->h_t.data(), d_t, m * sizeof(int64_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) { hipFree(d_t); return cleanup(hip_fail(e, "graph upload")); }
    g->t_min = m ? g->h_t[0] : 0;
    g->t_max = m ? g->h_t[m - 1] : 0;
    // relative times fit int32 when the span (plus the clamped window end) does
    const int64_t span = g->t_max - g->t_min;
    if (span < 0) { hipFree(d_t); return cleanup(fail(TM_E_INVALID, "time span overflows int64")); }
    g->key_bytes = span <= (int64_t)0x7ffffffe ? 4 : 8;

    // node ids in range
    uint32_t *d_bad = nullptr;
    uint32_t h_bad = 0;
    e = hipMalloc(&d_bad, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemsetAsync(d_bad, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) e = tmo::dev_check_ids(m, n, g->d_src, g->d_dst, d_bad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&h_bad, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (d_bad) hipFree(d_bad);
    if (e != hipSuccess) { hipFree(d_t); return cleanup(hip_fail(e, "id check")); }
    if (h_bad) { hipFree(d_t); return cleanup(fail(TM_E_INVALID, "node id out of range [0, n_nodes)")); }

    e = hipMalloc(&g->d_tk, std::max<int64_t>(m, 1) * g->key_bytes);
    if (e == hipSuccess) acc += std::max<int64_t>(m, 1) * g->key_bytes;
    if (e == hipSuccess) e = tmo::dev_make_keys(m, d_t, g->t_min, g->key_bytes, g->d_tk, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(d_t);
    if (e != hipSuccess) return cleanup(hip_fail(e, "time keys"));

    e = hipMalloc(&g->d_adj_t, std::max<int64_t>(2 * m, 1) * g->key_bytes);
    if (e == hipSuccess) acc += std::max<int64_t>(2 * m, 1) * g->key_bytes;
    if (e == hipSuccess) e = dmalloc(&g->d_adj_nbr, 2 * m, &acc);
    if (e == hipSuccess) e = dmalloc(&g->d_adj_eid, 2 * m, &acc);
    if (e == hipSuccess && g->has_w) e = dmalloc(&g->d_adj_w, 2 * m, &acc);
    if (e == hipSuccess) e = dmalloc(&g->d_off_out, n + 1, &acc);
    if (e == hipSuccess) e = dmalloc(&g->d_off_in, n + 1, &acc);
    if (e == hipSuccess) e = dmalloc(&g->d_pos_out, m, &acc);
    if (e == hipSuccess) e = dmalloc(&g->d_pos_in, m, &acc);
    if (e != hipSuccess) return cleanup(hip_fail(e, "adjacency allocation"));
    e = tmo::dev_build_csr(n, m, g->d_src, g->d_dst, g->d_tk, g->key_bytes, g->d_w, 0u, g->d_off_out, g->d_adj_t,
                          g->d_adj_nbr, g->d_adj_eid, g->d_adj_w, g->d_pos_out, s);
    if (e == hipSuccess)
        e = tmo::dev_build_csr(n, m, g->d_dst, g->d_src, g->d_tk, g->key_bytes, g->d_w, (uint32_t)m, g->d_off_in,
                              g->d_adj_t, g->d_adj_nbr, g->d_adj_eid, g->d_adj_w, g->d_pos_in, s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "adjacency build"));
    // the same lists sorted by (neighbour, time): out at [0, m), in at [m, 2m)
    e = dmalloc(&g->d_pr_nbr, 2 * m, &acc);
    if (e == hipSuccess) e = hipMalloc(&g->d_pr_t, std::max<int64_t>(2 * m, 1) * g->key_bytes);
    if (e == hipSuccess) acc += std::max<int64_t>(2 * m, 1) * g->key_bytes;
    if (e == hipSuccess) e = dmalloc(&g->d_pr_pos, 2 * m, &acc);
    if (e != hipSuccess) return cleanup(hip_fail(e, "pair list allocation"));
    e = tmo::dev_build_pairs(n, m, g->d_src, g->d_dst, g->d_tk, g->key_bytes, g->d_pr_nbr, g->d_pr_t, g->d_pos_out,
                             0u, g->d_pr_pos, s);
    if (e == hipSuccess)
        e = tmo::dev_build_pairs(n, m, g->d_dst, g->d_src, g->d_tk, g->key_bytes, g->d_pr_nbr + m,
                                 (char *)g->d_pr_t + m * g->key_bytes, g->d_pos_in, (uint32_t)m, g->d_pr_pos, s);
    if (e != hipSuccess) return cleanup(hip_fail(e, "pair list build"));
    e = build_hub_table(g, s, &acc);
    if (e != hipSuccess) return cleanup(hip_fail(e, "hub table build"));
    // line samples: one key per 128 bytes of keys (a cache line)
    g->samp_lg = g->key_bytes == 4 ? 5 : 4;
    {
        const int64_t ns = (2 * m + (int64_t(1) << g->samp_lg) - 1) >> g->samp_lg;
        e = hipMalloc(&g->d_samp, std::max<int64_t>(ns, 1) * g->key_bytes);
        if (e == hipSuccess) acc += std::max<int64_t>(ns, 1) * g->key_bytes;
        if (e == hipSuccess) e = tmo::dev_line_samples(ns, g->d_adj_t, g->key_bytes, g->samp_lg, g->d_samp, s);
        // and every 32nd neighbour id of the pair-sorted lists (int32: one per line)
        const int64_t np = (2 * m + 31) >> 5;
        if (e == hipSuccess) e = dmalloc(&g->d_pr_samp, np, &acc);
        if (e == hipSuccess) e = tmo::dev_line_samples(np, g->d_pr_nbr, 4, 5, g->d_pr_samp, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return cleanup(hip_fail(e, "line samples"));
    }
    g->device_bytes = acc;
    hipStreamDestroy(s);
    *out = g;
    return TM_OK;
}

void tm_free_graph(tm_graph *g) {
    if (!g) return;
    DeviceGuard dg(g->device);
    hipDeviceSynchronize();
    free_graph_buffers(g);
    delete g;
}

tm_status tm_graph_get_info(const tm_graph *g, tm_graph_info *info) {
    if (!g || !info) return fail(TM_E_INVALID, "null argument");
    info->n_nodes = g->n;
    info->n_edges = g->m;
    info->t_min = g->t_min;
    info->t_max = g->t_max;
    info->key_bytes = g->key_bytes;
    info->has_weights = g->has_w ? 1 : 0;
    info->device_bytes = g->device_bytes;
    info->was_sorted = g->was_sorted ? 1 : 0;
    info->has_labels = g->has_labels ? 1 : 0;
    info->has_edge_labels = g->has_edge_labels ? 1 : 0;
    info->hub_lists = g->hub_lists;
    info->hub_bytes = (int32_t)(g->hub_words * 4u);
    return TM_OK;
}

tm_status tm_graph_set_node_labels(tm_graph *g, const int32_t *labels) {
    if (!g || (!labels && g->n > 0)) return fail(TM_E_INVALID, "null argument");
    for (int64_t v = 0; v < g->n; v++)
        if (labels[v] < 0) return fail(TM_E_INVALID, "vertex labels must be >= 0");
    DeviceGuard dg(g->device);
    if (!g->d_nlab) HIP_TRY(dmalloc(&g->d_nlab, g->n, &g->device_bytes), "hipMalloc labels");
    if (g->n > 0) {
        HIP_TRY(hipMemcpy(g->d_nlab, labels, (size_t)g->n * sizeof(int32_t), hipMemcpyHostToDevice), "upload labels");
        // a copy from pageable memory may return before it lands; kernels on
        // non-blocking streams are not ordered after it, so wait here
        HIP_TRY(hipDeviceSynchronize(), "upload labels");
    }
    g->has_labels = true;
    return TM_OK;
}

tm_status tm_graph_set_edge_labels(tm_graph *g, const int32_t *labels) {
    if (!g || (!labels && g->m > 0)) return fail(TM_E_INVALID, "null argument");
    for (int64_t e = 0; e < g->m; e++)
        if (labels[e] < 0) return fail(TM_E_INVALID, "edge labels must be >= 0");
    DeviceGuard dg(g->device);
    // input order -> edge-id order (ids are positions after the time sort)
    std::vector<int32_t> by_id;
    const int32_t *src = labels;
    if (!g->perm.empty()) {
        by_id.resize(g->m);
        for (int64_t e = 0; e < g->m; e++) by_id[e] = labels[g->perm[e]];
        src = by_id.data();
    }
    if (!g->d_el) HIP_TRY(dmalloc(&g->d_el, std::max<int64_t>(g->m, 1), &g->device_bytes), "hipMalloc edge labels");
    if (!g->d_adj_el)
        HIP_TRY(dmalloc(&g->d_adj_el, std::max<int64_t>(2 * g->m, 1), &g->device_bytes), "hipMalloc edge labels");
    if (g->m > 0) {
        HIP_TRY(hipMemcpy(g->d_el, src, (size_t)g->m * sizeof(int32_t), hipMemcpyHostToDevice), "upload edge labels");
        HIP_TRY(hipDeviceSynchronize(), "upload edge labels");
        HIP_TRY(tmo::dev_gather_i32(2 * g->m, g->d_adj_eid, g->d_el, g->d_adj_el, nullptr), "edge labels by list");
        HIP_TRY(hipDeviceSynchronize(), "edge labels by list");
    }
    g->has_edge_labels = true;
    return TM_OK;
}

tm_status tm_graph_edge_order(const tm_graph *g, int64_t *perm_out) {
    if (!g || (!perm_out && g->m)) return fail(TM_E_INVALID, "null argument");
    for (int64_t i = 0; i < g->m; i++) perm_out[i] = g->perm.empty() ? i : g->perm[i];
    return TM_OK;
}

tm_status tm_graph_copy_csr(const tm_graph *g, int32_t dir, uint32_t *off, int32_t *nbr, int32_t *eid,
                            int64_t *t_rel) {
    if (!g || dir < 0 || dir > 3) return fail(TM_E_INVALID, "bad argument");
    DeviceGuard dg(g->device);
    const bool pair = dir >= 2;
    const int64_t m = g->m, base = (dir & 1) ? m : 0;
    if (off) HIP_TRY(hipMemcpy(off, (dir & 1) ? g->d_off_in : g->d_off_out, (g->n + 1) * sizeof(uint32_t),
                               hipMemcpyDeviceToHost), "copy offsets");
    if (m == 0) return TM_OK;
    if (nbr) HIP_TRY(hipMemcpy(nbr, (pair ? g->d_pr_nbr : g->d_adj_nbr) + base, m * sizeof(int32_t),
                               hipMemcpyDeviceToHost), "copy nbr");
    if (eid && !pair)
        HIP_TRY(hipMemcpy(eid, g->d_adj_eid + base, m * sizeof(int32_t), hipMemcpyDeviceToHost), "copy eid");
    if (eid && pair) {
        // the pair-sorted lists keep no edge ids: place each time-sorted
        // entry's id at its pair-sorted position
        std::vector<int32_t> ids(m);
        std::vector<uint32_t> pos(m);
        HIP_TRY(hipMemcpy(ids.data(), g->d_adj_eid + base, m * sizeof(int32_t), hipMemcpyDeviceToHost), "copy eid");
        HIP_TRY(hipMemcpy(pos.data(), g->d_pr_pos + base, m * sizeof(uint32_t), hipMemcpyDeviceToHost), "copy pos");
        for (int64_t i = 0; i < m; i++) {
            const int64_t p = (int64_t)pos[i] - base;
            if (p < 0 || p >= m) return fail(TM_E_DEVICE, "pair-sorted position out of range");
            eid[p] = ids[i];
        }
    }
    if (t_rel) {
        const void *src = pair ? g->d_pr_t : g->d_adj_t;
        if (g->key_bytes == 8) {
            HIP_TRY(hipMemcpy(t_rel, (const int64_t *)src + base, m * sizeof(int64_t), hipMemcpyDeviceToHost),
                    "copy t");
        } else {
            std::vector<int32_t> tmp(m);
            HIP_TRY(hipMemcpy(tmp.data(), (const int32_t *)src + base, m * sizeof(int32_t), hipMemcpyDeviceToHost),
                    "copy t");
            for (int64_t i = 0; i < m; i++) t_rel[i] = tmp[i];
        }
    }
    return TM_OK;
}

// ------------------------------------------------------------------- motif

tm_status tm_compile_motif(tm_ctx *ctx, const tm_motif_desc *desc, tm_motif **out) {
    if (!ctx || !out) return fail(TM_E_INVALID, "null context or out");
    *out = nullptr;
    if (desc && (desc->n_edges > TM_MAX_EDGES || desc->n_nodes > TM_MAX_NODES))
        return fail(TM_E_UNSUPPORTED, "motif too large (at most 8 edges and 8 nodes)");
    tm_motif *m = new (std::nothrow) tm_motif();
    if (!m) return fail(TM_E_OOM, "host allocation");
    std::string err;
    if (!tmo::build_plan(desc, &m->plan, m->gaps, &err)) {
        delete m;
        return fail(TM_E_INVALID, err);
    }
    m->ctx = ctx;
    m->delta = desc->delta;
    DeviceGuard dg(ctx->device);
    // compile eagerly for 32-bit time keys (the common case) so errors surface
    // here; with the generic tier this is the shared module of the motif length
    const tmo::Plan gp = tmo::generic_plan(m->plan.l);
    if (!ctx->compiler.get(use_generic(ctx->tier, m) ? gp : m->plan, 4, ctx->block, &err, ctx->min_waves,
                           tmo::mode_group(tmo::MODE_COUNT), ctx->step_form | (ctx->xcd_order << 1))) {
        delete m;
        return fail(TM_E_COMPILE, err);
    }
    *out = m;
    return TM_OK;
}

void tm_free_motif(tm_motif *m) { delete m; }

// Emitted HIP source of a motif's kernel (for inspection). Writes at most
// `cap` bytes including the terminator; *len gets the full length.
tm_status tm_motif_source(const tm_motif_desc *desc, int32_t key_bytes, char *buf, int64_t cap, int64_t *len) {
    tmo::Plan p;
    int64_t gaps[TM_MAX_EDGES];
    std::string err;
    if (!tmo::build_plan(desc, &p, gaps, &err)) return fail(TM_E_INVALID, err);
    if (key_bytes != 4 && key_bytes != 8) return fail(TM_E_INVALID, "key_bytes must be 4 or 8");
    std::string s = tmo::generate_source(p, key_bytes, 256);
    if (len) *len = (int64_t)s.size();
    if (buf && cap > 0) {
        int64_t n = std::min<int64_t>(cap - 1, (int64_t)s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = '\0';
    }
    return TM_OK;
}

// Compile (or find in the on-disk cache) the modules a motif's calls load:
// one per group of kernel modes, as get_module builds them at the default
// block size. *code_bytes gets their total size.
static tm_status compile_groups(const tmo::Plan &p, int32_t key_bytes, int64_t *code_bytes) {
    const unsigned groups[3] = {tmo::mode_group(tmo::MODE_COUNT), tmo::mode_group(tmo::MODE_STATS),
                                tmo::mode_group(tmo::MODE_ENUM_COUNT)};
    int64_t total = 0;
    for (unsigned gm : groups) {
        std::vector<char> code;
        std::string err;
        if (!tmo::cached_code(tmo::generate_source(p, key_bytes, tmo::kDefaultBlock, 0, gm), &code, &err))
            return fail(TM_E_COMPILE, err);
        total += (int64_t)code.size();
    }
    if (code_bytes) *code_bytes = total;
    return TM_OK;
}

tm_status tm_batch_compile_check(const tm_motif_desc *descs, int32_t q, int32_t tier, int32_t key_bytes,
                                 int64_t *code_bytes) {
    if (!descs || q < 1) return fail(TM_E_INVALID, "need at least one motif");
    if (key_bytes != 4 && key_bytes != 8) return fail(TM_E_INVALID, "key_bytes must be 4 or 8");
    if (tier != 0 && tier != 1) return fail(TM_E_INVALID, "tier must be 0 or 1");
    std::vector<tmo::Plan> plans(q);
    std::vector<const tmo::Plan *> qp(q), mods;
    for (int i = 0; i < q; i++) {
        int64_t gaps[TM_MAX_EDGES];
        std::string err;
        if (!tmo::build_plan(&descs[i], &plans[i], gaps, &err)) return fail(TM_E_INVALID, err);
        qp[i] = &plans[i];
    }
    std::vector<int> fn;
    std::vector<tmo::Plan> gplans;
    batch_plans(qp, tier, &gplans, &mods, &fn);
    std::vector<char> code;
    std::string err;
    if (!tmo::batch_code(mods, key_bytes, tmo::kDefaultBlock, 0, &code, &err)) return fail(TM_E_COMPILE, err);
    if (code_bytes) *code_bytes = (int64_t)code.size();
    return TM_OK;
}

tm_status tm_motif_compile_check(const tm_motif_desc *descs, int32_t q, int32_t key_bytes, int64_t *code_bytes) {
    if (!descs || q < 1) return fail(TM_E_INVALID, "need at least one motif");
    if (key_bytes != 4 && key_bytes != 8) return fail(TM_E_INVALID, "key_bytes must be 4 or 8");
    if (q > 1) return tm_batch_compile_check(descs, q, 0, key_bytes, code_bytes);
    tmo::Plan plan;
    {
        int64_t gaps[TM_MAX_EDGES];
        std::string err;
        if (!tmo::build_plan(&descs[0], &plan, gaps, &err)) return fail(TM_E_INVALID, err);
    }
    return compile_groups(plan, key_bytes, code_bytes);
}

tm_status tm_generic_compile_check(int32_t l, int32_t key_bytes, int64_t *code_bytes) {
    if (l < 0 || l > TM_MAX_EDGES) return fail(TM_E_INVALID, "motif length out of range");
    if (key_bytes != 4 && key_bytes != 8) return fail(TM_E_INVALID, "key_bytes must be 4 or 8");
    if (l > 0) return compile_groups(tmo::generic_plan(l), key_bytes, code_bytes);
    std::vector<tmo::Plan> gplans;
    for (int k = 1; k <= TM_MAX_EDGES; k++) gplans.push_back(tmo::generic_plan(k));
    std::vector<const tmo::Plan *> ptrs;
    for (auto &gp : gplans) ptrs.push_back(&gp);
    std::vector<char> code;
    std::string err;
    if (!tmo::batch_code(ptrs, key_bytes, tmo::kDefaultBlock, 0, &code, &err)) return fail(TM_E_COMPILE, err);
    if (code_bytes) *code_bytes = (int64_t)code.size();
    return TM_OK;
}

// ------------------------------------------------------------------ mining

tm_status tm_count(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range, hipStream_t stream,
                   uint64_t *count_out) {
    tm_status st = check_pair(ctx, g, m);
    if (st != TM_OK) return st;
    if (!count_out) return fail(TM_E_INVALID, "count_out is null");
    WsLease lease(ctx);
    return tmo::count_impl(ctx, g, m, range, ctx->tier, ctx->work_budget, stream, lease.w, count_out);
}

tm_status tm_work_stats(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range,
                        hipStream_t stream, uint64_t *stats_out) {
    tm_status st = check_pair(ctx, g, m);
    if (st != TM_OK) return st;
    if (!stats_out) return fail(TM_E_INVALID, "stats_out is null");
    DeviceGuard dg(ctx->device);
    std::shared_ptr<tmo::Module> mod;
    if ((st = get_module(ctx, g, m, ctx->tier, tmo::MODE_STATS, &mod)) != TM_OK) return st;
    WsLease lease(ctx);
    tm_ctx::Workspace *w = lease.w;
    int64_t chunks = 0, r0 = 0;
    tmo::LaunchCfg cfg = default_cfg(ctx);
    cfg.split = 0;  // the counters describe the unsplit search
    cfg.timed = false;
    st = run_single(ctx, g, m, range, stream, tmo::MODE_STATS, w, mod.get(), cfg, 0, &chunks, &r0, nullptr);
    if (st != TM_OK) return st;
    if (chunks == 0) HIP_TRY(tmo::dev_fill_u64(w->ctl, 0, tmo::CTL_WORDS, stream), "reset counters");
    HIP_TRY(hipMemcpyAsync(w->h_ctl, w->ctl, tmo::CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
            "read stats");
    HIP_TRY(hipMemcpyAsync(w->h_counts, w->counts, sizeof(uint64_t), hipMemcpyDeviceToHost, stream), "read count");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    for (int i = 0; i < 5; i++) stats_out[i] = w->h_ctl[tmo::CTL_STATS + i];
    stats_out[5] = w->h_counts[0];
    for (int i = 0; i < 3; i++) stats_out[6 + i] = w->h_ctl[tmo::CTL_LEAF + i];
    return TM_OK;
}

}  // extern "C"

namespace tmo {

tm_status count_impl(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range, int tier,
                     int64_t budget, hipStream_t stream, tm_ctx::Workspace *w, uint64_t *count_out) {
    DeviceGuard dg(ctx->device);
    std::shared_ptr<tmo::Module> mod;
    tm_status st;
    if ((st = get_module(ctx, g, m, tier, tmo::MODE_COUNT, &mod)) != TM_OK) return st;
    int64_t r0, r1, chunks = 0;
    root_ids(g, range, &r0, &r1);
    auto once = [&](const tmo::LaunchCfg &c, double *ms, std::vector<uint64_t> *res) -> tm_status {
        int64_t rr0 = 0;
        tm_status s =
            run_single(ctx, g, m, range, stream, tmo::MODE_COUNT, w, mod.get(), c, budget, &chunks, &rr0, ms);
        if (s != TM_OK) return s;
        HIP_TRY(hipMemcpyAsync(w->h_counts, w->counts, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
                "read count");
        HIP_TRY(hipMemcpyAsync(w->h_ctl, w->ctl, tmo::CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
                "read control words");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
        if (chunks && w->h_ctl[tmo::CTL_ERROR]) return fail(TM_E_DEVICE, "work item handoff timed out");
        res->assign(1, budget > 0 && (int64_t)w->h_counts[1] > budget ? kCancelled : w->h_counts[0]);
        return TM_OK;
    };
    const tmo::Plan gp = tmo::generic_plan(m->plan.l);
    const std::string key = ctx->autotune ? tune_key(g, module_key(ctx, g, use_generic(tier, m) ? gp : m->plan),
                                                     m->delta,
                                                     r1 - r0, 1)
                                          : std::string();
    std::vector<uint64_t> res;
    tmo::LaunchCfg used;
    bool tuned = false;
    double ms = 0;
    st = run_tuned(ctx, key, r1 - r0, once, &res, &used, &tuned, &ms);
    if (st != TM_OK) return st;
    note_launch(ctx, used, tuned, ms, chunks ? 1 : 0);
    if (res[0] == kCancelled) return fail(TM_E_CANCELLED, "work budget exceeded");
    *count_out = res[0];
    return TM_OK;
}


tm_status load_count_module(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, int tier) {
    DeviceGuard dg(ctx->device);
    std::shared_ptr<tmo::Module> mod;
    return get_module(ctx, g, m, tier, tmo::MODE_COUNT, &mod);
}

tm_status enumerate_impl(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range, int tier,
                         int64_t budget, hipStream_t stream, tm_ctx::Workspace *w, const RowAlloc &alloc,
                         uint64_t *n_out, int64_t **rows_out) {
    DeviceGuard dg(ctx->device);
    std::shared_ptr<tmo::Module> mod;
    tm_status st;
    if (rows_out) *rows_out = nullptr;
    if ((st = get_module(ctx, g, m, tier, tmo::MODE_ENUM_COUNT, &mod)) != TM_OK) return st;
    int64_t r0, r1;
    root_ids(g, range, &r0, &r1);
    // the setting a count of this key was tuned to, else the defaults
    tmo::LaunchCfg cfg = default_cfg(ctx);
    bool tuned = false;
    if (ctx->autotune) {
        const tmo::Plan gp = tmo::generic_plan(m->plan.l);
        tuned = tune_lookup(
            ctx, tune_key(g, module_key(ctx, g, use_generic(tier, m) ? gp : m->plan), m->delta, r1 - r0, 1), &cfg);
    }
    const int64_t rch = chunk_for(ctx, cfg, r1 - r0);  // the same split as run_single's pass
    const int64_t chunks = (r1 - r0 + rch - 1) / rch;
    HIP_TRY(ws_prepare(w, chunks, 1), "workspace");
    if (chunks == 0) {
        *n_out = 0;
        return TM_OK;
    }
    // pass 1: per-chunk counts
    HIP_TRY(tmo::dev_fill_u64(w->chunk_cnt, 0, chunks, stream), "reset chunk counts");
    int64_t c0 = 0, rr0 = 0;
    double ms = 0;
    st = run_single(ctx, g, m, range, stream, tmo::MODE_ENUM_COUNT, w, mod.get(), cfg, budget, &c0, &rr0, &ms);
    if (st != TM_OK) return st;
    // exclusive scan -> per-chunk output offsets (one extra entry: the total)
    HIP_TRY(tmo::dev_fill_u64(w->chunk_cnt + chunks, 0, 1, stream), "scan tail");
    const size_t need = (size_t)tmo::scan_tmp_elems(chunks + 1) * sizeof(uint64_t);
    if (need > w->scan_tmp_bytes) {
        if (w->scan_tmp) hipFree(w->scan_tmp);
        w->scan_tmp = nullptr;
        w->scan_tmp_bytes = 0;
        HIP_TRY(hipMalloc(&w->scan_tmp, need), "scan workspace");
        w->scan_tmp_bytes = need;
    }
    HIP_TRY(tmo::dev_exclusive_scan_u64(w->chunk_cnt, w->chunk_off, chunks + 1, (uint64_t *)w->scan_tmp, stream),
            "scan");
    HIP_TRY(hipMemcpyAsync(w->h_ctl + 64, w->chunk_off + chunks, sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
            "read total");
    HIP_TRY(hipMemcpyAsync(w->h_counts, w->counts, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
            "read count");
    HIP_TRY(hipMemcpyAsync(w->h_ctl, w->ctl, tmo::CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
            "read control words");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (w->h_ctl[tmo::CTL_ERROR]) return fail(TM_E_DEVICE, "work item handoff timed out");
    if (budget > 0 && (int64_t)w->h_counts[1] > budget) return fail(TM_E_CANCELLED, "work budget exceeded");
    const uint64_t total = w->h_ctl[64];
    if (total != w->h_counts[0]) return fail(TM_E_DEVICE, "enumeration pass 1 disagrees with its own total");
    *n_out = total;
    if (total == 0) return TM_OK;
    uint64_t capacity = 0;
    tm_status ast = TM_OK;
    int64_t *d_out = alloc(total, &capacity, &ast);
    if (!d_out || capacity < total) return ast;
    if (rows_out) *rows_out = d_out;
    // pass 2: write rows; chunk_cnt is reused as the per-chunk write cursor. It
    // repeats pass 1's search, which finished within the budget, so it has none.
    ((QArgs *)w->h_qa)->budget = 0;
    HIP_TRY(tmo::dev_fill_u64(w->chunk_cnt, 0, chunks, stream), "reset cursors");
    HIP_TRY(hipMemcpyAsync(w->qa, w->h_qa, sizeof(QArgs), hipMemcpyHostToDevice, stream), "upload query");
    HIP_TRY(tmo::dev_fill_u64(w->counts, 0, 2, stream), "reset count");
    GArgs a = base_args(ctx, g, w, cfg);
    a.xlen = ((QArgs *)w->h_qa)->xns;
    a.total_chunks = chunks;
    a.rch = (int32_t)rch;
    a.nq = 1;
    a.out = d_out;
    a.capacity = capacity;
    const bool timed = cfg.timed;
    st = launch(ctx, w, mod.get(), tmo::MODE_ENUM_WRITE, &a, stream, timed, cfg.bpc);
    if (st != TM_OK) return st;
    HIP_TRY(hipMemcpyAsync(w->h_ctl, w->ctl, tmo::CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
            "read overflow");
    HIP_TRY(hipMemcpyAsync(w->h_counts, w->counts, sizeof(uint64_t), hipMemcpyDeviceToHost, stream), "read count");
    HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (w->h_ctl[tmo::CTL_ERROR]) return fail(TM_E_DEVICE, "work item handoff timed out");
    if (timed) {
        float k = 0.f;
        if (hipEventElapsedTime(&k, w->ev0, w->ev1) == hipSuccess) ms += k;
    }
    note_launch(ctx, cfg, tuned, ms, 2);
    if (w->h_ctl[tmo::CTL_OVERFLOW] != 0 || w->h_counts[0] != total)
        return fail(TM_E_DEVICE, "enumeration pass 2 wrote a different number of rows than pass 1 counted");
    return TM_OK;
}

tm_status count_batch_impl(tm_ctx *ctx, const tm_graph *g, int32_t q, const tm_motif *const *motifs,
                           const tm_root_range *ranges, const int64_t *budgets, int tier, hipStream_t stream,
                           tm_ctx::Workspace *w, uint64_t *counts_out, uint8_t *cancelled, bool no_alloc) {
    DeviceGuard dg(ctx->device);
    std::vector<const tmo::Plan *> qp(q), plans;
    for (int i = 0; i < q; i++) qp[i] = &motifs[i]->plan;
    std::vector<int> fn;
    std::vector<tmo::Plan> gplans;
    batch_plans(qp, tier, &gplans, &plans, &fn);
    std::string err;
    std::shared_ptr<tmo::Module> mod;
    if (no_alloc) {
        mod = ctx->compiler.find_batch(plans, g->key_bytes, ctx->block, ctx->min_waves, ctx->step_form | (ctx->xcd_order << 1));
        if (!mod)
            return fail(TM_E_INVALID, "the batched kernel of these motifs is not loaded: run tm_count_batch with "
                                      "them once first");
    } else {
        mod = ctx->compiler.get_batch(plans, g->key_bytes, ctx->block, &err, ctx->min_waves, ctx->step_form | (ctx->xcd_order << 1));
        if (!mod) return fail(TM_E_COMPILE, err);
        HIP_TRY(ws_prepare(w, 0, q), "workspace");
    }
    std::vector<int64_t> rlo(q), rhi(q);
    int64_t roots = 0, dmax = 0;
    const int64_t span = g->m ? g->t_max - g->t_min : 0;
    for (int i = 0; i < q; i++) {
        root_ids(g, ranges ? &ranges[i] : nullptr, &rlo[i], &rhi[i]);
        roots += rhi[i] - rlo[i];
        dmax = std::max(dmax, motifs[i]->delta);
    }
    // Queries go into the shared chunk queue heaviest first (by roots times
    // window, a cheap estimate of their search), so the long ones start early
    // and the short ones fill in behind them.
    std::vector<int> order(q);
    for (int i = 0; i < q; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        const double wa = (double)(rhi[a] - rlo[a]) * (double)std::min(motifs[a]->delta, span);
        const double wb = (double)(rhi[b] - rlo[b]) * (double)std::min(motifs[b]->delta, span);
        return wa > wb;
    });
    // Every query of a batch takes the batch's splitting setting: once any
    // query splits, idle wavefronts poll the donation queues of all of them,
    // so settings tuned for queries alone do not carry over (measured: mixing
    // them made a 64-query batch 5x slower).
    int64_t c0 = 0;
    auto once = [&](const tmo::LaunchCfg &c, double *ms, std::vector<uint64_t> *res) -> tm_status {
        const int64_t rch = chunk_for(ctx, c, roots);
        QArgs *h = (QArgs *)w->h_qa;
        c0 = 0;
        int any_split = 0;
        for (int j = 0; j < q; j++) {
            const int i = order[j];
            fill_qargs(g, motifs[i], rlo[i], rhi[i], c0, rch, fn[i], budgets ? budgets[i] : 0, c.split,
                       c.split_min, &h[j]);
            any_split |= c.split;
            c0 += h[j].nchunks;
        }
        const int64_t xlen = xcd_prefix(h, q);
        HIP_TRY(hipMemcpyAsync(w->qa, w->h_qa, q * sizeof(QArgs), hipMemcpyHostToDevice, stream), "upload queries");
        HIP_TRY(tmo::dev_fill_u64(w->counts, 0, 2 * (int64_t)q, stream), "reset counts and step tallies");
        if (c0 > 0) {
            GArgs a = base_args(ctx, g, w, c);
            a.xlen = xlen;
            a.split = any_split;
            a.total_chunks = c0;
            a.rch = (int32_t)rch;
            a.nq = q;
            tm_status st = launch(ctx, w, mod.get(), tmo::MODE_COUNT, &a, stream, c.timed, c.bpc);
            if (st != TM_OK) return st;
            if (c.timed) {
                HIP_TRY(hipEventSynchronize(w->ev1), "hipEventSynchronize");
                float k = 0.f;
                if (hipEventElapsedTime(&k, w->ev0, w->ev1) == hipSuccess) *ms = k;
            }
        }
        HIP_TRY(hipMemcpyAsync(w->h_counts, w->counts, 2 * q * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
                "read counts");
        HIP_TRY(hipMemcpyAsync(w->h_ctl, w->ctl, tmo::CTL_WORDS * sizeof(uint64_t), hipMemcpyDeviceToHost, stream),
                "read control words");
        HIP_TRY(hipStreamSynchronize(stream), "hipStreamSynchronize");
        if (c0 > 0 && w->h_ctl[tmo::CTL_ERROR]) return fail(TM_E_DEVICE, "work item handoff timed out");
        res->assign(q, 0);
        for (int j = 0; j < q; j++) {
            const int i = order[j];
            (*res)[i] = w->h_counts[j];
            if (budgets && budgets[i] > 0 && (int64_t)w->h_counts[q + j] > budgets[i]) (*res)[i] = kCancelled;
        }
        return TM_OK;
    };
    std::string mkey;
    if (ctx->autotune) {
        mkey = "B" + std::to_string(g->key_bytes) + "b" + std::to_string(ctx->block) +
               (ctx->min_waves ? "w" + std::to_string(ctx->min_waves) : std::string()) +
               (ctx->xcd_order ? "x" : "") + ":";
        for (auto *p : plans) mkey += p->key() + "|";
    }
    const std::string key = ctx->autotune ? tune_key(g, mkey, dmax, roots, q) : std::string();
    std::vector<uint64_t> res;
    tmo::LaunchCfg used;
    bool tuned = false;
    double ms = 0;
    tm_status st;
    if (no_alloc) {
        // no tuning trials (they need timing events): the tuned setting of
        // the key if there is one, else the defaults; untimed
        used = default_cfg(ctx);
        tuned = ctx->autotune && roots > 0 && tune_lookup(ctx, key, &used);
        used.timed = false;
        st = once(used, &ms, &res);
    } else {
        st = run_tuned(ctx, key, roots, once, &res, &used, &tuned, &ms);
    }
    if (st != TM_OK) return st;
    note_launch(ctx, used, tuned, ms, c0 > 0 ? 1 : 0);
    for (int i = 0; i < q; i++) {
        counts_out[i] = res[i];
        if (cancelled) cancelled[i] = res[i] == kCancelled;
    }
    return TM_OK;
}

tm_ctx::Workspace *ws_acquire(tm_ctx *ctx) {
    std::lock_guard<std::mutex> lk(ctx->ws_mu);
    for (auto &p : ctx->ws)
        if (!p->busy) {
            p->busy = true;
            return p.get();
        }
    ctx->ws.emplace_back(new tm_ctx::Workspace());
    ctx->ws.back()->busy = true;
    return ctx->ws.back().get();
}

void ws_release(tm_ctx *ctx, tm_ctx::Workspace *w) {
    std::lock_guard<std::mutex> lk(ctx->ws_mu);
    w->busy = false;
}

tm_status set_error(tm_status st, const std::string &msg) { return fail(st, msg); }

tm_status check_query(tm_ctx *ctx, const tm_graph *g, const tm_motif *m) { return check_pair(ctx, g, m); }

void resolve_roots(const tm_graph *g, const tm_root_range *range, int64_t *r0, int64_t *r1) {
    root_ids(g, range, r0, r1);
}

}  // namespace tmo

extern "C" {

tm_status tm_enumerate(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range,
                       hipStream_t stream, int64_t *d_out, uint64_t capacity, uint64_t *n_out) {
    tm_status st = check_pair(ctx, g, m);
    if (st != TM_OK) return st;
    if (!n_out) return fail(TM_E_INVALID, "n_out is null");
    if (capacity > 0 && !d_out) return fail(TM_E_INVALID, "d_out is null with capacity > 0");
    // the caller's buffer, if it holds every row; a size query (no buffer) is not an error
    tmo::RowAlloc alloc = [&](uint64_t total, uint64_t *cap, tm_status *ast) -> int64_t * {
        *cap = capacity;
        if (capacity >= total) return d_out;
        *ast = d_out ? fail(TM_E_CAPACITY, "enumeration buffer too small") : TM_OK;
        return nullptr;
    };
    WsLease lease(ctx);
    return tmo::enumerate_impl(ctx, g, m, range, ctx->tier, ctx->work_budget, stream, lease.w, alloc, n_out,
                               nullptr);
}

tm_status tm_count_batch(tm_ctx *ctx, const tm_graph *g, int32_t q, const tm_motif *const *motifs,
                         const tm_root_range *ranges, hipStream_t stream, uint64_t *counts_out) {
    if (!ctx || !g || q < 0 || (q > 0 && (!motifs || !counts_out))) return fail(TM_E_INVALID, "bad argument");
    if (q == 0) return TM_OK;
    for (int i = 0; i < q; i++) {
        tm_status st = check_pair(ctx, g, motifs[i]);
        if (st != TM_OK) return st;
    }
    WsLease lease(ctx);
    std::vector<int64_t> budgets(q, ctx->work_budget);
    std::vector<uint8_t> cancelled(q, 0);
    tm_status st = tmo::count_batch_impl(ctx, g, q, motifs, ranges, budgets.data(), ctx->tier, stream, lease.w,
                                         counts_out, cancelled.data());
    if (st != TM_OK) return st;
    const int64_t n_cancelled = std::count(cancelled.begin(), cancelled.end(), 1);
    if (n_cancelled)
        return fail(TM_E_CANCELLED, std::to_string(n_cancelled) + " of the queries exceeded the work budget");
    return TM_OK;
}

// tm_count_batch on the device scratch array: no device memory, event or
// stream is allocated. Scratch layout (256-byte aligned parts): control words,
// per-query counts and step tallies, per-query item queue heads and tails,
// the queries' launch arguments, then the donated-work items.
tm_status tm_count_batch_noalloc(tm_ctx *ctx, const tm_graph *g, int32_t q, const tm_motif *const *motifs,
                                 const tm_root_range *ranges, hipStream_t stream, uint64_t *counts_out) {
    if (!ctx || !g || q < 0 || (q > 0 && (!motifs || !counts_out))) return fail(TM_E_INVALID, "bad argument");
    if (q > tmo::kScratchMaxQueries)
        return fail(TM_E_INVALID, "at most " + std::to_string(tmo::kScratchMaxQueries) +
                                      " queries fit the no-allocation scratch");
    if (q == 0) return TM_OK;
    if (!ctx->scratch) return fail(TM_E_DEVICE, "no scratch address for this device");
    for (int i = 0; i < q; i++) {
        tm_status st = check_pair(ctx, g, motifs[i]);
        if (st != TM_OK) return st;
    }
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_counts = up(tmo::CTL_WORDS * sizeof(uint64_t));
    const size_t o_qctl = o_counts + up(2 * tmo::kScratchMaxQueries * sizeof(uint64_t));
    const size_t o_qa = o_qctl + up(2 * tmo::kScratchMaxQueries * sizeof(uint64_t));
    const size_t o_items = o_qa + up(tmo::kScratchMaxQueries * sizeof(QArgs));
    static_assert(tmo::kScratchBytes > (size_t(1) << 20), "scratch too small for its item region");
    char *base = (char *)ctx->scratch;
    // host mirrors (pageable; every copy is waited for before they go)
    std::vector<QArgs> h_qa(q);
    std::vector<uint64_t> h_counts(2 * (size_t)q), h_ctl(tmo::CTL_WORDS + 65);
    tm_ctx::Workspace w;
    w.no_alloc = true;
    w.ctl = (uint64_t *)base;
    w.counts = (uint64_t *)(base + o_counts);
    w.qctl = (uint64_t *)(base + o_qctl);
    w.qa = base + o_qa;
    w.items = (uint32_t *)(base + o_items);
    w.items_total = (tmo::kScratchBytes - o_items) / (tmo::kItemWords * sizeof(uint32_t));
    w.q_cap = tmo::kScratchMaxQueries;
    w.h_qa = h_qa.data();
    w.h_counts = h_counts.data();
    w.h_ctl = h_ctl.data();
    w.shared_epoch = tmo::scratch_epoch(ctx->device);
    std::vector<int64_t> budgets(q, ctx->work_budget);
    std::vector<uint8_t> cancelled(q, 0);
    tm_status st;
    {
        // one call at a time uses a device's scratch
        std::lock_guard<std::mutex> lk(*tmo::scratch_mutex(ctx->device));
        st = tmo::count_batch_impl(ctx, g, q, motifs, ranges, budgets.data(), ctx->tier, stream, &w, counts_out,
                                   cancelled.data(), true);
    }
    if (st != TM_OK) return st;
    const int64_t n_cancelled = std::count(cancelled.begin(), cancelled.end(), 1);
    if (n_cancelled)
        return fail(TM_E_CANCELLED, std::to_string(n_cancelled) + " of the queries exceeded the work budget");
    return TM_OK;
}

}  // extern "C"
