// Query server: a request loop that keeps one graph on the device and serves a
// stream of motif queries with continuous batching.
//
// * Submissions (any host thread) are validated, copied and appended to one
//   FIFO admission queue (bounded: TM_E_BUSY when full).
// * Each of `stream_slots` host threads owns a HIP stream and a workspace.
//   Whenever a slot is free it takes what is pending: up to `max_batch`
//   consecutive count queries become one batched persistent launch; an
//   enumeration runs on its own. Batches on different slots overlap on the
//   device, so queries that arrive while others run are admitted as soon as a
//   slot frees up.
// * An enumeration is admitted by the memory its output needs: after its
//   counting pass, 8 * l * rows bytes are reserved from a fixed device pool
//   (waiting while other results hold the memory); an output larger than the
//   whole pool completes with TM_E_CAPACITY and its count.
// * Results (count, rows, status, and arrival / admit / launch / done
//   timestamps on the host's monotonic clock) are collected by tm_poll;
//   enumeration rows stay in the pool until tm_release.
// * Tier 2: count queries run table-driven in batches under a probe budget; a
//   query over it is moved to a per-structure wait list, one compile thread
//   builds that structure's specialised counting kernel, and the query then
//   runs on its own with it (the ready list, which slots serve first). A slot
//   with nothing else to do runs a waiting query whose compile has not
//   started with the table-driven kernel instead.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "tm_internal.h"

namespace {

int64_t now_ns() {
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Pending {
    uint64_t ticket = 0, tag = 0;
    tm_motif motif;
    tm_root_range range{};
    bool has_range = false;
    bool enumerate = false;
    int64_t budget = 0;  // wavefront loop steps (0 = no limit)
    int64_t t_arrival = 0, t_admit = 0;
    int kernel_tier = 1;
    bool capped = false;   // its batch ran it under the probe budget
    bool probed = false;   // it exceeded the probe budget and runs again alone
    bool spec_ok = false;  // its specialised kernel is loaded
};

}  // namespace

struct tm_server {
    tm_ctx *ctx = nullptr;
    const tm_graph *g = nullptr;
    tm_server_cfg cfg{};
    std::string tune_path;  // empty: no tune table file
    std::mutex mu;
    std::condition_variable cv_pending, cv_results, cv_pool;
    std::deque<Pending *> pending;
    std::deque<tm_result> results;
    std::vector<std::thread> slots;
    bool stopping = false;
    uint64_t next_ticket = 1;
    // enumeration memory pool (bytes), first-fit over free ranges
    char *pool = nullptr;
    uint64_t pool_bytes = 0;
    std::map<uint64_t, uint64_t> free_ranges;               // offset -> size
    std::map<uint64_t, std::pair<uint64_t, uint64_t>> held;  // ticket -> (offset, size)
    uint64_t served = 0, batches = 0;
    // tier 2 (all under mu)
    std::deque<Pending *> ready;                            // heavy queries ready to run alone
    std::map<std::string, std::vector<Pending *>> waiting;  // heavy queries by structure, awaiting its compile
    std::deque<std::pair<std::string, tm_motif>> compile_q; // structures to compile, oldest first
    std::map<std::string, bool> compiled;                   // structure -> its compile succeeded
    std::string compiling;                                  // the structure being compiled, if any
    std::thread compiler;
    bool compile_stop = false;
    std::condition_variable cv_compile;
};

namespace {

// Reserve `bytes` (rounded to 256) from the pool; waits while it does not fit.
char *pool_alloc(tm_server *s, uint64_t ticket, uint64_t bytes, tm_status *st) {
    bytes = (bytes + 255) & ~uint64_t(255);
    std::unique_lock<std::mutex> lk(s->mu);
    if (bytes > s->pool_bytes) {
        *st = TM_E_CAPACITY;
        return nullptr;
    }
    for (;;) {
        for (auto it = s->free_ranges.begin(); it != s->free_ranges.end(); ++it) {
            if (it->second >= bytes) {
                const uint64_t off = it->first, rest = it->second - bytes;
                s->free_ranges.erase(it);
                if (rest) s->free_ranges[off + bytes] = rest;
                s->held[ticket] = {off, bytes};
                return s->pool + off;
            }
        }
        if (s->stopping) {
            *st = TM_E_CANCELLED;
            return nullptr;
        }
        s->cv_pool.wait(lk);
    }
}

void pool_free_locked(tm_server *s, uint64_t ticket) {
    auto it = s->held.find(ticket);
    if (it == s->held.end()) return;
    uint64_t off = it->second.first, size = it->second.second;
    s->held.erase(it);
    auto nx = s->free_ranges.lower_bound(off);
    if (nx != s->free_ranges.end() && off + size == nx->first) {
        size += nx->second;
        nx = s->free_ranges.erase(nx);
    }
    if (nx != s->free_ranges.begin()) {
        auto pv = std::prev(nx);
        if (pv->first + pv->second == off) {
            pv->second += size;
            s->cv_pool.notify_all();
            return;
        }
    }
    s->free_ranges[off] = size;
    s->cv_pool.notify_all();
}

// `why` describes a failure the calling thread's last error does not (a query
// cancelled inside a batch that itself succeeded).
void publish(tm_server *s, const Pending &p, tm_status st, uint64_t count, int64_t *rows, uint64_t n_rows,
             int64_t t_launch, const char *why = nullptr) {
    tm_result r;
    std::memset(&r, 0, sizeof(r));
    r.ticket = p.ticket;
    r.tag = p.tag;
    r.status = st;
    r.count = count;
    r.rows = rows;
    r.n_rows = n_rows;
    r.n_edges = p.motif.plan.l;
    r.t_arrival_ns = p.t_arrival;
    r.t_admit_ns = p.t_admit;
    r.t_launch_ns = t_launch;
    r.t_done_ns = now_ns();
    r.kernel_tier = p.kernel_tier;
    r.probed = p.probed ? 1 : 0;
    if (st != TM_OK) std::snprintf(r.error, sizeof(r.error), "%s", why ? why : tm_last_error());
    std::lock_guard<std::mutex> lk(s->mu);
    s->results.push_back(r);
    s->served++;
    s->cv_results.notify_all();
}

// A query launched on its own: an enumeration, or under the generic tier a
// count with anti-edges (which the table-driven matchers lack; alone it runs
// its own specialised matcher, compiled once per structure, instead of making
// every batch it joins a module of its own).
bool alone(const tm_server *s, const Pending *p) { return p->enumerate || (s->cfg.tier && p->motif.plan.n_anti > 0); }

// Tier 2, under mu: a waiting query whose structure is not being compiled
// (taken out of the wait list when `take`).
Pending *stealable(tm_server *s, bool take) {
    for (auto it = s->waiting.begin(); it != s->waiting.end(); ++it) {
        if (it->first == s->compiling || it->second.empty()) continue;
        Pending *p = it->second.front();
        if (take) {
            it->second.erase(it->second.begin());
            if (it->second.empty()) s->waiting.erase(it);
        }
        return p;
    }
    return nullptr;
}

// Tier 2: a query that exceeded the probe budget waits for its structure's
// specialised kernel (queued for compilation once), or is ready at once when
// that compile already ran.
void to_heavy(tm_server *s, Pending *p) {
    p->probed = true;
    const std::string key = p->motif.plan.key();
    std::lock_guard<std::mutex> lk(s->mu);
    auto c = s->compiled.find(key);
    if (c != s->compiled.end()) {
        p->spec_ok = c->second;
        s->ready.push_back(p);
    } else {
        auto &v = s->waiting[key];
        bool queued = key == s->compiling;
        for (auto &q : s->compile_q) queued = queued || q.first == key;
        if (!queued) {
            s->compile_q.emplace_back(key, p->motif);
            s->cv_compile.notify_one();
        }
        v.push_back(p);
    }
    s->cv_pending.notify_all();
}

// Tier 2: the compile thread. Builds one structure's specialised counting
// kernel at a time, oldest request first, and moves the queries waiting for
// it to the ready list (table-driven there if the compile failed).
void compile_main(tm_server *s) {
    for (;;) {
        std::pair<std::string, tm_motif> job;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_compile.wait(lk, [&] { return s->compile_stop || !s->compile_q.empty(); });
            if (s->compile_stop) break;
            job = s->compile_q.front();
            s->compile_q.pop_front();
            s->compiling = job.first;
        }
        const bool ok = tmo::load_count_module(s->ctx, s->g, &job.second, 0) == TM_OK;
        std::lock_guard<std::mutex> lk(s->mu);
        s->compiling.clear();
        s->compiled[job.first] = ok;
        auto it = s->waiting.find(job.first);
        if (it != s->waiting.end()) {
            for (Pending *p : it->second) {
                p->spec_ok = ok;
                s->ready.push_back(p);
            }
            s->waiting.erase(it);
        }
        s->cv_pending.notify_all();
    }
}

void slot_main(tm_server *s) {
    tm_ctx *ctx = s->ctx;
    hipSetDevice(ctx->device);
    hipStream_t stream = nullptr;
    if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
    tm_ctx::Workspace *w = tmo::ws_acquire(ctx);
    std::vector<Pending *> batch;
    std::vector<const tm_motif *> motifs;
    std::vector<tm_root_range> ranges;
    std::vector<uint64_t> counts;
    std::vector<int64_t> budgets;
    std::vector<uint8_t> cancelled;
    const int base_tier = s->cfg.tier == 2 ? 1 : s->cfg.tier;
    for (;;) {
        batch.clear();
        bool heavy = false;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_pending.wait(lk, [&] {
                return !s->pending.empty() || !s->ready.empty() || stealable(s, false) ||
                       (s->stopping && s->waiting.empty());
            });
            if (!s->ready.empty()) {
                batch.push_back(s->ready.front());
                s->ready.pop_front();
                heavy = true;
            } else if (s->pending.empty()) {
                Pending *p = stealable(s, true);
                if (!p) break;  // stopping and drained
                batch.push_back(p);
                heavy = true;
            } else if (alone(s, s->pending.front())) {
                batch.push_back(s->pending.front());
                s->pending.pop_front();
            } else {
                while (!s->pending.empty() && !alone(s, s->pending.front()) &&
                       (int)batch.size() < s->cfg.max_batch) {
                    batch.push_back(s->pending.front());
                    s->pending.pop_front();
                }
            }
            s->batches++;
        }
        if (heavy) {
            // alone, with the specialised kernel when it compiled, else table-driven
            Pending *p = batch[0];
            p->kernel_tier = p->spec_ok ? 0 : 1;
            uint64_t c = 0;
            const int64_t t_launch = now_ns();
            const tm_status st = tmo::count_impl(ctx, s->g, &p->motif, p->has_range ? &p->range : nullptr,
                                                 p->kernel_tier, p->budget, stream, w, &c);
            publish(s, *p, st, st == TM_OK ? c : 0, nullptr, 0, t_launch);
            delete p;
            continue;
        }
        const int64_t t_admit = now_ns();
        for (Pending *p : batch) p->t_admit = t_admit;
        if (batch[0]->enumerate) {
            Pending *p = batch[0];
            const uint64_t l = (uint64_t)p->motif.plan.l;
            tmo::RowAlloc alloc = [&](uint64_t rows, uint64_t *cap, tm_status *ast) -> int64_t * {
                char *mem = pool_alloc(s, p->ticket, rows * l * sizeof(int64_t), ast);
                *cap = mem ? rows : 0;
                return (int64_t *)mem;
            };
            uint64_t n = 0;
            int64_t *rows = nullptr;
            const int64_t t_launch = now_ns();
            p->kernel_tier = base_tier;
            tm_status st = tmo::enumerate_impl(ctx, s->g, &p->motif, p->has_range ? &p->range : nullptr,
                                               base_tier, p->budget, stream, w, alloc, &n, &rows);
            if (st == TM_OK && n > 0 && !rows) st = TM_E_CAPACITY;
            if (st != TM_OK) {
                std::lock_guard<std::mutex> lk(s->mu);
                pool_free_locked(s, p->ticket);
                rows = nullptr;
            }
            publish(s, *p, st, n, rows, rows ? n : 0, t_launch,
                    st == TM_E_CAPACITY ? "rows exceed the enumeration pool" : nullptr);
            delete p;
        } else {
            motifs.clear();
            ranges.clear();
            budgets.clear();
            const int tier = batch[0]->motif.plan.n_anti > 0 ? 0 : base_tier;
            // tier 2: a table-driven batch caps each query at the probe budget
            const bool probe = s->cfg.tier == 2 && tier == 1;
            for (Pending *p : batch) {
                motifs.push_back(&p->motif);
                tm_root_range r = p->range;
                if (!p->has_range) r = {INT64_MIN, INT64_MAX};
                ranges.push_back(r);
                p->capped = probe && (p->budget == 0 || p->budget > s->cfg.probe_budget);
                p->kernel_tier = tier;
                budgets.push_back(p->capped ? s->cfg.probe_budget : p->budget);
            }
            counts.assign(batch.size(), 0);
            cancelled.assign(batch.size(), 0);
            const int64_t t_launch = now_ns();
            tm_status st = tmo::count_batch_impl(ctx, s->g, (int)batch.size(), motifs.data(), ranges.data(),
                                                 budgets.data(), tier, stream, w, counts.data(), cancelled.data());
            for (size_t i = 0; i < batch.size(); i++) {
                if (st == TM_OK && cancelled[i] && batch[i]->capped) {
                    to_heavy(s, batch[i]);
                    continue;
                }
                const tm_status qs = st != TM_OK ? st : cancelled[i] ? TM_E_CANCELLED : TM_OK;
                publish(s, *batch[i], qs, qs == TM_OK ? counts[i] : 0, nullptr, 0, t_launch,
                        st == TM_OK && cancelled[i] ? "work budget exceeded" : nullptr);
                delete batch[i];
            }
        }
    }
    tmo::ws_release(ctx, w);
    if (stream) hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

tm_status tm_server_start(tm_ctx *ctx, const tm_graph *g, const tm_server_cfg *cfg, tm_server **out) {
    if (!ctx || !g || !cfg || !out) return tmo::set_error(TM_E_INVALID, "null argument");
    *out = nullptr;
    if (g->ctx != ctx) return tmo::set_error(TM_E_INVALID, "graph belongs to another context");
    if (cfg->stream_slots < 1 || cfg->stream_slots > 64 || cfg->max_batch < 1 || cfg->max_batch > 4096 ||
        cfg->queue_capacity < 1 || cfg->enum_pool_bytes < 0 || cfg->tier < 0 || cfg->tier > 2 ||
        cfg->work_budget < 0 || (cfg->tier == 2 && cfg->probe_budget < 1))
        return tmo::set_error(TM_E_INVALID, "server configuration out of range");
    tm_server *s = new (std::nothrow) tm_server();
    if (!s) return tmo::set_error(TM_E_OOM, "host allocation");
    s->ctx = ctx;
    s->g = g;
    s->cfg = *cfg;
    s->cfg.tune_path = nullptr;
    if (cfg->tune_path) {
        s->tune_path = cfg->tune_path;
        if (FILE *f = std::fopen(cfg->tune_path, "rb")) {
            std::fclose(f);
            const tm_status st = tm_tune_load(ctx, cfg->tune_path);
            if (st != TM_OK) {
                delete s;
                return st;
            }
        }
    }
    hipSetDevice(ctx->device);
    s->pool_bytes = (uint64_t)cfg->enum_pool_bytes;
    if (s->pool_bytes) {
        if (hipMalloc((void **)&s->pool, s->pool_bytes) != hipSuccess) {
            delete s;
            return tmo::set_error(TM_E_OOM, "enumeration pool");
        }
        s->free_ranges[0] = s->pool_bytes;
    }
    if (cfg->tier == 2) s->compiler = std::thread(compile_main, s);
    for (int i = 0; i < cfg->stream_slots; i++) s->slots.emplace_back(slot_main, s);
    *out = s;
    return TM_OK;
}

tm_status tm_submit_query(tm_server *s, const tm_query *q, uint64_t *ticket) {
    if (!s || !q) return tmo::set_error(TM_E_INVALID, "null argument");
    Pending *p = new (std::nothrow) Pending();
    if (!p) return tmo::set_error(TM_E_OOM, "host allocation");
    p->t_arrival = now_ns();
    std::string err;
    if (!tmo::build_plan(&q->motif, &p->motif.plan, p->motif.gaps, &err)) {
        delete p;
        return tmo::set_error(TM_E_INVALID, err);
    }
    p->motif.ctx = s->ctx;
    p->motif.delta = q->motif.delta;
    tm_status st = tmo::check_query(s->ctx, s->g, &p->motif);
    if (st != TM_OK) {
        delete p;
        return st;
    }
    p->has_range = q->has_range != 0;
    p->range = q->range;
    p->enumerate = q->enumerate != 0;
    p->tag = q->tag;
    if (q->work_budget < 0) {
        delete p;
        return tmo::set_error(TM_E_INVALID, "work budget must be >= 0");
    }
    p->budget = q->work_budget ? q->work_budget : s->cfg.work_budget;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) {
        delete p;
        return tmo::set_error(TM_E_CANCELLED, "server is stopping");
    }
    if ((int64_t)s->pending.size() >= s->cfg.queue_capacity) {
        delete p;
        return tmo::set_error(TM_E_BUSY, "admission queue full");
    }
    p->ticket = s->next_ticket++;
    if (ticket) *ticket = p->ticket;
    s->pending.push_back(p);
    s->cv_pending.notify_one();
    return TM_OK;
}

tm_status tm_poll(tm_server *s, tm_result *out, int32_t max, int32_t *n, int32_t timeout_ms) {
    if (!s || !n || (max > 0 && !out) || max < 0) return tmo::set_error(TM_E_INVALID, "bad argument");
    *n = 0;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->results.empty() && timeout_ms != 0) {
        auto pred = [&] { return !s->results.empty(); };
        if (timeout_ms < 0)
            s->cv_results.wait(lk, pred);
        else
            s->cv_results.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
    }
    while (*n < max && !s->results.empty()) {
        out[(*n)++] = s->results.front();
        s->results.pop_front();
    }
    return TM_OK;
}

tm_status tm_release(tm_server *s, uint64_t ticket) {
    if (!s) return tmo::set_error(TM_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    pool_free_locked(s, ticket);
    return TM_OK;
}

tm_status tm_server_stats(tm_server *s, uint64_t *served, uint64_t *batches, uint64_t *pending) {
    if (!s) return tmo::set_error(TM_E_INVALID, "null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (served) *served = s->served;
    if (batches) *batches = s->batches;
    if (pending) *pending = s->pending.size();
    return TM_OK;
}

tm_status tm_server_stop(tm_server *s) {
    if (!s) return TM_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->cv_pending.notify_all();
        s->cv_pool.notify_all();
    }
    for (auto &t : s->slots) t.join();
    if (s->compiler.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->compile_stop = true;
            s->cv_compile.notify_all();
        }
        s->compiler.join();
    }
    hipSetDevice(s->ctx->device);
    if (s->pool) hipFree(s->pool);
    const tm_status st = s->tune_path.empty() ? TM_OK : tm_tune_save(s->ctx, s->tune_path.c_str());
    delete s;
    return st;
}

}  // extern "C"
