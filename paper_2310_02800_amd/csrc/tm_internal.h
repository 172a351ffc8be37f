// Internal structures of the temporal motif library (not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <atomic>
#include <condition_variable>
#include <string>
#include <vector>

#include "../../include/tmotif.h"

namespace tmo {

// Launch arguments of the mining kernels. The generated device source declares
// the same two structs (QArgs per query, GArgs per launch); sizes are checked
// by static_assert on both sides.
struct QArgs {
    int64_t r0, r1;     // root id range [r0, r1)
    int64_t delta;      // clamped to the graph's time span
    int64_t gap[8];     // fine-grained limits, clamped to delta
    int64_t c0, nchunks;  // this query's slice of the launch's root-chunk queue
    int64_t budget;     // wavefront loop steps this query may use (0 = no limit)
    int32_t fn;         // which specialised matcher of the module runs it
    int32_t split;      // 1: busy lanes of this query hand pending windows to idle ones
    int32_t split_min;  // smallest pending window this query splits
    int32_t pred_mask;  // bit i: motif edge i has at least one weight predicate
    // plan tables read by the generic (table-driven) matchers, per level:
    // list kind, source and destination motif node, mask of motif nodes bound
    // before the level, window-start rule (0 search, 1 after the root in its
    // source's out-list, 2 after the root in its destination's in-list, 3 after
    // the previous level's candidate)
    uint8_t pk[8], pa[8], pb[8], pm[8], pj[8];
    int32_t glob_mask;  // bit i: level i scans the whole edge list
    int32_t lab_mask;   // bit v: motif node v requires a vertex label in [nlab[v], nlab_hi[v]]
    int32_t elab_mask;  // bit i: motif edge i requires an edge label in [elo[i], ehi[i]]
    int32_t npred;      // weight predicates: pth, pop, plev [0, npred), sorted by edge
    int32_t nlab[8], nlab_hi[8];
    int32_t elo[8], ehi[8];
    float pth[12];
    uint8_t pop[12], plev[12];
    // XCD order (GArgs.xcd): this query's chunks cut into 8 slices of xns
    // chunks; xs0 = the slices' start in every XCD's chunk sequence
    int64_t xns, xs0;
};
static_assert(sizeof(QArgs) == 400, "QArgs layout");

struct GArgs {
    const int32_t *src;
    const int32_t *dst;
    const void *tk;        // relative edge times, int32 or int64, edge-id order
    const float *w;        // edge weights or null
    const void *adj_t;     // unified adjacency: out-lists at [0,m), in-lists at [m,2m)
    const int32_t *adj_nbr;
    const int32_t *adj_eid;
    const float *adj_w;
    const uint32_t *off_out;  // n+1 offsets into [0,m)
    const uint32_t *off_in;   // n+1 offsets into [m,2m)
    const QArgs *qa;          // device array of nq queries
    uint64_t *ctl;            // [0] chunk cursor [1] output overflow [2..6] work counters
    uint64_t *counts;         // per query: counts[0, nq), then steps used counts[nq, 2 nq)
    uint64_t *chunk_cnt;      // enumeration: per-chunk counts, then write cursors
    const uint64_t *chunk_off;
    int64_t *out;
    uint64_t capacity;
    int64_t m_edges;
    int64_t total_chunks;
    int32_t rch;              // roots per chunk
    int32_t nq;
    int32_t split;            // bit 0: idle lanes take pending candidates from busy lanes; bit 1: and unstarted roots
    int32_t leaf_min;         // smallest last-level window counted in closed form (0 = never)
    uint32_t *items;          // donated work items, item_cap per query, 32 words each
    uint64_t *qctl;           // per query: (head, tail) of its item queue
    uint32_t item_cap;
    uint32_t epoch;           // launch number; an item is ready when its word 0 equals it
    const uint32_t *pos_out;  // per edge: its position in its source's out-list
    const uint32_t *pos_in;   // per edge: its position in its destination's in-list
    const int32_t *pr_nbr;    // adjacency sorted by (neighbour, time), same offsets
    const void *pr_t;
    const int32_t *nlab;      // vertex labels (n entries) or null
    const uint32_t *pr_pos;   // per adjacency entry: its position in the pair-sorted lists
    const int32_t *el;        // edge labels in edge-id order (m entries) or null
    const int32_t *adj_el;    // edge labels in adjacency order (2m entries) or null
    const uint32_t *hub;      // hub-list sample table staged in LDS by every workgroup, or null
    uint32_t hub_words;       // its size in 32-bit words (0: no staging)
    uint32_t hub_dmin;        // shortest hub list: only windows over lists this long look it up
    const void *samp;         // line samples of adj_t: samp[j] = adj_t[j << samp_lg]
    uint32_t samp_min;        // windows over at least this many entries search the samples first (0: never)
    int32_t samp_lg;
    const int32_t *pr_samp;   // line samples of pr_nbr: pr_samp[j] = pr_nbr[32 j], or null
    int32_t xcd;              // 1: chunks are contiguous root ranges, taken per XCD from 8 time slices
    int32_t pad_;
    int64_t xlen;             // chunks in one XCD's sequence (sum of the queries' xns)
};
static_assert(sizeof(GArgs) == 312, "GArgs layout");

// Hub-list staging (LDS): the longest adjacency lists each get up to
// kHubSamplesPerList time keys sampled at a power-of-two stride (at least 32,
// one cache line of keys), kHubMaxLists lists at most and kHubMaxWords words
// of table in all, so that a workgroup's copy stays within its share of LDS
// at full occupancy. Lists shorter than kHubMinLen are never staged.
constexpr uint32_t kHubMaxWords = 7168, kHubMaxLists = 64, kHubSamplesPerList = 512, kHubMinLen = 512;
constexpr uint32_t kLdsPerCu = 160u * 1024u;  // gfx950

// ctl words: [10..12] work counters of the windows counted without a scan,
// [13] donated items waiting in all queues
enum { CTL_CURSOR = 0, CTL_OVERFLOW = 1, CTL_STATS = 2, CTL_ERROR = 7, CTL_BUSY = 8, CTL_HUNGRY = 9,
       CTL_LEAF = 10, CTL_AVAIL = 13, CTL_HANDED = 14, CTL_XCD = 16, CTL_WORDS = 24 };
constexpr uint32_t kItemWords = 32;
constexpr uint64_t kItemsTotal = uint64_t(1) << 20;  // donated work items per launch (128 MiB)
constexpr int kTraceCols = 8;            // t_ns, cursor, chunks, busy, waiting, items, done, handed
constexpr int64_t kTraceMaxSamples = 1 << 20;
enum Mode { MODE_COUNT = 0, MODE_STATS = 1, MODE_ENUM_COUNT = 2, MODE_ENUM_WRITE = 3, MODE_COUNT_ = 4 };

// Where a level takes its candidates from (Algorithm 1, GetCandidateEdgeList).
enum ListKind { LIST_OUT = 0, LIST_IN = 1, LIST_BOTH = 2, LIST_GLOBAL = 3 };

struct Plan {
    int l = 0, k = 0;
    int a[TM_MAX_EDGES] = {}, b[TM_MAX_EDGES] = {};
    int kind[TM_MAX_EDGES] = {};            // per level >= 1
    std::vector<int> mapped[TM_MAX_EDGES];  // motif nodes bound before level i
    // weight predicates (Sec. 2.1 attribute constraints), sorted by motif
    // edge: which edge each tests (structure) and its operator and threshold
    // (launch arguments)
    int np = 0;
    int pred_lvl[TM_MAX_PREDS + 1] = {}, pred_op[TM_MAX_PREDS + 1] = {};
    float pred_th[TM_MAX_PREDS + 1] = {};
    bool generic = false;  // table-driven matcher for every motif with l edges
    // temporal anti-edges: motif nodes, attach edge, and the level at which
    // each is checked (its attach edge matched and both nodes bound)
    int n_anti = 0;
    int anti_a[TM_MAX_ANTI] = {}, anti_b[TM_MAX_ANTI] = {}, anti_at[TM_MAX_ANTI] = {}, anti_lvl[TM_MAX_ANTI] = {};
    // anti-edge windows: launch values (in the gap slots the motif leaves
    // free), not part of the structure key
    int64_t anti_delta[TM_MAX_ANTI] = {};
    // vertex labels: bit v of lab_mask = motif node v requires a label in
    // [lab_val[v], lab_hi[v]]; edge labels: bit i of elab_mask = motif edge i
    // requires a label in [elab_lo[i], elab_hi[i]] (masks are structure,
    // values launch arguments)
    int lab_mask = 0;
    int32_t lab_val[TM_MAX_NODES] = {}, lab_hi[TM_MAX_NODES] = {};
    int elab_mask = 0;
    int32_t elab_lo[TM_MAX_EDGES] = {}, elab_hi[TM_MAX_EDGES] = {};
    // bit i: motif edge i has at least one weight predicate
    uint32_t pred_mask() const {
        uint32_t m = 0;
        for (int j = 0; j < np; j++) m |= 1u << pred_lvl[j];
        return m;
    }
    std::string key() const;
};

// Launch-argument slot of anti-edge j's window: the gap slots from the top
// down, which a motif of l edges leaves free when l + n_anti <= 9.
inline int anti_slot(int j) { return 7 - j; }

Plan generic_plan(int l);
// Fill the plan tables a generic matcher reads (and that specialised ones ignore).
void fill_plan_tables(const Plan &p, QArgs *q);

// Loop step form of the generated matchers: 0 = search probe and candidate scan
// as separate branches; 1 = one read round per step (TM_PARAM_STEP_FORM).
constexpr int kDefaultStepForm = 0;

struct Module {
    hipModule_t mod = nullptr;
    hipFunction_t fn[MODE_COUNT_] = {};
    int max_blocks_per_cu = 0;
    double compile_ms = 0.0;
};

struct Graph;

// Module cache key: plan structure + timestamp width + block size.
struct Compiler {
    std::mutex mu;
    std::condition_variable cv;                // signalled when a compile ends
    std::map<std::string, std::shared_ptr<Module>> cache;
    std::set<std::string> inflight;            // keys some thread is compiling now
    int device = 0;
    // min_waves > 0 asks the compiler to fit that many waves per SIMD
    // `modes`: the kernels the module holds (bit i = Mode i; see mode_group)
    std::shared_ptr<Module> get(const Plan &p, int key_bytes, int block, std::string *err, int min_waves,
                                unsigned modes, int form = kDefaultStepForm);
    std::shared_ptr<Module> get_batch(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                      std::string *err, int min_waves = 0, int form = kDefaultStepForm);
    // the batched module if it is already built and loaded, else null
    // (never compiles or loads)
    std::shared_ptr<Module> find_batch(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                       int min_waves = 0, int form = kDefaultStepForm);
    // the cached module for `key`, else one built by `make` (holding the
    // kernels of `modes`, 0 = the batched kernel); concurrent callers of one
    // key share a single compile
    // produces a module's code object (from the on-disk cache or by compiling)
    using CodeFn = std::function<bool(std::vector<char> *code, std::string *err)>;
    std::shared_ptr<Module> lookup_or_build(const std::string &key, int block, unsigned modes, const CodeFn &make,
                                            std::string *err);
};

constexpr int kDefaultBlock = 256;  // threads per workgroup of the mining kernels
// every single-query kernel; a module is compiled per group of modes one call
// needs (mode_group), so a count compiles one kernel, not four
constexpr unsigned kAllModes = 0xFu;
inline unsigned mode_group(int mode) {
    return mode == MODE_ENUM_COUNT || mode == MODE_ENUM_WRITE ? (1u << MODE_ENUM_COUNT) | (1u << MODE_ENUM_WRITE)
                                                              : 1u << mode;
}
std::string generate_source(const Plan &p, int key_bytes, int block, int min_waves = 0, unsigned modes = kAllModes,
                            int form = kDefaultStepForm);
std::string generate_batch_source(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                  int min_waves = 0, int form = kDefaultStepForm);
bool build_plan(const tm_motif_desc *d, Plan *p, int64_t *gaps, std::string *err);
bool compile_to_code(const std::string &src, std::vector<char> *code, std::string *err);
bool cached_code(const std::string &src, std::vector<char> *code, std::string *err);
// Code of a batched module. min_waves 0: compiled as is, then again to fit one
// more wave per SIMD when that needs at most kSqueezeRegs fewer registers and
// spills at most kSqueezeSpills (the second build is used then).
constexpr int kSqueezeRegs = 8, kSqueezeSpills = 8;
bool batch_code(const std::vector<const Plan *> &plans, int key_bytes, int block, int min_waves,
                std::vector<char> *code, std::string *err, int form = kDefaultStepForm);

// device helpers (tm_device.hip)
hipError_t dev_build_pairs(int64_t n, int64_t m, const int32_t *d_key, const int32_t *d_other, const void *d_tk,
                           int key_bytes, int32_t *d_pr_nbr, void *d_pr_t, const uint32_t *d_pos, uint32_t add,
                           uint32_t *d_pr_pos, hipStream_t s);
hipError_t dev_build_csr(int64_t n, int64_t m, const int32_t *d_key, const int32_t *d_other, const void *d_tk,
                         int key_bytes, const float *d_w, uint32_t add, uint32_t *d_off, void *d_adj_t,
                         int32_t *d_adj_nbr, int32_t *d_adj_eid, float *d_adj_w, uint32_t *d_pos, hipStream_t s);
hipError_t dev_sort_by_time(int64_t m, int64_t *d_t, int64_t *d_perm, hipStream_t s);
hipError_t dev_gather_edges(int64_t m, const int64_t *d_perm, const int32_t *src_in, const int32_t *dst_in,
                            const float *w_in, int32_t *src_out, int32_t *dst_out, float *w_out, hipStream_t s);
hipError_t dev_make_keys(int64_t m, const int64_t *d_t, int64_t t_min, int key_bytes, void *d_tk, hipStream_t s);
hipError_t dev_check_ids(int64_t m, int64_t n, const int32_t *d_src, const int32_t *d_dst, uint32_t *d_bad,
                         hipStream_t s);
hipError_t dev_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s);
// The device scratch array of tm_count_batch_noalloc: its address on the
// current device (looked up once per device), its launch counter and the lock
// that serialises its users.
constexpr size_t kScratchBytes = TM_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchMaxQueries = TM_NOALLOC_MAX_QUERIES;
hipError_t scratch_for_device(int device, void **out);
std::atomic<uint32_t> *scratch_epoch(int device);
std::mutex *scratch_mutex(int device);
// out[p] = el[eid[p]] for p < n (edge labels into adjacency order)
hipError_t dev_gather_i32(int64_t n, const int32_t *eid, const int32_t *el, int32_t *out, hipStream_t s);
// samp[j] = adj_t[j << lg] for j < n (line samples of the unified adjacency).
hipError_t dev_line_samples(int64_t n, const void *adj_t, int key_bytes, int lg, void *samp, hipStream_t s);
// Fill the samples of a hub table whose header is in place (see build_hub_table).
hipError_t dev_hub_samples(uint32_t *d_tab, uint32_t base, uint32_t total, const void *adj_t, int key_bytes,
                           hipStream_t s);
// own scan and radix sort (tm_sort.hip). Scans: exclusive, in == out allowed,
// `tmp` holds scan_tmp_elems(n) elements. Radix sort: stable, keys below
// 2^end_bit, ping-pong between (keys, vals) and the *_alt buffers (*in_alt
// tells where the result is); hist holds radix_hist_elems(n) entries and
// scan_tmp scan_tmp_elems(radix_hist_elems(n)).
int64_t scan_tmp_elems(int64_t n);
int64_t radix_hist_elems(int64_t n);
hipError_t dev_exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s);
hipError_t dev_exclusive_scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t s);
template <typename K, typename V>
hipError_t dev_radix_sort_pairs(K *keys, V *vals, K *keys_alt, V *vals_alt, int64_t n, int end_bit, uint32_t *hist,
                                uint32_t *scan_tmp, hipStream_t s, bool *in_alt);

}  // namespace tmo

namespace tmo {

// Launch settings of one mining launch; none of them changes a result.
struct LaunchCfg {
    int64_t rch = 256;      // roots per chunk (an upper bound unless `exact`)
    bool exact = false;     // use rch as is instead of shrinking it for small ranges
    int split = 0;          // hand pending windows of busy lanes to idle lanes / wavefronts
    int64_t split_min = 2;  // smallest pending window worth splitting
    int64_t leaf_min = 512; // smallest last-level window counted in closed form (0 = never)
    int bpc = 0;            // workgroups per CU at most (0: as many as fit)
    bool timed = false;     // record HIP events around the launch
};

// The setting the autotuner kept for one key, and its kernel time.
struct TuneEntry {
    int64_t rch = 0;
    int split = 0;
    int64_t split_min = 2;
    int64_t leaf_min = 512;
    int bpc = 0;
    double ms = 0.0;
};

}  // namespace tmo

struct tm_ctx {
    int device = 0;
    int num_cus = 0;
    int block = tmo::kDefaultBlock;
    int64_t root_chunk = 256;
    int64_t grid = 0;
    int profile = 0;
    int split = 1;
    int64_t split_min = 32;
    int tier = 0;  // 0: kernels specialised per motif structure, 1: generic per motif length
    int min_waves = 0;  // waves per SIMD the kernels are compiled to fit (0: compiler's choice)
    int64_t leaf_min = 512;  // smallest last-level window counted in closed form (0 = never)
    int autotune = 0;
    int64_t work_budget = 0;  // wavefront loop steps per query (0 = no limit)
    std::mutex tune_mu;
    std::map<std::string, tmo::TuneEntry> tune;  // key: graph, module, delta and size buckets
    tmo::Compiler compiler;
    std::mutex ws_mu;
    struct Workspace {
        uint64_t *ctl = nullptr;     // CTL_WORDS
        uint64_t *h_ctl = nullptr;   // pinned host mirror
        uint64_t *chunk_cnt = nullptr;
        uint64_t *chunk_off = nullptr;
        int64_t chunk_cap = 0;
        void *scan_tmp = nullptr;
        size_t scan_tmp_bytes = 0;
        uint64_t *counts = nullptr;  // per query results
        void *qa = nullptr;          // device QArgs[q_cap]
        void *h_qa = nullptr;        // pinned staging for qa
        uint64_t *h_counts = nullptr;
        int q_cap = 0;
        uint64_t *qctl = nullptr;    // 2 words per query
        uint32_t *items = nullptr;   // items_total * kItemWords, zeroed once
        uint64_t items_total = tmo::kItemsTotal;
        uint32_t epoch = 0;
        // set for a view of the device scratch (tm_count_batch_noalloc): no
        // buffer, event or stream is ever created for it, launches are never
        // timed or sampled, and launch numbers come from one counter per
        // device (the scratch's items outlive any one call)
        bool no_alloc = false;
        std::atomic<uint32_t> *shared_epoch = nullptr;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        // launch sampler (TM_PARAM_TRACE_US): side stream, events, pinned mirror
        hipStream_t tr_stream = nullptr;
        hipEvent_t tr_go = nullptr, tr_done = nullptr;
        uint64_t *h_tr = nullptr;
        bool busy = false;
    };
    std::vector<std::unique_ptr<Workspace>> ws;
    std::mutex prof_mu;
    double last_ms = 0.0;
    int last_launches = 0;
    tmo::LaunchCfg last_cfg;  // setting of the last mining launch
    int last_tuned = 0;       // 1: it came from the tune table
    int64_t trace_us = 0;     // launch sampling period (0 = off)
    int root_handoff = 1;     // hand unstarted roots to waiting wavefronts once the queue is empty
    int hub_lds = 0;          // stage the hub lists' sampled keys in LDS (TM_PARAM_HUB_LDS)
    int64_t samp_min = 64;    // windows this long search the line samples first (TM_PARAM_LINE_SAMPLES, 0 = off)
    int step_form = tmo::kDefaultStepForm;  // matcher loop step form (TM_PARAM_STEP_FORM)
    int xcd_order = 0;        // root chunks in XCD time slices (TM_PARAM_XCD_ORDER)
    std::vector<int64_t> trace;  // samples of the last sampled launch, kTraceCols each
    void *scratch = nullptr;     // this device's no-allocation scratch (tm_count_batch_noalloc)
};

struct tm_graph {
    tm_ctx *ctx = nullptr;  // for the same-context check only; never dereferenced
    int device = 0;         // the device holding the buffers (freeing needs no context)
    int64_t n = 0, m = 0;
    int64_t t_min = 0, t_max = 0;
    int key_bytes = 4;
    bool has_w = false;
    bool was_sorted = true;
    int32_t *d_src = nullptr, *d_dst = nullptr;
    void *d_tk = nullptr;
    float *d_w = nullptr;
    void *d_adj_t = nullptr;
    int32_t *d_adj_nbr = nullptr, *d_adj_eid = nullptr;
    float *d_adj_w = nullptr;
    uint32_t *d_off_out = nullptr, *d_off_in = nullptr;
    uint32_t *d_pos_out = nullptr, *d_pos_in = nullptr;
    int32_t *d_pr_nbr = nullptr;  // adjacency sorted by (neighbour, time): out [0,m), in [m,2m)
    void *d_pr_t = nullptr;
    uint32_t *d_pr_pos = nullptr;  // per adjacency entry: its position in the pair-sorted lists
    int32_t *d_nlab = nullptr;    // vertex labels (n entries), once attached
    bool has_labels = false;
    int32_t *d_el = nullptr;      // edge labels (m entries, id order), once attached
    int32_t *d_adj_el = nullptr;  // the same in adjacency order (2m entries)
    bool has_edge_labels = false;
    uint32_t *d_hub = nullptr;    // hub-list sample table (see kHubMaxWords), or null
    void *d_samp = nullptr;       // line samples of d_adj_t (one key per 128 bytes of keys)
    int32_t *d_pr_samp = nullptr; // line samples of d_pr_nbr (every 32nd neighbour id)
    int samp_lg = 5;              // log2 of the sample stride
    uint32_t hub_words = 0, hub_dmin = 0;
    int32_t hub_lists = 0;
    std::vector<int64_t> h_t;     // sorted absolute times (root-range lookup)
    std::vector<int64_t> perm;    // empty when the input was sorted
    int64_t device_bytes = 0;
};

struct tm_motif {
    tm_ctx *ctx = nullptr;
    tmo::Plan plan;
    int64_t delta = 0;
    int64_t gaps[TM_MAX_EDGES] = {};
};

namespace tmo {

// After the counting pass of an enumeration: given the total number of rows,
// return a device buffer and its capacity in rows, or nullptr (with *st) to
// stop after reporting the total.
using RowAlloc = std::function<int64_t *(uint64_t rows, uint64_t *capacity, tm_status *st)>;

// Blocking building blocks shared by the C entry points and the server; each
// runs on `stream` with an explicit workspace and kernel tier.
// A positive budget caps the wavefront loop steps of the query's counting
// pass: past it the query stops and reports TM_E_CANCELLED (batch: its flag in
// `cancelled`, which may be null, and count ~0).
tm_status enumerate_impl(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range, int tier,
                         int64_t budget, hipStream_t stream, tm_ctx::Workspace *w, const RowAlloc &alloc,
                         uint64_t *n_out, int64_t **rows_out);
// One query counted on its own (its module compiled first if not loaded),
// with the context's launch settings or its tuned ones.
tm_status count_impl(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range, int tier,
                     int64_t budget, hipStream_t stream, tm_ctx::Workspace *w, uint64_t *count_out);
// The single-query counting module of this motif under `tier`, compiled if it
// is not loaded (TM_E_COMPILE on failure).
tm_status load_count_module(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, int tier);
// no_alloc: the workspace is a view of the device scratch; the batched module
// must already be loaded (TM_E_INVALID otherwise) and the launch uses the
// key's tuned setting or the defaults, untimed, with no tuning trials.
tm_status count_batch_impl(tm_ctx *ctx, const tm_graph *g, int32_t q, const tm_motif *const *motifs,
                           const tm_root_range *ranges, const int64_t *budgets, int tier, hipStream_t stream,
                           tm_ctx::Workspace *w, uint64_t *counts_out, uint8_t *cancelled, bool no_alloc = false);
tm_ctx::Workspace *ws_acquire(tm_ctx *ctx);
void ws_release(tm_ctx *ctx, tm_ctx::Workspace *w);
tm_status set_error(tm_status st, const std::string &msg);
tm_status check_query(tm_ctx *ctx, const tm_graph *g, const tm_motif *m);
void resolve_roots(const tm_graph *g, const tm_root_range *range, int64_t *r0, int64_t *r1);

}  // namespace tmo
