/*
 * tmotif.h — C ABI of the MI355X temporal motif miner.
 *
 * The library counts and enumerates the instances of a temporal motif in a
 * time-ordered edge list that stays resident in the GPU's HBM.
 *
 * Problem (Sec. 2.1, "Problem definition"): a temporal graph is a list of
 * directed edges (u, v, t). A motif is an ordered list of l directed edges
 * (a_i, b_i) on k motif nodes. An instance is an l-tuple of graph edge ids
 * (e_0, ..., e_{l-1}) such that
 *   1. t(e_0) < t(e_1) < ... < t(e_{l-1})      (strict; equal times never match),
 *   2. t(e_{l-1}) - t(e_0) <= delta            (delta-temporal motif, inclusive),
 *   3. t(e_{i+1}) - t(e_i) <= gap_max[i]       (fine-grained delta_i, Sec. 2.1),
 *   4. phi(a_i) = src(e_i), phi(b_i) = dst(e_i) for one injective node map phi
 *      (isomorphism semantics: a bijection between motif and matched nodes),
 *   5. optionally w(e_j) OP theta for one motif edge j (edge-attribute
 *      constraint, Sec. 5.4.1; an exact IEEE float32 comparison),
 *   6. t_lo <= t(e_0) <= t_hi when a root range is given,
 *   7. optionally, every motif node with a required vertex label maps to a
 *      graph node carrying it (Sec. 5.4.1; labels attached with
 *      tm_graph_set_node_labels),
 *   8. optionally, for each temporal anti-edge (a, b, attached to edge i,
 *      window w), no graph edge phi(a) -> phi(b) has a time in
 *      [t(e_i), t(e_i) + w] (Sec. 2.1).
 * Graph self-loops can never match (condition 4). Edge ids are positions in
 * the time-sorted edge list (ties keep input order).
 *
 * Conventions for every entry point:
 *   - Every function returns a tm_status; nothing throws across the ABI.
 *   - On failure no output is written except where stated, and no partial
 *     state is left behind. tm_last_error() returns a message for the last
 *     failure on the calling thread.
 *   - "Host" pointers are ordinary CPU memory read or written during the call;
 *     the caller keeps ownership. "Device" pointers are GPU memory on the
 *     context's device, owned by the caller.
 *   - Calls on one context may come from several host threads. Calls that use
 *     the same hipStream_t are ordered by that stream; blocking calls return
 *     after their work on the stream has completed.
 */
#ifndef TMOTIF_H
#define TMOTIF_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tm_status;
enum {
    TM_OK = 0,
    TM_E_INVALID = 1,     /* bad argument, malformed motif, negative delta, node id out of range */
    TM_E_OOM = 2,         /* device allocation failed */
    TM_E_COMPILE = 3,     /* runtime kernel compilation failed; log in tm_last_error() */
    TM_E_DEVICE = 4,      /* HIP runtime error */
    TM_E_CAPACITY = 5,    /* enumeration buffer too small; the total is still written */
    TM_E_UNSUPPORTED = 6, /* e.g. more than 8 motif edges */
    TM_E_BUSY = 7,        /* server admission queue full */
    TM_E_CANCELLED = 8    /* query stopped: over its work budget, or the server is stopping */
};

/* Edge-attribute predicate operators: w(e_j) OP theta. */
enum { TM_PRED_GE = 0, TM_PRED_GT = 1, TM_PRED_LE = 2, TM_PRED_LT = 3 };

#define TM_MAX_EDGES 8
#define TM_MAX_NODES 8
#define TM_MAX_ANTI 4
#define TM_MAX_PREDS 8 /* weight predicates beyond pred_edge/pred_op/pred_theta */

typedef struct tm_ctx tm_ctx;
typedef struct tm_graph tm_graph;
typedef struct tm_motif tm_motif;

/* Message of the last failed call on this host thread ("" if none). The
 * string stays valid until the next failing call on the same thread. */
const char *tm_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t tm_version(void);

/* ------------------------------------------------------------------ context
 * A context binds one GPU (HIP device ordinal `device`) and owns the compiled
 * motif kernels and the internal work buffers. tm_destroy frees those; graphs
 * and motifs of the context are freed by their own calls, before or after
 * tm_destroy (after it, freeing is the only valid use of them). */
tm_status tm_create(int32_t device, tm_ctx **out);
void tm_destroy(tm_ctx *ctx);

/* Tunables (runtime launch parameters; they never change a result).
 *   TM_PARAM_BLOCK         threads per workgroup (64..1024, multiple of 64)
 *   TM_PARAM_ROOT_CHUNK    most roots a wavefront takes from the global queue at once
 *                          (>= 1); launches over few roots use smaller chunks (about
 *                          four per compute unit, at least 64 roots). A chunk
 *                          interleaves its roots across the range (see tm_enumerate)
 *                          and is the enumeration output segment
 *   TM_PARAM_GRID          workgroups per launch (0 = fill the GPU by occupancy)
 *   TM_PARAM_PROFILE       1 = time every mining kernel with HIP events
 *   TM_PARAM_SPLIT         1 (default) = hand the pending candidates of busy lanes to
 *                          idle lanes and, through per-query queues, to idle wavefronts
 *                          once the root chunks are gone (Sec. 5.2); 0 = never
 *   TM_PARAM_SPLIT_MIN     smallest pending window worth splitting (>= 2; default 32)
 *   TM_PARAM_TIER          0 = kernels specialised to each motif structure (compiled
 *                          once per structure); 1 = table-driven kernels, one per
 *                          motif length, that read the motif's plan at run time (no
 *                          compilation per structure)
 *   TM_PARAM_AUTOTUNE      1 = pick root chunk and splitting per key by measurement
 *                          (see tm_tune_save); 0 (default) = use the values above
 *   TM_PARAM_WORK_BUDGET   most wavefront loop steps (one memory step of up to 64
 *                          lanes each) one query may use in tm_count, tm_count_batch
 *                          and the counting pass of tm_enumerate; past it the query
 *                          stops with TM_E_CANCELLED and no result. Checked every
 *                          1024 steps of each wavefront, so a query may run up to
 *                          1024 steps per wavefront past the budget, and one within
 *                          that margin may or may not be cancelled. 0 (default) =
 *                          no limit. This plays the role of the paper's abort signal,
 *                          checked every fixed number of iterations (Sec. 5.2.2),
 *                          except that the query ends instead of being resumed.
 *   TM_PARAM_MIN_WAVES     0 (default) = registers as the compiler chooses; 1..8 = compile
 *                          the mining kernels to fit at least that many waves per SIMD
 *                          (more resident waves hide more memory latency; fewer
 *                          registers each). Kernels compiled with each value are
 *                          cached apart.
 *   TM_PARAM_LEAF_MIN      counting: a last-level window of at least this many
 *                          candidates (default 512) whose count has a closed form is
 *                          counted with binary searches instead of a scan (see
 *                          tm_work_stats); 0 = always scan; else 32..2^24
 *   TM_PARAM_ROOT_HANDOFF  1 (default) = with splitting on, once the root chunks are
 *                          gone, a wavefront whose chunk still holds 16 or more unstarted
 *                          roots hands the last half of them, one per work item, to
 *                          waiting wavefronts (tail redistribution, Sec. 5.2.2); 0 = never
 *   TM_PARAM_HUB_LDS       0 (default) = off; 1 = every workgroup of a mining kernel
 *                          first copies the graph's hub table into LDS: for the
 *                          longest adjacency lists (up to 64, chosen longest first
 *                          at load time while the table fits 28 KiB), time keys
 *                          sampled every 2^k positions (k >= 5, at most 512 per
 *                          list). A window opened over such a list is first located
 *                          among its samples in LDS, and the search in HBM then
 *                          covers one stride (candidate caching, Sec. 5.1.1).
 *                          Results are identical either way; see
 *                          tm_graph_info.hub_lists
 *   TM_PARAM_STEP_FORM     loop step of the generated kernels (results are the same):
 *                          0 = the search probe and the candidate scan are separate
 *                          branches, each waiting for its own reads, and binding a
 *                          candidate opens the next level's window at once; 1 = each
 *                          step issues the reads of all lanes (search pivots,
 *                          candidate key and neighbour, list offsets of a level to
 *                          open) before using any, one wait per step
 *   TM_PARAM_LINE_SAMPLES  64 (default) or more: windows over lists of at least this
 *                          many entries first search the graph's line samples (one time
 *                          key per 128 bytes of keys, built at load time; Sec. 5.1.1
 *                          candidate caching), then one line of the list: a window
 *                          opened on a long list reads about two cache lines from
 *                          beyond the L2 instead of one per halving; 0 = off.
 *                          Results are the same
 *   TM_PARAM_XCD_ORDER     0 (default) = chunk j of a query holds its roots j, j + C,
 *                          j + 2C, ... (C chunks: a burst of heavy roots spreads over
 *                          many wavefronts); 1 = chunks are contiguous root ranges in
 *                          time order, cut into 8 slices, and workgroup b takes
 *                          chunks from slice b mod 8 (its XCD under round-robin
 *                          dispatch; a slice that runs dry hands over to the next),
 *                          so one XCD's L2 serves the adjacency of a narrow time
 *                          range. Results are the same
 *   TM_PARAM_TRACE_US      0 (default) = off; 10..100000 = while each mining kernel
 *                          runs, sample its control words every this many
 *                          microseconds from a side stream (the kernel is not
 *                          changed; the call blocks until the kernel ends); read
 *                          the samples of the last launch with tm_last_trace
 */
enum {
    TM_PARAM_BLOCK = 1,
    TM_PARAM_ROOT_CHUNK = 2,
    TM_PARAM_GRID = 3,
    TM_PARAM_PROFILE = 5,
    TM_PARAM_SPLIT = 6,
    TM_PARAM_SPLIT_MIN = 7,
    TM_PARAM_TIER = 8,
    TM_PARAM_AUTOTUNE = 9,
    TM_PARAM_WORK_BUDGET = 10,
    TM_PARAM_MIN_WAVES = 11,
    TM_PARAM_LEAF_MIN = 12,
    TM_PARAM_TRACE_US = 13,
    TM_PARAM_ROOT_HANDOFF = 14,
    TM_PARAM_HUB_LDS = 15,
    TM_PARAM_STEP_FORM = 16,
    TM_PARAM_LINE_SAMPLES = 17,
    TM_PARAM_XCD_ORDER = 18
};
tm_status tm_set_param(tm_ctx *ctx, int32_t param, int64_t value);

/* Samples of the last mining launch taken with TM_PARAM_TRACE_US > 0, 8 int64
 * per sample in time order (the load balance over time, Sec. 5.2.2):
 *   0 host nanoseconds since the launch was queued
 *   1 root chunks taken from the queue (>= column 2 once the queue is empty;
 *     every wavefront that finds it empty adds one)
 *   2 root chunks of the launch
 *   3 wavefronts inside a matcher
 *   4 wavefronts waiting for donated work
 *   5 donated work items waiting in the queues
 *   6 1 on the last sample, taken after the kernel ended
 *   7 unstarted roots handed to waiting wavefronts so far (TM_PARAM_ROOT_HANDOFF)
 * out: host int64[cap][8], may be NULL when cap is 0; *n_out (host) receives
 * the number of samples (at most cap rows are written). */
tm_status tm_last_trace(tm_ctx *ctx, int64_t *out, int64_t cap, int64_t *n_out);
tm_status tm_get_param(tm_ctx *ctx, int32_t param, int64_t *value);

/* Autotuning (the launch-setting counterpart of the paper's hyper-parameter
 * study, Appendix "Impact of Hyper-parameters": stealing threshold and
 * signal interval there; roots per chunk and splitting here). With
 * TM_PARAM_AUTOTUNE = 1 the first tm_count or tm_count_batch of a key runs
 * its launch under each candidate setting (roots per chunk in {16, 64, 256,
 * 1024}, each with splitting off and with splitting of windows of 32 or more;
 * at 256 roots also splitting from 2, 8 and 128; then half and twice the
 * best roots per chunk at its splitting setting; then, at the best of those,
 * TM_PARAM_LEAF_MIN in {0, 128, 2048}; then, at the best, at most 3 and 2
 * workgroups per CU instead of as many as fit), checks that every trial returns the
 * same counts (else TM_E_DEVICE), returns them, and keeps the fastest setting for
 * the key. Later counts, batches and enumerations with the key use it. The
 * key is the graph (node and edge counts, time span), the kernel module, and
 * power-of-two buckets of the largest delta (clamped to the span), of the
 * number of roots and of the number of queries. Results never depend on
 * tuning; only the first call of a key pays for the trials.
 *
 * tm_last_launch: the setting of the last count / batch / enumerate on ctx
 * (root chunk used or its upper bound, split flag, smallest split window,
 * smallest window counted in closed form, 1 if it came from the tune table);
 * each output may be NULL. tm_tune_save writes the table as text to path (host string;
 * a "tmotif-tune 3" header, then per key: root chunk, split flag, smallest split
 * window, closed-form threshold, workgroups per CU (0 = as many as fit), ms);
 * tm_tune_load merges a saved table into ctx (version 2 tables, without the
 * workgroups column, are read as 0 there; TM_E_INVALID if the file
 * cannot be read or is not a table; then nothing is merged); tm_tune_clear
 * empties it (n_removed, may be NULL, receives the number of entries). */
tm_status tm_last_launch(tm_ctx *ctx, int64_t *root_chunk, int32_t *split, int64_t *split_min, int64_t *leaf_min,
                         int32_t *tuned);
tm_status tm_tune_save(tm_ctx *ctx, const char *path);
tm_status tm_tune_load(tm_ctx *ctx, const char *path);
tm_status tm_tune_clear(tm_ctx *ctx, int64_t *n_removed);

/* Duration in milliseconds of the mining kernels of the last count or
 * enumerate call on this context (summed over their launches), measured with
 * HIP events on the caller's stream; requires TM_PARAM_PROFILE = 1. */
tm_status tm_last_kernel_ms(tm_ctx *ctx, double *ms, int32_t *launches);

/* -------------------------------------------------------------------- graph
 * Ingest a temporal edge list (Sec. 2.2: a chronologically sorted edge list
 * plus CSR-like incoming and outgoing edge lists per node; Sec. 4.2 step 0:
 * preprocessing runs on the GPU, once, off the query path).
 *
 *   n_nodes        node ids must lie in [0, n_nodes); 1 <= n_nodes < 2^31
 *   n_edges        0 <= n_edges < 2^31
 *   src, dst       host int32[n_edges]
 *   t              host int64[n_edges]; any order (stably sorted if needed)
 *   w              host float32[n_edges] edge weights, or NULL (then motifs
 *                  with a predicate are rejected at count time)
 *   flags          0 (reserved)
 *
 * The graph is copied to the device: the edge list in time order, and for each
 * node its out-edges and in-edges sorted by (time, edge id). Timestamps are
 * stored relative to the minimum (int32 when the span allows, else int64);
 * comparisons stay exact. Errors: TM_E_INVALID (ids out of range, sizes),
 * TM_E_OOM, TM_E_DEVICE. */
tm_status tm_load_graph(tm_ctx *ctx, int64_t n_nodes, int64_t n_edges, const int32_t *src, const int32_t *dst,
                        const int64_t *t, const float *w, uint32_t flags, tm_graph **out);
void tm_free_graph(tm_graph *g);

typedef struct {
    int64_t n_nodes, n_edges;
    int64_t t_min, t_max;    /* over all edges; 0, 0 when empty */
    int32_t key_bytes;       /* 4 or 8: width of the stored relative timestamps */
    int32_t has_weights;
    int64_t device_bytes;    /* HBM held by the graph */
    int32_t was_sorted;      /* 1 if the input was already in non-decreasing time order */
    int32_t has_labels;      /* 1 once vertex labels are attached */
    int32_t has_edge_labels; /* 1 once edge labels are attached */
    int32_t hub_lists;       /* adjacency lists in the hub table (TM_PARAM_HUB_LDS) */
    int32_t hub_bytes;       /* the table's size: the LDS each workgroup stages */
} tm_graph_info;
tm_status tm_graph_get_info(const tm_graph *g, tm_graph_info *info);

/* Attach vertex labels (Sec. 5.4.1; the paper's example labels nodes by
 * role, Sec. 4.3): labels is a host int32[n_nodes] array of values >= 0,
 * copied to device memory (4 bytes per node; a second call replaces them).
 * Motifs that require labels run only on a graph that has them. Not while
 * queries on this graph are running. Blocking. Errors: TM_E_INVALID (null
 * argument, a negative label), TM_E_OOM, TM_E_DEVICE. */
tm_status tm_graph_set_node_labels(tm_graph *g, const int32_t *labels);

/* Attach edge labels (Sec. 2.1: edges may carry discrete attributes; Sec.
 * 5.4.1: an edge's label is checked when the edge is matched; Sec. 6: random
 * edge features): labels is a host int32[n_edges] array of values >= 0 in the
 * input order of tm_load_graph (the library moves them to edge-id order when
 * it re-sorted the input). Copied to device memory twice, in edge-id and in
 * adjacency order (12 bytes per edge); a second call replaces them. Motifs
 * with edge label ranges run only on a graph that has them. Not while
 * queries on this graph are running. Blocking. Errors: TM_E_INVALID (null
 * argument, a negative label), TM_E_OOM, TM_E_DEVICE. */
tm_status tm_graph_set_edge_labels(tm_graph *g, const int32_t *labels);

/* perm_out: host int64[n_edges]; perm_out[id] = input position of edge id. */
tm_status tm_graph_edge_order(const tm_graph *g, int64_t *perm_out);

/* Copy one direction of the device adjacency back to host memory, for
 * inspection (dir 0 = out-lists, 1 = in-lists; 2 and 3 = the same lists
 * sorted by (neighbour, time, edge id) instead, as the closed-form counts
 * read them). Any output may be NULL.
 *   off     host uint32[n_nodes+1]: list of node v = positions [off[v], off[v+1])
 *           (in-list positions start at n_edges)
 *   nbr     host int32[n_edges]: the other endpoint, in list order
 *   eid     host int32[n_edges]: the edge id, in list order
 *   t_rel   host int64[n_edges]: time minus t_min, in list order
 * Lists of dir 0 and 1 are sorted by (time, edge id). */
tm_status tm_graph_copy_csr(const tm_graph *g, int32_t dir, uint32_t *off, int32_t *nbr, int32_t *eid,
                            int64_t *t_rel);

/* -------------------------------------------------------------------- motif
 * A motif query (Sec. 4.3, user-defined query: pattern plus the coarse delta
 * and fine-grained delta_i constraints and attribute constraints on nodes and
 * edges).
 *
 *   n_nodes     k, 2..8; every node 0..k-1 must appear on some edge
 *   n_edges     l, 1..8
 *   edges       host int32[2*l]: a_0, b_0, a_1, b_1, ... in motif time order; a_i != b_i
 *   delta       >= 0
 *   gap_max     host int64[l-1] or NULL; entry i bounds t(e_{i+1}) - t(e_i);
 *               INT64_MAX means none; entries must be >= 0
 *   pred_edge   -1 for none, else the motif edge j whose weight is tested
 *   pred_op     TM_PRED_*; pred_theta the float32 threshold
 *   n_anti      number of temporal anti-edges (Sec. 2.1), 0..TM_MAX_ANTI, with
 *               n_edges + n_anti <= 9
 *   anti        host int32[3*n_anti] or NULL when n_anti is 0: a, b, i per
 *               anti-edge; a != b are motif nodes that appear on edges, i is the
 *               motif edge it is attached to
 *   anti_delta  host int64[n_anti], entries >= 0: a match is rejected when the
 *               graph has any edge phi(a) -> phi(b) (one of the match's own
 *               edges included) whose time lies in the closed range
 *               [t(e_i), t(e_i) + anti_delta]
 *   node_label  host int32[n_nodes] or NULL: the vertex label each motif node
 *               requires (Sec. 5.4.1), -1 = any; checked when the node is
 *               first matched. Label values are launch arguments; which nodes
 *               carry one is part of the structure.
 *   n_pred      0..TM_MAX_PREDS further weight predicates (Sec. 2.1 attribute
 *               constraints), all of which must hold besides pred_edge's; several
 *               may test one motif edge (an interval of weights)
 *   preds       host tm_edge_pred[n_pred] or NULL when n_pred is 0: motif edge,
 *               TM_PRED_* operator and float32 threshold of each
 *   node_label_hi  host int32[n_nodes] or NULL: with node_label, node v's label
 *               must lie in [node_label[v], node_label_hi[v]] (inclusive,
 *               node_label_hi[v] >= node_label[v] where node_label[v] >= 0);
 *               NULL means node_label_hi = node_label (one value)
 *   edge_label  host int32[2*n_edges] or NULL: (lo, hi) per motif edge; the
 *               graph edge matched to motif edge i must carry an edge label in
 *               [lo, hi] (lo = -1: any; else hi >= lo >= 0); checked when the
 *               edge is matched. Which edges carry a range is structure, the
 *               bounds are launch arguments.
 *
 * An anti-edge is checked when the candidate of level max(i, first level
 * binding a, first level binding b) is accepted, and a hit ends that branch of
 * the search (Sec. 5.4.3). Anti-edge windows are launch arguments like delta.
 * A motif with anti-edges always runs a matcher specialised to it, also under
 * TM_PARAM_TIER = 1.
 *
 * Compiling specialises a GPU kernel to the motif's structure (Sec. 5.1.2:
 * per-level candidate list, mapped-node checks and bookkeeping fixed ahead of
 * time) with the runtime compiler. Kernels are cached per structure: delta,
 * gaps, threshold and root range are launch arguments and never recompile.
 * A motif whose edge i shares no node with edges 0..i-1 is accepted; that
 * level scans the whole edge list (Algorithm 1, GetCandidateEdgeList, case
 * neither endpoint mapped). Errors: TM_E_INVALID, TM_E_UNSUPPORTED,
 * TM_E_COMPILE. */
/* One weight predicate: w(e_edge) op theta, as a float32 comparison. */
typedef struct {
    int32_t edge;
    int32_t op;  /* TM_PRED_* */
    float theta;
} tm_edge_pred;

typedef struct {
    int32_t n_nodes;
    int32_t n_edges;
    const int32_t *edges;
    int64_t delta;
    const int64_t *gap_max;
    int32_t pred_edge;
    int32_t pred_op;
    float pred_theta;
    int32_t n_anti;
    const int32_t *anti;
    const int64_t *anti_delta;
    const int32_t *node_label;
    int32_t n_pred;
    const tm_edge_pred *preds;
    const int32_t *node_label_hi;
    const int32_t *edge_label;
} tm_motif_desc;

tm_status tm_compile_motif(tm_ctx *ctx, const tm_motif_desc *desc, tm_motif **out);
void tm_free_motif(tm_motif *m);

/* The HIP source the motif compiler emits for `desc` (key_bytes 4 or 8 = the
 * width of relative timestamps), for inspection; needs no device. Writes at
 * most `cap` bytes including the terminating NUL into `buf` (host, may be
 * NULL when cap is 0); *len (host) receives the full length. */
tm_status tm_motif_source(const tm_motif_desc *desc, int32_t key_bytes, char *buf, int64_t cap, int64_t *len);

/* Run the motif compiler down to a gfx950 code object without loading it
 * (needs no device): q = 1 compiles the single-query module of descs[0],
 * q > 1 the batched module of descs[0..q-1] (host array). *code_bytes (host,
 * may be NULL) receives the code object's size. Errors: TM_E_INVALID,
 * TM_E_COMPILE (log in tm_last_error()). */
tm_status tm_motif_compile_check(const tm_motif_desc *descs, int32_t q, int32_t key_bytes, int64_t *code_bytes);

/* Compile, without loading it, the batched module that tm_count_batch (and the
 * server's count batches) would launch for descs[0..q-1] (host array) under
 * `tier` (as TM_PARAM_TIER: 0 one matcher per distinct structure, 1 the
 * table-driven matchers plus specialised ones for motifs with anti-edges), so
 * that a later launch finds it in the code-object cache. Needs no device.
 * *code_bytes (host, may be NULL) receives the code object's size. Errors:
 * TM_E_INVALID, TM_E_COMPILE. */
tm_status tm_batch_compile_check(const tm_motif_desc *descs, int32_t q, int32_t tier, int32_t key_bytes,
                                 int64_t *code_bytes);

/* Compile a table-driven module (TM_PARAM_TIER = 1) without loading it: l in
 * 1..8 the single-query module for motifs of l edges, l = 0 the batched module
 * covering every length. Needs no device. Errors: TM_E_INVALID, TM_E_COMPILE. */
tm_status tm_generic_compile_check(int32_t l, int32_t key_bytes, int64_t *code_bytes);

/* Root range: only instances whose first edge has t_lo <= t <= t_hi (both
 * inclusive); later edges may exceed t_hi. Counts add over disjoint ranges.
 * A NULL range pointer means every root. */
typedef struct {
    int64_t t_lo, t_hi;
} tm_root_range;

/* ------------------------------------------------------------------ mining
 * Count instances (Sec. 2.1, "count" flavour). Blocking: the work is queued
 * on `stream` (0 = the null stream) and the call returns after it finished.
 * count_out: host uint64. Errors: TM_E_INVALID (a predicate on a graph
 * without weights, graph and motif from different contexts), TM_E_DEVICE,
 * TM_E_OOM, TM_E_COMPILE, TM_E_CANCELLED (over TM_PARAM_WORK_BUDGET; count_out
 * not written). */
tm_status tm_count(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range,
                   hipStream_t stream, uint64_t *count_out);

/* Enumerate instances (Sec. 2.1, "enumerate" flavour). A first pass counts the
 * instances of every segment of consecutive roots, an exclusive prefix sum
 * turns those counts into output offsets, and a second pass writes each
 * instance (e_0, ..., e_{l-1}) as l int64 edge ids into its segment.
 *   d_out      device int64[capacity][l] (row-major), caller-owned; may be
 *              NULL when capacity is 0 (size query)
 *   capacity   rows available in d_out
 *   n_out      host uint64: total number of instances (always written on
 *              TM_OK and TM_E_CAPACITY)
 * Rows are grouped by root chunk (chunk j of C holds the roots j, j+C, j+2C,
 * ... of the range, C set by the range size and TM_PARAM_ROOT_CHUNK); the
 * order of chunks is fixed, the order inside a chunk is unspecified. With
 * capacity < total, returns TM_E_CAPACITY and leaves d_out unspecified. A
 * counting pass over TM_PARAM_WORK_BUDGET returns TM_E_CANCELLED (n_out not
 * written, d_out untouched). */
tm_status tm_enumerate(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range,
                       hipStream_t stream, int64_t *d_out, uint64_t capacity, uint64_t *n_out);

/* Work counters of one query, for the byte model of the benchmark: roots
 * read, candidate windows opened, sum over windows of ceil(log2(L+1)) where
 * L is the searched list's length (the shorter of the two lists when both
 * endpoints are mapped), candidates read (including the read that ends a
 * window), candidate reads at the predicate level, and instances: the
 * search of the method as the paper describes it (Alg. 1), whatever shortcut
 * the count kernels take. Then three counters of that shortcut: last-level
 * windows of TM_PARAM_LEAF_MIN or more candidates whose count has a closed form (both
 * endpoints bound, or one new endpoint, and no weight predicate on the level),
 * which the count kernels count with binary searches in per-node lists sorted
 * by (neighbour, time) instead of scanning; the candidate reads of those
 * windows (included in the fourth counter); and the reads their counts take.
 * stats_out: host uint64[9]. Blocking like tm_count. */
tm_status tm_work_stats(tm_ctx *ctx, const tm_graph *g, const tm_motif *m, const tm_root_range *range,
                        hipStream_t stream, uint64_t *stats_out);

/* Batched count: q queries (motifs[i] with ranges[i], ranges may be NULL) in
 * one persistent launch; work items (query, root chunk) are drawn from one
 * device queue, the queries' chunks in decreasing order of roots times delta
 * (heaviest first); one launch setting (tuned per batch key with
 * TM_PARAM_AUTOTUNE) applies to all of them. counts_out: host uint64[q], in
 * the order of motifs. Blocking. TM_PARAM_WORK_BUDGET
 * applies to each query on its own: a query over it gets count UINT64_MAX and
 * the call returns TM_E_CANCELLED; the other counts are exact. */
tm_status tm_count_batch(tm_ctx *ctx, const tm_graph *g, int32_t q, const tm_motif *const *motifs,
                         const tm_root_range *ranges, hipStream_t stream, uint64_t *counts_out);

/* tm_count_batch for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc. It
 * allocates no device memory, event or stream (its host-side argument copies
 * are ordinary pageable memory). Its control words, per-query counts, launch
 * arguments and donated-work items live in one device array of 16 MiB
 * (TM_NOALLOC_SCRATCH_BYTES) that each GPU the library runs on holds until
 * the process ends, shared by every call on that GPU: each call resets what
 * must start at zero and keeps nothing from earlier calls. Calls on one GPU
 * are serialised by the library (a second one waits for the first); calls
 * from other processes or overlapping with the same scratch by any other
 * route race. Arguments and results as tm_count_batch, except:
 *   - q <= TM_NOALLOC_MAX_QUERIES (256), else TM_E_INVALID;
 *   - the batched kernel of exactly these motifs (same structures, tier and
 *     graph timestamp width) must already be compiled and loaded by an
 *     earlier tm_count_batch on ctx, else TM_E_INVALID (nothing is compiled or
 *     loaded here);
 *   - the launch uses the batch key's tuned setting when TM_PARAM_AUTOTUNE
 *     has one, else the context's defaults, with no tuning trials and no
 *     timing or sampling (TM_PARAM_PROFILE and TM_PARAM_TRACE_US are ignored);
 *   - at most about 130,000 pending windows can be donated between
 *     wavefronts per launch (a donor keeps work it cannot hand over), which
 *     changes speed, never a count. */
#define TM_NOALLOC_SCRATCH_BYTES (16 << 20)
#define TM_NOALLOC_MAX_QUERIES 256
tm_status tm_count_batch_noalloc(tm_ctx *ctx, const tm_graph *g, int32_t q, const tm_motif *const *motifs,
                                 const tm_root_range *ranges, hipStream_t stream, uint64_t *counts_out);

/* ----------------------------------------------------------------- serving
 * A request loop over one resident graph with continuous batching. Queries
 * are copied at submission into a FIFO admission queue. Each of stream_slots
 * host threads owns a HIP stream; whenever one is free it takes what is
 * pending: up to max_batch consecutive count queries as one batched launch,
 * or one enumeration. Batches on different slots overlap on the GPU, so
 * queries arriving while others run are admitted as slots free up. An
 * enumeration is admitted by the memory its rows need (8 * l bytes per row,
 * known after its counting pass) against a device pool of enum_pool_bytes,
 * waiting while other results hold the pool; rows that would not fit in the
 * whole pool complete with TM_E_CAPACITY and the count. There is no per-query
 * compilation when tier = 1 (see TM_PARAM_TIER), except once per structure of
 * a motif with anti-edges: under tier 1 such a count query is launched on its
 * own, with its specialised matcher.
 * tier = 2 (specialise heavy queries; the paper compiles a kernel per query,
 * Sec. 4.2, which a stream of thousands of structures cannot wait for): count
 * queries run first in table-driven batches, each capped at probe_budget
 * steps. A query that exceeds the cap leaves its batch (the partial work is
 * dropped) and its structure's specialised counting kernel is compiled on the
 * server's compile thread while the slots go on serving; the query then runs
 * on its own with that kernel and its full budget. A slot that would be idle
 * takes a query still waiting for a compile that has not started and runs it
 * with the table-driven kernel instead. Compiled kernels stay loaded, so a
 * later heavy query of the same structure starts at once. Enumerations run
 * table-driven, as under tier 1.
 * Timestamps are host monotonic-clock nanoseconds (CLOCK_MONOTONIC). */
typedef struct tm_server tm_server;

typedef struct {
    int32_t stream_slots;     /* concurrent launches (1..64) */
    int32_t max_batch;        /* count queries per batched launch (1..4096) */
    int64_t enum_pool_bytes;  /* device memory for enumeration rows (>= 0) */
    int32_t queue_capacity;   /* pending queries before TM_E_BUSY (>= 1) */
    int32_t tier;             /* kernel tier, as TM_PARAM_TIER, or 2 (see above) */
    int64_t work_budget;      /* default work budget of a query, as TM_PARAM_WORK_BUDGET (0 = none) */
    const char *tune_path;    /* NULL, or a tune table (tm_tune_save) merged at start if the
                                 file exists and written back at stop; launches are tuned
                                 when the context has TM_PARAM_AUTOTUNE = 1 */
    int64_t probe_budget;     /* tier 2: steps a count query may take in a table-driven
                                 batch (>= 1); ignored by tiers 0 and 1 */
} tm_server_cfg;

typedef struct {
    tm_motif_desc motif;      /* copied at submission (arrays may be freed after) */
    tm_root_range range;      /* used when has_range != 0 */
    int32_t has_range;
    int32_t enumerate;        /* 0 = count, 1 = enumerate */
    uint64_t tag;             /* returned with the result */
    int64_t work_budget;      /* as TM_PARAM_WORK_BUDGET; 0 = the server's default; over it
                                 the result has status TM_E_CANCELLED */
} tm_query;

typedef struct {
    uint64_t ticket, tag;
    tm_status status;
    int32_t n_edges;          /* row width of rows */
    uint64_t count;           /* instances (also for TM_E_CAPACITY) */
    int64_t *rows;            /* device int64[n_rows][n_edges], owned by the server until tm_release */
    uint64_t n_rows;
    int64_t t_arrival_ns, t_admit_ns, t_launch_ns, t_done_ns;
    char error[128];          /* for a status other than TM_OK: what failed (NUL-terminated) */
    int32_t kernel_tier;      /* the kernels of the final run: 0 specialised, 1 table-driven */
    int32_t probed;           /* tier 2: 1 if the query exceeded probe_budget in a batch and was
                                 run again on its own (t_launch_ns is that run's) */
} tm_result;

/* Start serving graph g of ctx. The graph and the context must outlive the
 * server (stop it before destroying either). Errors:
 * TM_E_INVALID (configuration out of range), TM_E_OOM (pool). */
tm_status tm_server_start(tm_ctx *ctx, const tm_graph *g, const tm_server_cfg *cfg, tm_server **out);

/* Submit one query (thread-safe). ticket: host uint64 (may be NULL). Errors:
 * TM_E_INVALID (malformed motif, predicate without weights), TM_E_BUSY (queue
 * full), TM_E_CANCELLED (server stopping). */
tm_status tm_submit_query(tm_server *s, const tm_query *q, uint64_t *ticket);

/* Collect up to max finished results into out (host array), waiting up to
 * timeout_ms (0 = no wait, < 0 = until one is ready); *n receives how many. */
tm_status tm_poll(tm_server *s, tm_result *out, int32_t max, int32_t *n, int32_t timeout_ms);

/* Return an enumeration result's rows to the pool (no-op for other tickets). */
tm_status tm_release(tm_server *s, uint64_t ticket);

/* Queries finished, launches made and queries pending (each may be NULL). */
tm_status tm_server_stats(tm_server *s, uint64_t *served, uint64_t *batches, uint64_t *pending);

/* Finish every pending query, then stop the slots and free the pool (rows not
 * released are freed too). With a tune_path, writes the tune table there and
 * returns that write's status; the server is stopped and freed either way. */
tm_status tm_server_stop(tm_server *s);

#ifdef __cplusplus
}
#endif
#endif /* TMOTIF_H */
