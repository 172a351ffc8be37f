/*
 * Reference CPU oracle for exact temporal motif mining.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file; it exists so the tests, the smoke check and the benchmark's
 * CPU baseline can compare the GPU results against an independent, plain
 * implementation. It shares no code, header or table with the GPU path.
 *
 * What it computes (problem definition, Sec. 2.1): the number (or the list) of
 * l-tuples of edge ids (e_0..e_{l-1}) such that
 *   - timestamps increase strictly in motif order (delta-temporal motif);
 *   - t(e_{l-1}) - t(e_0) <= delta, inclusive (delta-temporal motif);
 *   - t(e_{i+1}) - t(e_i) <= gap_i for every i (fine-grained delta_i);
 *   - a node map phi with phi(a_i) = src(e_i), phi(b_i) = dst(e_i) exists and
 *     is injective (isomorphism semantics: bijections onto the sub-graph);
 *   - every edge-attribute predicate w(e_j) OP theta holds (float32
 *     comparisons; several may name one edge; attribute constraints, Sec. 2.1
 *     and Sec. 5.4.1);
 *   - the root edge's time lies in [t_lo, t_hi] (a root-range filter; later
 *     edges may exceed t_hi by up to delta, so counts add over root ranges);
 *   - every motif node v with a required label range [lo(v), hi(v)] (lo >= 0)
 *     maps to a graph node whose label lies in it (vertex labels, Sec. 5.4.1:
 *     checked when the node is newly matched; one label is lo == hi);
 *   - every motif edge i with a required label range [elo(i), ehi(i)] is
 *     matched by a graph edge whose label lies in it (edge labels, Sec. 5.4.1:
 *     checked when the edge is matched);
 *   - for every temporal anti-edge (a, b, attached to motif edge i, delta_ab)
 *     the graph has no edge phi(a) -> phi(b) with time in the closed range
 *     [t(e_i), t(e_i) + delta_ab] (absence of an edge, Sec. 2.1), whether or
 *     not that edge belongs to the match.
 *
 * How (Sec. 2.2, Algorithm 1): chronological depth-first search in the style of
 * Mackey et al. The first motif edge is mapped onto every graph edge in time
 * order; each later level takes its candidate list from the mapping state
 * (GetCandidateEdgeList: out-list of the mapped source, in-list of the mapped
 * destination, or the whole edge list), filters it by binary search for
 * t_e > t_prev, keeps candidates whose endpoints are consistent with the
 * partial map (StructConstraints, using MapGM), and maintains MapMG / MapGM /
 * eCount with the update and rollback steps of the algorithm. The window end
 * is inclusive, following the definition (the printed loop tests time < t',
 * which would exclude t_last - t_first == delta).
 *
 * Anti-edges (Sec. 5.4.3): an anti-edge is checked as soon as its attach edge
 * is matched and both its nodes are bound, i.e. when the candidate of level
 * max(i, first level binding a, first level binding b) is accepted; a
 * matching graph edge ends that branch. The check scans phi(a)'s out-list
 * over the closed range. It reads no candidate the work counters count.
 *
 * Readings where the paper is silent: equal timestamps are allowed in the
 * graph and never both used in one match (strict order); a candidate whose two
 * endpoints are both new must have src != dst (otherwise two motif nodes would
 * share one graph node); the predicate is a pure float32 comparison; root-range
 * filtering applies to the root edge's time only.
 *
 * The optional "stats" output counts the work of the method as the byte model
 * defines it: roots scanned, windows opened, sum over windows of
 * ceil(log2(L+1)) (L = length of the list searched), candidates visited
 * (including the one read that ends a window early) and visits at the predicate
 * level. With list_rule = 1, a level whose two endpoints are both mapped
 * searches the shorter of the two lists (ties: the out-list); with
 * list_rule = 0 it always uses the out-list. The result does not depend on it.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_MAXL 8
#define OR_MAXK 8
#define OR_MAXA 4
#define OR_MAXP 9 /* weight predicates: the single one plus up to 8 more */

enum { OR_GE = 0, OR_GT = 1, OR_LE = 2, OR_LT = 3 };

typedef struct {
    int64_t n, m;
    const int32_t *src, *dst;
    const int64_t *t;
    const float *w;
    const int32_t *lab;        /* node labels (n entries, >= 0) or NULL */
    const int32_t *elab;       /* edge labels (m entries, >= 0) or NULL */
    int64_t *out_off, *in_off; /* n+1 each */
    int64_t *out_ids, *in_ids; /* edge ids per node, ascending id order */
} or_graph;

typedef struct {
    int l, k;
    int a[OR_MAXL], b[OR_MAXL];
    int64_t delta;
    int64_t gap[OR_MAXL];
    int np; /* weight predicates: edge, operator, threshold */
    int p_edge[OR_MAXP], p_op[OR_MAXP];
    float p_th[OR_MAXP];
    int pred_level[OR_MAXL]; /* 1: level i has at least one predicate */
    int64_t t_lo, t_hi;
    int list_rule;
    int n_anti;
    int anti_a[OR_MAXA], anti_b[OR_MAXA], anti_at[OR_MAXA], anti_lvl[OR_MAXA];
    int64_t anti_delta[OR_MAXA];
    int32_t nlab[OR_MAXK], nlab_hi[OR_MAXK]; /* required label range per motif node, lo -1 = any */
    int32_t elab_lo[OR_MAXL], elab_hi[OR_MAXL]; /* required label range per motif edge, lo -1 = any */
} or_query;

typedef struct {
    uint64_t roots, windows, probes, visits, pred_visits, matches;
} or_stats;

/* Execution context of one search (Algorithm 1): MapMG, MapGM, eCount, eStack. */
typedef struct {
    const or_graph *g;
    const or_query *q;
    int64_t map_mg[OR_MAXK];
    int32_t *map_gm; /* n entries, -1 = unmapped */
    int32_t *ecount; /* n entries */
    int64_t estack[OR_MAXL];
    int64_t tprime; /* t' = t_root + delta (saturating) */
    uint64_t count;
    or_stats st;
    int64_t *enum_out;
    uint64_t enum_cap, enum_n;
} or_ctx;

static int64_t sat_add(int64_t a, int64_t b) {
    if (b > 0 && a > INT64_MAX - b) return INT64_MAX;
    return a + b;
}

/* ceil(log2(L+1)) */
static uint64_t probe_bits(int64_t L) {
    uint64_t r = 0;
    uint64_t v = (uint64_t)L;
    while (v) { r++; v >>= 1; }
    return r;
}

/* First index in ids[lo,hi) whose edge time is > x (ids are in time order). */
static int64_t upper_bound_ids(const int64_t *t, const int64_t *ids, int64_t lo, int64_t hi, int64_t x) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (t[ids[mid]] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int64_t upper_bound_all(const int64_t *t, int64_t lo, int64_t hi, int64_t x) {
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (t[mid] <= x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

static int cmp_ok(int op, float w, float th) {
    switch (op) {
    case OR_GE: return w >= th;
    case OR_GT: return w > th;
    case OR_LE: return w <= th;
    default: return w < th;
    }
}

/* Every weight predicate on motif edge i holds for weight w. */
static int preds_ok(const or_query *q, int i, float w) {
    for (int j = 0; j < q->np; j++)
        if (q->p_edge[j] == i && !cmp_ok(q->p_op[j], w, q->p_th[j])) return 0;
    return 1;
}

/* Edge labels (Sec. 5.4.1): graph edge e matched to motif edge i carries a
 * label in the edge's required range. */
static int elabel_ok(const or_query *q, const int32_t *elab, int i, int64_t e) {
    if (q->elab_lo[i] < 0) return 1;
    return elab[e] >= q->elab_lo[i] && elab[e] <= q->elab_hi[i];
}

/* UpdateDataStructures: bind both endpoints of motif edge i to graph edge e. */
static void update_ds(or_ctx *c, int i, int64_t e) {
    int64_t ug = c->g->src[e], vg = c->g->dst[e];
    int um = c->q->a[i], vm = c->q->b[i];
    c->map_mg[um] = ug;
    c->map_mg[vm] = vg;
    c->map_gm[ug] = um;
    c->map_gm[vg] = vm;
    c->ecount[ug] += 1;
    c->ecount[vg] += 1;
}

/* RollbackDataStructures: release nodes whose mapped-edge count drops to 0. */
static void rollback_ds(or_ctx *c, int64_t e) {
    int64_t ug = c->g->src[e], vg = c->g->dst[e];
    c->ecount[ug] -= 1;
    c->ecount[vg] -= 1;
    if (c->ecount[ug] == 0) {
        int um = c->map_gm[ug];
        c->map_gm[ug] = -1;
        c->map_mg[um] = -1;
    }
    if (c->ecount[vg] == 0) {
        int vm = c->map_gm[vg];
        c->map_gm[vg] = -1;
        c->map_mg[vm] = -1;
    }
}

/* StructConstraints: each endpoint is either the already-mapped graph node or
 * a graph node that no motif node maps to yet. */
static int struct_ok(const or_ctx *c, int64_t e, int64_t ug, int64_t vg) {
    int64_t ue = c->g->src[e], ve = c->g->dst[e];
    int u_cons = (ug >= 0) ? (ue == ug) : (c->map_gm[ue] < 0);
    int v_cons = (vg >= 0) ? (ve == vg) : (c->map_gm[ve] < 0);
    if (ug < 0 && vg < 0 && ue == ve) return 0; /* two new motif nodes, one graph node */
    return u_cons && v_cons;
}

static int needs_labels(const or_query *q) {
    for (int v = 0; v < q->k; v++)
        if (q->nlab[v] >= 0) return 1;
    return 0;
}

static int needs_edge_labels(const or_query *q) {
    for (int i = 0; i < q->l; i++)
        if (q->elab_lo[i] >= 0) return 1;
    return 0;
}

/* Vertex labels (Sec. 5.4.1): a newly matched graph node carries the label
 * its motif node requires. Nodes bound earlier were checked then. */
static int label_ok(const or_ctx *c, int v, int64_t gnode) {
    const int32_t lo = c->q->nlab[v];
    if (lo < 0) return 1;
    const int32_t x = c->g->lab[gnode];
    return x >= lo && x <= c->q->nlab_hi[v];
}

/* Absence check of anti-edge j once its nodes are bound and its attach edge
 * matched: no edge phi(a) -> phi(b) with time in [t_at, t_at + delta]. */
static int anti_free(const or_ctx *c, int j) {
    const or_graph *g = c->g;
    const or_query *q = c->q;
    const int64_t u = c->map_mg[q->anti_a[j]], v = c->map_mg[q->anti_b[j]];
    const int64_t t0 = g->t[c->estack[q->anti_at[j]]];
    const int64_t t1 = sat_add(t0, q->anti_delta[j]);
    int64_t lo = g->out_off[u], hi = g->out_off[u + 1];
    while (lo < hi) { /* first out-edge of u with time >= t0 */
        int64_t mid = lo + (hi - lo) / 2;
        if (g->t[g->out_ids[mid]] < t0) lo = mid + 1; else hi = mid;
    }
    for (int64_t p = lo; p < g->out_off[u + 1]; p++) {
        const int64_t e = g->out_ids[p];
        if (g->t[e] > t1) break;
        if (g->dst[e] == v) return 0;
    }
    return 1;
}

/* All anti-edges checked at level i hold. */
static int anti_ok(const or_ctx *c, int i) {
    for (int j = 0; j < c->q->n_anti; j++)
        if (c->q->anti_lvl[j] == i && !anti_free(c, j)) return 0;
    return 1;
}

static void emit(or_ctx *c) {
    c->count++;
    c->st.matches++;
    if (c->enum_out) {
        if (c->enum_n < c->enum_cap) {
            for (int j = 0; j < c->q->l; j++) c->enum_out[c->enum_n * c->q->l + j] = c->estack[j];
        }
        c->enum_n++;
    }
}

/* Extend the partial match to motif edge i; t_prev is the time of edge i-1. */
static void dfs(or_ctx *c, int i, int64_t t_prev) {
    const or_graph *g = c->g;
    const or_query *q = c->q;
    if (i == q->l) { emit(c); return; }
    int64_t hi = c->tprime;
    int64_t gcap = sat_add(t_prev, q->gap[i - 1]);
    if (gcap < hi) hi = gcap;

    int64_t ug = c->map_mg[q->a[i]], vg = c->map_mg[q->b[i]];
    /* GetCandidateEdgeList */
    const int64_t *ids = NULL;
    int64_t lo, end, L;
    int use_out;
    if (ug >= 0 && vg >= 0) {
        int64_t ln_o = g->out_off[ug + 1] - g->out_off[ug];
        int64_t ln_i = g->in_off[vg + 1] - g->in_off[vg];
        use_out = (q->list_rule == 0) || (ln_o <= ln_i);
    } else {
        use_out = (ug >= 0);
    }
    if (ug >= 0 && use_out) {
        ids = g->out_ids; lo = g->out_off[ug]; end = g->out_off[ug + 1];
    } else if (vg >= 0) {
        ids = g->in_ids; lo = g->in_off[vg]; end = g->in_off[vg + 1];
    } else {
        ids = NULL; lo = 0; end = g->m;
    }
    L = end - lo;
    lo = ids ? upper_bound_ids(g->t, ids, lo, end, t_prev) : upper_bound_all(g->t, lo, end, t_prev);
    c->st.windows++;
    c->st.probes += probe_bits(L);

    /* FindNextMatchingEdge, repeated until the window is exhausted */
    for (int64_t p = lo; p < end; p++) {
        int64_t e = ids ? ids[p] : p;
        c->st.visits++;
        if (q->pred_level[i]) c->st.pred_visits++;
        if (g->t[e] > hi) break;
        if (!struct_ok(c, e, ug, vg)) continue;
        if (ug < 0 && !label_ok(c, q->a[i], g->src[e])) continue;
        if (vg < 0 && !label_ok(c, q->b[i], g->dst[e])) continue;
        if (q->pred_level[i] && !preds_ok(q, i, g->w[e])) continue;
        if (!elabel_ok(q, g->elab, i, e)) continue;
        /* NextLevel: bookkeeping and push, then descend; Backtrack on return */
        update_ds(c, i, e);
        c->estack[i] = e;
        if (anti_ok(c, i)) dfs(c, i + 1, g->t[e]);
        rollback_ds(c, e);
    }
}

static void run_root(or_ctx *c, int64_t r) {
    const or_graph *g = c->g;
    const or_query *q = c->q;
    c->st.roots++;
    if (q->pred_level[0]) c->st.pred_visits++;
    if (g->src[r] == g->dst[r]) return; /* both motif nodes new: must differ */
    if (!label_ok(c, q->a[0], g->src[r]) || !label_ok(c, q->b[0], g->dst[r])) return;
    if (q->pred_level[0] && !preds_ok(q, 0, g->w[r])) return;
    if (!elabel_ok(q, g->elab, 0, r)) return;
    update_ds(c, 0, r);
    c->estack[0] = r;
    c->tprime = sat_add(g->t[r], q->delta);
    if (anti_ok(c, 0)) dfs(c, 1, g->t[r]);
    rollback_ds(c, r);
}

/* ---------------------------------------------------------------- graph */

static void build_lists(const int32_t *key, int64_t n, int64_t m, int64_t **off_out, int64_t **ids_out) {
    int64_t *off = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *ids = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    int64_t *fill = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) off[key[e] + 1]++;
    for (int64_t v = 0; v < n; v++) off[v + 1] += off[v];
    memcpy(fill, off, (size_t)(n + 1) * sizeof(int64_t));
    for (int64_t e = 0; e < m; e++) ids[fill[key[e]]++] = e; /* ascending id order per node */
    free(fill);
    *off_out = off;
    *ids_out = ids;
}

void *oracle_graph_new(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const int64_t *t,
                       const float *w) {
    or_graph *g = (or_graph *)calloc(1, sizeof(or_graph));
    g->n = n; g->m = m; g->src = src; g->dst = dst; g->t = t; g->w = w;
    build_lists(src, n, m, &g->out_off, &g->out_ids);
    build_lists(dst, n, m, &g->in_off, &g->in_ids);
    return g;
}

void oracle_graph_free(void *h) {
    or_graph *g = (or_graph *)h;
    if (!g) return;
    free(g->out_off); free(g->in_off); free(g->out_ids); free(g->in_ids);
    free(g);
}

/* Attribute constraints beyond the single predicate: extra weight predicates,
 * upper ends of node label ranges, edge label ranges (each may be NULL). */
typedef struct {
    int n_pred;
    const int32_t *pred_edge, *pred_op;
    const float *pred_theta;
    const int32_t *node_label_hi; /* k entries */
    const int32_t *edge_label;    /* 2*l entries: lo, hi per motif edge */
} or_attrs;

static int make_query(or_query *q, int l, int k, const int32_t *edges, int64_t delta, const int64_t *gaps,
                      int pred_edge, int pred_op, float theta, int64_t t_lo, int64_t t_hi, int list_rule,
                      int n_anti, const int32_t *anti, const int64_t *anti_delta, const int32_t *node_label,
                      const or_attrs *at) {
    if (l < 1 || l > OR_MAXL || k < 2 || k > OR_MAXK || delta < 0) return 1;
    memset(q, 0, sizeof(*q));
    q->l = l; q->k = k; q->delta = delta;
    for (int i = 0; i < l; i++) {
        q->a[i] = edges[2 * i]; q->b[i] = edges[2 * i + 1];
        if (q->a[i] < 0 || q->a[i] >= k || q->b[i] < 0 || q->b[i] >= k || q->a[i] == q->b[i]) return 1;
    }
    for (int i = 0; i + 1 < l; i++) {
        q->gap[i] = gaps ? gaps[i] : INT64_MAX;
        if (q->gap[i] < 0) return 1;
    }
    q->np = 0;
    if (pred_edge >= 0) {
        if (pred_edge >= l || pred_op < OR_GE || pred_op > OR_LT) return 1;
        q->p_edge[0] = pred_edge; q->p_op[0] = pred_op; q->p_th[0] = theta; q->np = 1;
    }
    if (at && at->n_pred) {
        if (at->n_pred < 0 || at->n_pred > OR_MAXP - 1 || !at->pred_edge || !at->pred_op || !at->pred_theta) return 1;
        for (int j = 0; j < at->n_pred; j++) {
            if (at->pred_edge[j] < 0 || at->pred_edge[j] >= l || at->pred_op[j] < OR_GE || at->pred_op[j] > OR_LT)
                return 1;
            q->p_edge[q->np] = at->pred_edge[j]; q->p_op[q->np] = at->pred_op[j]; q->p_th[q->np] = at->pred_theta[j];
            q->np++;
        }
    }
    for (int j = 0; j < q->np; j++) q->pred_level[q->p_edge[j]] = 1;
    q->t_lo = t_lo; q->t_hi = t_hi; q->list_rule = list_rule;
    for (int v = 0; v < OR_MAXK; v++) q->nlab[v] = q->nlab_hi[v] = -1;
    if (node_label)
        for (int v = 0; v < k; v++) {
            if (node_label[v] < -1) return 1;
            q->nlab[v] = node_label[v];
            q->nlab_hi[v] = (at && at->node_label_hi) ? at->node_label_hi[v] : node_label[v];
            if (q->nlab[v] >= 0 && q->nlab_hi[v] < q->nlab[v]) return 1;
        }
    for (int i = 0; i < OR_MAXL; i++) q->elab_lo[i] = q->elab_hi[i] = -1;
    if (at && at->edge_label)
        for (int i = 0; i < l; i++) {
            const int32_t lo = at->edge_label[2 * i], hi = at->edge_label[2 * i + 1];
            if (lo < -1 || (lo >= 0 && hi < lo)) return 1;
            q->elab_lo[i] = lo; q->elab_hi[i] = hi;
        }
    /* anti-edges: (a, b, attach edge) triples; checked at the level where the
     * attach edge is matched and both nodes are bound */
    if (n_anti < 0 || n_anti > OR_MAXA || (n_anti > 0 && (!anti || !anti_delta))) return 1;
    int first[OR_MAXK];
    for (int v = 0; v < k; v++) first[v] = -1;
    for (int i = l - 1; i >= 0; i--) { first[q->a[i]] = i; first[q->b[i]] = i; }
    q->n_anti = n_anti;
    for (int j = 0; j < n_anti; j++) {
        const int a = anti[3 * j], b = anti[3 * j + 1], at = anti[3 * j + 2];
        if (a < 0 || a >= k || b < 0 || b >= k || a == b || at < 0 || at >= l || anti_delta[j] < 0) return 1;
        if (first[a] < 0 || first[b] < 0) return 1;
        int lvl = at;
        if (first[a] > lvl) lvl = first[a];
        if (first[b] > lvl) lvl = first[b];
        q->anti_a[j] = a; q->anti_b[j] = b; q->anti_at[j] = at; q->anti_lvl[j] = lvl;
        q->anti_delta[j] = anti_delta[j];
    }
    return 0;
}

static int64_t first_root(const or_graph *g, int64_t t_lo) {
    /* first edge with t >= t_lo */
    int64_t lo = 0, hi = g->m;
    while (lo < hi) { int64_t mid = lo + (hi - lo) / 2; if (g->t[mid] < t_lo) lo = mid + 1; else hi = mid; }
    return lo;
}

static int64_t end_root(const or_graph *g, int64_t t_hi) {
    return upper_bound_all(g->t, 0, g->m, t_hi);
}

static void ctx_init(or_ctx *c, const or_graph *g, const or_query *q) {
    memset(c, 0, sizeof(*c));
    c->g = g; c->q = q;
    for (int i = 0; i < OR_MAXK; i++) c->map_mg[i] = -1;
    c->map_gm = (int32_t *)malloc((size_t)(g->n > 0 ? g->n : 1) * sizeof(int32_t));
    c->ecount = (int32_t *)calloc((size_t)(g->n > 0 ? g->n : 1), sizeof(int32_t));
    for (int64_t v = 0; v < g->n; v++) c->map_gm[v] = -1;
}

static void ctx_free(or_ctx *c) { free(c->map_gm); free(c->ecount); }

typedef struct {
    const or_graph *g;
    const or_query *q;
    int64_t r0, r1, chunk;
    volatile int64_t *next;
    uint64_t count;
    or_stats st;
} or_worker;

static void *worker_main(void *arg) {
    or_worker *wk = (or_worker *)arg;
    or_ctx c;
    ctx_init(&c, wk->g, wk->q);
    for (;;) {
        int64_t b = __sync_fetch_and_add(wk->next, wk->chunk);
        if (b >= wk->r1) break;
        int64_t e = b + wk->chunk < wk->r1 ? b + wk->chunk : wk->r1;
        for (int64_t r = b; r < e; r++) run_root(&c, r);
    }
    wk->count = c.count;
    wk->st = c.st;
    ctx_free(&c);
    return NULL;
}

/* Count instances. stats (nullable) receives roots, windows, probes, visits,
 * pred_visits, matches. Returns 0 on success, 1 on an invalid query. */
int oracle_count(void *gh, int l, int k, const int32_t *edges, int64_t delta, const int64_t *gaps,
                 int pred_edge, int pred_op, float theta, int64_t t_lo, int64_t t_hi, int list_rule,
                 int n_anti, const int32_t *anti, const int64_t *anti_delta, const int32_t *node_label,
                 int n_pred, const int32_t *p_edge, const int32_t *p_op, const float *p_theta,
                 const int32_t *node_label_hi, const int32_t *edge_label,
                 int nthreads, uint64_t *count_out, uint64_t *stats_out) {
    const or_graph *g = (const or_graph *)gh;
    or_query q;
    const or_attrs at = {n_pred, p_edge, p_op, p_theta, node_label_hi, edge_label};
    if (make_query(&q, l, k, edges, delta, gaps, pred_edge, pred_op, theta, t_lo, t_hi, list_rule, n_anti, anti,
                   anti_delta, node_label, &at))
        return 1;
    if (needs_labels(&q) && !g->lab) return 1; /* labels required, graph has none */
    if (needs_edge_labels(&q) && !g->elab) return 1;
    if (q.np > 0 && !g->w) return 1;
    int64_t r0 = first_root(g, t_lo), r1 = end_root(g, t_hi);
    if (r1 < r0) r1 = r0;
    if (nthreads < 1) nthreads = 1;
    volatile int64_t next = r0;
    or_worker *wk = (or_worker *)calloc((size_t)nthreads, sizeof(or_worker));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int i = 0; i < nthreads; i++) {
        wk[i].g = g; wk[i].q = &q; wk[i].r0 = r0; wk[i].r1 = r1; wk[i].chunk = 256; wk[i].next = &next;
    }
    if (nthreads == 1) {
        worker_main(&wk[0]);
    } else {
        for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, worker_main, &wk[i]);
        for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    }
    uint64_t total = 0;
    or_stats st;
    memset(&st, 0, sizeof(st));
    for (int i = 0; i < nthreads; i++) {
        total += wk[i].count;
        st.roots += wk[i].st.roots; st.windows += wk[i].st.windows; st.probes += wk[i].st.probes;
        st.visits += wk[i].st.visits; st.pred_visits += wk[i].st.pred_visits; st.matches += wk[i].st.matches;
    }
    *count_out = total;
    if (stats_out) {
        stats_out[0] = st.roots; stats_out[1] = st.windows; stats_out[2] = st.probes;
        stats_out[3] = st.visits; stats_out[4] = st.pred_visits; stats_out[5] = st.matches;
    }
    free(wk); free(th);
    return 0;
}

/* Enumerate instances in root order, then depth-first candidate order. Writes
 * at most `capacity` rows of l int64 edge ids; *n_out gets the total. */
int oracle_enumerate(void *gh, int l, int k, const int32_t *edges, int64_t delta, const int64_t *gaps,
                     int pred_edge, int pred_op, float theta, int64_t t_lo, int64_t t_hi,
                     int n_anti, const int32_t *anti, const int64_t *anti_delta, const int32_t *node_label,
                     int n_pred, const int32_t *p_edge, const int32_t *p_op, const float *p_theta,
                     const int32_t *node_label_hi, const int32_t *edge_label,
                     int64_t *out, uint64_t capacity, uint64_t *n_out) {
    const or_graph *g = (const or_graph *)gh;
    or_query q;
    const or_attrs at = {n_pred, p_edge, p_op, p_theta, node_label_hi, edge_label};
    if (make_query(&q, l, k, edges, delta, gaps, pred_edge, pred_op, theta, t_lo, t_hi, 0, n_anti, anti,
                   anti_delta, node_label, &at))
        return 1;
    if (needs_labels(&q) && !g->lab) return 1; /* labels required, graph has none */
    if (needs_edge_labels(&q) && !g->elab) return 1;
    if (q.np > 0 && !g->w) return 1;
    int64_t r0 = first_root(g, t_lo), r1 = end_root(g, t_hi);
    or_ctx c;
    ctx_init(&c, g, &q);
    c.enum_out = out; c.enum_cap = capacity;
    for (int64_t r = r0; r < r1; r++) run_root(&c, r);
    *n_out = c.enum_n;
    ctx_free(&c);
    return 0;
}

/* Attach node labels (n entries, >= 0; the caller keeps them alive). */
void oracle_graph_set_labels(void *gh, const int32_t *lab) { ((or_graph *)gh)->lab = lab; }

/* Attach edge labels (m entries in edge id order, >= 0; kept alive by the caller). */
void oracle_graph_set_edge_labels(void *gh, const int32_t *elab) { ((or_graph *)gh)->elab = elab; }

int oracle_version(void) { return 4; }
