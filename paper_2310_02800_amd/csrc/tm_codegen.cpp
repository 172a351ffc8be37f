// Motif compiler: validates a motif, derives its per-level plan and emits a
// HIP kernel specialised to it, compiled at run time for gfx950.
//
// The plan is the paper's `minfo` idea (Sec. 5.1.2): for every level of the
// search tree it fixes ahead of time where candidates come from (out-list of
// the mapped source, in-list of the mapped destination, the shorter of the two
// when both are mapped, or the whole edge list when neither is), which motif
// nodes are already bound (so only those are compared), and which new node a
// candidate binds. The emitted kernel holds that context in registers, one
// named variable per level and motif node (Sec. 5.1.3), with every level
// unrolled and no interpretation of the motif at run time.
//
// Execution model of the emitted kernel (one wavefront = 64 lanes):
//   * each lane runs its own depth-first search over one root edge at a time
//     (Algorithm 1 with cached candidate windows, Sec. 5.1.1);
//   * a lane whose tree is finished takes the next root from its wavefront's
//     pool at once, and the pool refills from one global queue of root chunks
//     (a work queue as in Sec. 5.2.2, here at root-chunk granularity), so lanes
//     stay busy until the queue drains;
//   * every loop iteration performs one memory step per lane: a root fetch, one
//     binary-search probe, or one candidate read. Lanes at different stages
//     therefore issue their dependent loads together instead of waiting for
//     each other's searches to finish.
#include <dlfcn.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>
#include <utime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <sstream>

#include "tm_internal.h"

namespace tmo {

// Batched modules with more matchers than this emit them as separate
// functions (see Emitter::matcher).
constexpr int kMaxInlinedMatchers = 8;

Plan generic_plan(int l) {
    Plan p;
    p.l = l;
    p.k = TM_MAX_NODES;
    p.generic = true;
    p.a[0] = 0;
    p.b[0] = 1;
    return p;
}

void fill_plan_tables(const Plan &p, QArgs *q) {
    q->glob_mask = 0;
    for (int i = 0; i < 8; i++) q->pk[i] = q->pa[i] = q->pb[i] = q->pm[i] = q->pj[i] = 0;
    for (int i = 1; i < p.l; i++) {
        q->pk[i] = (uint8_t)p.kind[i];
        q->pa[i] = (uint8_t)p.a[i];
        q->pb[i] = (uint8_t)p.b[i];
        uint32_t mask = 0;
        for (int v : p.mapped[i]) mask |= 1u << v;
        q->pm[i] = (uint8_t)mask;
        if (p.kind[i] == LIST_GLOBAL) q->glob_mask |= 1 << i;
        // window-start rule, as in the specialised emitter
        int j = 0;
        if (p.kind[i] == LIST_OUT && p.a[i] == p.a[i - 1]) j = i == 1 ? 1 : (p.kind[i - 1] == LIST_OUT ? 3 : 0);
        if (p.kind[i] == LIST_IN && p.b[i] == p.b[i - 1]) j = i == 1 ? 2 : (p.kind[i - 1] == LIST_IN ? 3 : 0);
        q->pj[i] = (uint8_t)j;
    }
}

std::string Plan::key() const {
    if (generic) return "G" + std::to_string(l);
    std::ostringstream o;
    o << "l" << l << "k" << k << "p";
    if (np == 0) o << "-1";  // no predicate (the key of motifs without one is unchanged)
    for (int j = 0; j < np; j++) o << (j ? "." : "") << pred_lvl[j];
    o << ":";
    for (int i = 0; i < l; i++) o << a[i] << b[i] << ",";
    if (lab_mask) o << "L" << lab_mask;
    if (elab_mask) o << "E" << elab_mask;
    if (n_anti > 0) {
        o << "n";
        for (int j = 0; j < n_anti; j++) o << anti_a[j] << anti_b[j] << anti_at[j] << ",";
    }
    return o.str();
}

bool build_plan(const tm_motif_desc *d, Plan *p, int64_t *gaps, std::string *err) {
    if (!d || !d->edges) { *err = "motif descriptor or edge array is null"; return false; }
    if (d->n_edges < 1) { *err = "motif needs at least one edge"; return false; }
    if (d->n_edges > TM_MAX_EDGES || d->n_nodes > TM_MAX_NODES) {
        *err = "motif too large (at most 8 edges and 8 nodes)";
        return false;
    }
    if (d->n_nodes < 2) { *err = "motif needs at least two nodes"; return false; }
    if (d->delta < 0) { *err = "delta must be >= 0"; return false; }
    const int l = d->n_edges, k = d->n_nodes;
    int relabel[TM_MAX_NODES];
    for (int i = 0; i < TM_MAX_NODES; i++) relabel[i] = -1;
    int next = 0;
    for (int i = 0; i < l; i++) {
        int a = d->edges[2 * i], b = d->edges[2 * i + 1];
        if (a < 0 || a >= k || b < 0 || b >= k) { *err = "motif node id out of range"; return false; }
        if (a == b) { *err = "motif edge with a == b"; return false; }
        if (relabel[a] < 0) relabel[a] = next++;
        if (relabel[b] < 0) relabel[b] = next++;
        p->a[i] = relabel[a];
        p->b[i] = relabel[b];
    }
    if (next != k) { *err = "every motif node must appear on an edge"; return false; }
    p->l = l;
    p->k = k;
    for (int i = 0; i + 1 < l; i++) {
        int64_t g = d->gap_max ? d->gap_max[i] : INT64_MAX;
        if (g < 0) { *err = "gap_max entries must be >= 0"; return false; }
        gaps[i] = g;
    }
    for (int i = l - 1; i < TM_MAX_EDGES; i++) gaps[i] = INT64_MAX;
    if (d->pred_edge < -1 || d->pred_edge >= l) { *err = "pred_edge out of range"; return false; }
    if (d->pred_edge >= 0 && (d->pred_op < TM_PRED_GE || d->pred_op > TM_PRED_LT)) {
        *err = "unknown predicate operator";
        return false;
    }
    // weight predicates: the single one and the list, sorted by motif edge
    // (stable, so a launch's thresholds follow the caller's order per edge)
    if (d->n_pred < 0 || d->n_pred > TM_MAX_PREDS) { *err = "at most 8 further weight predicates"; return false; }
    if (d->n_pred > 0 && !d->preds) { *err = "predicate array is null"; return false; }
    {
        struct P { int lvl, op; float th; };
        std::vector<P> ps;
        if (d->pred_edge >= 0) ps.push_back({d->pred_edge, d->pred_op, d->pred_theta});
        for (int j = 0; j < d->n_pred; j++) {
            const tm_edge_pred &x = d->preds[j];
            if (x.edge < 0 || x.edge >= l) { *err = "predicate edge out of range"; return false; }
            if (x.op < TM_PRED_GE || x.op > TM_PRED_LT) { *err = "unknown predicate operator"; return false; }
            ps.push_back({x.edge, x.op, x.theta});
        }
        std::stable_sort(ps.begin(), ps.end(), [](const P &x, const P &y) { return x.lvl < y.lvl; });
        p->np = (int)ps.size();
        for (int j = 0; j < p->np; j++) {
            p->pred_lvl[j] = ps[j].lvl;
            p->pred_op[j] = ps[j].op;
            p->pred_th[j] = ps[j].th;
        }
    }
    // edge labels (Sec. 5.4.1): an inclusive range per motif edge
    p->elab_mask = 0;
    for (int i = 0; i < TM_MAX_EDGES; i++) p->elab_lo[i] = p->elab_hi[i] = 0;
    if (d->edge_label)
        for (int i = 0; i < l; i++) {
            const int32_t lo = d->edge_label[2 * i], hi = d->edge_label[2 * i + 1];
            if (lo < -1 || (lo >= 0 && hi < lo)) { *err = "edge label ranges need -1 or 0 <= lo <= hi"; return false; }
            if (lo >= 0) {
                p->elab_mask |= 1 << i;
                p->elab_lo[i] = lo;
                p->elab_hi[i] = hi;
            }
        }
    bool bound[TM_MAX_NODES] = {};
    bound[p->a[0]] = bound[p->b[0]] = true;
    for (int i = 1; i < l; i++) {
        p->mapped[i].clear();
        for (int v = 0; v < k; v++)
            if (bound[v]) p->mapped[i].push_back(v);
        bool am = bound[p->a[i]], bm = bound[p->b[i]];
        p->kind[i] = am && bm ? LIST_BOTH : am ? LIST_OUT : bm ? LIST_IN : LIST_GLOBAL;
        bound[p->a[i]] = bound[p->b[i]] = true;
    }
    // vertex labels (Sec. 5.4.1), in the relabelled node order
    p->lab_mask = 0;
    for (int v = 0; v < TM_MAX_NODES; v++) p->lab_val[v] = p->lab_hi[v] = 0;
    if (d->node_label)
        for (int v = 0; v < k; v++) {
            const int32_t want = d->node_label[v];
            const int32_t top = d->node_label_hi ? d->node_label_hi[v] : want;
            if (want < -1) { *err = "node labels must be -1 (any) or >= 0"; return false; }
            if (want >= 0 && top < want) { *err = "node label ranges need node_label_hi >= node_label"; return false; }
            if (want >= 0) {
                p->lab_mask |= 1 << relabel[v];
                p->lab_val[relabel[v]] = want;
                p->lab_hi[relabel[v]] = top;
            }
        }
    // temporal anti-edges (Sec. 2.1): each is checked at the first level where
    // its attach edge is matched and both its nodes are bound (Sec. 5.4.3)
    const int na = d->n_anti;
    if (na < 0 || na > TM_MAX_ANTI) { *err = "at most 4 anti-edges"; return false; }
    if (na > 0 && (!d->anti || !d->anti_delta)) { *err = "anti-edge arrays are null"; return false; }
    if (l + na > TM_MAX_EDGES + 1) { *err = "edges plus anti-edges must not exceed 9"; return false; }
    int first[TM_MAX_NODES];
    for (int v = 0; v < TM_MAX_NODES; v++) first[v] = -1;
    for (int i = l - 1; i >= 0; i--) first[p->a[i]] = first[p->b[i]] = i;
    p->n_anti = na;
    for (int j = 0; j < na; j++) {
        const int a = d->anti[3 * j], b = d->anti[3 * j + 1], at = d->anti[3 * j + 2];
        if (a < 0 || a >= k || b < 0 || b >= k) { *err = "anti-edge node id out of range"; return false; }
        if (a == b) { *err = "anti-edge with a == b"; return false; }
        if (at < 0 || at >= l) { *err = "anti-edge attach edge out of range"; return false; }
        if (d->anti_delta[j] < 0) { *err = "anti-edge windows must be >= 0"; return false; }
        const int ra = relabel[a], rb = relabel[b];
        p->anti_a[j] = ra;
        p->anti_b[j] = rb;
        p->anti_at[j] = at;
        p->anti_lvl[j] = std::max(at, std::max(first[ra], first[rb]));
        p->anti_delta[j] = d->anti_delta[j];
    }
    return true;
}

// ------------------------------------------------------------------ emitter

static const char *kPrelude = R"HIP(
typedef unsigned long long u64;
typedef long long i64;
typedef unsigned int u32;

struct QArgs {
  i64 r0, r1, delta;
  i64 gap[8];
  i64 c0, nchunks;
  i64 budget;
  int fn, split, split_min, pred_mask;
  unsigned char pk[8], pa[8], pb[8], pm[8], pj[8];
  int glob_mask, lab_mask, elab_mask, npred;
  int nlab[8], nlab_hi[8];
  int elo[8], ehi[8];
  float pth[12];
  unsigned char pop[12], plev[12];
  i64 xns, xs0;
};

// Query arguments are read-only during a launch and uniform per wavefront; in the
// constant address space the compiler reads them with scalar loads.
typedef const __attribute__((address_space(4))) QArgs* qptr;

struct GArgs {
  const int* src; const int* dst; const tkey* tk; const float* w;
  const tkey* adj_t; const int* adj_nbr; const int* adj_eid; const float* adj_w;
  const u32* off_out; const u32* off_in;
  const QArgs* qa;
  u64* ctl;
  u64* counts;
  u64* chunk_cnt; const u64* chunk_off; i64* out; u64 capacity;
  i64 m_edges; i64 total_chunks; int rch; int nq;
  int split; int leaf_min;
  u32* items; u64* qctl; u32 item_cap; u32 epoch;
  const u32* pos_out; const u32* pos_in;
  const int* pr_nbr; const tkey* pr_t;
  const int* nlab;
  const u32* pr_pos;
  const int* el; const int* adj_el;
  const u32* hub; u32 hub_words; u32 hub_dmin;
  const tkey* samp; u32 samp_min; int samp_lg;
  const int* pr_samp;
  int xcd; int pad_; i64 xlen;
};
static_assert(sizeof(QArgs) == 400, "QArgs layout");
static_assert(sizeof(GArgs) == 312, "GArgs layout");
// Hub-list samples staged by the workgroup (launches with hub_words > 0):
// [0] H, [1, 1+H) list starts (ascending), [1+H, 2+2H) sample offsets,
// [2+2H, 2+3H) log2 strides, time keys from word 2+3H rounded up to even.
extern __shared__ u32 lds_hub[];
// The next root chunk for this wavefront (lane 0 calls it), or total_chunks
// when none is left; ctl[0] counts the chunks taken. In XCD order each
// query's chunks are contiguous root ranges in time order, cut into 8 slices;
// workgroup b takes from slice b mod 8 first (its XCD under round-robin
// dispatch, so that XCD's L2 serves a narrow time range of the adjacency) and
// moves to the next slice when its own runs dry.
__device__ __forceinline__ i64 next_chunk_x(const GArgs& g) {
  const int x = (int)(blockIdx.x & 7u);
  for (int k = 0; k < 8; ++k) {
    const int y = (x + k) & 7;
    for (;;) {
      const u64 pos = atomicAdd(&g.ctl[16 + y], 1ull);
      if (pos >= (u64)g.xlen) break;
      int lo = 0, hi = g.nq - 1;
      while (lo < hi) { const int md = (lo + hi + 1) >> 1; if ((u64)g.qa[md].xs0 <= pos) lo = md; else hi = md - 1; }
      const i64 loc = (i64)y * g.qa[lo].xns + ((i64)pos - g.qa[lo].xs0);
      if (loc < g.qa[lo].nchunks) { atomicAdd(&g.ctl[0], 1ull); return g.qa[lo].c0 + loc; }
    }
  }
  return g.total_chunks;
}
// A window over [lo, hi) of the unified adjacency: the line samples
// (smp[j] = key at position j << lg) inside the range are searched first, which
// leaves to the search over the list the positions between the last sample
// <= x and the next one: one line of keys instead of one line per halving.
__device__ __forceinline__ void line_narrow(const tkey* smp, int lg, u32 lo, u32 hi, tkey x, u32& sb, u32& sn) {
  const u32 j0 = (lo + (1u << lg) - 1u) >> lg, j1 = (hi - 1u) >> lg;
  if (j0 > j1) return;
  u32 b = j0, k = j1 - j0 + 1u;
  while (k > 0u) { const u32 h2 = k >> 1; if (smp[b + h2] <= x) { b += h2 + 1u; k -= h2 + 1u; } else { k = h2; } }
  // b: the first sample in range with key > x (j1 + 1 if none)
  const u32 nlo = b == j0 ? lo : ((b - 1u) << lg) + 1u;
  const u32 nhi = b <= j1 ? (b << lg) : hi;
  sb = nlo; sn = nhi - nlo;
}
// A window over the hub list that starts at adjacency position lo: locate the
// first key > x among the list's samples in LDS and leave [sb, sb+sn) to the
// search in HBM, one stride at most; lists not in the table are left as they are.
__device__ __forceinline__ void hub_narrow(u32 lo, tkey x, u32& sb, u32& sn) {
  const u32 H = lds_hub[0];
  u32 a = 0u, n = H;
  while (n > 0u) { const u32 h2 = n >> 1; if (lds_hub[1u + a + h2] < lo) { a += h2 + 1u; n -= h2 + 1u; } else { n = h2; } }
  if (a >= H || lds_hub[1u + a] != lo) return;
  const u32 s0 = lds_hub[1u + H + a], s1 = lds_hub[2u + H + a], lg = lds_hub[2u + 2u * H + a];
  const tkey* smp = (const tkey*)(lds_hub + ((2u + 3u * H + 1u) & ~1u));
  u32 b = s0, k = s1 - s0;
  while (k > 0u) { const u32 h2 = k >> 1; if (smp[b + h2] <= x) { b += h2 + 1u; k -= h2 + 1u; } else { k = h2; } }
  const u32 c = b - s0;  // samples <= x: sample c (if any) is the first key > x among them
  if (c == 0u) { sn = 0u; return; }  // the list's first key already exceeds x
  const u32 end = sb + sn, nb = lo + ((c - 1u) << lg) + 1u, nx = lo + (c << lg);
  sb = nb; sn = (nx < end ? nx : end) - nb;
}
// generic matchers: motif node slot by run-time index, and the bound-node check
#define mget(ix) ((ix) == 0 ? m0 : (ix) == 1 ? m1 : (ix) == 2 ? m2 : (ix) == 3 ? m3 : \
                  (ix) == 4 ? m4 : (ix) == 5 ? m5 : (ix) == 6 ? m6 : m7)
#define lget(ix) ((ix) == 0 ? l0 : (ix) == 1 ? l1 : (ix) == 2 ? l2 : (ix) == 3 ? l3 : \
                  (ix) == 4 ? l4 : (ix) == 5 ? l5 : (ix) == 6 ? l6 : l7)
#define hget(ix) ((ix) == 0 ? h0 : (ix) == 1 ? h1 : (ix) == 2 ? h2 : (ix) == 3 ? h3 : \
                  (ix) == 4 ? h4 : (ix) == 5 ? h5 : (ix) == 6 ? h6 : h7)
#define mset(ix, val) do { const int v_ = (val); const int i_ = (ix); \
    m0 = i_ == 0 ? v_ : m0; m1 = i_ == 1 ? v_ : m1; m2 = i_ == 2 ? v_ : m2; m3 = i_ == 3 ? v_ : m3; \
    m4 = i_ == 4 ? v_ : m4; m5 = i_ == 5 ? v_ : m5; m6 = i_ == 6 ? v_ : m6; m7 = i_ == 7 ? v_ : m7; } while (0)
__device__ __forceinline__ bool notin(u32 mask, int x, int a0, int a1, int a2, int a3, int a4, int a5, int a6,
                                      int a7) {
  return !(((mask & 1u) && x == a0) || ((mask & 2u) && x == a1) || ((mask & 4u) && x == a2) ||
           ((mask & 8u) && x == a3) || ((mask & 16u) && x == a4) || ((mask & 32u) && x == a5) ||
           ((mask & 64u) && x == a6) || ((mask & 128u) && x == a7));
}


__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}
__device__ __forceinline__ u64 ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ __forceinline__ int rank_in(u64 mask) {
  return (int)__builtin_amdgcn_mbcnt_hi((u32)(mask >> 32), __builtin_amdgcn_mbcnt_lo((u32)mask, 0u));
}
__device__ __forceinline__ i64 bcast64(i64 v) {
  u32 lo = (u32)__builtin_amdgcn_readfirstlane((int)(u32)(u64)v);
  u32 hi = (u32)__builtin_amdgcn_readfirstlane((int)(u32)((u64)v >> 32));
  return (i64)(((u64)hi << 32) | lo);
}
__device__ __forceinline__ u32 xor32(u32 v, int mask, int lane) {
  return (u32)__builtin_amdgcn_ds_bpermute((lane ^ mask) << 2, (int)v);
}
__device__ __forceinline__ u64 wave_sum(u64 v, int lane) {
  for (int s = 32; s >= 1; s >>= 1) {
    u32 lo = xor32((u32)v, s, lane), hi = xor32((u32)(v >> 32), s, lane);
    v += ((u64)hi << 32) | (u64)lo;
  }
  return v;
}
__device__ __forceinline__ bool pred_ok(float w, int op, float th) {
  return op == 0 ? (w >= th) : op == 1 ? (w > th) : op == 2 ? (w <= th) : (w < th);
}
// every weight predicate of level lv holds (table-driven matchers)
__device__ __forceinline__ bool preds_at(qptr q, int lv, float w) {
  bool ok = true;
  for (int j = 0; j < q->npred; ++j)
    if (q->plev[j] == lv) ok = ok && pred_ok(w, q->pop[j], q->pth[j]);
  return ok;
}
// a label in the inclusive range [lo, hi]
__device__ __forceinline__ bool in_range(int x, int lo, int hi) { return x >= lo && x <= hi; }
__device__ __forceinline__ u32 bitlen(u32 x) { return x ? 32u - (u32)__builtin_clz(x) : 0u; }
// Roots in chunk L of a query of n roots cut into contiguous runs of rch.
__device__ __forceinline__ i64 ch_roots_x(i64 L, i64 n, i64 rch) {
  const i64 left = n - L * rch;
  return left < rch ? left : rch;
}
// Counting a last-level window without scanning it. `pr` counts the reads.
// Entries of [c, e) (sorted by time) with time <= t, galloping from c.
__device__ __forceinline__ u32 win_len(const tkey* at, u32 c, u32 e, tkey t, u32& pr) {
  u32 lo = c, bound = e;
  for (u64 step = 1u;; step <<= 1) {
    const u64 q = (u64)lo + step - 1u;
    if (q >= (u64)e) { bound = e; break; }
    ++pr;
    if (at[q] > t) { bound = (u32)q; break; }
    lo = (u32)q + 1u;
  }
  u32 n = bound - lo;
  while (n > 0u) { const u32 h = n >> 1, m = lo + h; ++pr; if (at[m] <= t) { lo = m + 1u; n -= h + 1u; } else n = h; }
  return lo - c;
}
// In one node's list [lo, hi) sorted by (neighbour, time): the first entry
// with neighbour >= x. With ps (every 32nd neighbour id of the lists), a list
// of 64+ entries is first narrowed to the line after the last sample < x.
__device__ __forceinline__ u32 nbr_lb(const int* pn, const int* ps, u32 lo, u32 hi, int x, u32& pr) {
  if (ps && hi - lo >= 64u) {
    const u32 j0 = (lo + 31u) >> 5, j1 = (hi - 1u) >> 5;
    u32 b = j0, k = j1 - j0 + 1u;
    while (k > 0u) { const u32 h = k >> 1; if (ps[b + h] < x) { b += h + 1u; k -= h + 1u; } else k = h; }
    const u32 nlo = b == j0 ? lo : ((b - 1u) << 5) + 1u, nhi = b <= j1 ? (b << 5) : hi;
    lo = nlo; hi = nhi;
  }
  u32 n = hi - lo;
  while (n > 0u) { const u32 h = n >> 1, m = lo + h; ++pr; if (pn[m] < x) { lo = m + 1u; n -= h + 1u; } else n = h; }
  return lo;
}
// From s (the first entry with neighbour x), the first entry past those with
// neighbour x and time <= t: galloping, then binary search.
__device__ __forceinline__ u32 run_ub(const int* pn, const tkey* pt, u32 s, u32 hi, int x, tkey t, u32& pr) {
  u32 lo = s, bound = hi;
  for (u64 step = 1u;; step <<= 1) {
    const u64 q = (u64)lo + step - 1u;
    if (q >= (u64)hi) { bound = hi; break; }
    ++pr;
    if (pn[q] != x || pt[q] > t) { bound = (u32)q; break; }
    lo = (u32)q + 1u;
  }
  u32 n = bound - lo;
  while (n > 0u) {
    const u32 h = n >> 1, m = lo + h; ++pr;
    if (pn[m] == x && pt[m] <= t) { lo = m + 1u; n -= h + 1u; } else n = h;
  }
  return lo;
}
// Entries of [lo, hi) with neighbour x and time in (t0, t1], t0 < t1.
__device__ __forceinline__ u32 pair_cnt(const int* pn, const int* ps, const tkey* pt, u32 lo, u32 hi, int x, tkey t0,
                                        tkey t1, u32& pr) {
  const u32 s = nbr_lb(pn, ps, lo, hi, x, pr);
  ++pr;
  if (s >= hi || pn[s] != x) return 0u;
  return run_ub(pn, pt, s, hi, x, t1, pr) - run_ub(pn, pt, s, hi, x, t0, pr);
}
// read lane `src`'s value (all 64 lanes must be active)
__device__ __forceinline__ int shf(int v, int src) { return __builtin_amdgcn_ds_bpermute(src << 2, v); }
__device__ __forceinline__ u32 shf(u32 v, int src) { return (u32)__builtin_amdgcn_ds_bpermute(src << 2, (int)v); }
__device__ __forceinline__ i64 shf(i64 v, int src) {
  u32 lo = shf((u32)(u64)v, src), hi = shf((u32)((u64)v >> 32), src);
  return (i64)(((u64)hi << 32) | lo);
}
// value of a register in lane j (j uniform)
__device__ __forceinline__ int rl(int v, int j) { return __builtin_amdgcn_readlane(v, j); }
__device__ __forceinline__ u32 rl(u32 v, int j) { return (u32)__builtin_amdgcn_readlane((int)v, j); }
__device__ __forceinline__ i64 rl(i64 v, int j) {
  const u32 lo = rl((u32)(u64)v, j), hi = rl((u32)((u64)v >> 32), j);
  return (i64)(((u64)hi << 32) | lo);
}
// lane index of the r-th set bit of mask (r < popcount(mask))
__device__ __forceinline__ int nth_bit(u64 mask, int r) {
  int pos = 0;
  for (int step = 32; step >= 1; step >>= 1) {
    const int cand = pos + step;
    if (__builtin_popcountll(mask & ((1ull << cand) - 1ull)) <= r) pos = cand;
  }
  return pos;
}
// Control words (g.ctl): 0 root-chunk cursor, 1 output overflow, 2..6 work
// counters, 7 handoff error, 8 wavefronts inside a matcher, 9 wavefronts
// waiting for donated work. g.qctl holds (head, tail) of each query's queue.
// A donated work item is 32 words: 0 ready (= launch epoch), 1 level,
// 2 window start, 3 window end, 4-5 window time bound, 6 wanted neighbour,
// 7 root edge, 8-9 output chunk, 10-11 time limit, 12-19 bound motif nodes,
// 20-26 edge ids of levels 1..7.
#define ITEM_WORDS 32u
// Item words are written and read with device-coherent (agent-scope) relaxed
// atomics, so no whole-cache writeback or invalidation is needed; ordering
// comes from waiting for the field stores before the ready word is stored,
// and for the ready word before the fields are read.
__device__ __forceinline__ void st_ag(u32* p, u32 v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32 ld_ag(const u32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_ag64(u32* p, i64 v) { st_ag(p, (u32)(u64)v); st_ag(p + 1, (u32)((u64)v >> 32)); }
__device__ __forceinline__ i64 ld_ag64(const u32* p) { return (i64)(((u64)ld_ag(p + 1) << 32) | (u64)ld_ag(p)); }
__device__ __forceinline__ void mem_order() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ u64 ld_rlx64(const u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u32* item_at(const GArgs& g, int qi, u64 slot) {
  return g.items + ((u64)qi * (u64)g.item_cap + slot) * ITEM_WORDS;
}
// Reserve up to `want` donated items of query qi for this wavefront (uniform
// call, all lanes active). Returns the first slot; *n receives the count.
__device__ __forceinline__ i64 try_pop(const GArgs& g, int qi, int want, int* n) {
  i64 h = 0; int k = 0;
  if (lane_id() == 0 && want > 0) {
    u64* qc = g.qctl + 2 * qi;
    const u64 hh = ld_rlx64(&qc[0]);
    u64 tt = ld_rlx64(&qc[1]);
    if (tt > (u64)g.item_cap) tt = (u64)g.item_cap;
    if (hh < tt) {
      u64 kk = tt - hh;
      if (kk > (u64)want) kk = (u64)want;
      if (atomicCAS(&qc[0], hh, hh + kk) == hh) {
        h = (i64)hh; k = (int)kk;
        atomicAdd(&g.ctl[13], (u64)(-(i64)kk));  // items waiting in all queues
      }
    }
  }
  *n = __builtin_amdgcn_readfirstlane(k);
  return bcast64(h);
}
// Wait until a reserved item has been published by its donor.
__device__ __forceinline__ bool item_ready(const GArgs& g, const u32* it) {
  u32 spins = 0u;
  while (ld_ag(it) != g.epoch) {
    if (++spins > (1u << 22)) { atomicOr((u32*)&g.ctl[7], 1u); return false; }
    __builtin_amdgcn_s_sleep(2);
  }
  mem_order();
  return true;
}
)HIP";

namespace {

// The emitter writes either a matcher specialised to one motif (every plan
// property a constant) or, with `G`, a generic matcher for all motifs of p.l
// edges whose per-level properties (list kind, motif nodes, bound-node mask,
// window-start rule, predicate level) are read from the query's plan tables
// at run time: it trades some instructions for needing no compilation per
// motif (used when a query stream holds thousands of distinct structures).
struct Emitter {
    std::ostringstream o;
    const Plan &p;
    const bool G;
    // Step form. false: a loop step runs the search probe and the candidate
    // scan as separate branches, each waiting for its own reads, and a
    // candidate that binds opens the next level (reads its offsets) at once.
    // true: a step first issues the reads of every lane (search pivots,
    // candidate key and neighbour, or the offsets of a level to open) and
    // then consumes them, so that a wavefront waits once per step; a binding
    // candidate leaves the next level's open to the following step (phase 4).
    bool F = false;
    // Root order: false, chunk L of a query holds roots L, L + C, L + 2C, ...;
    // true (XCD order), chunks are contiguous root ranges taken per XCD from
    // 8 time slices (next_chunk).
    bool X = false;
    explicit Emitter(const Plan &pl, bool generic = false, int form = 0)
        : p(pl), G(generic), F((form & 1) != 0), X((form & 2) != 0) {}

    std::string I(int i) const { return std::to_string(i); }

    // Vertex labels (Sec. 5.4.1): a node newly bound by a candidate must carry
    // a label in its motif node's range (registers nl<v>, nh<v>: launch
    // arguments).
    bool labelled(int v) const { return !G && ((p.lab_mask >> v) & 1); }
    std::string lab_cond(int v, const std::string &node) const {
        return "in_range(g.nlab[" + node + "], nl" + I(v) + ", nh" + I(v) + ")";
    }
    // Weight predicates (attribute constraints, Sec. 2.1 / 5.4.1): every
    // predicate on motif edge i holds for weight w (pop<j>, pth<j>: launch
    // arguments of predicate slot j).
    bool has_pred(int i) const { return !G && ((p.pred_mask() >> i) & 1u); }
    std::string preds_cond(int i, const std::string &w) const {
        std::string c;
        for (int j = 0; j < p.np; j++)
            if (p.pred_lvl[j] == i) c += (c.empty() ? "" : " && ") + std::string("pred_ok(") + w + ", pop" + I(j) + ", pth" + I(j) + ")";
        return c.empty() ? "true" : c;
    }
    // Edge labels: the graph edge matched to motif edge i carries a label in
    // [elo<i>, ehi<i>] (launch arguments).
    bool has_elab(int i) const { return !G && ((p.elab_mask >> i) & 1); }
    std::string elab_cond(int i, const std::string &el) const {
        return "in_range(" + el + ", elo" + I(i) + ", ehi" + I(i) + ")";
    }
    // The motif node a level's candidate binds, for list kinds OUT and IN.
    int new_node(int i) const { return p.kind[i] == LIST_OUT ? p.b[i] : p.a[i]; }

    // Temporal anti-edges (Sec. 2.1, Sec. 5.4.3). Each is checked when the
    // candidate of its check level is accepted: the candidate is rejected when
    // the graph holds an edge between the two mapped nodes inside the
    // anti-edge's window.
    bool anti_on(int i) const {
        for (int j = 0; j < p.n_anti; j++)
            if (p.anti_lvl[j] == i) return true;
        return false;
    }
    // Level j's edge id is kept in every mode (not only when writing rows)
    // when an anti-edge attached to it is checked at a deeper level.
    bool keep_e(int j) const {
        for (int x = 0; x < p.n_anti; x++)
            if (j >= 1 && p.anti_at[x] == j && p.anti_lvl[x] > j) return true;
        return false;
    }
    std::string e_cond(int j) const { return keep_e(j) ? "true" : "MODE == 3"; }
    // The root edge id: written with each instance, and read by an anti-edge
    // attached to the root edge that is checked at a deeper level.
    std::string root_cond() const {
        for (int x = 0; x < p.n_anti; x++)
            if (p.anti_at[x] == 0 && p.anti_lvl[x] > 0) return "true";
        return "MODE == 3";
    }
    // Graph node of motif node v while level i's candidate is checked.
    std::string node_at(int i, int v) const {
        if (i == 0) return v == p.a[0] ? "s" : "d";
        for (int u : p.mapped[i])
            if (u == v) return "m" + I(v);
        if (p.kind[i] == LIST_GLOBAL) return v == p.a[i] ? "cs" : "cd";
        return "nb";  // the node the candidate binds
    }
    // Time of the edge matched at level `at` while level i's candidate is checked.
    std::string time_at(int i, int at) const {
        if (at == i) return i == 0 ? "tr" : "tt";
        if (at == 0) return "g.tk[root]";
        return "g.tk[e" + I(at) + "]";
    }
    std::string anti_cond(int i) const {
        std::ostringstream c;
        bool first = true;
        for (int j = 0; j < p.n_anti; j++) {
            if (p.anti_lvl[j] != i) continue;
            c << (first ? "" : " && ") << "anti_free(g, " << node_at(i, p.anti_a[j]) << ", "
              << node_at(i, p.anti_b[j]) << ", " << time_at(i, p.anti_at[j]) << ", adl" << j << ")";
            first = false;
        }
        return c.str();
    }

    bool has_global() const {
        if (G) return true;
        for (int i = 1; i < p.l; i++)
            if (p.kind[i] == LIST_GLOBAL) return true;
        return false;
    }

    // Where level i's window can start without a search: when level i reads
    // the list that holds the edge matched at level i-1 (the out-list of its
    // source or the in-list of its destination), the window begins right after
    // that edge's position, then skips equal timestamps. Returns the position
    // expression ("" if a search is needed); `c` is the scan position of level
    // i-1, `r` the root edge.
    std::string jump_of(int i) const {
        if (i < 1 || p.kind[i] == LIST_BOTH || p.kind[i] == LIST_GLOBAL) return "";
        if (p.kind[i] == LIST_OUT && p.a[i] == p.a[i - 1]) {
            if (i == 1) return "g.pos_out[r] + 1u";
            if (p.kind[i - 1] == LIST_OUT) return "c + 1u";
        }
        if (p.kind[i] == LIST_IN && p.b[i] == p.b[i - 1]) {
            if (i == 1) return "g.pos_in[r] + 1u";
            if (p.kind[i - 1] == LIST_IN) return "c + 1u";
        }
        return "";
    }

    // Open level i's window after binding edge i-1 at time `tp`; with a known
    // start the search collapses to the tie skip (not in the work-counter mode,
    // which follows the byte model's one search per window).
    void open(int i, const char *tp, const char *ind) {
        if (leaf_cache() && i == p.l - 2) o << ind << "lq = false;\n";
        if (F) {
            // the next step reads the list offsets; a known window start (see
            // jump_of) is kept in sb until then, the bound edge's time in sx
            if (G) {
                if (i == 1)
                    o << ind << "if (MODE != 1 && gj1 != 0) sb = (gj1 == 1 ? g.pos_out[r] : g.pos_in[r]) + 1u;\n";
                else
                    o << ind << "if (MODE != 1 && gj" << i << " != 0) sb = c + 1u;\n";
            } else {
                const std::string jump = jump_of(i);
                if (!jump.empty()) o << ind << "if (MODE != 1) sb = " << jump << ";\n";
            }
            o << ind << "sx = (" << tp << "); lvl = " << i << "; ph = 4;\n";
            return;
        }
        if (G) {
            const std::string in2 = std::string(ind) + "  ";
            o << ind << "if (MODE != 1 && gj" << i << " != 0) {\n";
            if (i == 1)
                o << in2 << "const u32 lo_ = (gj1 == 1 ? g.pos_out[r] : g.pos_in[r]) + 1u;\n";
            else
                o << in2 << "const u32 lo_ = c + 1u;\n";
            o << in2 << "const u32 hi_ = gk" << i << " == 0 ? g.off_out[mget(ga" << i << ") + 1] : g.off_in[mget(gb"
              << i << ") + 1];\n";
            o << in2 << "end" << i << " = hi_; exact &= ~" << (1 << i) << "u;\n";
            o << in2 << "{ i64 h_ = (i64)(" << tp << ") + gap" << (i - 1) << "; hi" << i
              << " = (tkey)(h_ < (i64)tmaxk ? h_ : (i64)tmaxk); }\n";
            o << in2 << "sb = lo_; sn = hi_ - lo_; sx = (" << tp << "); lvl = " << i << ";\n";
            o << in2 << "if (sn == 0u) { cur" << i << " = lo_; ph = 0; } else { ph = 2; }\n";
            o << ind << "} else {\n";
            open_search(i, tp, in2.c_str());
            o << ind << "}\n";
            return;
        }
        const std::string jump = jump_of(i);
        if (jump.empty()) {
            open_search(i, tp, ind);
            return;
        }
        std::string in2 = std::string(ind) + "  ";
        o << ind << "if (MODE == 1) {\n";
        open_search(i, tp, in2.c_str());
        o << ind << "} else {\n";
        o << in2 << "const u32 lo_ = " << jump << ";\n";
        if (p.kind[i] == LIST_OUT)
            o << in2 << "const u32 hi_ = g.off_out[m" << p.a[i] << " + 1];\n";
        else
            o << in2 << "const u32 hi_ = g.off_in[m" << p.b[i] << " + 1];\n";
        o << in2 << "end" << i << " = hi_; exact &= ~" << (1 << i) << "u;\n";
        o << in2 << "{ i64 h_ = (i64)(" << tp << ") + gap" << (i - 1) << "; hi" << i
          << " = (tkey)(h_ < (i64)tmaxk ? h_ : (i64)tmaxk); }\n";
        o << in2 << "sb = lo_; sn = hi_ - lo_; sx = (" << tp << "); lvl = " << i << ";\n";
        o << in2 << "if (sn == 0u) { cur" << i << " = lo_; ph = 0; } else { ph = 2; }\n";
        o << ind << "}\n";
    }

    void open_search(int i, const char *tp, const char *ind) {
        const int A = p.a[i], B = p.b[i];
        o << ind << "{ // open level " << i << "\n";
        o << ind << "  u32 lo_, hi_;\n";
        if (G) {
            const std::string s = I(i);
            o << ind << "  if (gk" << s << " == 0) { const int v_ = mget(ga" << s
              << "); lo_ = g.off_out[v_]; hi_ = g.off_out[v_ + 1]; }\n";
            o << ind << "  else if (gk" << s << " == 1) { const int v_ = mget(gb" << s
              << "); lo_ = g.off_in[v_]; hi_ = g.off_in[v_ + 1]; }\n";
            o << ind << "  else if (gk" << s << " == 2) {\n";
            o << ind << "    const int va = mget(ga" << s << "), vb = mget(gb" << s << ");\n";
            o << ind << "    const u32 la = g.off_out[va], ha = g.off_out[va + 1], lb = g.off_in[vb], hb = g.off_in[vb + 1];\n";
            o << ind << "    const bool uo = (ha - la) <= (hb - lb);\n";
            o << ind << "    lo_ = uo ? la : lb; hi_ = uo ? ha : hb; want" << s << " = uo ? vb : va;\n";
            o << ind << "  } else { lo_ = 0u; hi_ = (u32)g.m_edges; }\n";
        } else switch (p.kind[i]) {
        case LIST_OUT:
            o << ind << "  lo_ = g.off_out[m" << A << "]; hi_ = g.off_out[m" << A << " + 1];\n";
            break;
        case LIST_IN:
            o << ind << "  lo_ = g.off_in[m" << B << "]; hi_ = g.off_in[m" << B << " + 1];\n";
            break;
        case LIST_BOTH:
            o << ind << "  { u32 la = g.off_out[m" << A << "], ha = g.off_out[m" << A << " + 1];\n";
            o << ind << "    u32 lb = g.off_in[m" << B << "], hb = g.off_in[m" << B << " + 1];\n";
            o << ind << "    bool uo = (ha - la) <= (hb - lb);\n";
            o << ind << "    lo_ = uo ? la : lb; hi_ = uo ? ha : hb; want" << i << " = uo ? m" << B << " : m" << A
              << "; }\n";
            break;
        default:
            o << ind << "  lo_ = 0u; hi_ = (u32)g.m_edges;\n";
        }
        o << ind << "  end" << i << " = hi_; exact &= ~" << (1 << i) << "u;\n";
        o << ind << "  { i64 h_ = (i64)(" << tp << ") + gap" << (i - 1) << "; hi" << i
          << " = (tkey)(h_ < (i64)tmaxk ? h_ : (i64)tmaxk); }\n";
        o << ind << "  sb = lo_; sn = hi_ - lo_; sx = (" << tp << "); lvl = " << i << ";\n";
        o << ind << "  if (MODE == 1) { st_win++; st_probe += bitlen(sn); }\n";
        // a long window first searches the line samples inside the list
        // (phase 5: sb, sn index the samples; cur<i> keeps the list start)
        o << ind << "  bool ls_ = false;\n";
        if (G) {
            o << ind << "  if (MODE != 1 && g.hub_words != 0u && gk" << i << " != 3 && sn >= g.hub_dmin) hub_narrow(lo_, sx, sb, sn);\n";
            o << ind << "  if (MODE != 1 && g.samp_min != 0u && gk" << i << " != 3 && sn >= g.samp_min) {\n";
        } else if (p.kind[i] != LIST_GLOBAL) {
            o << ind << "  if (MODE != 1 && g.hub_words != 0u && sn >= g.hub_dmin) hub_narrow(lo_, sx, sb, sn);\n";
            o << ind << "  if (MODE != 1 && g.samp_min != 0u && sn >= g.samp_min) {\n";
        }
        if (G || p.kind[i] != LIST_GLOBAL) {
            o << ind << "    const u32 j0 = (lo_ + (1u << g.samp_lg) - 1u) >> g.samp_lg, j1 = (hi_ - 1u) >> g.samp_lg;\n";
            o << ind << "    if (j0 <= j1) { cur" << i << " = lo_; sb = j0; sn = j1 - j0 + 1u; ls_ = true; }\n";
            o << ind << "  }\n";
        }
        o << ind << "  if (ls_) ph = 5; else if (sn == 0u) { cur" << i << " = sb; ph = 0; } else { ph = 1; }\n";
        o << ind << "}\n";
    }

    // Phase 4 reads: the offsets of the list level i opens.
    void open_reads(int i, const char *ind) {
        if (G) {
            const std::string s = I(i);
            o << ind << "if (gk" << s << " == 0 || gk" << s << " == 2) { const int x_ = mget(ga" << s
              << "); f1 = g.off_out[x_]; f2 = g.off_out[x_ + 1]; }\n";
            o << ind << "else if (gk" << s << " == 1) { const int y_ = mget(gb" << s
              << "); f1 = g.off_in[y_]; f2 = g.off_in[y_ + 1]; }\n";
            o << ind << "if (gk" << s << " == 2) { const int y_ = mget(gb" << s
              << "); f3 = g.off_in[y_]; f4 = g.off_in[y_ + 1]; }\n";
            return;
        }
        const int A = p.a[i], B = p.b[i];
        switch (p.kind[i]) {
        case LIST_OUT:
            o << ind << "f1 = g.off_out[m" << A << "]; f2 = g.off_out[m" << A << " + 1];\n";
            break;
        case LIST_IN:
            o << ind << "f1 = g.off_in[m" << B << "]; f2 = g.off_in[m" << B << " + 1];\n";
            break;
        case LIST_BOTH:
            o << ind << "f1 = g.off_out[m" << A << "]; f2 = g.off_out[m" << A << " + 1];\n";
            o << ind << "f3 = g.off_in[m" << B << "]; f4 = g.off_in[m" << B << " + 1];\n";
            break;
        default:
            break;
        }
    }

    // Level i's window once lo_, hi_ are known; `jump`: the start needs only
    // the tie skip (phase 2), else a search (phase 1).
    void open_tail(int i, bool jump, bool hub, const char *ind) {
        o << ind << "end" << i << " = hi_; exact &= ~" << (1 << i) << "u;\n";
        o << ind << "{ i64 h_ = (i64)sx + gap" << (i - 1) << "; hi" << i
          << " = (tkey)(h_ < (i64)tmaxk ? h_ : (i64)tmaxk); }\n";
        o << ind << "sb = lo_; sn = hi_ - lo_;\n";
        if (jump) {
            o << ind << "if (sn == 0u) { cur" << i << " = lo_; ph = 0; } else { ph = 2; }\n";
            return;
        }
        o << ind << "if (MODE == 1) { st_win++; st_probe += bitlen(sn); }\n";
        if (hub) {
            o << ind << "if (MODE != 1 && g.hub_words != 0u && sn >= g.hub_dmin) hub_narrow(lo_, sx, sb, sn);\n";
            o << ind << "if (MODE != 1 && g.samp_min != 0u && sn >= g.samp_min) line_narrow(g.samp, g.samp_lg, lo_, hi_, sx, sb, sn);\n";
        }
        o << ind << "if (sn == 0u) { cur" << i << " = sb; ph = 0; } else { ph = 1; }\n";
    }

    // Phase 4: open level i from the offsets read this step.
    void open_use(int i, const char *ind) {
        const std::string in2 = std::string(ind) + "  ";
        o << ind << "u32 lo_ = 0u, hi_ = 0u;\n";
        if (G) {
            const std::string s = I(i);
            o << ind << "if (MODE != 1 && gj" << s << " != 0) {\n";
            o << in2 << "lo_ = sb; hi_ = f2;\n";
            open_tail(i, true, false, in2.c_str());
            o << ind << "} else {\n";
            o << in2 << "if (gk" << s << " == 0 || gk" << s << " == 1) { lo_ = f1; hi_ = f2; }\n";
            o << in2 << "else if (gk" << s << " == 2) { const bool uo = (f2 - f1) <= (f4 - f3);\n";
            o << in2 << "  lo_ = uo ? f1 : f3; hi_ = uo ? f2 : f4; want" << s << " = uo ? mget(gb" << s << ") : mget(ga"
              << s << "); }\n";
            o << in2 << "else { lo_ = 0u; hi_ = (u32)g.m_edges; }\n";
            o << in2 << "end" << i << " = hi_; exact &= ~" << (1 << i) << "u;\n";
            o << in2 << "{ i64 h_ = (i64)sx + gap" << (i - 1) << "; hi" << i
              << " = (tkey)(h_ < (i64)tmaxk ? h_ : (i64)tmaxk); }\n";
            o << in2 << "sb = lo_; sn = hi_ - lo_;\n";
            o << in2 << "if (MODE == 1) { st_win++; st_probe += bitlen(sn); }\n";
            o << in2 << "if (MODE != 1 && g.hub_words != 0u && gk" << s
              << " != 3 && sn >= g.hub_dmin) hub_narrow(lo_, sx, sb, sn);\n";
            o << in2 << "if (MODE != 1 && g.samp_min != 0u && gk" << s
              << " != 3 && sn >= g.samp_min) line_narrow(g.samp, g.samp_lg, lo_, hi_, sx, sb, sn);\n";
            o << in2 << "if (sn == 0u) { cur" << i << " = sb; ph = 0; } else { ph = 1; }\n";
            o << ind << "}\n";
            return;
        }
        const bool jump = !jump_of(i).empty();
        std::string in = ind;
        if (jump) {
            o << ind << "if (MODE != 1) {\n";
            o << in2 << "lo_ = sb; hi_ = f2;\n";
            open_tail(i, true, false, in2.c_str());
            o << ind << "} else {\n";
            in = in2;
        }
        const int A = p.a[i], B = p.b[i];
        switch (p.kind[i]) {
        case LIST_OUT:
        case LIST_IN:
            o << in << "lo_ = f1; hi_ = f2;\n";
            break;
        case LIST_BOTH:
            o << in << "{ const bool uo = (f2 - f1) <= (f4 - f3);\n";
            o << in << "  lo_ = uo ? f1 : f3; hi_ = uo ? f2 : f4; want" << i << " = uo ? m" << B << " : m" << A << "; }\n";
            break;
        default:
            o << in << "lo_ = 0u; hi_ = (u32)g.m_edges;\n";
        }
        open_tail(i, false, p.kind[i] != LIST_GLOBAL, in.c_str());
        if (jump) o << ind << "}\n";
    }

    // One loop step in the fused form (see F): the reads of every lane first,
    // then their use. Phase 4 opens the level chosen in the previous step.
    void step_fused() {
        const int L = p.l;
        const bool glob = has_global();
        bool any_pred = false, any_elab = false;
        for (int i = 1; i < L; i++) {
            any_pred |= has_pred(i);
            any_elab |= has_elab(i);
        }
        o << "    if (lvl > 0 && ph != 3) {\n";
        if (G) {
            o << "      const bool glv = ((gglob >> lvl) & 1u) != 0u;\n";
        } else if (glob) {
            o << "      bool glv = false;\n";
            for (int i = 1; i < L; i++)
                if (p.kind[i] == LIST_GLOBAL) o << "      glv = glv || lvl == " << i << ";\n";
        }
        o << "      const tkey* sarr = " << (G || glob ? "glv ? g.tk : g.adj_t" : "g.adj_t") << ";\n";
        o << "      u32 c = 0u, e = 0u; tkey h = 0;\n";
        o << "      if (ph == 0) {\n";
        o << "        switch (lvl) {\n";
        for (int i = 1; i < L; i++)
            o << "          case " << i << ": c = cur" << i << "; e = end" << i << "; h = hi" << i << "; break;\n";
        o << "          default: break;\n";
        o << "        }\n";
        o << "      }\n";
        o << "      // the step's reads, issued together so that the wavefront waits once\n";
        o << "      tkey v1 = 0, v2 = 0, v3 = 0; int nb = 0; u32 f1 = 0u, f2 = 0u, f3 = 0u, f4 = 0u;";
        if (G || any_pred) o << " float wv = 0.0f;";
        if (G || any_elab) o << " int ev = 0;";
        o << "\n";
        o << "      u32 o1 = 0u, o2 = 0u, o3 = 0u;\n";
        o << "      const bool four = ph == 1 && sn >= 3u;  // three pivots, else one\n";
        o << "      if (ph == 4) {\n";
        o << "        switch (lvl) {\n";
        for (int i = 1; i < L; i++) {
            o << "          case " << i << ": {\n";
            open_reads(i, "            ");
            o << "          } break;\n";
        }
        o << "          default: break;\n";
        o << "        }\n";
        o << "      } else if (ph == 0) {\n";
        o << "        if (c < e) {\n";
        o << "          v1 = sarr[c];\n";
        if (G) {
            o << "          if (!glv) nb = g.adj_nbr[c];\n";
            o << "          if ((gpm >> lvl) & 1u) wv = glv ? g.w[c] : g.adj_w[c];\n";
            o << "          if ((gelm >> lvl) & 1u) ev = glv ? g.el[c] : g.adj_el[c];\n";
        } else {
            o << "          " << (glob ? "if (!glv) " : "") << "nb = g.adj_nbr[c];\n";
            for (int i = 1; i < L; i++) {
                if (has_pred(i))
                    o << "          if (lvl == " << i << ") wv = " << (p.kind[i] == LIST_GLOBAL ? "g.w[c]" : "g.adj_w[c]")
                      << ";\n";
                if (has_elab(i))
                    o << "          if (lvl == " << i << ") ev = " << (p.kind[i] == LIST_GLOBAL ? "g.el[c]" : "g.adj_el[c]")
                      << ";\n";
            }
        }
        o << "        }\n";
        o << "      } else if (four) {\n";
        o << "        o1 = ((sn + 1u) >> 2) - 1u; o2 = ((2u * (sn + 1u)) >> 2) - 1u; o3 = ((3u * (sn + 1u)) >> 2) - 1u;\n";
        o << "        v1 = sarr[sb + o1]; v2 = sarr[sb + o2]; v3 = sarr[sb + o3];\n";
        o << "      } else {\n";
        o << "        o1 = ph == 2 ? 0u : (sn >> 1);\n";
        o << "        v1 = sarr[sb + o1];\n";
        o << "      }\n";
        o << "      if (ph == 4) {\n";
        o << "        switch (lvl) {\n";
        for (int i = 1; i < L; i++) {
            o << "          case " << i << ": {\n";
            open_use(i, "            ");
            o << "          } break;\n";
        }
        o << "          default: break;\n";
        o << "        }\n";
        o << "      } else if (ph == 0) {\n";
        o << "      const tkey tt = v1; const bool inwin = c < e && tt <= h;\n";
        if (G)
            o << "      if (MODE == 1 && c < e) { st_visit++; if ((gpm >> lvl) & 1u) st_pv++; }\n";
        else
            o << "      if (MODE == 1 && c < e) { st_visit++;"
              << (any_pred ? " if ((" + std::to_string(p.pred_mask()) + "u >> lvl) & 1u) st_pv++;" : std::string())
              << " }\n";
        visit_accept();
        o << "      } else {\n";
        o << "      if (four) {\n";
        o << "        if (v3 <= sx) { sb += o3 + 1u; sn -= o3 + 1u; }\n";
        o << "        else if (v2 <= sx) { sb += o2 + 1u; sn = o3 - o2 - 1u; }\n";
        o << "        else if (v1 <= sx) { sb += o1 + 1u; sn = o2 - o1 - 1u; }\n";
        o << "        else { sn = o1; }\n";
        o << "      } else {\n";
        o << "        if (v1 <= sx) { sb += o1 + 1u; sn = sn - o1 - 1u; } else { sn = o1; }\n";
        o << "      }\n";
        o << "      ph = 1;\n";
        search_done();
        o << "      }\n";
        o << "    }\n";
    }

    // A search has ended (sn == 0): the window starts at sb.
    void search_done() {
        const int L = p.l;
        o << "      if (sn == 0u) {\n";
        o << "        bool park = false;\n";
        o << "        switch (lvl) {\n";
        for (int i = 1; i < L; i++) {
            if (i == L - 1 && coop_ok()) {
                // peek 32 candidates ahead: a window that reaches that far is
                // scanned by the whole wavefront, or, when counting and the
                // window's count has a closed form, counted without a scan
                o << "          case " << i << ": cur" << i << " = sb;\n";
                o << "            if (MODE != 1" << (G ? " && !((gglob >> " + I(i) + ") & 1u)" : std::string())
                  << ") { const u32 pk = sb + 31u; wide = pk < end" << i << " && g.adj_t[pk] <= hi" << i << "; }\n";
                leaf_count(i);
                o << "            break;\n";
            } else {
                o << "          case " << i << ": cur" << i << " = sb; break;\n";
            }
        }
        o << "          default: break;\n";
        o << "        }\n";
        o << "        ph = park ? 3 : 0;\n";
        o << "      }\n";
    }

    // The candidate read at position c of level lvl (tt, nb, wv, ev): leave the
    // level when it is past the window, else check it and bind or count it.
    void visit_accept() {
        const int L = p.l;
        o << "      if (!inwin) {\n";
        o << "        lvl -= 1;\n";
        o << "        if (lvl < base) {\n";
        o << "          lvl = 0;\n";
        o << "          if (MODE == 2 && rcnt) { atomicAdd(&g.chunk_cnt[mych], rcnt); cnt += rcnt; rcnt = 0; }\n";
        o << "        }\n";
        o << "      } else {\n";
        o << "        switch (lvl) {\n";
        for (int i = 1; i < L; i++) {
            const int A = p.a[i], B = p.b[i];
            o << "        case " << i << ": {\n";
            o << "          cur" << i << " = c + 1u;\n";
            if (G) {
                const std::string s = I(i);
                const std::string ms = "m0, m1, m2, m3, m4, m5, m6, m7";
                const std::string eidx = "(gk" + s + " == 3 ? (int)c : g.adj_eid[c])";
                o << "          int cs = 0, cd = 0; bool ok;\n";
                o << "          if (gk" << s << " == 2) ok = nb == want" << s << ";\n";
                o << "          else if (gk" << s << " == 3) { cs = g.src[c]; cd = g.dst[c];\n";
                o << "            ok = cs != cd && notin(gm" << s << ", cs, " << ms << ") && notin(gm" << s
                  << ", cd, " << ms << "); }\n";
                o << "          else ok = notin(gm" << s << ", nb, " << ms << ");\n";
                o << "          if (glm != 0u) {\n";
                o << "            if (gk" << s << " == 3) {\n";
                o << "              if ((glm >> ga" << s << ") & 1u) ok = ok && in_range(g.nlab[cs], lget(ga" << s
                  << "), hget(ga" << s << "));\n";
                o << "              if ((glm >> gb" << s << ") & 1u) ok = ok && in_range(g.nlab[cd], lget(gb" << s
                  << "), hget(gb" << s << "));\n";
                o << "            } else if (gk" << s << " != 2 && ((glm >> gn" << s << ") & 1u)) {\n";
                o << "              ok = ok && in_range(g.nlab[nb], lget(gn" << s << "), hget(gn" << s << "));\n";
                o << "            }\n";
                o << "          }\n";
                o << "          if ((gpm >> " << i << ") & 1u) ok = ok && preds_at(q, " << i << ", wv);\n";
                o << "          if ((gelm >> " << i << ") & 1u) ok = ok && in_range(ev, q->elo[" << i << "], q->ehi[" << i
                  << "]);\n";
                o << "          if (ok) {\n";
                if (i == L - 1) {
                    leaf("            ", eidx.c_str());
                } else {
                    o << "            if (gk" << s << " == 0) mset(gb" << s << ", nb);\n";
                    o << "            else if (gk" << s << " == 1) mset(ga" << s << ", nb);\n";
                    o << "            else if (gk" << s << " == 3) { mset(ga" << s << ", cs); mset(gb" << s
                      << ", cd); }\n";
                    o << "            if (MODE == 3) e" << i << " = " << eidx << ";\n";
                    open(i + 1, "tt", "            ");
                }
                o << "          }\n";
                o << "        } break;\n";
                continue;
            }
            std::ostringstream ok;
            std::string bind;
            std::string eid;
            switch (p.kind[i]) {
            case LIST_OUT:
            case LIST_IN: {
                ok << "true";
                for (int v : p.mapped[i]) ok << " && nb != m" << v;
                if (labelled(new_node(i))) ok << " && " << lab_cond(new_node(i), "nb");
                bind = "m" + std::to_string(p.kind[i] == LIST_OUT ? B : A) + " = nb;";
                eid = "g.adj_eid[c]";
                break;
            }
            case LIST_BOTH:
                ok << "nb == want" << i;
                eid = "g.adj_eid[c]";
                break;
            default: {
                o << "          const int cs = g.src[c], cd = g.dst[c];\n";
                ok << "cs != cd";
                for (int v : p.mapped[i]) ok << " && cs != m" << v << " && cd != m" << v;
                if (labelled(A)) ok << " && " << lab_cond(A, "cs");
                if (labelled(B)) ok << " && " << lab_cond(B, "cd");
                bind = "m" + std::to_string(A) + " = cs; m" + std::to_string(B) + " = cd;";
                eid = "(int)c";
            }
            }
            o << "          bool ok = " << ok.str() << ";\n";
            if (has_pred(i)) o << "          ok = ok && " << preds_cond(i, "wv") << ";\n";
            if (has_elab(i)) o << "          ok = ok && " << elab_cond(i, "ev") << ";\n";
            if (anti_on(i)) o << "          ok = ok && " << anti_cond(i) << ";\n";
            o << "          if (ok) {\n";
            if (i == L - 1) {
                leaf("            ", eid.c_str());
            } else {
                if (!bind.empty()) o << "            " << bind << "\n";
                o << "            if (" << e_cond(i) << ") e" << i << " = " << eid << ";\n";
                open(i + 1, "tt", "            ");
            }
            o << "          }\n";
            o << "        } break;\n";
        }
        o << "        default: break;\n";
        o << "        }\n";
        o << "      }\n";
    }

    void leaf(const char *ind, const char *last_eid) {
        o << ind << "if (MODE == 0 || MODE == 1) { cnt++; }\n";
        o << ind << "else if (MODE == 2) { rcnt++; }\n";
        o << ind << "else {\n";
        o << ind << "  u64 slot = g.chunk_off[mych] + atomicAdd(&g.chunk_cnt[mych], 1ull);\n";
        o << ind << "  if (slot < g.capacity) {\n";
        o << ind << "    i64* row = g.out + slot * " << p.l << "ull;\n";
        o << ind << "    row[0] = (i64)root;\n";
        for (int j = 1; j + 1 < p.l; j++) o << ind << "    row[" << j << "] = (i64)e" << j << ";\n";
        if (p.l > 1) o << ind << "    row[" << (p.l - 1) << "] = (i64)(" << last_eid << ");\n";
        o << ind << "  } else { atomicAdd(&g.ctl[1], 1ull); }\n";
        o << ind << "  cnt++;\n";
        o << ind << "}\n";
    }

    // Intra-wavefront work splitting (sub-tree-level parallelism, Sec. 5.2,
    // in the spirit of intra-warp work stealing, Sec. 5.2.1). Once the root
    // queue is drained, every busy lane finds its shallowest level that still
    // holds at least two candidates inside the time window (an upper-bound
    // search on the window's end also trims the cached window to its exact
    // extent, as the paper's context refinement does), and gives a later part
    // of those pending candidates, with the bound state above that level, to
    // one idle lane through cross-lane permutes. Donor and thief keep disjoint
    // candidate ranges, so every instance is still found exactly once.
    void steal() {
        const int L = p.l, K = p.k;
        o << "    if (q_split && drained && MODE != 1) {\n";
        o << "      iter++;\n";
        // Tail redistribution of unstarted roots (Sec. 5.2.2 redistributes
        // the tail's work): once the root queue is empty, a wavefront whose
        // pool still holds 16 or more roots of its chunk hands the last half
        // of them, one root per item, to the query's queue while some
        // wavefronts wait for work
        o << "      if ((g.split & 2) && g.items != 0 && ghungry > 0 && (iter & 31u) == 8u && pend - pnext >= 16) {\n";
        o << "        const i64 give = (pend - pnext) >> 1;\n";
        o << "        i64 s0 = 0;\n";
        o << "        if (lane == 0) s0 = (i64)atomicAdd(&g.qctl[2 * qi + 1], (u64)give);\n";
        o << "        s0 = bcast64(s0);\n";
        o << "        const i64 room = (i64)g.item_cap - s0;\n";
        o << "        const i64 fit = room <= 0 ? 0 : (room < give ? room : give);\n";
        o << "        for (i64 t = lane; t < fit; t += 64) {\n";
        o << "          const i64 k = pend - fit + t;\n";
        o << "          u32* it = item_at(g, qi, (u64)(s0 + t));\n";
        o << "          st_ag(it + 1, 0u); st_ag(it + 7, (u32)(" << (X ? "q_r0 + (pchunk - q_c0) * q_rch + k" : "q_r0 + (pchunk - q_c0) + k * q_nch") << ")); st_ag64(it + 8, pchunk);\n";
        o << "          mem_order();\n";
        o << "          st_ag(it, g.epoch);\n";
        o << "        }\n";
        // items waiting in all queues; roots handed so far
        o << "        if (lane == 0 && fit > 0) { atomicAdd(&g.ctl[13], (u64)fit); atomicAdd(&g.ctl[14], (u64)fit); }\n";
        o << "        pend -= fit;\n";
        o << "      }\n";
        o << "      if ((iter & 31u) == 0u && g.items != 0) {\n";
        o << "        i64 hv = 0; if (lane == 0) hv = (i64)ld_rlx64(&g.ctl[9]); ghungry = bcast64(hv);\n";
        o << "      }\n";
        o << "      const u64 idle = ballot(lvl < 0);\n";
        o << "      const bool gl = g.items != 0 && ghungry > 0 && (iter & 31u) == 0u;\n";
        o << "      if ((idle != 0ull || gl) && cool == 0) {\n";
        o << "        const u64 busy = ballot(lvl > 0);\n";
        o << "        if (busy != 0ull) {\n";
        o << "          int dj = 0; u32 ds = 0u, de = 0u; tkey dh = 0; int dw = 0;\n";
        o << "          if (lvl > 0) {\n";
        o << "            const int top = ph >= 1 ? lvl - 1 : lvl;\n";
        for (int i = 1; i < L; i++) {
            // wide last-level windows are scanned by the whole wavefront already
            if (!G && i == L - 1 && coop_ok()) continue;
            std::string arr = p.kind[i] == LIST_GLOBAL ? "g.tk" : "g.adj_t";
            std::string extra;
            if (G) {
                arr = "(((gglob >> " + I(i) + ") & 1u) ? g.tk : g.adj_t)";
                if (i == L - 1) extra = " && ((gglob >> " + I(i) + ") & 1u)";
            }
            o << "            if (dj == 0 && base <= " << i << " && " << i << " <= top && end" << i << " - cur" << i
              << " >= q_smin" << extra << ") {\n";
            o << "              u32 lo = cur" << i << ", n = end" << i << " - cur" << i << ";\n";
            o << "              if (exact & " << (1 << i) << "u) { lo = end" << i << "; n = 0u; }\n";
            o << "              while (n > 0u) { const u32 h2 = n >> 1; if (" << arr << "[lo + h2] <= hi" << i
              << ") { lo += h2 + 1u; n -= h2 + 1u; } else { n = h2; } }\n";
            o << "              const u32 P = lo - cur" << i << ";\n";
            o << "              end" << i << " = lo; exact |= " << (1 << i) << "u;\n";
            o << "              if (P >= 2u) {\n";
            o << "                dj = " << i << "; de = lo; dh = hi" << i << ";";
            if (G || p.kind[i] == LIST_BOTH) o << " dw = want" << i << ";";
            o << "\n";
            if (i == L - 1)
                o << "                ds = cur" << i << " + (P >> 1);\n";
            else
                o << "                { u32 f = (P * 3u) / 10u; ds = cur" << i << " + (f < 1u ? 1u : f); }\n";
            o << "              }\n";
            o << "            }\n";
        }
        o << "          }\n";
        // A donor at the level just above a wavefront-cooperative last level
        // whose last leaf window was wide gives nothing to idle lanes of its
        // own wavefront: every candidate it hands over opens another wide leaf
        // that the same wavefront scans one at a time anyway. Such work only
        // moves to other wavefronts (below).
        const int cp = coop_ok() ? L - 2 : -1;
        o << "          const u64 donors = ballot(dj > 0 && !(dj == " << cp << " && wide));\n";
        o << "          const int ni = __builtin_popcountll(idle), nd = __builtin_popcountll(donors);\n";
        o << "          const int np = ni < nd ? ni : nd;\n";
        o << "          const int rd = rank_in(donors);\n";
        o << "          if (np > 0) {\n";
        o << "            const int rt = rank_in(idle);\n";
        o << "            const bool thief = lvl < 0 && rt < np;\n";
        o << "            const int srcl = thief ? nth_bit(donors, rt) : lane;\n";
        o << "            const int t_dj = shf(dj, srcl); const u32 t_ds = shf(ds, srcl), t_de = shf(de, srcl);\n";
        o << "            const tkey t_dh = shf(dh, srcl); const int t_dw = shf(dw, srcl);\n";
        o << "            const int t_root = " << root_cond() << " ? shf(root, srcl) : 0;\n";
        o << "            const i64 t_mych = MODE >= 2 ? shf(mych, srcl) : 0;\n";
        o << "            const tkey t_tmax = shf(tmaxk, srcl);\n";
        for (int v = 0; v < K; v++) o << "            const int t_m" << v << " = shf(m" << v << ", srcl);\n";
        for (int j = 1; j + 1 < L; j++)
            o << "            const int t_e" << j << " = " << e_cond(j) << " ? shf(e" << j << ", srcl) : 0;\n";
        o << "            if (thief) {\n";
        o << "              lvl = t_dj; base = t_dj; ph = 0; root = t_root; mych = t_mych; tmaxk = t_tmax;\n";
        if (leaf_cache()) o << "              lq = false;\n";
        o << "              exact = 1u << t_dj;\n";
        for (int v = 0; v < K; v++) o << "              m" << v << " = t_m" << v << ";\n";
        for (int j = 1; j + 1 < L; j++) o << "              if (" << e_cond(j) << ") e" << j << " = t_e" << j << ";\n";
        o << "              switch (t_dj) {\n";
        for (int i = 1; i < L; i++) {
            o << "                case " << i << ": cur" << i << " = t_ds; end" << i << " = t_de; hi" << i
              << " = t_dh;";
            if (G || p.kind[i] == LIST_BOTH) o << " want" << i << " = t_dw;";
            o << " break;\n";
        }
        o << "                default: break;\n";
        o << "              }\n";
        o << "            } else if (((donors >> lane) & 1ull) && rd < np) {\n";
        o << "              switch (dj) {\n";
        for (int i = 1; i < L; i++) o << "                case " << i << ": end" << i << " = ds; break;\n";
        o << "                default: break;\n";
        o << "              }\n";
        o << "            }\n";
        o << "          }\n";
        // donors not paired inside the wavefront publish their split part for
        // wavefronts that ran out of work (cross-wavefront redistribution)
        o << "          bool pushed = false;\n";
        o << "          const bool gave = ((donors >> lane) & 1ull) && rd < np;\n";
        o << "          const u64 pushers = ballot(dj > 0 && !gave);\n";
        o << "          if (gl && dj > 0 && !gave && rank_in(pushers) < 16) {\n";
        o << "            const u64 slot = atomicAdd(&g.qctl[2 * qi + 1], 1ull);\n";
        o << "            if (slot < (u64)g.item_cap) {\n";
        o << "              atomicAdd(&g.ctl[13], 1ull);  // items waiting in all queues\n";
        o << "              u32* it = item_at(g, qi, slot);\n";
        o << "              st_ag(it + 1, (u32)dj); st_ag(it + 2, ds); st_ag(it + 3, de); st_ag64(it + 4, (i64)dh);\n";
        o << "              st_ag(it + 6, (u32)dw); st_ag(it + 7, (u32)root); st_ag64(it + 8, mych);\n";
        o << "              st_ag64(it + 10, (i64)tmaxk);\n";
        for (int v = 0; v < K; v++) o << "              st_ag(it + " << 12 + v << ", (u32)m" << v << ");\n";
        for (int j = 1; j + 1 < L; j++)
            o << "              if (" << e_cond(j) << ") st_ag(it + " << 19 + j << ", (u32)e" << j << ");\n";
        o << "              mem_order();\n";
        o << "              st_ag(it, g.epoch);\n";
        o << "              pushed = true;\n";
        o << "              switch (dj) {\n";
        for (int i = 1; i < L; i++) o << "                case " << i << ": end" << i << " = ds; break;\n";
        o << "                default: break;\n";
        o << "              }\n";
        o << "            }\n";
        o << "          }\n";
        o << "          const bool any_push = ballot(pushed) != 0ull;\n";
        o << "          cool = (np > 0 || any_push) ? 0 : 16;\n";
        o << "        }\n";
        o << "      }\n";
        o << "      if (cool > 0) cool--;\n";
        // idle lanes still without work take donated items of this query
        o << "      if (g.items != 0 && (iter & 31u) == 16u) {\n";
        o << "        const u64 idle2 = ballot(lvl < 0);\n";
        o << "        if (idle2 != 0ull) {\n";
        o << "          int n = 0;\n";
        o << "          const i64 h = try_pop(g, qi, __builtin_popcountll(idle2), &n);\n";
        o << "          const int r2 = rank_in(idle2);\n";
        o << "          if (n > 0 && lvl < 0 && r2 < n) {\n";
        adopt("            ", "(u64)(h + r2)");
        o << "          }\n";
        o << "        }\n";
        o << "      }\n";
        o << "    }\n";
    }

    // A lane takes over a donated work item (same state a thief receives).
    void adopt(const char *ind, const char *slot) {
        const int L = p.l, K = p.k;
        o << ind << "const u32* it = item_at(g, qi, " << slot << ");\n";
        o << ind << "if (item_ready(g, it)) {\n";
        o << ind << "  const int j = (int)ld_ag(it + 1);\n";
        // level 0: a handed root, which the lane fetches at its next refill
        o << ind << "  if (j == 0) { proot = (int)ld_ag(it + 7); if (MODE >= 2) pmy = ld_ag64(it + 8); lvl = 0; ph = 0; base = 1; exact = 0u; }\n";
        o << ind << "  else {\n";
        o << ind << "  lvl = j; base = j; ph = 0; exact = 1u << j;\n";
        if (leaf_cache()) o << ind << "  lq = false;\n";
        o << ind << "  if (" << root_cond() << ") root = (int)ld_ag(it + 7);\n";
        o << ind << "  if (MODE >= 2) mych = ld_ag64(it + 8);\n";
        o << ind << "  tmaxk = (tkey)ld_ag64(it + 10);\n";
        for (int v = 0; v < K; v++) o << ind << "  m" << v << " = (int)ld_ag(it + " << 12 + v << ");\n";
        for (int j = 1; j + 1 < L; j++)
            o << ind << "  if (" << e_cond(j) << ") e" << j << " = (int)ld_ag(it + " << 19 + j << ");\n";
        o << ind << "  const u32 i_s = ld_ag(it + 2), i_e = ld_ag(it + 3); const tkey i_h = (tkey)ld_ag64(it + 4);\n";
        o << ind << "  const int i_w = (int)ld_ag(it + 6);\n";
        o << ind << "  switch (j) {\n";
        for (int i = 1; i < L; i++) {
            o << ind << "    case " << i << ": cur" << i << " = i_s; end" << i << " = i_e; hi" << i << " = i_h;";
            if (G || p.kind[i] == LIST_BOTH) o << " want" << i << " = i_w;";
            o << " break;\n";
        }
        o << ind << "    default: break;\n";
        o << ind << "  }\n";
        o << ind << "  }\n";
        o << ind << "}\n";
    }

    // (not when an anti-edge is checked on the last level: each candidate
    // then needs its own search)
    bool coop_ok() const { return p.l > 1 && (G || p.kind[p.l - 1] != LIST_GLOBAL) && !anti_on(p.l - 1); }

    // Whether the last level's count has a closed form: both endpoints bound
    // (the edges between two given nodes in the time window), or one new
    // endpoint (the window's size minus the edges to each already bound node,
    // the node itself included, since the new node must differ from all of
    // them). Not with a weight predicate, an anti-edge or a label on the new node of that level. Generic matchers decide
    // at run time.
    bool leaf_countable() const {
        const int i = p.l - 1;
        return G || (p.l > 1 && p.kind[i] != LIST_GLOBAL && !has_pred(i) && !has_elab(i) && !anti_on(i) &&
                     !(p.kind[i] != LIST_BOTH && labelled(new_node(i))));
    }

    // Closed-form last level whose list (the out- or in-list of one node) and
    // some of whose subtracted nodes were bound before the level above it:
    // while that level iterates, they stay fixed, so the start of each fixed
    // node's run in the pair-sorted list is searched once per window of the
    // level above (registers ls<v>, valid while lq). When the level above has
    // no gap tighter than delta, every last-level window ends at the same time
    // (t_root + delta), so the window's end position (lE) and each fixed run's
    // end (le<v>) are kept too; a window then costs one search per new node
    // and one per fixed node instead of three each plus the window's own.
    bool leaf_cache() const {
        if (G || p.l < 3 || !leaf_countable() || p.kind[p.l - 1] == LIST_BOTH) return false;
        return fixed_at_leaf(new_node_list(p.l - 1));
    }
    int new_node_list(int i) const { return p.kind[i] == LIST_OUT ? p.a[i] : p.b[i]; }
    // The node the level above binds when it scans the last level's own list
    // (-1 otherwise): its candidate is then an entry of that node's run.
    int parent_node() const {
        const int i = p.l - 1, j = p.l - 2;
        if (j < 1 || p.kind[j] != p.kind[i]) return -1;
        if (p.kind[i] == LIST_OUT && p.a[j] == p.a[i]) return p.b[j];
        if (p.kind[i] == LIST_IN && p.b[j] == p.b[i]) return p.a[j];
        return -1;
    }
    bool fixed_at_leaf(int v) const {
        for (int x : p.mapped[p.l - 2])
            if (x == v) return true;
        return false;
    }

    // Closed-form count of the last level's window (registers cur, end, hi of
    // that level and sx = the previous edge's time) into lc_; w_ = the
    // window's length when computed; pr_ = entries read.
    void leaf_body(int i, const char *in, bool need_w) {
        const std::string s = I(i);
        o << in << "u32 pr_ = 0u; u64 lc_ = 0; u32 w_ = 0u;\n";
        if (G) {
            o << in << "if (gk" << s << " == 2) {\n";
            o << in << "  const int u_ = mget(ga" << s << ");\n";
            o << in << "  lc_ = pair_cnt(g.pr_nbr, prs, g.pr_t, g.off_out[u_], g.off_out[u_ + 1], mget(gb" << s
              << "), sx, hi" << s << ", pr_);\n";
            if (need_w)
                o << in << "  w_ = win_len(g.adj_t, cur" << s << ", end" << s << ", hi" << s << ", pr_);\n";
            o << in << "} else {\n";
            o << in << "  const bool o_ = gk" << s << " == 0; const int u_ = o_ ? mget(ga" << s << ") : mget(gb" << s
              << ");\n";
            o << in << "  const u32 plo = o_ ? g.off_out[u_] : g.off_in[u_], phi = o_ ? g.off_out[u_ + 1] : "
              << "g.off_in[u_ + 1];\n";
            o << in << "  w_ = win_len(g.adj_t, cur" << s << ", end" << s << ", hi" << s << ", pr_); lc_ = w_;\n";
            o << in << "  for (int v_ = 0; v_ < 8; ++v_)\n";
            o << in << "    if ((gm" << s << " >> v_) & 1u) lc_ -= pair_cnt(g.pr_nbr, prs, g.pr_t, plo, phi, mget(v_), sx, hi"
              << s << ", pr_);\n";
            o << in << "}\n";
        } else if (p.kind[i] == LIST_BOTH) {
            o << in << "lc_ = pair_cnt(g.pr_nbr, prs, g.pr_t, g.off_out[m" << p.a[i] << "], g.off_out[m" << p.a[i]
              << " + 1], m" << p.b[i] << ", sx, hi" << s << ", pr_);\n";
            if (need_w) o << in << "w_ = win_len(g.adj_t, cur" << s << ", end" << s << ", hi" << s << ", pr_);\n";
        } else if (leaf_cache()) {
            const bool out = p.kind[i] == LIST_OUT;
            const int u = out ? p.a[i] : p.b[i];
            const char *off = out ? "g.off_out" : "g.off_in";
            const std::string h = "hi" + s;
            o << in << "const u32 plo = " << off << "[m" << u << "], phi = " << off << "[m" << u << " + 1];\n";
            o << in << "if (!lq) {\n";
            o << in << "  lq = true;\n";
            o << in << "  if (q_gf) lE = plo + win_len(g.adj_t, plo, phi, " << h << ", pr_);\n";
            for (int v : p.mapped[i]) {
                if (!fixed_at_leaf(v)) continue;
                const std::string V = I(v);
                o << in << "  ls" << V << " = nbr_lb(g.pr_nbr, prs, plo, phi, m" << V << ", pr_); ++pr_;\n";
                o << in << "  if (ls" << V << " >= phi || g.pr_nbr[ls" << V << "] != m" << V << ") ls" << V << " = ~0u;\n";
                o << in << "  else if (q_gf) le" << V << " = run_ub(g.pr_nbr, g.pr_t, ls" << V << ", phi, m" << V << ", "
                  << h << ", pr_);\n";
            }
            o << in << "}\n";
            o << in << "w_ = q_gf ? (lE > cur" << s << " ? lE - cur" << s << " : 0u) : win_len(g.adj_t, cur" << s
              << ", end" << s << ", " << h << ", pr_);\n";
            o << in << "lc_ = w_;\n";
            for (int v : p.mapped[i]) {
                const std::string V = I(v);
                if (fixed_at_leaf(v))
                    o << in << "if (ls" << V << " != ~0u) lc_ -= (u64)((q_gf ? le" << V << " : run_ub(g.pr_nbr, g.pr_t, ls"
                      << V << ", phi, m" << V << ", " << h << ", pr_)) - run_ub(g.pr_nbr, g.pr_t, ls" << V << ", phi, m"
                      << V << ", sx, pr_));\n";
                else if (v == parent_node()) {
                    // the level above's own candidate is an entry of this node's
                    // run: start there (when this lane scanned that level itself)
                    const std::string P = I(p.l - 2);
                    o << in << "if (base <= " << P << ") {\n";
                    o << in << "  const u32 s_ = g.pr_pos[cur" << P << " - 1u]; ++pr_;\n";
                    o << in << "  lc_ -= (u64)(run_ub(g.pr_nbr, g.pr_t, s_, phi, m" << V << ", " << h
                      << ", pr_) - run_ub(g.pr_nbr, g.pr_t, s_, phi, m" << V << ", sx, pr_));\n";
                    o << in << "} else {\n";
                    o << in << "  lc_ -= pair_cnt(g.pr_nbr, prs, g.pr_t, plo, phi, m" << V << ", sx, " << h << ", pr_);\n";
                    o << in << "}\n";
                } else
                    o << in << "lc_ -= pair_cnt(g.pr_nbr, prs, g.pr_t, plo, phi, m" << V << ", sx, " << h << ", pr_);\n";
            }
        } else {
            const bool out = p.kind[i] == LIST_OUT;
            const int u = out ? p.a[i] : p.b[i];
            const char *off = out ? "g.off_out" : "g.off_in";
            o << in << "const u32 plo = " << off << "[m" << u << "], phi = " << off << "[m" << u << " + 1];\n";
            o << in << "w_ = win_len(g.adj_t, cur" << s << ", end" << s << ", hi" << s << ", pr_); lc_ = w_;\n";
            for (int v : p.mapped[i])
                o << in << "lc_ -= pair_cnt(g.pr_nbr, prs, g.pr_t, plo, phi, m" << v << ", sx, hi" << s << ", pr_);\n";
        }
    }

    // At the end of the last level's window search. Count modes: a window of
    // g.leaf_min or more candidates whose count has a closed form parks its
    // lane (phase 3) until the wavefront counts the parked windows together
    // (park_flush). The work-counter mode, which still scans (the byte model
    // of the method), computes the same count on the side to record what the
    // count modes read instead.
    void leaf_count(int i) {
        if (!leaf_countable()) return;
        const std::string s = I(i);
        const char *ind = "            ";
        const std::string gc = G ? " && gcf" : std::string();
        o << ind << "if ((MODE == 0 || MODE == 2) && wide && g.leaf_min > 0 && sb + (u32)g.leaf_min - 1u < end" << s
          << " && g.adj_t[sb + (u32)g.leaf_min - 1u] <= hi" << s << gc << ") park = true;\n";
        const std::string gcond = G ? " && !((gglob >> " + s + ") & 1u) && gcf" : std::string();
        o << ind << "if (MODE == 1 && g.leaf_min > 0" << gcond << ") {\n";
        o << ind << "  const u32 pk = sb + (u32)g.leaf_min - 1u;\n";
        o << ind << "  if (pk < end" << s << " && g.adj_t[pk] <= hi" << s << ") {\n";
        leaf_body(i, "                ", true);
        o << ind << "    st_lc++; st_lcp += pr_;\n";
        o << ind << "    st_lcw += (u64)w_ + (cur" << s << " + w_ < end" << s << " ? 1u : 0u);\n";
        o << ind << "  }\n";
        o << ind << "}\n";
    }

    // Count the parked windows: once half the wavefront is parked, or no
    // other lane can move, every parked lane runs its closed form at the same
    // time (their searches overlap instead of running one lane at a time),
    // then backtracks as if it had scanned the window.
    void park_flush() {
        if (!leaf_countable()) return;
        const int i = p.l - 1;
        o << "    if (MODE == 0 || MODE == 2) {\n";
        o << "      const u64 parked = ballot(ph == 3);\n";
        o << "      if (parked != 0ull && (__builtin_popcountll(parked) >= 32 || ballot(lvl >= 0 && ph != 3) == 0ull)) {\n";
        o << "        if (ph == 3) {\n";
        leaf_body(i, "          ", false);
        o << "          if (MODE == 2) rcnt += lc_; else cnt += lc_;\n";
        o << "          ph = 0; wide = false; lvl = " << i - 1 << ";\n";
        o << "          if (lvl < base) {\n";
        o << "            lvl = 0;\n";
        o << "            if (MODE == 2 && rcnt) { atomicAdd(&g.chunk_cnt[mych], rcnt); cnt += rcnt; rcnt = 0; }\n";
        o << "          }\n";
        o << "        }\n";
        o << "      }\n";
        o << "    }\n";
    }

    // Wavefront-cooperative last level. A lane whose last-level window is
    // wide hands it to the whole wavefront: the 64 lanes read 64 consecutive
    // candidates per step (coalesced), apply the owner's checks, and one
    // ballot counts (or places) the matches. Owners are served one at a time;
    // each owner's window is finished and the owner backtracks.
    void coop() {
        const int L = p.l, K = p.k, i = p.l - 1;
        o << "    if (MODE != 1) {\n";
        o << "      u64 lm = ballot(lvl == " << i << " && ph == 0 && wide);\n";
        o << "      while (lm != 0ull) {\n";
        o << "        const int j = __builtin_ctzll(lm); lm &= lm - 1ull;\n";
        o << "        u32 c = rl(cur" << i << ", j); const u32 e = rl(end" << i << ", j); const tkey h = rl(hi" << i
          << ", j);\n";
        std::ostringstream ok;
        if (G) {
            o << "        const int w_ = rl(want" << i << ", j);\n";
            for (int v = 0; v < 8; v++) o << "        const int x" << v << " = rl(m" << v << ", j);\n";
            ok << "(gk" << i << " == 2 ? nb == w_ : notin(gm" << i << ", nb, x0, x1, x2, x3, x4, x5, x6, x7))";
            ok << " && (gk" << i << " == 2 || ((glm >> gn" << i << ") & 1u) == 0u || in_range(g.nlab[nb], lget(gn"
               << i << "), hget(gn" << i << ")))";
        } else if (p.kind[i] == LIST_BOTH) {
            o << "        const int w_ = rl(want" << i << ", j);\n";
            ok << "nb == w_";
        } else {
            ok << "true";
            for (int v : p.mapped[i]) {
                o << "        const int x" << v << " = rl(m" << v << ", j);\n";
                ok << " && nb != x" << v;
            }
            if (labelled(new_node(i))) ok << " && " << lab_cond(new_node(i), "nb");
        }
        o << "        int o_root = 0; i64 o_ch = 0;\n";
        o << "        if (MODE == 3) { o_root = rl(root, j); o_ch = rl(mych, j); }\n";
        for (int k = 1; k + 1 < L; k++) o << "        const int o_e" << k << " = MODE == 3 ? rl(e" << k << ", j) : 0;\n";
        o << "        u64 tot = 0;\n";
        o << "        for (;;) {\n";
        o << "          const u32 idx = c + (u32)lane;\n";
        o << "          bool v = idx < e;\n";
        o << "          tkey t = 0; int nb = 0;\n";
        o << "          if (v) { t = g.adj_t[idx]; nb = g.adj_nbr[idx]; }\n";
        o << "          v = v && t <= h;\n";
        o << "          bool ok = v && " << ok.str() << ";\n";
        if (G) {
            o << "          if (ok && ((gpm >> " << i << ") & 1u)) ok = preds_at(q, " << i << ", g.adj_w[idx]);\n";
            o << "          if (ok && ((gelm >> " << i << ") & 1u)) ok = in_range(g.adj_el[idx], q->elo[" << i << "], q->ehi["
              << i << "]);\n";
        } else {
            if (has_pred(i)) o << "          if (ok) ok = " << preds_cond(i, "g.adj_w[idx]") << ";\n";
            if (has_elab(i)) o << "          if (ok) ok = " << elab_cond(i, "g.adj_el[idx]") << ";\n";
        }
        o << "          const u64 okm = ballot(ok);\n";
        o << "          tot += (u64)__builtin_popcountll(okm);\n";
        o << "          if (MODE == 3 && okm != 0ull) {\n";
        o << "            i64 b0 = 0;\n";
        o << "            if (lane == 0) b0 = (i64)(g.chunk_off[o_ch] + atomicAdd(&g.chunk_cnt[o_ch], (u64)__builtin_popcountll(okm)));\n";
        o << "            b0 = bcast64(b0);\n";
        o << "            if (ok) {\n";
        o << "              const u64 slot = (u64)b0 + (u64)rank_in(okm);\n";
        o << "              if (slot < g.capacity) {\n";
        o << "                i64* row = g.out + slot * " << L << "ull;\n";
        o << "                row[0] = (i64)o_root;\n";
        for (int k = 1; k + 1 < L; k++) o << "                row[" << k << "] = (i64)o_e" << k << ";\n";
        o << "                row[" << (L - 1) << "] = (i64)g.adj_eid[idx];\n";
        o << "              } else { atomicAdd(&g.ctl[1], 1ull); }\n";
        o << "            }\n";
        o << "          }\n";
        o << "          if (ballot(v) != ~0ull) break;\n";
        o << "          c += 64u;\n";
        o << "        }\n";
        o << "        if (lane == j) {\n";
        o << "          if (MODE == 2) rcnt += tot; else cnt += tot;\n";
        o << "          wide = false;\n";
        o << "          lvl -= 1;\n";
        o << "          if (lvl < base) {\n";
        o << "            lvl = 0;\n";
        o << "            if (MODE == 2 && rcnt) { atomicAdd(&g.chunk_cnt[mych], rcnt); cnt += rcnt; rcnt = 0; }\n";
        o << "          }\n";
        o << "        }\n";
        o << "      }\n";
        o << "    }\n";
        (void)K;
    }

    // `outlined`: the matcher is a separate (non-inlined) function of the
    // kernel. A module with many matchers compiles in time superlinear in the
    // kernel's size when all of them are inlined into it (register
    // coalescing over one huge function); as separate functions each is
    // compiled on its own. Such a matcher reads the launch arguments from the
    // kernel argument segment (scalar loads, as the inlined form does) and
    // makes its uniform parameters wave-uniform again on entry.
    void matcher(int fi, bool outlined = false) {
        const int L = p.l, K = p.k;
        const bool glob = has_global();
        o << "// motif " << p.key() << "\n";
        if (p.n_anti > 0) {
            o << "#ifndef TM_ANTI_FREE\n#define TM_ANTI_FREE\n";
            o << "// No edge u -> v with time in [t0, t0 + d]: find v's run in u's out-list\n";
            o << "// sorted by (neighbour, time), then the run's first entry with time >= t0.\n";
            o << "__device__ __forceinline__ bool anti_free(const GArgs& g, int u, int v, tkey t0, i64 d) {\n";
            o << "  const u32 lo = g.off_out[u], hi = g.off_out[u + 1];\n";
            o << "  u32 pr = 0u;\n";
            o << "  const u32 s = nbr_lb(g.pr_nbr, g.samp_min != 0u ? g.pr_samp : nullptr, lo, hi, v, pr);\n";
            o << "  if (s >= hi || g.pr_nbr[s] != v) return true;\n";
            o << "  const u32 f = run_ub(g.pr_nbr, g.pr_t, s, hi, v, (tkey)(t0 - 1), pr);\n";
            o << "  if (f >= hi || g.pr_nbr[f] != v) return true;\n";
            o << "  return (i64)g.pr_t[f] > (i64)t0 + d;\n";
            o << "}\n#endif\n";
        }
        if (outlined) {
            // `ga_` is the address of the kernel's argument segment (the
            // kernel's only argument is the GArgs); a callee cannot read that
            // address itself, so the kernel passes it
            o << "template <int MODE>\n__device__ __noinline__ i64 match" << fi
              << "(u64 ga_, int qi_, i64 chunk_, i64 ih_, int in_) {\n";
            o << "  const GArgs g = *(const __attribute__((address_space(4))) GArgs*)(u64)bcast64((i64)ga_);\n";
            o << "  const int qi = __builtin_amdgcn_readfirstlane(qi_), in = __builtin_amdgcn_readfirstlane(in_);\n";
            o << "  const i64 chunk = bcast64(chunk_), ih = bcast64(ih_);\n";
        } else {
            o << "template <int MODE>\n__device__ __forceinline__ i64 match" << fi
              << "(const GArgs& g, int qi, i64 chunk, i64 ih, int in) {\n";
        }
        o << "  const int lane = lane_id();\n";
        o << "  const qptr q = (qptr)(g.qa + qi);  // uniform: scalar loads\n";
        o << "  const int* const prs = MODE != 1 ? g.pr_samp : nullptr;  // pair-list line samples (not in the byte model's mode)\n";
        o << "  const i64 q_r0 = q->r0, q_delta = q->delta, q_c0 = q->c0, q_c1 = q->c0 + q->nchunks;\n";
        o << "  // chunk j of a query holds its roots j, j + nchunks, j + 2 nchunks, ...: a burst of\n";
        o << "  // consecutive heavy roots spreads over many wavefronts\n";
        o << "  const i64 q_nch = q->nchunks, q_n = q->r1 - q->r0, q_budget = q->budget;\n";
        // root i of the query's chunk L: interleaved, q_r0 + L + i * nchunks; in
        // XCD order, contiguous: q_r0 + L * q_rch + i
        if (X) o << "  const i64 q_rch = q_nch > 0 ? (q_n + q_nch - 1) / q_nch : 0;\n";
        o << "  const bool q_split = g.split && q->split; const u32 q_smin = (u32)q->split_min;\n";
        for (int i = 0; i + 1 < L; i++) o << "  const i64 gap" << i << " = q->gap[" << i << "];\n";
        for (int j = 0; j < p.n_anti; j++) o << "  const i64 adl" << j << " = q->gap[" << anti_slot(j) << "];\n";
        if (!G)
            for (int j = 0; j < p.np; j++)
                o << "  const int pop" << j << " = q->pop[" << j << "]; const float pth" << j << " = q->pth[" << j << "];\n";
        for (int v = 0; v < K; v++)
            if (labelled(v)) o << "  const int nl" << v << " = q->nlab[" << v << "], nh" << v << " = q->nlab_hi[" << v << "];\n";
        for (int i = 0; i < L; i++)
            if (has_elab(i)) o << "  const int elo" << i << " = q->elo[" << i << "], ehi" << i << " = q->ehi[" << i << "];\n";
        if (G) {
            o << "  const u32 gpm = (u32)q->pred_mask, gelm = (u32)q->elab_mask; const u32 gglob = (u32)q->glob_mask;\n";
            for (int i = 1; i < L; i++)
                o << "  const int gk" << i << " = q->pk[" << i << "], ga" << i << " = q->pa[" << i << "], gb" << i
                  << " = q->pb[" << i << "], gj" << i << " = q->pj[" << i << "]; const u32 gm" << i << " = q->pm["
                  << i << "];\n";
            o << "  const u32 glm = (u32)q->lab_mask;\n";
            o << "  const int l0 = q->nlab[0], l1 = q->nlab[1], l2 = q->nlab[2], l3 = q->nlab[3], l4 = q->nlab[4], "
                 "l5 = q->nlab[5], l6 = q->nlab[6], l7 = q->nlab[7];\n";
            o << "  const int h0 = q->nlab_hi[0], h1 = q->nlab_hi[1], h2 = q->nlab_hi[2], h3 = q->nlab_hi[3], "
                 "h4 = q->nlab_hi[4], h5 = q->nlab_hi[5], h6 = q->nlab_hi[6], h7 = q->nlab_hi[7];\n";
            for (int i = 1; i < L; i++)
                o << "  const int gn" << i << " = gk" << i << " == 0 ? gb" << i << " : ga" << i << ";\n";
            if (L > 1)
                o << "  const bool glabl = gk" << L - 1 << " != 2 && ((glm >> gn" << L - 1 << ") & 1u) != 0u;\n";
            // the last level's count has a closed form (no predicate, edge
            // label or label on its new node there)
            if (L > 1)
                o << "  const bool gcf = !glabl && !((gpm >> " << L - 1 << ") & 1u) && !((gelm >> " << L - 1
                  << ") & 1u);\n";
        }
        o << "  int lvl = 0, ph = 0, root = 0, base = 1, cool = 0;\n";
        o << "  u32 exact = 0u;  // bit i: end of level i's window is its exact extent\n";
        o << "  bool wide = false;  // last-level window reaches 32+ candidates\n";
        o << "  i64 mych = 0;\n";
        o << "  int";
        for (int v = 0; v < K; v++) o << (v ? ", " : " ") << "m" << v << " = 0";
        o << ";\n";
        for (int i = 1; i < L; i++) {
            o << "  u32 cur" << i << " = 0u, end" << i << " = 0u; tkey hi" << i << " = 0;";
            if (G || p.kind[i] == LIST_BOTH) o << " int want" << i << " = 0;";
            if (i + 1 < L) o << " int e" << i << " = 0;";
            o << "\n";
        }
        o << "  tkey tmaxk = 0, sx = 0; u32 sb = 0u, sn = 0u;\n";
        o << "  u64 cnt = 0, rcnt = 0, st_win = 0, st_probe = 0, st_visit = 0, st_pv = 0, st_root = 0;\n";
        o << "  u64 st_lc = 0, st_lcw = 0, st_lcp = 0;  // windows counted without a scan: number, visits, reads\n";
        if (leaf_cache()) {
            o << "  bool lq = false; const bool q_gf = gap" << L - 2 << " >= q_delta; u32 lE = 0u;"
              << "  // fixed-node searches of the closed-form last level\n";
            for (int v : p.mapped[L - 1])
                if (fixed_at_leaf(v)) o << "  u32 ls" << v << " = 0u, le" << v << " = 0u;\n";
        }
        o << "  u32 iter = 0u, steps = 0u; i64 ghungry = 0;\n";
        o << "  int proot = -1; i64 pmy = 0;  // a root handed to this lane (tail redistribution)\n";
        o << "  u32 dchk = 0u, dcur = 0u;  // queue-cursor look: step counter, value read (lane 0)\n";
        o << "  i64 pnext = 0, pend = 0, pchunk = chunk, pending = -1;\n";
        o << "  bool drained = chunk < 0;\n";
        o << "  if (chunk >= 0) {\n";
        if (X) o << "    pnext = 0; pend = ch_roots_x(chunk - q_c0, q_n, q_rch);\n";
        else o << "    pnext = 0; pend = (q_n - (chunk - q_c0) + q_nch - 1) / q_nch;\n";
        o << "  } else {\n";
        o << "    // start from donated work items [ih, ih + in) of this query\n";
        o << "    lvl = -1;\n";
        if (L > 1) {
            o << "    if (lane < in) {\n";
            adopt("      ", "(u64)(ih + lane)");
            o << "    }\n";
        }
        o << "  }\n";
        o << "  for (;;) {\n";
        // ---------------- refill
        // lanes holding a handed root (proot) take it instead of a pool root
        o << "    const bool wantp = lvl == 0 && proot < 0;\n";
        o << "    const u64 need = ballot(wantp);\n";
        o << "    if (need || ballot(lvl == 0) != 0ull) {\n";
        o << "      const i64 nneed = (i64)__builtin_popcountll(need);\n";
        o << "      const i64 rk = (i64)rank_in(need);\n";
        o << "      const i64 avail = pend - pnext;\n";
        o << "      i64 myr = -1, myc = pchunk;\n";
        if (X) o << "      if (wantp && rk < avail) myr = q_r0 + (pchunk - q_c0) * q_rch + pnext + rk;\n";
        else o << "      if (wantp && rk < avail) myr = q_r0 + (pchunk - q_c0) + (pnext + rk) * q_nch;\n";
        o << "      if (avail >= nneed) { pnext += nneed; }\n";
        o << "      else {\n";
        o << "        pnext = pend;\n";
        o << "        if (!drained) {\n";
        o << "          i64 c = 0;\n";
        o << "          if (lane == 0) c = " << (X ? "next_chunk_x(g)" : "(i64)atomicAdd(&g.ctl[0], 1ull)") << ";\n";
        o << "          c = bcast64(c);\n";
        o << "          if (" << (X ? "c < q_c0 || " : "") << "c >= q_c1) { drained = true; pending = c < g.total_chunks ? c : -1; }\n";
        o << "          else {\n";
        o << "            pchunk = c;\n";
        if (X) o << "            pnext = 0; pend = ch_roots_x(c - q_c0, q_n, q_rch);\n";
        else o << "            pnext = 0; pend = (q_n - (c - q_c0) + q_nch - 1) / q_nch;\n";
        o << "            const i64 k2 = rk - avail;\n";
        if (X) o << "            if (wantp && myr < 0 && k2 < pend) { myr = q_r0 + (c - q_c0) * q_rch + k2; myc = c; }\n";
        else o << "            if (wantp && myr < 0 && k2 < pend) { myr = q_r0 + (c - q_c0) + k2 * q_nch; myc = c; }\n";
        o << "            const i64 take = nneed - avail < pend - pnext ? nneed - avail : pend - pnext;\n";
        o << "            pnext += take;\n";
        o << "          }\n";
        o << "        }\n";
        o << "      }\n";
        o << "      if (lvl == 0 && proot >= 0) { myr = proot; myc = pmy; proot = -1; }\n";
        o << "      if (lvl == 0) {\n";
        o << "        if (myr >= 0) {\n";
        o << "          const int r = (int)myr;\n";
        o << "          const int s = g.src[r], d = g.dst[r];\n";
        o << "          const tkey tr = g.tk[r];\n";
        if (G) {
            o << "          if (MODE == 1) { st_root++; if (gpm & 1u) st_pv++; }\n";
            o << "          bool ok = s != d;\n";
            o << "          if (gpm & 1u) ok = ok && preds_at(q, 0, g.w[r]);\n";
            o << "          if (gelm & 1u) ok = ok && in_range(g.el[r], q->elo[0], q->ehi[0]);\n";
            o << "          if (glm & 1u) ok = ok && in_range(g.nlab[s], l0, h0);\n";
            o << "          if (glm & 2u) ok = ok && in_range(g.nlab[d], l1, h1);\n";
        } else {
            o << "          if (MODE == 1) { st_root++;" << (has_pred(0) ? " st_pv++;" : "") << " }\n";
            o << "          bool ok = s != d;\n";
            if (has_pred(0)) o << "          ok = ok && " << preds_cond(0, "g.w[r]") << ";\n";
            if (has_elab(0)) o << "          ok = ok && " << elab_cond(0, "g.el[r]") << ";\n";
            if (labelled(p.a[0])) o << "          ok = ok && " << lab_cond(p.a[0], "s") << ";\n";
            if (labelled(p.b[0])) o << "          ok = ok && " << lab_cond(p.b[0], "d") << ";\n";
            if (anti_on(0)) o << "          ok = ok && " << anti_cond(0) << ";\n";
        }
        o << "          if (ok) {\n";
        o << "            base = 1;\n";
        o << "            if (" << root_cond() << ") root = r;\n";
        o << "            if (MODE >= 2) mych = myc;  // its chunk orders the instances\n";
        if (L == 1) {
            leaf("            ", "0");
            o << "            if (MODE == 2 && rcnt) { atomicAdd(&g.chunk_cnt[mych], rcnt); cnt += rcnt; rcnt = 0; }\n";
        } else {
            o << "            m" << p.a[0] << " = s; m" << p.b[0] << " = d;\n";
            o << "            { i64 x = (i64)tr + q_delta; tmaxk = (tkey)(x < (i64)TKEY_MAX ? x : (i64)TKEY_MAX); }\n";
            open(1, "tr", "            ");
        }
        o << "          }\n";
        o << "        } else if (drained) {\n";
        o << "          lvl = -1;\n";
        o << "        }\n";
        o << "      }\n";
        o << "    }\n";
        o << "    if (ballot(lvl >= 0) == 0ull) break;\n";
        // work budget: every 1024 loop steps a wavefront adds them to its query's
        // tally; once the tally passes the budget the query is abandoned (the host
        // reports it cancelled): skip its remaining root chunks, keeping the first
        // chunk of a later query for the caller
        o << "    if (q_budget > 0 && (++steps & 1023u) == 0u) {\n";
        o << "      i64 used = 0;\n";
        o << "      if (lane == 0) used = (i64)atomicAdd(&g.counts[g.nq + qi], 1024ull) + 1024;\n";
        o << "      used = bcast64(used);\n";
        o << "      if (used > q_budget) {\n";
        o << "        if (!drained) {\n";
        o << "          i64 c = 0;\n";
        if (X) o << "          do { if (lane == 0) c = next_chunk_x(g); c = bcast64(c); } while (c >= q_c0 && c < q_c1);\n";
        else o << "          do { if (lane == 0) c = (i64)atomicAdd(&g.ctl[0], 1ull); c = bcast64(c); } while (c < q_c1);\n";
        o << "          drained = true; pending = c < g.total_chunks ? c : -1;\n";
        o << "        }\n";
        o << "        break;\n";
        o << "      }\n";
        o << "    }\n";
        // A wavefront still working through its chunk learns that the whole
        // root queue is empty (it only fetches again once its pool is used
        // up): a relaxed look at the queue cursor every 256 steps, read one
        // step after it is issued so that the wavefront does not wait on the
        // contended line. From then on it splits pending work and hands out
        // unstarted roots.
        if (L > 1) {
            o << "    if (q_split && !drained && g.items != 0) {\n";
            o << "      const u32 dk = ++dchk & 255u;\n";
            o << "      if (dk == 0u) { if (lane == 0) { const u64 v = ld_rlx64(&g.ctl[0]); dcur = v < 0xffffffffull ? (u32)v : 0xffffffffu; } }\n";
            o << "      else if (dk == 1u && (i64)(u32)__builtin_amdgcn_readfirstlane((int)dcur) >= g.total_chunks) drained = true;  // no chunk of any query is left\n";
            o << "    }\n";
            steal();
        }
        if (L > 1 && coop_ok()) coop();
        if (L > 1 && coop_ok()) park_flush();
        if (L > 1 && F) step_fused();
        if (L > 1 && !F) {
            // ---------------- search probe
            o << "    if (lvl > 0 && (ph == 1 || ph == 2 || ph == 5)) {\n";
            if (G) {
                o << "      const tkey* sarr = ph == 5 ? g.samp : ((gglob >> lvl) & 1u) ? g.tk : g.adj_t;\n";
            } else if (glob) {
                o << "      bool gl = false;\n";
                for (int i = 1; i < L; i++)
                    if (p.kind[i] == LIST_GLOBAL) o << "      gl = gl || lvl == " << i << ";\n";
                o << "      const tkey* sarr = ph == 5 ? g.samp : gl ? g.tk : g.adj_t;\n";
            } else {
                o << "      const tkey* sarr = ph == 5 ? g.samp : g.adj_t;\n";
            }
            // ph 2: first probe at the window start (tie skip after a jump).
            // A search of 3 or more unknown entries reads three pivots at
            // once and keeps one of the four ranges between them: half as
            // many dependent steps as a binary search, the three reads in
            // flight together.
            o << "      if (ph != 2 && sn >= 3u) {\n";
            o << "        const u32 o1 = ((sn + 1u) >> 2) - 1u, o2 = ((2u * (sn + 1u)) >> 2) - 1u, "
                 "o3 = ((3u * (sn + 1u)) >> 2) - 1u;\n";
            o << "        const tkey v1 = sarr[sb + o1], v2 = sarr[sb + o2], v3 = sarr[sb + o3];\n";
            o << "        if (v3 <= sx) { sb += o3 + 1u; sn -= o3 + 1u; }\n";
            o << "        else if (v2 <= sx) { sb += o2 + 1u; sn = o3 - o2 - 1u; }\n";
            o << "        else if (v1 <= sx) { sb += o1 + 1u; sn = o2 - o1 - 1u; }\n";
            o << "        else { sn = o1; }\n";
            o << "      } else {\n";
            o << "        const u32 half = ph == 2 ? 0u : (sn >> 1); const u32 mid = sb + half;\n";
            o << "        const tkey v = sarr[mid];\n";
            o << "        if (v <= sx) { sb = mid + 1u; sn = sn - half - 1u; } else { sn = half; }\n";
            o << "      }\n";
            o << "      if (ph == 2) ph = 1;\n";
            // the samples' search ended at the first sample > sx (index sb):
            // the list's first key > sx lies after the sample before it and
            // at or before that one
            o << "      if (ph == 5 && sn == 0u) {\n";
            o << "        u32 lo_ = 0u, hi_ = 0u;\n";
            o << "        switch (lvl) {\n";
            for (int i = 1; i < L; i++) o << "          case " << i << ": lo_ = cur" << i << "; hi_ = end" << i << "; break;\n";
            o << "          default: break;\n";
            o << "        }\n";
            o << "        const u32 j0 = (lo_ + (1u << g.samp_lg) - 1u) >> g.samp_lg, j1 = (hi_ - 1u) >> g.samp_lg;\n";
            o << "        const u32 nlo = sb == j0 ? lo_ : ((sb - 1u) << g.samp_lg) + 1u;\n";
            o << "        const u32 nhi = sb <= j1 ? (sb << g.samp_lg) : hi_;\n";
            o << "        sb = nlo; sn = nhi - nlo; ph = 1;\n";
            o << "      }\n";
            search_done();
            o << "    } else if (lvl > 0 && ph == 0) {\n";
            // ---------------- candidate scan
            o << "      u32 c = 0u, e = 0u; tkey h = 0;\n";
            o << "      switch (lvl) {\n";
            for (int i = 1; i < L; i++)
                o << "        case " << i << ": c = cur" << i << "; e = end" << i << "; h = hi" << i << "; break;\n";
            o << "        default: break;\n";
            o << "      }\n";
            bool any_pred = false, any_elab = false;
            for (int i = 1; i < L; i++) {
                any_pred |= has_pred(i);
                any_elab |= has_elab(i);
            }
            o << "      bool inwin = false; tkey tt = 0; int nb = 0;";
            if (G || any_pred) o << " float wv = 0.0f;";
            if (G || any_elab) o << " int ev = 0;";
            o << "\n";
            o << "      if (c < e) {\n";
            if (G) {
                o << "        const bool gl = ((gglob >> lvl) & 1u) != 0u;\n";
                o << "        tt = gl ? g.tk[c] : g.adj_t[c];\n";
                o << "        if (!gl) nb = g.adj_nbr[c];\n";
                o << "        if ((gpm >> lvl) & 1u) wv = gl ? g.w[c] : g.adj_w[c];\n";
                o << "        if ((gelm >> lvl) & 1u) ev = gl ? g.el[c] : g.adj_el[c];\n";
            } else if (glob) {
                o << "        bool gl = false;\n";
                for (int i = 1; i < L; i++)
                    if (p.kind[i] == LIST_GLOBAL) o << "        gl = gl || lvl == " << i << ";\n";
                o << "        tt = gl ? g.tk[c] : g.adj_t[c];\n";
                o << "        if (!gl) nb = g.adj_nbr[c];\n";
            } else {
                o << "        tt = g.adj_t[c];\n";
                o << "        nb = g.adj_nbr[c];\n";
            }
            for (int i = 1; i < L; i++) {
                if (has_pred(i))
                    o << "        if (lvl == " << i << ") wv = " << (p.kind[i] == LIST_GLOBAL ? "g.w[c]" : "g.adj_w[c]")
                      << ";\n";
                if (has_elab(i))
                    o << "        if (lvl == " << i << ") ev = " << (p.kind[i] == LIST_GLOBAL ? "g.el[c]" : "g.adj_el[c]")
                      << ";\n";
            }
            o << "        inwin = tt <= h;\n";
            if (G)
                o << "        if (MODE == 1) { st_visit++; if ((gpm >> lvl) & 1u) st_pv++; }\n";
            else
                o << "        if (MODE == 1) { st_visit++;"
                  << (any_pred ? " if ((" + std::to_string(p.pred_mask()) + "u >> lvl) & 1u) st_pv++;" : std::string())
                  << " }\n";
            o << "      }\n";
            visit_accept();
            o << "    }\n";
        }
        o << "  }\n";
        // ---------------- reductions
        o << "  cnt = wave_sum(cnt, lane);\n";
        o << "  if (lane == 0 && cnt) atomicAdd(&g.counts[qi], cnt);\n";
        o << "  if (MODE == 1) {\n";
        o << "    u64 v0 = wave_sum(st_root, lane), v1 = wave_sum(st_win, lane), v2 = wave_sum(st_probe, lane);\n";
        o << "    u64 v3 = wave_sum(st_visit, lane), v4 = wave_sum(st_pv, lane);\n";
        o << "    if (lane == 0) { atomicAdd(&g.ctl[2], v0); atomicAdd(&g.ctl[3], v1); atomicAdd(&g.ctl[4], v2);\n";
        o << "                     atomicAdd(&g.ctl[5], v3); atomicAdd(&g.ctl[6], v4); }\n";
        o << "    u64 v5 = wave_sum(st_lc, lane), v6 = wave_sum(st_lcw, lane), v7 = wave_sum(st_lcp, lane);\n";
        o << "    if (lane == 0) { atomicAdd(&g.ctl[10], v5); atomicAdd(&g.ctl[11], v6); atomicAdd(&g.ctl[12], v7); }\n";
        o << "  }\n";
        o << "  return pending;\n";
        o << "}\n\n";
    }
};

// Kernel entry names: a single-query module has all four modes; a batched
// module has one counting kernel, named apart so profiles separate the forms.
const char *const kSingleNames[4] = {"tm_count", "tm_stats", "tm_enum_count", "tm_enum_write"};
const char *const kBatchName = "tm_count_batch";

// `modes`: bit set of the single-query kernels to emit (bit i = mode i), or
// 0 for the batched module's one counting kernel.
void emit_kernels(std::ostringstream &o, int nfn, int block, unsigned modes, int min_waves, bool outlined, int form) {
    const bool batch = modes == 0;
    const char *const *names = batch ? &kBatchName : kSingleNames;
    const int nmodes = batch ? 1 : 4;
    for (int mode = 0; mode < nmodes; mode++) {
        if (!batch && !((modes >> mode) & 1u)) continue;
        auto run = [&](const char *ind, const char *qv, const char *cv, const char *ih, const char *in) {
            o << ind << "{ const int fn = __builtin_amdgcn_readfirstlane(g.qa[" << qv << "].fn);\n";
            o << ind << "  switch (fn) {\n";
            for (int f = 0; f < nfn; f++)
                o << ind << "    case " << f << ": c = match" << f << "<" << mode << ">(" << (outlined ? "ga, " : "g, ")
                  << qv << ", " << cv
                  << ", " << ih << ", " << in << "); break;\n";
            o << ind << "    default: c = -1; break;\n";
            o << ind << "  } }\n";
        };
        o << "extern \"C\" __global__ __launch_bounds__(" << block;
        if (min_waves > 0) o << ", " << min_waves;  // minimum waves per SIMD
        o << ") void " << names[mode] << "(GArgs g) {\n";
        o << "  const int lane = lane_id();\n";
        o << "  if (g.hub_words != 0u) {  // stage the hub samples (the same for all workgroups)\n";
        o << "    for (u32 i = threadIdx.x; i < g.hub_words; i += blockDim.x) lds_hub[i] = g.hub[i];\n";
        o << "    __syncthreads();\n";
        o << "  }\n";
        if (outlined) o << "  const u64 ga = (u64)__builtin_amdgcn_kernarg_segment_ptr();\n";
        o << "  i64 c = 0;\n";
        o << "  if (lane == 0) { atomicAdd(&g.ctl[8], 1ull); c = " << ((form & 2) ? "next_chunk_x(g)" : "(i64)atomicAdd(&g.ctl[0], 1ull)") << "; }\n";
        o << "  c = bcast64(c);\n";
        o << "  bool busy = true, hung = false;\n";
        o << "  u32 polls = 0u, nap = 1u;\n";
        o << "  for (;;) {\n";
        o << "    if (c >= 0 && c < g.total_chunks) {\n";
        o << "      int qi = 0;\n";
        o << "      if (g.nq > 1) { int lo = 0, hi = g.nq - 1;\n";
        o << "        while (lo < hi) { int md = (lo + hi + 1) >> 1; if (g.qa[md].c0 <= c) lo = md; else hi = md - 1; }\n";
        o << "        qi = lo; }\n";
        o << "      qi = __builtin_amdgcn_readfirstlane(qi);\n";
        run("      ", "qi", "c", "0", "0");
        o << "      continue;\n";
        o << "    }\n";
        // root chunks are gone: wait for work donated by busy wavefronts
        o << "    if (busy) { if (lane == 0) atomicAdd(&g.ctl[8], ~0ull); busy = false; }\n";
        o << "    if (" << mode << " == 1 || !g.split || g.items == 0) break;\n";
        o << "    if (!hung) { if (lane == 0) atomicAdd(&g.ctl[9], 1ull); hung = true; }\n";
        // look at the queues only when some item waits (one word), and once
        // more, whatever that word says, before leaving: every wavefront that
        // donated was busy at the time and looks at the queues itself when it
        // stops being busy, so no item is left behind
        o << "    i64 b = 0, av = 0, hq = 0;\n";
        o << "    if (lane == 0) { b = (i64)ld_rlx64(&g.ctl[8]); av = (i64)ld_rlx64(&g.ctl[13]); hq = (i64)ld_rlx64(&g.ctl[9]); }\n";
        o << "    b = bcast64(b); av = bcast64(av); hq = bcast64(hq);\n";
        // surplus waiters leave, freeing their compute units for other
        // launches (a few per busy wavefront take all it can donate)
        o << "    if (av <= 0 && b > 0 && hq > 2 * b + 32) break;\n";
        o << "    int fq = -1, n = 0; i64 h = 0;\n";
        o << "    for (int qq = 0; (av > 0 || b == 0) && qq < g.nq; ++qq) {\n";
        o << "      int ne = 0;\n";
        o << "      if (lane == 0) {\n";
        o << "        const u64 hh = ld_rlx64(&g.qctl[2 * qq]);\n";
        o << "        u64 tt = ld_rlx64(&g.qctl[2 * qq + 1]);\n";
        o << "        if (tt > (u64)g.item_cap) tt = (u64)g.item_cap;\n";
        o << "        ne = hh < tt ? 1 : 0;\n";
        o << "      }\n";
        o << "      ne = __builtin_amdgcn_readfirstlane(ne);\n";
        o << "      if (ne) {\n";
        o << "        if (lane == 0) atomicAdd(&g.ctl[8], 1ull);  // counted busy before taking items\n";
        o << "        h = try_pop(g, qq, 64, &n);\n";
        o << "        if (n > 0) { fq = qq; break; }\n";
        o << "        if (lane == 0) atomicAdd(&g.ctl[8], ~0ull);\n";
        o << "      }\n";
        o << "    }\n";
        o << "    if (fq >= 0) {\n";
        o << "      busy = true;\n";
        o << "      if (lane == 0) atomicAdd(&g.ctl[9], ~0ull);\n";
        o << "      hung = false; polls = 0u; nap = 1u;\n";
        run("      ", "fq", "-1", "h", "n");
        o << "      continue;\n";
        o << "    }\n";
        o << "    if (b == 0) break;\n";
        // back off exponentially (1 to 16 long sleeps between looks), so that
        // thousands of waiting wavefronts do not hammer the few queue words the
        // working ones also use; give up after about 2^18 long sleeps in all
        o << "    polls += nap;\n";
        o << "    if (polls > (1u << 18)) break;\n";
        o << "    for (u32 k = 0u; k < nap; ++k) __builtin_amdgcn_s_sleep(127);\n";
        o << "    if (nap < 16u) nap <<= 1;\n";
        o << "  }\n";
        o << "  if (busy && lane == 0) atomicAdd(&g.ctl[8], ~0ull);\n";
        o << "  if (hung && lane == 0) atomicAdd(&g.ctl[9], ~0ull);\n";
        o << "}\n";
    }
}

}  // namespace

static std::string header(int key_bytes) {
    std::ostringstream o;
    o << "// generated by the tmotif motif compiler\n";
    o << "typedef " << (key_bytes == 4 ? "int" : "long long") << " tkey;\n";
    o << "#define TKEY_MAX " << (key_bytes == 4 ? "2147483647LL" : "9223372036854775807LL") << "\n";
    o << kPrelude;
    return o.str();
}

std::string generate_source(const Plan &p, int key_bytes, int block, int min_waves, unsigned modes, int form) {
    Emitter e(p, p.generic, form);
    e.o << header(key_bytes);
    e.matcher(0);
    emit_kernels(e.o, 1, block, modes & kAllModes, min_waves, false, form);
    return e.o.str();
}

std::string generate_batch_source(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                  int min_waves, int form) {
    std::ostringstream all;
    all << header(key_bytes);
    int n_generic = 0;
    for (auto *pl : plans) n_generic += pl->generic ? 1 : 0;
    const bool outlined = (int)plans.size() > kMaxInlinedMatchers || n_generic > 1;
    for (size_t f = 0; f < plans.size(); f++) {
        Emitter e(*plans[f], plans[f]->generic, form);
        e.matcher((int)f, outlined);
        all << e.o.str();
    }
    emit_kernels(all, (int)plans.size(), block, 0u, min_waves, outlined, form);
    return all.str();
}

// ---------------------------------------------------------------- compiling

// hipRTC options of every motif module (packed fp32 instructions disabled)
static const char *const kRtcOpts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                                       "-Xclang", "-packed-fp32-ops"};
static const int kRtcNopts = (int)(sizeof(kRtcOpts) / sizeof(kRtcOpts[0]));

bool compile_to_code(const std::string &src, std::vector<char> *code, std::string *err) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "tm_motif.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return false;
    }
    hiprtcResult rc = hiprtcCompileProgram(prog, kRtcNopts, kRtcOpts);
    if (rc != HIPRTC_SUCCESS) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n + 1, '\0');
        hiprtcGetProgramLog(prog, &log[0]);
        *err = std::string("motif kernel compilation failed: ") + log;
        hiprtcDestroyProgram(&prog);
        return false;
    }
    size_t code_size = 0;
    hiprtcGetCodeSize(prog, &code_size);
    code->resize(code_size);
    hiprtcGetCode(prog, code->data());
    hiprtcDestroyProgram(&prog);
    return true;
}

// On-disk code-object cache. A cache file holds a magic word, the full
// source text it was compiled from and the code object; it is used only when
// the stored source equals the requested one byte for byte, so a stale or
// colliding entry is recompiled, never loaded. Directory: $TMOTIF_KERNEL_CACHE,
// else `_kcache` beside the library; an unwritable directory disables it. A
// hit refreshes the file's modification time, so entries not used since a
// given time can be deleted safely.
static std::string cache_dir() {
    static std::string dir = [] {
        const char *env = std::getenv("TMOTIF_KERNEL_CACHE");
        if (env) return std::string(env);
        Dl_info info;
        if (dladdr((const void *)&cache_dir, &info) && info.dli_fname) {
            std::string p(info.dli_fname);
            size_t s = p.find_last_of('/');
            return (s == std::string::npos ? std::string(".") : p.substr(0, s)) + "/_kcache";
        }
        return std::string();
    }();
    return dir;
}

static std::string cache_path(const std::string &src) {
    uint64_t h1 = 1469598103934665603ull, h2 = 0x9e3779b97f4a7c15ull;
    for (unsigned char ch : src) {
        h1 = (h1 ^ ch) * 1099511628211ull;
        h2 = (h2 ^ ch) * 0x100000001b3ull + 0x7f4a7c15ull;
    }
    char name[64];
    std::snprintf(name, sizeof(name), "/%016llx%016llx.co", (unsigned long long)h1, (unsigned long long)h2);
    return cache_dir() + name;
}

static const uint64_t kCacheMagic = 0x31304f434d544d54ull;  // file format tag

static bool cache_load(const std::string &src, std::vector<char> *code) {
    const std::string dir = cache_dir();
    if (dir.empty()) return false;
    FILE *f = std::fopen(cache_path(src).c_str(), "rb");
    if (!f) return false;
    uint64_t hdr[2] = {0, 0};
    bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == kCacheMagic && hdr[1] == src.size();
    if (ok) {
        std::string stored(src.size(), '\0');
        ok = std::fread(&stored[0], 1, src.size(), f) == src.size() && stored == src;
    }
    if (ok) {
        std::vector<char> buf;
        char tmp[1 << 16];
        size_t n;
        while ((n = std::fread(tmp, 1, sizeof(tmp), f)) > 0) buf.insert(buf.end(), tmp, tmp + n);
        ok = !buf.empty();
        if (ok) code->swap(buf);
    }
    std::fclose(f);
    if (ok) utime(cache_path(src).c_str(), nullptr);  // mark as recently used
    return ok;
}

static void cache_store(const std::string &src, const std::vector<char> &code) {
    const std::string dir = cache_dir();
    if (dir.empty()) return;
    mkdir(dir.c_str(), 0755);
    const std::string path = cache_path(src);
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return;
    uint64_t hdr[2] = {kCacheMagic, (uint64_t)src.size()};
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 && std::fwrite(src.data(), 1, src.size(), f) == src.size() &&
              std::fwrite(code.data(), 1, code.size(), f) == code.size();
    ok = (std::fclose(f) == 0) && ok;
    if (ok) ok = std::rename(tmp.c_str(), path.c_str()) == 0;
    if (!ok) std::remove(tmp.c_str());
}

bool cached_code(const std::string &src, std::vector<char> *code, std::string *err) {
    // the cache key is the compiler version, its options and the exact source text
    int major = 0, minor = 0;
    hiprtcVersion(&major, &minor);
    std::string key = "// hiprtc " + std::to_string(major) + "." + std::to_string(minor);
    for (int i = 0; i < kRtcNopts; i++) key += std::string(" ") + kRtcOpts[i];
    key += "\n" + src;
    if (cache_load(key, code)) return true;
    if (!compile_to_code(src, code, err)) return false;
    cache_store(key, *code);
    return true;
}

// `modes` as for emit_kernels: the kernels the module holds.
// An unsigned field of the first kernel's metadata in a code object: the
// metadata note is MessagePack, where the field name is a short string (one
// prefix byte 0xa0 | length) followed by the value as a positive fixint or a
// uint8/16/32. -1 when absent.
static long meta_uint(const std::vector<char> &code, const char *field) {
    const size_t n = std::strlen(field);
    std::string pat(1, (char)(0xa0u | (unsigned)n));
    pat += field;
    auto it = std::search(code.begin(), code.end(), pat.begin(), pat.end());
    if (it == code.end()) return -1;
    const size_t i = (size_t)(it - code.begin()) + pat.size();
    if (i >= code.size()) return -1;
    const unsigned char b = (unsigned char)code[i];
    auto be = [&](int k) {
        if (i + (size_t)k >= code.size()) return -1L;
        long v = 0;
        for (int j = 1; j <= k; j++) v = (v << 8) | (unsigned char)code[i + j];
        return v;
    };
    if (b < 0x80) return b;
    if (b == 0xcc) return be(1);
    if (b == 0xcd) return be(2);
    if (b == 0xce) return be(4);
    return -1;
}

// Waves per SIMD that `vgprs` registers per lane leave room for on gfx950
// (512 registers per lane across the SIMD's waves, allocated in granules of 8).
static int waves_for(long vgprs) {
    const long a = (vgprs + 7) / 8 * 8;
    return a <= 0 ? 8 : (int)std::min(8L, 512 / a);
}

bool batch_code(const std::vector<const Plan *> &plans, int key_bytes, int block, int min_waves,
                std::vector<char> *code, std::string *err, int form) {
    if (!cached_code(generate_batch_source(plans, key_bytes, block, min_waves, form), code, err)) return false;
    if (min_waves != 0) return true;
    // A batched kernel a few registers above a wave boundary runs one wave
    // more per SIMD when compiled to fit it (the persistent kernel hides its
    // dependent loads with waves); kept if the squeeze spills little.
    const long v = meta_uint(*code, ".vgpr_count");
    const int w = waves_for(v);
    if (v < 0 || w >= 8) return true;
    const long fit = (512 / (w + 1)) / 8 * 8;
    if (v - fit > kSqueezeRegs) return true;
    std::vector<char> c2;
    std::string e2;
    if (!cached_code(generate_batch_source(plans, key_bytes, block, w + 1, form), &c2, &e2)) return true;
    const long spill = meta_uint(c2, ".vgpr_spill_count");
    if (spill < 0 || spill > kSqueezeSpills) return true;
    code->swap(c2);
    return true;
}

static bool compile_module(const std::vector<char> &code, int block, unsigned modes, Module *out, std::string *err) {
    const bool batch = modes == 0;
    const char *const *names = batch ? &kBatchName : kSingleNames;
    const int nmodes = batch ? 1 : 4;
    hipError_t he = hipModuleLoadData(&out->mod, code.data());
    if (he != hipSuccess) {
        *err = std::string("hipModuleLoadData: ") + hipGetErrorString(he);
        return false;
    }
    for (int mode = 0; mode < nmodes; mode++) {
        if (!batch && !((modes >> mode) & 1u)) continue;
        he = hipModuleGetFunction(&out->fn[mode], out->mod, names[mode]);
        if (he != hipSuccess) {
            *err = std::string("hipModuleGetFunction(") + names[mode] + "): " + hipGetErrorString(he);
            hipModuleUnload(out->mod);
            out->mod = nullptr;
            return false;
        }
    }
    int nb = 0;
    hipFunction_t any = nullptr;
    for (int mode = 0; mode < MODE_COUNT_ && !any; mode++) any = out->fn[mode];
    if (any && hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, any, block, 0) == hipSuccess)
        out->max_blocks_per_cu = nb;
    return true;
}

std::shared_ptr<Module> Compiler::lookup_or_build(const std::string &key, int block, unsigned modes,
                                                  const CodeFn &make, std::string *err) {
    {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
            auto it = cache.find(key);
            if (it != cache.end()) return it->second;
            if (!inflight.count(key)) break;
            cv.wait(lk);  // another thread is compiling this key; a failed compile is retried here
        }
        inflight.insert(key);
    }
    auto m = std::make_shared<Module>();
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<char> code;
    const bool ok = make(&code, err) && compile_module(code, block, modes, m.get(), err);
    m->compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::lock_guard<std::mutex> lk(mu);
    inflight.erase(key);
    if (ok) cache[key] = m;
    cv.notify_all();
    return ok ? m : nullptr;
}

std::shared_ptr<Module> Compiler::get(const Plan &p, int key_bytes, int block, std::string *err, int min_waves,
                                      unsigned modes, int form) {
    const std::string key = "S" + std::to_string(key_bytes) + "b" + std::to_string(block) +
                            (min_waves ? "w" + std::to_string(min_waves) : std::string()) +
                            (form ? "f" + std::to_string(form) : std::string()) + "m" + std::to_string(modes) + ":" +
                            p.key();
    return lookup_or_build(key, block, modes, [&](std::vector<char> *code, std::string *e) {
        return cached_code(generate_source(p, key_bytes, block, min_waves, modes, form), code, e);
    }, err);
}

static std::string batch_key(const std::vector<const Plan *> &plans, int key_bytes, int block, int min_waves,
                             int form) {
    std::string key = "B" + std::to_string(key_bytes) + "b" + std::to_string(block) +
                      (min_waves ? "w" + std::to_string(min_waves) : std::string()) +
                      (form ? "f" + std::to_string(form) : std::string()) + ":";
    for (auto *p : plans) key += p->key() + "|";
    return key;
}

std::shared_ptr<Module> Compiler::get_batch(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                            std::string *err, int min_waves, int form) {
    return lookup_or_build(batch_key(plans, key_bytes, block, min_waves, form), block, 0u,
                           [&](std::vector<char> *code, std::string *e) {
                               return batch_code(plans, key_bytes, block, min_waves, code, e, form);
                           }, err);
}

std::shared_ptr<Module> Compiler::find_batch(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                             int min_waves, int form) {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(batch_key(plans, key_bytes, block, min_waves, form));
    return it == cache.end() ? nullptr : it->second;
}

}  // namespace tmo
