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
#include <hip/hiprtc.h>

#include <chrono>
#include <cstring>
#include <sstream>

#include "tm_internal.h"

namespace tmo {

std::string Plan::key() const {
    std::ostringstream o;
    o << "l" << l << "k" << k << "p" << pred_level << ":";
    for (int i = 0; i < l; i++) o << a[i] << b[i] << ",";
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
    p->pred_level = d->pred_edge;
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
  float theta;
  int pred_op;
  int fn;
  int pad;
  i64 reserved;
};

struct GArgs {
  const int* src; const int* dst; const tkey* tk; const float* w;
  const tkey* adj_t; const int* adj_nbr; const int* adj_eid; const float* adj_w;
  const u32* off_out; const u32* off_in;
  const QArgs* qa;
  u64* ctl;
  u64* counts;
  u64* chunk_cnt; const u64* chunk_off; i64* out; u64 capacity;
  i64 m_edges; i64 total_chunks; int rch; int nq;
};
static_assert(sizeof(QArgs) == 128, "QArgs layout");
static_assert(sizeof(GArgs) == 160, "GArgs layout");

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
__device__ __forceinline__ u32 bitlen(u32 x) { return x ? 32u - (u32)__builtin_clz(x) : 0u; }
)HIP";

namespace {

struct Emitter {
    std::ostringstream o;
    const Plan &p;
    explicit Emitter(const Plan &pl) : p(pl) {}

    bool has_global() const {
        for (int i = 1; i < p.l; i++)
            if (p.kind[i] == LIST_GLOBAL) return true;
        return false;
    }

    // Open the candidate window of level i after binding edge i-1 at time `tp`.
    void open(int i, const char *tp, const char *ind) {
        const int A = p.a[i], B = p.b[i];
        o << ind << "{ // open level " << i << "\n";
        o << ind << "  u32 lo_, hi_;\n";
        switch (p.kind[i]) {
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
        o << ind << "  end" << i << " = hi_;\n";
        o << ind << "  { i64 h_ = (i64)(" << tp << ") + gap" << (i - 1) << "; hi" << i
          << " = (tkey)(h_ < (i64)tmaxk ? h_ : (i64)tmaxk); }\n";
        o << ind << "  sb = lo_; sn = hi_ - lo_; sx = (" << tp << "); lvl = " << i << ";\n";
        o << ind << "  if (sn == 0u) { cur" << i << " = lo_; ph = 0; } else { ph = 1; }\n";
        o << ind << "  if (MODE == 1) { st_win++; st_probe += bitlen(sn); }\n";
        o << ind << "}\n";
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

    void matcher(int fi) {
        const int L = p.l, K = p.k;
        const bool glob = has_global();
        o << "// motif " << p.key() << "\n";
        o << "template <int MODE>\n__device__ __forceinline__ i64 match" << fi
          << "(const GArgs& g, int qi, i64 chunk) {\n";
        o << "  const int lane = lane_id();\n";
        o << "  const QArgs* q = g.qa + qi;\n";
        o << "  const i64 q_r0 = q->r0, q_r1 = q->r1, q_delta = q->delta, q_c0 = q->c0, q_c1 = q->c0 + q->nchunks;\n";
        for (int i = 0; i + 1 < L; i++) o << "  const i64 gap" << i << " = q->gap[" << i << "];\n";
        if (p.pred_level >= 0) o << "  const float theta = q->theta; const int pop = q->pred_op;\n";
        o << "  int lvl = 0, ph = 0, root = 0;\n";
        o << "  i64 mych = 0;\n";
        o << "  int";
        for (int v = 0; v < K; v++) o << (v ? ", " : " ") << "m" << v << " = 0";
        o << ";\n";
        for (int i = 1; i < L; i++) {
            o << "  u32 cur" << i << " = 0u, end" << i << " = 0u; tkey hi" << i << " = 0;";
            if (p.kind[i] == LIST_BOTH) o << " int want" << i << " = 0;";
            if (i + 1 < L) o << " int e" << i << " = 0;";
            o << "\n";
        }
        o << "  tkey tmaxk = 0, sx = 0; u32 sb = 0u, sn = 0u;\n";
        o << "  u64 cnt = 0, rcnt = 0, st_win = 0, st_probe = 0, st_visit = 0, st_pv = 0, st_root = 0;\n";
        o << "  i64 pnext = q_r0 + (chunk - q_c0) * (i64)g.rch;\n";
        o << "  i64 pend = pnext + (i64)g.rch < q_r1 ? pnext + (i64)g.rch : q_r1;\n";
        o << "  i64 pchunk = chunk, pending = -1;\n";
        o << "  bool drained = false;\n";
        o << "  for (;;) {\n";
        // ---------------- refill
        o << "    const u64 need = ballot(lvl == 0);\n";
        o << "    if (need) {\n";
        o << "      const i64 nneed = (i64)__builtin_popcountll(need);\n";
        o << "      const i64 rk = (i64)rank_in(need);\n";
        o << "      const i64 avail = pend - pnext;\n";
        o << "      i64 myr = -1, myc = pchunk;\n";
        o << "      if (lvl == 0 && rk < avail) myr = pnext + rk;\n";
        o << "      if (avail >= nneed) { pnext += nneed; }\n";
        o << "      else {\n";
        o << "        pnext = pend;\n";
        o << "        if (!drained) {\n";
        o << "          i64 c = 0;\n";
        o << "          if (lane == 0) c = (i64)atomicAdd(&g.ctl[0], 1ull);\n";
        o << "          c = bcast64(c);\n";
        o << "          if (c >= q_c1) { drained = true; pending = c < g.total_chunks ? c : -1; }\n";
        o << "          else {\n";
        o << "            pchunk = c;\n";
        o << "            pnext = q_r0 + (c - q_c0) * (i64)g.rch;\n";
        o << "            pend = pnext + (i64)g.rch < q_r1 ? pnext + (i64)g.rch : q_r1;\n";
        o << "            const i64 k2 = rk - avail;\n";
        o << "            if (lvl == 0 && myr < 0 && k2 < pend - pnext) { myr = pnext + k2; myc = c; }\n";
        o << "            const i64 take = nneed - avail < pend - pnext ? nneed - avail : pend - pnext;\n";
        o << "            pnext += take;\n";
        o << "          }\n";
        o << "        }\n";
        o << "      }\n";
        o << "      if (lvl == 0) {\n";
        o << "        if (myr >= 0) {\n";
        o << "          const int r = (int)myr;\n";
        o << "          const int s = g.src[r], d = g.dst[r];\n";
        o << "          const tkey tr = g.tk[r];\n";
        o << "          if (MODE == 1) { st_root++;" << (p.pred_level == 0 ? " st_pv++;" : "") << " }\n";
        o << "          bool ok = s != d;\n";
        if (p.pred_level == 0) o << "          ok = ok && pred_ok(g.w[r], pop, theta);\n";
        o << "          if (ok) {\n";
        o << "            root = r; mych = myc;\n";
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
        if (L > 1) {
            // ---------------- search probe
            o << "    if (lvl > 0 && ph == 1) {\n";
            if (glob) {
                o << "      bool gl = false;\n";
                for (int i = 1; i < L; i++)
                    if (p.kind[i] == LIST_GLOBAL) o << "      gl = gl || lvl == " << i << ";\n";
                o << "      const tkey* sarr = gl ? g.tk : g.adj_t;\n";
            } else {
                o << "      const tkey* sarr = g.adj_t;\n";
            }
            o << "      const u32 half = sn >> 1; const u32 mid = sb + half;\n";
            o << "      const tkey v = sarr[mid];\n";
            o << "      if (v <= sx) { sb = mid + 1u; sn = sn - half - 1u; } else { sn = half; }\n";
            o << "      if (sn == 0u) {\n";
            o << "        switch (lvl) {\n";
            for (int i = 1; i < L; i++) o << "          case " << i << ": cur" << i << " = sb; break;\n";
            o << "          default: break;\n";
            o << "        }\n";
            o << "        ph = 0;\n";
            o << "      }\n";
            o << "    } else if (lvl > 0) {\n";
            // ---------------- candidate scan
            o << "      u32 c = 0u, e = 0u; tkey h = 0;\n";
            o << "      switch (lvl) {\n";
            for (int i = 1; i < L; i++)
                o << "        case " << i << ": c = cur" << i << "; e = end" << i << "; h = hi" << i << "; break;\n";
            o << "        default: break;\n";
            o << "      }\n";
            o << "      bool inwin = false; tkey tt = 0; int nb = 0;";
            if (p.pred_level >= 1) o << " float wv = 0.0f;";
            o << "\n";
            o << "      if (c < e) {\n";
            if (glob) {
                o << "        bool gl = false;\n";
                for (int i = 1; i < L; i++)
                    if (p.kind[i] == LIST_GLOBAL) o << "        gl = gl || lvl == " << i << ";\n";
                o << "        tt = gl ? g.tk[c] : g.adj_t[c];\n";
                o << "        if (!gl) nb = g.adj_nbr[c];\n";
            } else {
                o << "        tt = g.adj_t[c];\n";
                o << "        nb = g.adj_nbr[c];\n";
            }
            if (p.pred_level >= 1) {
                if (p.kind[p.pred_level] == LIST_GLOBAL)
                    o << "        if (lvl == " << p.pred_level << ") wv = g.w[c];\n";
                else
                    o << "        if (lvl == " << p.pred_level << ") wv = g.adj_w[c];\n";
            }
            o << "        inwin = tt <= h;\n";
            o << "        if (MODE == 1) { st_visit++;"
              << (p.pred_level >= 1 ? " if (lvl == " + std::to_string(p.pred_level) + ") st_pv++;" : std::string())
              << " }\n";
            o << "      }\n";
            o << "      if (!inwin) {\n";
            o << "        lvl -= 1;\n";
            o << "        if (lvl == 0 && MODE == 2 && rcnt) { atomicAdd(&g.chunk_cnt[mych], rcnt); cnt += rcnt; rcnt = 0; }\n";
            o << "      } else {\n";
            o << "        switch (lvl) {\n";
            for (int i = 1; i < L; i++) {
                const int A = p.a[i], B = p.b[i];
                o << "        case " << i << ": {\n";
                o << "          cur" << i << " = c + 1u;\n";
                std::ostringstream ok;
                std::string bind;
                std::string eid;
                switch (p.kind[i]) {
                case LIST_OUT:
                case LIST_IN: {
                    ok << "true";
                    for (int v : p.mapped[i]) ok << " && nb != m" << v;
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
                    bind = "m" + std::to_string(A) + " = cs; m" + std::to_string(B) + " = cd;";
                    eid = "(int)c";
                }
                }
                o << "          bool ok = " << ok.str() << ";\n";
                if (p.pred_level == i) o << "          ok = ok && pred_ok(wv, pop, theta);\n";
                o << "          if (ok) {\n";
                if (i == L - 1) {
                    leaf("            ", eid.c_str());
                } else {
                    if (!bind.empty()) o << "            " << bind << "\n";
                    o << "            if (MODE == 3) e" << i << " = " << eid << ";\n";
                    open(i + 1, "tt", "            ");
                }
                o << "          }\n";
                o << "        } break;\n";
            }
            o << "        default: break;\n";
            o << "        }\n";
            o << "      }\n";
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
        o << "  }\n";
        o << "  return pending;\n";
        o << "}\n\n";
    }
};

void emit_kernels(std::ostringstream &o, int nfn, int block, bool all_modes) {
    static const char *names[4] = {"tm_count", "tm_stats", "tm_enum_count", "tm_enum_write"};
    const int nmodes = all_modes ? 4 : 1;
    for (int mode = 0; mode < nmodes; mode++) {
        o << "extern \"C\" __global__ __launch_bounds__(" << block << ") void " << names[mode] << "(GArgs g) {\n";
        o << "  const int lane = lane_id();\n";
        o << "  i64 c = 0;\n";
        o << "  if (lane == 0) c = (i64)atomicAdd(&g.ctl[0], 1ull);\n";
        o << "  c = bcast64(c);\n";
        o << "  while (c >= 0 && c < g.total_chunks) {\n";
        o << "    int qi = 0;\n";
        o << "    if (g.nq > 1) { int lo = 0, hi = g.nq - 1;\n";
        o << "      while (lo < hi) { int md = (lo + hi + 1) >> 1; if (g.qa[md].c0 <= c) lo = md; else hi = md - 1; }\n";
        o << "      qi = lo; }\n";
        o << "    qi = __builtin_amdgcn_readfirstlane(qi);\n";
        o << "    const int fn = __builtin_amdgcn_readfirstlane(g.qa[qi].fn);\n";
        o << "    switch (fn) {\n";
        for (int f = 0; f < nfn; f++) o << "      case " << f << ": c = match" << f << "<" << mode << ">(g, qi, c); break;\n";
        o << "      default: c = -1; break;\n";
        o << "    }\n";
        o << "  }\n";
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

std::string generate_source(const Plan &p, int key_bytes, int block) {
    std::vector<const Plan *> v{&p};
    Emitter e(p);
    e.o << header(key_bytes);
    e.matcher(0);
    emit_kernels(e.o, 1, block, true);
    return e.o.str();
}

std::string generate_batch_source(const std::vector<const Plan *> &plans, int key_bytes, int block) {
    std::ostringstream all;
    all << header(key_bytes);
    for (size_t f = 0; f < plans.size(); f++) {
        Emitter e(*plans[f]);
        e.matcher((int)f);
        all << e.o.str();
    }
    emit_kernels(all, (int)plans.size(), block, false);
    return all.str();
}

// ---------------------------------------------------------------- compiling

bool compile_to_code(const std::string &src, std::vector<char> *code, std::string *err) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "tm_motif.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        *err = "hiprtcCreateProgram failed";
        return false;
    }
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
                          "-packed-fp32-ops"};
    hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof(opts) / sizeof(opts[0])), opts);
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

static bool compile_module(const std::string &src, int block, int nmodes, Module *out, std::string *err) {
    auto t0 = std::chrono::steady_clock::now();
    std::vector<char> code;
    if (!compile_to_code(src, &code, err)) return false;
    hipError_t he = hipModuleLoadData(&out->mod, code.data());
    if (he != hipSuccess) {
        *err = std::string("hipModuleLoadData: ") + hipGetErrorString(he);
        return false;
    }
    static const char *names[4] = {"tm_count", "tm_stats", "tm_enum_count", "tm_enum_write"};
    for (int mode = 0; mode < nmodes; mode++) {
        he = hipModuleGetFunction(&out->fn[mode], out->mod, names[mode]);
        if (he != hipSuccess) {
            *err = std::string("hipModuleGetFunction(") + names[mode] + "): " + hipGetErrorString(he);
            hipModuleUnload(out->mod);
            out->mod = nullptr;
            return false;
        }
    }
    int nb = 0;
    if (out->fn[0] && hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, out->fn[0], block, 0) == hipSuccess)
        out->max_blocks_per_cu = nb;
    out->compile_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return true;
}

std::shared_ptr<Module> Compiler::get(const Plan &p, int key_bytes, int block, std::string *err) {
    std::string key = "S" + std::to_string(key_bytes) + "b" + std::to_string(block) + ":" + p.key();
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    auto m = std::make_shared<Module>();
    if (!compile_module(generate_source(p, key_bytes, block), block, 4, m.get(), err)) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    cache[key] = m;
    return m;
}

std::shared_ptr<Module> Compiler::get_batch(const std::vector<const Plan *> &plans, int key_bytes, int block,
                                            std::string *err) {
    std::string key = "B" + std::to_string(key_bytes) + "b" + std::to_string(block) + ":";
    for (auto *p : plans) key += p->key() + "|";
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    auto m = std::make_shared<Module>();
    if (!compile_module(generate_batch_source(plans, key_bytes, block), block, 1, m.get(), err)) return nullptr;
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    cache[key] = m;
    return m;
}

}  // namespace tmo
