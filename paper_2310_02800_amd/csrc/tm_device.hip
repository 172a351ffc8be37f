// Device-side graph preprocessing and small utility kernels.
//
// Graph ingest (Sec. 2.2: a chronologically sorted temporal edge list plus
// CSR-like incoming and outgoing edge lists per node; Sec. 4.2, pipeline step
// 0: the data loader does all preprocessing on the GPU):
//   1. if the input is not time-ordered, a stable radix sort of (t, input
//      position) gives the edge order, and src/dst/w are gathered into it;
//   2. times are rebased to the minimum (int32 when the span allows);
//   3. per direction, a stable radix sort of (node, edge id) groups edge ids by
//      node while keeping id order, which is time order, inside each node; a
//      degree histogram and an exclusive scan give the offsets (the sort and
//      scan kernels are in tm_sort.hip);
//   4. a gather writes the adjacency as structure-of-arrays (time, neighbour,
//      edge id, weight), so the search kernels read contiguous windows.
// Out-lists occupy positions [0, m) and in-lists [m, 2m) of one unified
// adjacency, so a candidate window is a plain index range whichever list a
// motif level uses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kThreads = 256;

inline int blocks_for(int64_t n) {
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b > 65535LL * 32) b = 65535LL * 32;
    return (int)(b < 1 ? 1 : b);
}

__global__ void k_iota_i64(int64_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = i;
}

__global__ void k_iota_i32(int32_t *p, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_gather_edges(int64_t m, const int64_t *perm, const int32_t *src_in, const int32_t *dst_in,
                               const float *w_in, int32_t *src_out, int32_t *dst_out, float *w_out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t j = perm[i];
        src_out[i] = src_in[j];
        dst_out[i] = dst_in[j];
        if (w_in) w_out[i] = w_in[j];
    }
}

template <typename K>
__global__ void k_make_keys(int64_t m, const int64_t *t, int64_t t_min, K *tk) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        tk[i] = (K)(t[i] - t_min);
}

__global__ void k_check_ids(int64_t m, int64_t n, const int32_t *src, const int32_t *dst, uint32_t *bad) {
    uint32_t any = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t s = src[i], d = dst[i];
        any |= (s < 0 || s >= n || d < 0 || d >= n) ? 1u : 0u;
    }
    if (any) atomicOr(bad, 1u);
}

__global__ void k_degree(int64_t m, const int32_t *key, uint32_t *deg) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&deg[key[i]], 1u);
}

__global__ void k_add_u32(uint32_t *p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] += v;
}

template <typename K>
__global__ void k_gather_adj(int64_t m, const int32_t *eids, const int32_t *other, const K *tk, const float *w,
                             K *adj_t, int32_t *adj_nbr, int32_t *adj_eid, float *adj_w, uint32_t *pos,
                             uint32_t add) {
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
        int32_t e = eids[p];
        adj_t[p] = tk[e];
        adj_nbr[p] = other[e];
        adj_eid[p] = e;
        if (w) adj_w[p] = w[e];
        pos[e] = add + (uint32_t)p;
    }
}

// Launch errors are read back with hipGetLastError(), which also returns an
// error some earlier, unrelated call left on this thread; clearing it first
// makes the check report this helper's own launches.
void clear_stale_error() { (void)hipGetLastError(); }

// pr_pos[pos[e]] = add + i: where the adjacency entry of edge e sits in the
// pair-sorted order of the same lists
__global__ void k_pair_pos(int64_t m, const int32_t *ids, const uint32_t *pos, uint32_t add, uint32_t *pr_pos) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        pr_pos[pos[ids[i]]] = add + (uint32_t)i;
}

template <typename K>
__global__ void k_gather_pairs(int64_t m, const int32_t *ids, const int32_t *other, const K *tk, int32_t *pr_nbr,
                               K *pr_t) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = ids[i];
        pr_nbr[i] = other[e];
        pr_t[i] = tk[e];
    }
}

// int64 time -> unsigned key with the same order (sign bit flipped), and back
__global__ void k_time_keys(int64_t m, const int64_t *t, uint64_t *k) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        k[i] = (uint64_t)t[i] ^ (1ull << 63);
}

__global__ void k_untime_keys(int64_t m, const uint64_t *k, int64_t *t) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        t[i] = (int64_t)(k[i] ^ (1ull << 63));
}

// (node, neighbour) as one key: node in the high bits
__global__ void k_pair_keys(int64_t m, const int32_t *key, const int32_t *other, int nbits, uint64_t *k64) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        k64[i] = ((uint64_t)(uint32_t)key[i] << nbits) | (uint64_t)(uint32_t)other[i];
}

__global__ void k_copy_u32(int64_t m, const int32_t *in, uint32_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)in[i];
}

int bits_for(int64_t n) {
    int b = 1;
    while (b < 31 && (int64_t(1) << b) < n) b++;
    return b;
}

}  // namespace

hipError_t dev_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t s) {
    clear_stale_error();
    if (n <= 0) return hipSuccess;
    k_fill_u64<<<blocks_for(n), kThreads, 0, s>>>(p, v, n);
    return hipGetLastError();
}

__global__ void k_gather_i32(int64_t n, const int32_t *idx, const int32_t *vals, int32_t *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = vals[idx[i]];
}

hipError_t dev_gather_i32(int64_t n, const int32_t *eid, const int32_t *el, int32_t *out, hipStream_t s) {
    clear_stale_error();
    if (n <= 0) return hipSuccess;
    k_gather_i32<<<blocks_for(n), kThreads, 0, s>>>(n, eid, el, out);
    return hipGetLastError();
}

// Samples of the hub lists staged in LDS: sample i of hub h (slots
// soff[h] .. soff[h+1]) is the time key at adjacency position
// start[h] + (i - soff[h]) * 2^lg[h]. The table's header (hub count, starts,
// sample offsets, strides) is already in place; samples follow at word `base`.
template <typename K>
__global__ void k_hub_samples(uint32_t *tab, uint32_t base, const K *adj_t) {
    const uint32_t H = tab[0];
    const uint32_t *start = tab + 1, *soff = tab + 1 + H, *lg = tab + 2 + 2 * H;
    K *out = (K *)(tab + base);
    const uint32_t total = soff[H];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        uint32_t lo = 0, n = H;  // hub h: the last with soff[h] <= i
        while (n > 0) {
            const uint32_t h2 = n >> 1;
            if (soff[lo + h2 + 1] <= i) { lo += h2 + 1; n -= h2 + 1; } else { n = h2; }
        }
        out[i] = adj_t[start[lo] + ((i - soff[lo]) << lg[lo])];
    }
}

hipError_t dev_hub_samples(uint32_t *d_tab, uint32_t base, uint32_t total, const void *adj_t, int key_bytes,
                           hipStream_t s) {
    clear_stale_error();
    if (total == 0) return hipSuccess;
    const int blocks = (int)std::min<uint32_t>((total + kThreads - 1) / kThreads, 1024u);
    if (key_bytes == 4)
        k_hub_samples<int32_t><<<blocks, kThreads, 0, s>>>(d_tab, base, (const int32_t *)adj_t);
    else
        k_hub_samples<int64_t><<<blocks, kThreads, 0, s>>>(d_tab, base, (const int64_t *)adj_t);
    return hipGetLastError();
}

// Line samples of the unified adjacency: samp[j] = adj_t[j << lg], one time
// key per 2^lg positions (one cache line of keys), a search index that is
// 2^lg times smaller than the lists it covers.
template <typename K>
__global__ void k_line_samples(int64_t n, const K *adj_t, int lg, K *samp) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        samp[j] = adj_t[j << lg];
}

hipError_t dev_line_samples(int64_t n, const void *adj_t, int key_bytes, int lg, void *samp, hipStream_t s) {
    clear_stale_error();
    if (n <= 0) return hipSuccess;
    if (key_bytes == 4)
        k_line_samples<int32_t><<<blocks_for(n), kThreads, 0, s>>>(n, (const int32_t *)adj_t, lg, (int32_t *)samp);
    else
        k_line_samples<int64_t><<<blocks_for(n), kThreads, 0, s>>>(n, (const int64_t *)adj_t, lg, (int64_t *)samp);
    return hipGetLastError();
}

// Device scratch of tm_count_batch_noalloc, for callers that cannot allocate
// device memory: control words, per-query counts, queue heads and launch
// arguments, and the donated-work items, in one statically sized array each
// device holds until the process ends. Host code uses the address
// hipGetSymbolAddress returns for the current device, never the array's name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
std::atomic<uint32_t> g_scratch_epoch[kMaxDevices];
std::mutex g_scratch_use[kMaxDevices];
}  // namespace

hipError_t scratch_for_device(int device, void **out) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

std::atomic<uint32_t> *scratch_epoch(int device) { return &g_scratch_epoch[device]; }
std::mutex *scratch_mutex(int device) { return &g_scratch_use[device]; }

hipError_t dev_check_ids(int64_t m, int64_t n, const int32_t *d_src, const int32_t *d_dst, uint32_t *d_bad,
                         hipStream_t s) {
    clear_stale_error();
    if (m <= 0) return hipSuccess;
    k_check_ids<<<blocks_for(m), kThreads, 0, s>>>(m, n, d_src, d_dst, d_bad);
    return hipGetLastError();
}

hipError_t dev_sort_by_time(int64_t m, int64_t *d_t, int64_t *d_perm, hipStream_t s) {
    clear_stale_error();
    // stable sort of (t, position): returns sorted t in d_t and the input
    // position of each sorted edge in d_perm
    if (m <= 1) {
        if (m == 1) k_iota_i64<<<1, kThreads, 0, s>>>(d_perm, m);
        return hipGetLastError();
    }
    uint64_t *k = nullptr, *k_alt = nullptr;
    int64_t *v_alt = nullptr;
    uint32_t *hist = nullptr, *stmp = nullptr;
    bool in_alt = false;
    const int64_t nh = radix_hist_elems(m);
    hipError_t e = hipMalloc(&k, m * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&k_alt, m * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&v_alt, m * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&hist, nh * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&stmp, scan_tmp_elems(nh) * sizeof(uint32_t));
    if (e == hipSuccess) {
        k_time_keys<<<blocks_for(m), kThreads, 0, s>>>(m, d_t, k);
        k_iota_i64<<<blocks_for(m), kThreads, 0, s>>>(d_perm, m);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = dev_radix_sort_pairs<uint64_t, int64_t>(k, d_perm, k_alt, v_alt, m, 64, hist, stmp, s,
                                                                      &in_alt);
    if (e == hipSuccess && in_alt) e = hipMemcpyAsync(d_perm, v_alt, m * sizeof(int64_t), hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) {
        k_untime_keys<<<blocks_for(m), kThreads, 0, s>>>(m, in_alt ? k_alt : k, d_t);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipStreamSynchronize(s);
    (void)hipFree(stmp);
    (void)hipFree(hist);
    (void)hipFree(v_alt);
    (void)hipFree(k_alt);
    (void)hipFree(k);
    return e;
}

hipError_t dev_gather_edges(int64_t m, const int64_t *d_perm, const int32_t *src_in, const int32_t *dst_in,
                            const float *w_in, int32_t *src_out, int32_t *dst_out, float *w_out, hipStream_t s) {
    clear_stale_error();
    if (m <= 0) return hipSuccess;
    k_gather_edges<<<blocks_for(m), kThreads, 0, s>>>(m, d_perm, src_in, dst_in, w_in, src_out, dst_out, w_out);
    return hipGetLastError();
}

hipError_t dev_make_keys(int64_t m, const int64_t *d_t, int64_t t_min, int key_bytes, void *d_tk, hipStream_t s) {
    clear_stale_error();
    if (m <= 0) return hipSuccess;
    if (key_bytes == 4)
        k_make_keys<int32_t><<<blocks_for(m), kThreads, 0, s>>>(m, d_t, t_min, (int32_t *)d_tk);
    else
        k_make_keys<int64_t><<<blocks_for(m), kThreads, 0, s>>>(m, d_t, t_min, (int64_t *)d_tk);
    return hipGetLastError();
}

// Per-node lists sorted by (neighbour, time), for counting the edges between
// two given nodes inside a time window with binary searches. Same grouping by
// node (and so the same offsets) as the time-sorted lists below.
hipError_t dev_build_pairs(int64_t n, int64_t m, const int32_t *d_key, const int32_t *d_other, const void *d_tk,
                           int key_bytes, int32_t *d_pr_nbr, void *d_pr_t, const uint32_t *d_pos, uint32_t add,
                           uint32_t *d_pr_pos, hipStream_t s) {
    clear_stale_error();
    if (m <= 0) return hipSuccess;
    hipError_t e = hipSuccess;
    uint64_t *k = nullptr, *k_alt = nullptr;
    int32_t *ids = nullptr, *ids_alt = nullptr;
    uint32_t *hist = nullptr, *stmp = nullptr;
    bool in_alt = false;
    const int nbits = bits_for(n);
    const int64_t nh = radix_hist_elems(m);
    e = hipMalloc(&k, m * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&k_alt, m * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&ids, m * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&ids_alt, m * sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&hist, nh * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&stmp, scan_tmp_elems(nh) * sizeof(uint32_t));
    if (e != hipSuccess) goto done;
    k_pair_keys<<<blocks_for(m), kThreads, 0, s>>>(m, d_key, d_other, nbits, k);
    k_iota_i32<<<blocks_for(m), kThreads, 0, s>>>(ids, m);
    // the sort is stable: equal (node, neighbour) keys keep edge-id order,
    // which is time order
    e = dev_radix_sort_pairs<uint64_t, int32_t>(k, ids, k_alt, ids_alt, m, 2 * nbits, hist, stmp, s, &in_alt);
    if (e != hipSuccess) goto done;
    {
        const int32_t *sorted = in_alt ? ids_alt : ids;
        if (key_bytes == 4)
            k_gather_pairs<int32_t><<<blocks_for(m), kThreads, 0, s>>>(m, sorted, d_other, (const int32_t *)d_tk,
                                                                        d_pr_nbr, (int32_t *)d_pr_t);
        else
            k_gather_pairs<int64_t><<<blocks_for(m), kThreads, 0, s>>>(m, sorted, d_other, (const int64_t *)d_tk,
                                                                        d_pr_nbr, (int64_t *)d_pr_t);
        k_pair_pos<<<blocks_for(m), kThreads, 0, s>>>(m, sorted, d_pos, add, d_pr_pos);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
done:
    (void)hipStreamSynchronize(s);
    (void)hipFree(stmp);
    (void)hipFree(hist);
    (void)hipFree(ids_alt);
    (void)hipFree(ids);
    (void)hipFree(k_alt);
    (void)hipFree(k);
    return e;
}

// Build one direction of the adjacency. d_key = the node that owns the list
// (src for out-lists, dst for in-lists), d_other = the neighbour. Positions
// are offset by `add` (0 for out-lists, m for in-lists).
hipError_t dev_build_csr(int64_t n, int64_t m, const int32_t *d_key, const int32_t *d_other, const void *d_tk,
                         int key_bytes, const float *d_w, uint32_t add, uint32_t *d_off, void *d_adj_t,
                         int32_t *d_adj_nbr, int32_t *d_adj_eid, float *d_adj_w, uint32_t *d_pos, hipStream_t s) {
    clear_stale_error();
    hipError_t e = hipSuccess;
    uint32_t *deg = nullptr, *keys = nullptr, *keys_alt = nullptr, *hist = nullptr, *stmp = nullptr;
    int32_t *ids = nullptr, *ids_alt = nullptr;
    bool in_alt = false;
    const int nbits = bits_for(n);
    const int64_t nh = radix_hist_elems(std::max<int64_t>(m, 1));
    const int64_t ntmp = std::max(scan_tmp_elems(nh), scan_tmp_elems(n + 1));
    e = hipMalloc(&deg, (n + 1) * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&stmp, ntmp * sizeof(uint32_t));
    if (e != hipSuccess) goto done;
    k_fill_u32<<<blocks_for(n + 1), kThreads, 0, s>>>(deg, 0u, n + 1);
    if (m > 0) {
        e = hipMalloc(&keys, m * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&keys_alt, m * sizeof(uint32_t));
        if (e == hipSuccess) e = hipMalloc(&ids, m * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&ids_alt, m * sizeof(int32_t));
        if (e == hipSuccess) e = hipMalloc(&hist, nh * sizeof(uint32_t));
        if (e != hipSuccess) goto done;
        k_degree<<<blocks_for(m), kThreads, 0, s>>>(m, d_key, deg);
        k_copy_u32<<<blocks_for(m), kThreads, 0, s>>>(m, d_key, keys);
        k_iota_i32<<<blocks_for(m), kThreads, 0, s>>>(ids, m);
        e = hipGetLastError();
        if (e != hipSuccess) goto done;
        e = dev_radix_sort_pairs<uint32_t, int32_t>(keys, ids, keys_alt, ids_alt, m, nbits, hist, stmp, s, &in_alt);
        if (e != hipSuccess) goto done;
    }
    // offsets: exclusive scan of the degrees (n + 1 entries, the last one 0)
    e = dev_exclusive_scan_u32(deg, d_off, n + 1, stmp, s);
    if (e != hipSuccess) goto done;
    if (add) k_add_u32<<<blocks_for(n + 1), kThreads, 0, s>>>(d_off, add, n + 1);
    if (m > 0) {
        const int32_t *sorted = in_alt ? ids_alt : ids;
        if (key_bytes == 4)
            k_gather_adj<int32_t><<<blocks_for(m), kThreads, 0, s>>>(
                m, sorted, d_other, (const int32_t *)d_tk, d_w, (int32_t *)d_adj_t + add, d_adj_nbr + add,
                d_adj_eid + add, d_w ? d_adj_w + add : nullptr, d_pos, add);
        else
            k_gather_adj<int64_t><<<blocks_for(m), kThreads, 0, s>>>(
                m, sorted, d_other, (const int64_t *)d_tk, d_w, (int64_t *)d_adj_t + add, d_adj_nbr + add,
                d_adj_eid + add, d_w ? d_adj_w + add : nullptr, d_pos, add);
    }
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
done:
    (void)hipStreamSynchronize(s);
    (void)hipFree(hist);
    (void)hipFree(ids_alt);
    (void)hipFree(ids);
    (void)hipFree(keys_alt);
    (void)hipFree(keys);
    (void)hipFree(stmp);
    (void)hipFree(deg);
    return e;
}

}  // namespace tmo
