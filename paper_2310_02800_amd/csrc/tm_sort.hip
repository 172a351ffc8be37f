// Exclusive prefix sums and a stable LSD radix sort of (key, value) pairs,
// written for wave64: the graph ingest's counting sorts by node (Sec. 2.2,
// CSR-like in/out lists kept in time order; Sec. 4.2, preprocessing on the
// GPU) and the enumeration writer's chunk offsets.
//
// Scan: a tile of 4096 elements per 256-thread workgroup is staged in LDS,
// each thread sums 16 consecutive elements, a wavefront scan (shuffles) and a
// scan over the four wavefronts give the thread's base; multi-tile inputs
// first reduce every tile, scan the tile sums (recursively) and then scan each
// tile from its base.
//
// Radix sort, one pass per 8-bit digit from the least significant:
//   1. per tile (4096 elements), a digit histogram in LDS;
//   2. an exclusive scan of the histograms in digit-major order gives every
//      (digit, tile) its first output position;
//   3. per tile, each wavefront takes 16 rounds of 64 consecutive elements;
//      the lanes holding the same digit are found with 8 ballots, an element's
//      rank is its same-digit lanes below it plus the count of that digit in
//      the wavefront's earlier rounds (LDS), then the wavefronts' counts are
//      scanned in order. Elements keep their input order within a digit, so
//      every pass is stable and the passes compose into a sort by the whole
//      key.
#include <hip/hip_runtime.h>

#include "tm_internal.h"

namespace tmo {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;  // elements per workgroup
constexpr int kWaves = kThreads / 64;

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T v, int lane) {
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Exclusive scan of one value per thread over the workgroup.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *wave_tot) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const T inc = wave_inclusive_scan(v, lane);
    if (lane == 63) wave_tot[w] = inc;
    __syncthreads();
    T base = 0;
    for (int i = 0; i < w; i++) base += wave_tot[i];
    __syncthreads();
    return base + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_tile_sum(const T *in, int64_t n, T *sums) {
    __shared__ T wave_tot[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    T s = 0;
    for (int i = 0; i < kItems; i++) {
        const int64_t g = base + (int64_t)i * kThreads + threadIdx.x;
        if (g < n) s += in[g];
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    s = wave_inclusive_scan(s, lane);
    if (lane == 63) wave_tot[w] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int i = 0; i < kWaves; i++) t += wave_tot[i];
        sums[blockIdx.x] = t;
    }
}

// out[i] = carry[tile] + sum of in[tile start .. i) (in == out allowed)
template <typename T>
__global__ void __launch_bounds__(kThreads) k_tile_scan(const T *in, T *out, int64_t n, const T *carry) {
    __shared__ T tile[kTile];
    __shared__ T wave_tot[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; i++) {
        const int idx = i * kThreads + threadIdx.x;
        const int64_t g = base + idx;
        tile[idx] = g < n ? in[g] : T(0);
    }
    __syncthreads();
    T s = 0;
    for (int i = 0; i < kItems; i++) s += tile[threadIdx.x * kItems + i];
    T run = block_exclusive_scan(s, wave_tot) + (carry ? carry[blockIdx.x] : T(0));
    for (int i = 0; i < kItems; i++) {
        const int idx = threadIdx.x * kItems + i;
        const T x = tile[idx];
        tile[idx] = run;
        run += x;
    }
    __syncthreads();
    for (int i = 0; i < kItems; i++) {
        const int idx = i * kThreads + threadIdx.x;
        const int64_t g = base + idx;
        if (g < n) out[g] = tile[idx];
    }
}

int64_t tiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

template <typename T>
hipError_t scan_rec(const T *in, T *out, int64_t n, T *tmp, hipStream_t s) {
    const int64_t nb = tiles_of(n);
    if (nb <= 1) {
        k_tile_scan<T><<<1, kThreads, 0, s>>>(in, out, n, nullptr);
        return hipGetLastError();
    }
    k_tile_sum<T><<<(unsigned)nb, kThreads, 0, s>>>(in, n, tmp);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = scan_rec<T>(tmp, tmp, nb, tmp + nb, s);
    if (e != hipSuccess) return e;
    k_tile_scan<T><<<(unsigned)nb, kThreads, 0, s>>>(in, out, n, tmp);
    return hipGetLastError();
}

// Key digit for the radix sort.
template <typename K>
__device__ __forceinline__ uint32_t digit_of(K k, int shift) {
    return (uint32_t)((k >> shift) & (K)255);
}

template <typename K>
__global__ void __launch_bounds__(kThreads) k_radix_hist(const K *keys, int64_t n, int shift, uint32_t *hist,
                                                         int64_t nb) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile;
    for (int i = 0; i < kItems; i++) {
        const int64_t g = base + (int64_t)i * kThreads + threadIdx.x;
        if (g < n) atomicAdd(&cnt[digit_of(keys[g], shift)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

template <typename K, typename V>
__global__ void __launch_bounds__(kThreads) k_radix_scatter(const K *kin, const V *vin, int64_t n, int shift,
                                                            const uint32_t *offs, int64_t nb, K *kout, V *vout) {
    __shared__ uint32_t cnt[kWaves][256];
    __shared__ uint32_t first[256];
    for (int w = 0; w < kWaves; w++) cnt[w][threadIdx.x] = 0u;
    first[threadIdx.x] = offs[(int64_t)threadIdx.x * nb + blockIdx.x];
    __syncthreads();
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t below = (1ull << lane) - 1ull;
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)w * (kItems * 64);
    K k[kItems];
    V v[kItems];
    uint32_t rank[kItems];
    for (int r = 0; r < kItems; r++) {
        const int64_t g = base + r * 64 + lane;
        const bool valid = g < n;
        k[r] = valid ? kin[g] : K(0);
        v[r] = valid ? vin[g] : V(0);
        const uint32_t d = digit_of(k[r], shift);
        uint64_t same = __builtin_amdgcn_ballot_w64(valid);
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __builtin_amdgcn_ballot_w64(bit);
            same &= bit ? bb : ~bb;
        }
        const uint64_t lower = same & below;
        // every lane reads the count before the lowest lane of its digit adds
        // the round's elements (LDS operations of one wavefront run in order)
        const uint32_t prior = valid ? cnt[w][d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid && lower == 0ull) cnt[w][d] = prior + (uint32_t)__builtin_popcountll(same);
        __builtin_amdgcn_wave_barrier();
        rank[r] = prior + (uint32_t)__builtin_popcountll(lower);
    }
    __syncthreads();
    {  // exclusive scan of the wavefronts' counts per digit, in wavefront order
        uint32_t run = 0u;
        for (int x = 0; x < kWaves; x++) {
            const uint32_t c = cnt[x][threadIdx.x];
            cnt[x][threadIdx.x] = run;
            run += c;
        }
    }
    __syncthreads();
    for (int r = 0; r < kItems; r++) {
        const int64_t g = base + r * 64 + lane;
        if (g < n) {
            const uint32_t d = digit_of(k[r], shift);
            const uint64_t pos = (uint64_t)first[d] + cnt[w][d] + rank[r];
            kout[pos] = k[r];
            vout[pos] = v[r];
        }
    }
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) {
    int64_t tot = 0;
    for (int64_t nb = tiles_of(n); nb > 1; nb = tiles_of(nb)) tot += nb;
    return tot + 1;
}

hipError_t dev_exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t s) {
    (void)hipGetLastError();
    if (n <= 0) return hipSuccess;
    return scan_rec<uint32_t>(in, out, n, tmp, s);
}

hipError_t dev_exclusive_scan_u64(const uint64_t *in, uint64_t *out, int64_t n, uint64_t *tmp, hipStream_t s) {
    (void)hipGetLastError();
    if (n <= 0) return hipSuccess;
    return scan_rec<uint64_t>(in, out, n, tmp, s);
}

int64_t radix_hist_elems(int64_t n) { return 256 * std::max<int64_t>(tiles_of(n), 1); }

template <typename K, typename V>
hipError_t dev_radix_sort_pairs(K *keys, V *vals, K *keys_alt, V *vals_alt, int64_t n, int end_bit,
                                uint32_t *hist, uint32_t *scan_tmp, hipStream_t s, bool *in_alt) {
    (void)hipGetLastError();
    *in_alt = false;
    if (n <= 1) return hipSuccess;
    const int64_t nb = tiles_of(n);
    K *ka = keys, *kb = keys_alt;
    V *va = vals, *vb = vals_alt;
    for (int shift = 0; shift < end_bit; shift += 8) {
        k_radix_hist<K><<<(unsigned)nb, kThreads, 0, s>>>(ka, n, shift, hist, nb);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = scan_rec<uint32_t>(hist, hist, 256 * nb, scan_tmp, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<K, V><<<(unsigned)nb, kThreads, 0, s>>>(ka, va, n, shift, hist, nb, kb, vb);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ka, kb);
        std::swap(va, vb);
        *in_alt = !*in_alt;
    }
    return hipSuccess;
}

template hipError_t dev_radix_sort_pairs<uint32_t, int32_t>(uint32_t *, int32_t *, uint32_t *, int32_t *, int64_t,
                                                             int, uint32_t *, uint32_t *, hipStream_t, bool *);
template hipError_t dev_radix_sort_pairs<uint64_t, int32_t>(uint64_t *, int32_t *, uint64_t *, int32_t *, int64_t,
                                                             int, uint32_t *, uint32_t *, hipStream_t, bool *);
template hipError_t dev_radix_sort_pairs<uint64_t, int64_t>(uint64_t *, int64_t *, uint64_t *, int64_t *, int64_t,
                                                             int, uint32_t *, uint32_t *, hipStream_t, bool *);

}  // namespace tmo
