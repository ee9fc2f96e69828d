// Exclusive scan and stable LSD radix sort used by the binning step.
//
// Both take their element count from device memory (with a host-side capacity that sizes
// the grid), issue no memset and never synchronise, so the whole binning sequence can be
// captured in a hipGraph and replayed with different counts.
//
// Radix sort: 8-bit digits, least significant first.  Each pass is a stable counting
// sort: per-block digit histograms -> exclusive scan of the digit-major histogram matrix
// -> scatter with ranks that are stable inside the block (each wavefront ranks a contiguous
// slice of the block; equal digits inside a wavefront's slot are matched with ballots),
// staged in LDS so that each digit's run of the block is written contiguously.
#include <hip/hip_runtime.h>

#include "vista_internal.h"

namespace vista {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;   // elements per block
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;   // records per block
constexpr int kRadix = 256;

__device__ __forceinline__ uint64_t block_exclusive_u64(uint64_t x, uint64_t* sh, uint64_t* total) {
    // sh: at least kScanThreads / 64 entries.  Inclusive scan in each wavefront by shuffles,
    // then the wavefront totals through LDS.
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    uint64_t inc = x;
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    uint64_t before = 0, all = 0;
    for (int k = 0; k < kScanThreads / 64; ++k) {
        const uint64_t s = sh[k];
        if (k < w) before += s;
        all += s;
    }
    *total = all;
    __syncthreads();                      // sh is free again when this returns
    return before + inc - x;
}

// Per-block totals of in[0, n).
template <class T>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const T* __restrict__ in, const int64_t* __restrict__ n_dev,
                                                               int64_t n_host, uint64_t* __restrict__ sums) {
    __shared__ uint64_t sh[kScanThreads];
    int64_t n = n_dev ? *n_dev : n_host;
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint64_t acc = 0;
    for (int i = 0; i < kScanItems; ++i) {
        int64_t e = base + (int64_t)i * kScanThreads + threadIdx.x;
        if (e < n) acc += (uint64_t)in[e];
    }
    uint64_t tot;
    block_exclusive_u64(acc, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of sums[0, nb) in place by one workgroup; sums[nb] = total.
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(uint64_t* __restrict__ sums, int64_t nb) {
    __shared__ uint64_t sh[kScanThreads];
    uint64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += kScanThreads) {
        int64_t b = b0 + threadIdx.x;
        uint64_t x = b < nb ? sums[b] : 0;
        uint64_t tot;
        uint64_t ex = block_exclusive_u64(x, sh, &tot);
        if (b < nb) sums[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

// out[e] = sums[block] + exclusive prefix inside the block; out[n] = total.  The tile goes
// through LDS both ways, so that global loads and stores are coalesced while each thread
// scans kScanItems consecutive items (element e of the tile at LDS index e + e / 16, which
// keeps a thread's consecutive items off one bank).
template <class T, class U>
__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const T* __restrict__ in, const int64_t* __restrict__ n_dev,
                                                              int64_t n_host, const uint64_t* __restrict__ sums,
                                                              int64_t nb, U* __restrict__ out) {
    __shared__ uint64_t sh[kScanThreads];
    __shared__ uint64_t tile[kScanTile + kScanTile / 16];
    const int64_t n = n_dev ? *n_dev : n_host;
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    auto at = [](int e) { return e + (e >> 4); };
    for (int i = 0; i < kScanItems; ++i) {
        const int e = i * kScanThreads + (int)threadIdx.x;
        tile[at(e)] = base + e < n ? (uint64_t)in[base + e] : 0;
    }
    __syncthreads();
    uint64_t v[kScanItems];
    uint64_t acc = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = tile[at((int)threadIdx.x * kScanItems + i)];
        acc += v[i];
    }
    uint64_t tot;
    uint64_t ex = block_exclusive_u64(acc, sh, &tot) + sums[blockIdx.x];
    for (int i = 0; i < kScanItems; ++i) {
        tile[at((int)threadIdx.x * kScanItems + i)] = ex;
        ex += v[i];
    }
    __syncthreads();
    for (int i = 0; i < kScanItems; ++i) {
        const int e = i * kScanThreads + (int)threadIdx.x;
        if (base + e < n) out[base + e] = (U)tile[at(e)];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (U)sums[nb];
}

// Digit histogram of each block: hist[d * nblocks + b].
__global__ void __launch_bounds__(kSortThreads) k_rs_hist(const uint32_t* __restrict__ keys, const int64_t* __restrict__ n_dev,
                                                          int64_t n_host, int shift, uint32_t* __restrict__ hist,
                                                          int64_t nblocks) {
    __shared__ uint32_t h[kRadix];
    int64_t n = n_dev ? *n_dev : n_host;
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int s = 0; s < kSortItems; ++s) {
        int64_t e = base + (int64_t)s * kSortThreads + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Scatter of one tile: every record is ranked among the tile's records of its digit, placed
// at that rank in LDS, and the tile is then written out from LDS digit run by digit run, so
// that consecutive threads store to consecutive addresses.  Wavefront w takes the tile's
// w-th slice of kSortItems * 64 records (slot by slot, lanes in order) and ranks them with
// counters of its own, so the slots need no workgroup barrier; the slices' counts are
// combined per digit once.  Ranks follow the tile's index order: the sort is stable.
__global__ void __launch_bounds__(kSortThreads) k_rs_scatter(const uint32_t* __restrict__ kin, const uint64_t* __restrict__ vin,
                                                             const int64_t* __restrict__ n_dev, int64_t n_host, int shift,
                                                             const uint32_t* __restrict__ hist,
                                                             const uint32_t* __restrict__ off, int64_t nblocks,
                                                             uint32_t* __restrict__ kout, uint64_t* __restrict__ vout) {
    constexpr int NW = kSortThreads / 64;
    constexpr int kSlice = kSortItems * 64;   // records of one wavefront's slice
    static_assert(kSortThreads == kRadix, "one thread per digit");
    __shared__ uint32_t wcnt[NW][kRadix];      // per slice: running count, then the slice's base
    __shared__ uint32_t lstart[kRadix];        // start of each digit's run in the tile
    __shared__ uint32_t gstart[kRadix];        // where that run goes in the output
    __shared__ uint32_t wtot[NW];
    __shared__ uint32_t sk[kSortTile];
    __shared__ uint64_t sv[kSortTile];
    const int64_t n = n_dev ? *n_dev : n_host;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    {
        // the tile's digit counts (from the histogram pass), exclusive scan over digits
        const int64_t hd = (int64_t)threadIdx.x * nblocks + blockIdx.x;
        const uint32_t c = hist[hd];
        gstart[threadIdx.x] = off[hd];
        uint32_t x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wtot[wave] = x;
        for (int w = 0; w < NW; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < wave; ++w) add += wtot[w];
        lstart[threadIdx.x] = x - c + add;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const int64_t sbase = base + (int64_t)wave * kSlice;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t key[kSortItems], rank[kSortItems];
    uint64_t val[kSortItems];
    for (int s = 0; s < kSortItems; ++s) {
        const int64_t e = sbase + (int64_t)s * 64 + lane;
        const bool valid = e < n;
        key[s] = valid ? kin[e] : 0u;
        val[s] = valid ? vin[e] : 0ull;
    }
    for (int s = 0; s < kSortItems; ++s) {
        const bool valid = sbase + (int64_t)s * 64 + lane < n;
        const uint32_t d = (key[s] >> shift) & (kRadix - 1);
        // lanes of this slot holding the same digit
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            peers &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t before = wcnt[wave][d];                  // this slice's count so far
        rank[s] = before + (uint32_t)__popcll(peers & lt);
        if (valid && (peers & lt) == 0) wcnt[wave][d] = before + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // slice bases per digit: the counts of the slices before
        const int dd = threadIdx.x;
        uint32_t r = 0;
        for (int w = 0; w < NW; ++w) {
            const uint32_t c = wcnt[w][dd];
            wcnt[w][dd] = r;
            r += c;
        }
    }
    __syncthreads();
    for (int s = 0; s < kSortItems; ++s) {
        if (sbase + (int64_t)s * 64 + lane >= n) continue;
        const uint32_t d = (key[s] >> shift) & (kRadix - 1);
        const uint32_t p = lstart[d] + wcnt[wave][d] + rank[s];
        sk[p] = key[s];
        sv[p] = val[s];
    }
    __syncthreads();
    const int nvalid = (int)(n - base < (int64_t)kSortTile ? (n - base > 0 ? n - base : 0) : (int64_t)kSortTile);
    for (int i = threadIdx.x; i < nvalid; i += kSortThreads) {
        const uint32_t k = sk[i];
        const uint32_t d = (k >> shift) & (kRadix - 1);
        const uint32_t pos = gstart[d] + ((uint32_t)i - lstart[d]);
        kout[pos] = k;
        vout[pos] = sv[i];
    }
}

template <class T, class U>
hipError_t scan_impl(const T* in, const int64_t* n_dev, int64_t cap, U* out, uint64_t* sums, hipStream_t s) {
    int64_t nb = (cap + kScanTile - 1) / kScanTile;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL((k_scan_reduce<T>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n_dev, cap, sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
    hipLaunchKernelGGL((k_scan_apply<T, U>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n_dev, cap, sums, nb,
                       out);
    return hipGetLastError();
}

}  // namespace

size_t scan_temp_elems(int64_t cap) { return (size_t)std::max<int64_t>(1, (cap + kScanTile - 1) / kScanTile) + 1; }

hipError_t exclusive_scan_u64(const uint64_t* in, const int64_t* n_dev, int64_t cap, uint64_t* out, uint64_t* sums,
                              hipStream_t s) {
    return scan_impl<uint64_t, uint64_t>(in, n_dev, cap, out, sums, s);
}

hipError_t exclusive_scan_u32_to_u64(const uint32_t* in, const int64_t* n_dev, int64_t cap, uint64_t* out,
                                     uint64_t* sums, hipStream_t s) {
    return scan_impl<uint32_t, uint64_t>(in, n_dev, cap, out, sums, s);
}

hipError_t exclusive_scan_u32_to_u32(const uint32_t* in, const int64_t* n_dev, int64_t cap, uint32_t* out,
                                     uint64_t* sums, hipStream_t s) {
    return scan_impl<uint32_t, uint32_t>(in, n_dev, cap, out, sums, s);
}

size_t radix_sort_temp_bytes(int64_t cap) {
    int64_t nb = std::max<int64_t>(1, (cap + kSortTile - 1) / kSortTile);
    int64_t m = nb * kRadix;
    // histogram + offsets (u32, one extra) + scan sums + ping-pong keys/values
    return (size_t)m * 4 * 2 + 16 + scan_temp_elems(m) * 8 + (size_t)cap * (4 + 8) + 1024;
}

hipError_t radix_sort_pairs(uint32_t* keys, uint64_t* vals, const int64_t* n_dev, int64_t cap, int bits, void* temp,
                            hipStream_t s) {
    if (cap <= 0) return hipSuccess;
    int64_t nb = std::max<int64_t>(1, (cap + kSortTile - 1) / kSortTile);
    int64_t m = nb * kRadix;
    char* p = (char*)temp;
    auto take = [&p](size_t b) { char* q = p; p += (b + 255) & ~(size_t)255; return q; };
    uint32_t* hist = (uint32_t*)take((size_t)m * 4);
    uint32_t* off = (uint32_t*)take((size_t)m * 4 + 4);
    uint64_t* sums = (uint64_t*)take(scan_temp_elems(m) * 8);
    uint32_t* k2 = (uint32_t*)take((size_t)cap * 4);
    uint64_t* v2 = (uint64_t*)take((size_t)cap * 8);
    uint32_t* ka = keys;
    uint64_t* va = vals;
    uint32_t* kb = k2;
    uint64_t* vb = v2;
    int passes = (bits + 7) / 8;
    if (passes < 1) passes = 1;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ka, n_dev, cap, shift, hist, nb);
        hipError_t e = scan_impl<uint32_t, uint32_t>(hist, nullptr, m, off, sums, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kSortThreads), 0, s, ka, va, n_dev, cap, shift, hist,
                           off, nb, kb, vb);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (passes & 1) {
        // result is in the temporary arrays: copy back with a kernel-free async copy
        hipError_t e = hipMemcpyAsync(keys, ka, (size_t)cap * 4, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
        e = hipMemcpyAsync(vals, va, (size_t)cap * 8, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

}  // namespace vista
