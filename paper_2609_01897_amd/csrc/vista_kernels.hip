// gfx950 kernels of the ViSta stacking hot path.
//
//   track (count / emit) -- binning: each row's channels, walked in frequency order,
//       trace a radial line in uv (u_lambda = u_m nu/c); the cells along it are monotone,
//       so the channels that fall in one uv tile form one contiguous run.  Each run is
//       cut at the rest-channel block boundaries; every piece becomes one record keyed by
//       its (tile, block) unit.
//   sort (vista_sort.hip) / unit offsets -- stable grouping of the records by unit.
//   accum -- one workgroup owns one (uv tile, rest-channel block) unit of the grid state
//       in LDS, streams the unit's records (contiguous channel runs of one row), applies
//       the Eq. 2 phase shift with the phase argument formed and range-reduced in FP64,
//       splits every sample over the rest channels with the Eq. 3-4 fractions,
//       accumulates in LDS, and writes its cells once.
//
// Cell and channel indices follow the FP64 operation sequence of the definition exactly
// (this file is compiled with -ffp-contract=off, no fast-math): u = u_m * a_k,
// iu = rint(u * (1/du)) + nu/2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "vista_device.h"

namespace vista {

namespace {




// Channel scales a_k as the searches read them: from LDS (the block's staged copy) or from
// the target's channel table.
struct ScalesLds {
    const double* a;
    __device__ double operator[](int32_t k) const { return a[k]; }
};
struct ScalesGlobal {
    const DevChan* ch;
    __device__ double operator[](int32_t k) const { return ch[k].a; }
};

// First k in [lo, hi) with s * rint((c * a_k) * inv) >= A, or hi.  The key is
// non-decreasing in k for the given orientation s.  The continuous value s (c a_k) inv is
// close to linear in k, so one interpolation step from the range's end points guesses the
// answer g; the exact keys at g - 1 and g (two independent loads) confirm it or shrink the
// range, and bisection finishes what is left.  The answer is the same as plain bisection.
template <class A>
__device__ int32_t first_at_least(const A& a, int32_t lo, int32_t hi, double c, double inv, double s, double key_min) {
    if (hi - lo > 2) {
        const double x0 = s * ((c * a[lo]) * inv), x1 = s * ((c * a[hi - 1]) * inv);
        const double f = (key_min - 0.5 - x0) / (x1 - x0);           // rint reaches key_min at key_min - 1/2
        int32_t g = lo;
        if (f >= 1.0) g = hi;
        else if (f > 0.0) g = lo + (int32_t)ceil(f * (double)(hi - 1 - lo));    // also NaN -> lo
        g = min(max(g, lo), hi);
        const bool below = g > lo && s * cell_coord(c, a[g - 1], inv) < key_min;  // key(g - 1) < key_min
        const bool at = g == hi || s * cell_coord(c, a[g], inv) >= key_min;     // key(g) >= key_min
        if ((below || g == lo) && at) return g;
        if (!at) lo = g + 1;                   // key(g) < key_min: the answer is past g
        else hi = g - 1;                       // key(g - 1) >= key_min: the answer is at most g - 1
    }
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        double key = s * cell_coord(c, a[mid], inv);
        if (key >= key_min) hi = mid; else lo = mid + 1;
    }
    return lo;
}

struct Track {
    int32_t ga, gb;     // in-grid channel interval
    double su, sv;      // orientation of the u and v cell sequences
};

// In-grid interval of row (U, V) over channels [klo, khi).
template <class A>
__device__ Track in_grid(const A& a, int32_t klo, int32_t khi, double U, double V, double inv_du, double inv_dv,
                         int32_t nu, int32_t nv) {
    Track t;
    double u0 = cell_coord(U, a[klo], inv_du), u1 = cell_coord(U, a[khi - 1], inv_du);
    double v0 = cell_coord(V, a[klo], inv_dv), v1 = cell_coord(V, a[khi - 1], inv_dv);
    t.su = (u1 >= u0) ? 1.0 : -1.0;
    t.sv = (v1 >= v0) ? 1.0 : -1.0;
    // inside: -(n/2) <= r < n - n/2.  With key = s r: s>0 -> [lo_b, hi_b);
    // s<0 -> key in (-hi_b, -lo_b] = [1 - hi_b, 1 - lo_b) for integer-valued keys.
    double lob_u = -(double)(nu / 2), hib_u = (double)(nu - nu / 2);
    double lob_v = -(double)(nv / 2), hib_v = (double)(nv - nv / 2);
    double Au = t.su > 0 ? lob_u : 1.0 - hib_u, Bu = t.su > 0 ? hib_u : 1.0 - lob_u;
    double Av = t.sv > 0 ? lob_v : 1.0 - hib_v, Bv = t.sv > 0 ? hib_v : 1.0 - lob_v;
    int32_t a1 = first_at_least(a, klo, khi, U, inv_du, t.su, Au);
    int32_t b1 = first_at_least(a, a1, khi, U, inv_du, t.su, Bu);
    int32_t a2 = first_at_least(a, klo, khi, V, inv_dv, t.sv, Av);
    int32_t b2 = first_at_least(a, a2, khi, V, inv_dv, t.sv, Bv);
    t.ga = max(a1, a2);
    t.gb = min(b1, b2);
    if (t.gb < t.ga) t.gb = t.ga;
    return t;
}

// End (exclusive) of the run of channels starting at k that stay in k's uv tile.
template <class A>
__device__ int32_t tile_run_end(const A& a, int32_t k, int32_t gb, double U, double V, double inv_du,
                                double inv_dv, int32_t nu, int32_t nv, int32_t TU, int32_t TV, const Track& tr,
                                int32_t* tile_u, int32_t* tile_v) {
    double ru = cell_coord(U, a[k], inv_du), rv = cell_coord(V, a[k], inv_dv);
    int32_t iu = (int32_t)ru + nu / 2, iv = (int32_t)rv + nv / 2;
    int32_t tu = iu / TU, tv = iv / TV;
    *tile_u = tu;
    *tile_v = tv;
    // leave the tile upward: r >= (t+1) T - n/2; downward: r < t T - n/2, i.e.
    // -r >= -(t T - n/2) + 1.
    double Au = tr.su > 0 ? (double)((tu + 1) * TU - nu / 2) : (double)(-(tu * TU - nu / 2) + 1);
    double Av = tr.sv > 0 ? (double)((tv + 1) * TV - nv / 2) : (double)(-(tv * TV - nv / 2) + 1);
    int32_t nu_k = first_at_least(a, k + 1, gb, U, inv_du, tr.su, Au);
    int32_t nv_k = first_at_least(a, k + 1, gb, V, inv_dv, tr.sv, Av);
    return min(nu_k, nv_k);
}


// ----------------------------------------------------------------------------- binning

constexpr int kTrackThreads = 256;
constexpr int kTrackScales = 2048;     // channel scales of one target staged in LDS (16 KB)

// Records of row r of target T, whose uv cells come from (U, V): counted, or (EMIT)
// written from position `base` on.  Returns the count; `outside` gets the row's in-band
// samples that fall outside the grid.
template <bool EMIT, class A>
__device__ uint32_t track_row(const LaunchDesc& L, const DevTarget& T, const DevStack& S, const A& a, int64_t g,
                              double U, double V, uint32_t base, uint32_t* __restrict__ keys,
                              uint64_t* __restrict__ vals, unsigned long long* outside) {
    const Track tr = in_grid(a, T.kin_lo, T.kin_hi, U, V, S.inv_du, S.inv_dv, S.nu, S.nv);
    const int32_t inb_all = T.inband[T.kin_hi] - T.inband[T.kin_lo];
    const int32_t inb_in = T.inband[tr.gb] - T.inband[tr.ga];
    *outside = (unsigned long long)(inb_all - inb_in) * (unsigned long long)T.npol;
    uint32_t n = 0;
    int32_t k = tr.ga;
    while (k < tr.gb) {
        int32_t tu, tv;
        const int32_t k1 = tile_run_end(a, k, tr.gb, U, V, S.inv_du, S.inv_dv, S.nu, S.nv, L.tu, L.tv, tr, &tu, &tv);
        const int64_t unit0 = S.unit_base + ((int64_t)tv * S.tiles_u + tu) * S.nblocks;
        for (int32_t b = 0; b < T.nblocks; ++b) {
            const int32_t lo = max(k, T.blk[2 * b]), hi = min(k1, T.blk[2 * b + 1]);
            if (lo >= hi) continue;
            if (EMIT) {
                keys[base + n] = (uint32_t)(unit0 + b);
                vals[base + n] = ((uint64_t)g << 32) | ((uint64_t)lo << 16) | (uint64_t)hi;
            }
            ++n;
        }
        k = k1;
    }
    return n;
}

// Binning pass over the launch's rows, one thread per row: count (EMIT false, also writes
// each row's context for the packed accumulation) or emit the records.  The channel scales
// of the block's first target are staged in LDS when they fit, so the searches of its rows
// (nearly always every row of the block) read LDS instead of the channel table.
template <bool EMIT>
__global__ void __launch_bounds__(kTrackThreads) k_track(const LaunchDesc* __restrict__ Lp,
                                                         uint32_t* __restrict__ seg_count,
                                                         const uint32_t* __restrict__ seg_off,
                                                         uint32_t* __restrict__ keys,
                                                         uint64_t* __restrict__ vals) {
    __shared__ double s_scale[kTrackScales];
    const LaunchDesc& L = *Lp;
    const int64_t g0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t g = g0 + threadIdx.x;
    const int32_t t0 = g0 < L.nrows ? (int32_t)find_le_uniform(L.target_row_base, L.ntargets, g0) : -1;
    const bool staged = t0 >= 0 && L.targets[t0].nchan <= kTrackScales;
    if (staged) {
        const DevChan* ch = L.targets[t0].chan;
        for (int32_t k = threadIdx.x; k < L.targets[t0].nchan; k += blockDim.x) s_scale[k] = ch[k].a;
    }
    __syncthreads();
    unsigned long long outside = 0;
    int32_t stack_id = -1;
    if (g < L.nrows) {
        int32_t ti = t0;
        if (g >= L.targets[t0].row_base + L.targets[t0].nrow) ti = (int32_t)find_le(L.target_row_base, L.ntargets, g);
        const DevTarget& T = L.targets[ti];
        const DevStack& S = L.stacks[T.stack];
        stack_id = T.stack;
        const int64_t r = g - T.row_base;
        const double Um = T.uvw[3 * r], Vm = T.uvw[3 * r + 1], Wm = T.uvw[3 * r + 2];
        if (!EMIT && L.rowctx) {
            // the row's context for the packed accumulation
            RowCtx c;
            cell_uv(T, Um, Vm, Wm, &c.U, &c.V);     // uv cells: the (rotated) baseline
            if (L.phase_fp32)
                c.T = (double)((float)Um * (float)T.l + (float)Vm * (float)T.m + (float)Wm * (float)T.nm1);
            else
                c.T = Um * T.l + Vm * T.m + Wm * T.nm1;
            const size_t rs = (size_t)T.nchan * T.npol;     // samples per row
            c.w0 = T.weight_per_chan ? 0.f : T.weight[r * T.npol];
            c.w1 = (T.weight_per_chan || T.npol < 2) ? 0.f : T.weight[r * T.npol + 1];
            c.vis = (uint64_t)(T.vis + r * rs);
            c.flag = T.flag ? (uint64_t)(T.flag + r * rs) : (uint64_t)L.zero_flags;
            c.wrow = (uint64_t)(T.weight + (T.weight_per_chan ? r * rs : r * T.npol));
            c.chan0 = T.chan0;
            c.info = (uint32_t)T.npol | ((uint32_t)(T.weight_per_chan != 0) << 8);
            L.rowctx[g] = c;
        }
        uint32_t n = 0;
        if (T.kin_lo < T.kin_hi) {
            double U, V;
            cell_uv(T, Um, Vm, Wm, &U, &V);
            const uint32_t base = EMIT ? seg_off[g] : 0u;
            if (staged && ti == t0)
                n = track_row<EMIT>(L, T, S, ScalesLds{s_scale}, g, U, V, base, keys, vals, &outside);
            else
                n = track_row<EMIT>(L, T, S, ScalesGlobal{T.chan}, g, U, V, base, keys, vals, &outside);
        }
        if (!EMIT) seg_count[g] = n;
    }
    if (!EMIT) {
        // outside-uv samples: one atomic per wave and stack run (waves rarely straddle
        // two stacks; lanes of another stack add their own share)
        int32_t first = __shfl(stack_id, 0, kWave);
        unsigned long long mine = (stack_id == first) ? outside : 0ull;
        unsigned long long tot = wave_sum_u64(mine);
        if ((threadIdx.x & (kWave - 1)) == 0 && first >= 0 && tot) atomicAdd(&L.stacks[first].stats[3], tot);
        if (stack_id >= 0 && stack_id != first && outside) atomicAdd(&L.stacks[stack_id].stats[3], outside);
    }
}

// unit_off[u] = index of the first record of unit u (records sorted by unit).  Thread t
// covers record positions 4t .. 4t + 3 (position nrec stands for the end) and reads their
// keys with one 16-byte load where all four are records.
__global__ void k_unit_offsets(const uint32_t* __restrict__ keys, const int64_t* __restrict__ nrec_dev,
                               int64_t nrec_cap, const int64_t* __restrict__ nunits_dev,
                               uint32_t* __restrict__ off) {
    const int64_t nunits = *nunits_dev;
    const int64_t nrec = nrec_dev ? *nrec_dev : nrec_cap;
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 > nrec) return;
    int64_t cur[4];
    if (i0 + 4 <= nrec && ((uintptr_t)(keys + i0) & 15) == 0) {
        const uint4 k4 = *(const uint4*)(keys + i0);
        cur[0] = k4.x; cur[1] = k4.y; cur[2] = k4.z; cur[3] = k4.w;
    } else {
        for (int j = 0; j < 4; ++j) {
            const int64_t i = i0 + j;
            cur[j] = i < nrec ? (int64_t)keys[i] : nunits;
        }
    }
    int64_t prev = (i0 == 0) ? -1 : (int64_t)keys[i0 - 1];
    for (int j = 0; j < 4 && i0 + j <= nrec; ++j) {
        for (int64_t t = prev + 1; t <= cur[j] && t <= nunits; ++t) off[t] = (uint32_t)(i0 + j);
        prev = cur[j];
    }
}

// Fills walk the array in grid strides: a dispatch covers fewer than 2^32 work-items, and
// a carried grid state can hold more words than that.
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = v;
}

// flag <- 1 if a[i] != b[i] for some i (flag zeroed by the caller).
__global__ void k_diff_u32(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, int64_t n,
                           uint32_t* __restrict__ flag) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    bool d = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) d |= a[i] != b[i];
    if (__any(d) && (threadIdx.x & (kWave - 1)) == 0) atomicOr(flag, 1u);
}

// Plain 16-byte-vector copy: reads and writes every byte once (byte-counter calibration).
// Plain copy of n 16-byte vectors: four independent loads in flight per thread before their
// stores, streaming (nontemporal) hints.  It measures the device's copy bandwidth and
// calibrates the byte counters.
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));
__global__ void k_copy16(const v4u32* __restrict__ src, v4u32* __restrict__ dst, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const v4u32 a = __builtin_nontemporal_load(src + i);
        const v4u32 b = __builtin_nontemporal_load(src + i + stride);
        const v4u32 c = __builtin_nontemporal_load(src + i + 2 * stride);
        const v4u32 d = __builtin_nontemporal_load(src + i + 3 * stride);
        __builtin_nontemporal_store(a, dst + i);
        __builtin_nontemporal_store(b, dst + i + stride);
        __builtin_nontemporal_store(c, dst + i + 2 * stride);
        __builtin_nontemporal_store(d, dst + i + 3 * stride);
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

// ------------------------------------------------------------------------ accumulation


// LDS grid state of one unit: per cell sum(w f V') re/im, sum(w f) and the count.  The
// sums are FP64 (LDS has native FP64 atomic adds, far faster than its FP32 ones on
// gfx950), or, for the compensated mode, FP32 values with FP32 compensations.
template <int TU, int TV, int JC, int MODE, bool KAHAN>
struct AccumShape {
    static constexpr int JP = JC + 1;                 // padded channel stride
    static constexpr int NC = TU * TV * JP;           // LDS cells
    static constexpr size_t LDS = (size_t)NC * 28;
};

// Element i of a buffer-load result as float.  Elements are first copied to integers:
// bit-casting a vector element expression directly has been seen to read element 0.
template <class V>
__device__ __forceinline__ float fel(const V& v, int i) {
    const uint32_t x = (uint32_t)v[i];
    return __builtin_bit_cast(float, x);
}

// Raw buffer resource over [base, base + bytes): per-lane 32-bit offsets, uniform base in
// scalar registers, and reads past the end return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Wave-uniform description of one work item: up to 64 consecutive channels [k0, k1) of one
// row of one target.  Kept small: three of these live in scalar registers at once.
struct Item {
    int32_t ti;                    // target
    int32_t k0, k1;                // channels of this item
    int32_t r;                     // row within the target
    double U, V, trow;             // row u, v [m] and Eq. 2 turns per unit a_k
    float w[2];                    // row weights of the first two polarisations
};

__device__ __forceinline__ uint32_t ufl(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t ufl(uint64_t x) {
    return ((uint64_t)ufl((uint32_t)(x >> 32)) << 32) | ufl((uint32_t)x);
}
__device__ __forceinline__ double ufl(double x) { return __builtin_bit_cast(double, ufl(__builtin_bit_cast(uint64_t, x))); }
__device__ __forceinline__ float ufl(float x) { return __builtin_bit_cast(float, ufl(__builtin_bit_cast(uint32_t, x))); }

// The item with every field read from the first lane: the values are wave-uniform, so
// they stay in scalar registers and buffer resources built from them need no loops.
__device__ __forceinline__ Item uniform(const Item& a) {
    Item u;
    u.ti = (int32_t)ufl((uint32_t)a.ti);
    u.k0 = (int32_t)ufl((uint32_t)a.k0);
    u.k1 = (int32_t)ufl((uint32_t)a.k1);
    u.r = (int32_t)ufl((uint32_t)a.r);
    u.U = ufl(a.U); u.V = ufl(a.V); u.trow = ufl(a.trow);
    u.w[0] = ufl(a.w[0]); u.w[1] = ufl(a.w[1]);
    return u;
}

// Per-lane data of an item, loaded one item ahead of its use.
template <int NPOL>
struct LaneLoad {
    double a;
    uint32_t jn;
    float f0, f1;
    float vr[NPOL > 0 ? NPOL : 4], vi[NPOL > 0 ? NPOL : 4];
    uint32_t fl;
    float wc[NPOL > 0 ? 1 : 4];    // per-channel weights (generic path only)
};

template <int NPOL>
__device__ __forceinline__ void issue_loads(const VISTA_CONST DevTarget* tgts, const Item& itv, int lane,
                                            LaneLoad<NPOL>& ld) {
    const Item it = uniform(itv);
    const VISTA_CONST DevTarget& T = tgts[it.ti];
    const int npol = NPOL > 0 ? NPOL : T.npol;
    const uint32_t nch = ufl((uint32_t)T.nchan);
    const __amdgpu_buffer_rsrc_t ch = buf((const void*)ufl((uint64_t)T.chan), nch * (uint32_t)sizeof(DevChan));
    const __amdgpu_buffer_rsrc_t f1 = buf((const void*)ufl((uint64_t)T.f1), nch * 4u);
    // the row's visibilities, flags and per-channel weights
    const uint32_t rowe = nch * (uint32_t)npol;                   // samples per row
    const size_t re0 = (size_t)it.r * rowe;
    const __amdgpu_buffer_rsrc_t visr = buf((const char*)ufl((uint64_t)T.vis) + re0 * 8, rowe * 8u);
    const uint64_t fbase = ufl((uint64_t)T.flag);
    const __amdgpu_buffer_rsrc_t flagr = buf(fbase ? (const void*)((const char*)fbase + re0) : (const void*)T.vis,
                                             fbase ? rowe : 0u);
    const int has_flag = fbase != 0;
    const __amdgpu_buffer_rsrc_t wchr = buf((const char*)ufl((uint64_t)T.weight) + re0 * 4,
                                            T.weight_per_chan ? rowe * 4u : 0u);
    // whole offsets in the lane offset: the hardware range check covers exactly that part
    const int kl = it.k0 + lane;
    auto c = __builtin_amdgcn_raw_buffer_load_b128(ch, kl * 16, 0, 0);
    const uint32_t c0 = (uint32_t)c[0], c1 = (uint32_t)c[1], c2 = (uint32_t)c[2];
    ld.a = __builtin_bit_cast(double, ((uint64_t)c1 << 32) | c0);
    ld.jn = c2;
    ld.f0 = fel(c, 3);
    const uint32_t f1w = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(f1, kl * 4, 0, 0);
    ld.f1 = __builtin_bit_cast(float, f1w);
    if (NPOL == 0) {
        // polarisation slots beyond npol take part in the merge with weight 0: keep them 0
        for (int p = 0; p < 4; ++p) { ld.vr[p] = 0.f; ld.vi[p] = 0.f; }
    }
    if (npol == 2) {
        auto v = __builtin_amdgcn_raw_buffer_load_b128(visr, kl * 16, 0, 0);
        ld.vr[0] = fel(v, 0); ld.vi[0] = fel(v, 1);
        ld.vr[1] = fel(v, 2); ld.vi[1] = fel(v, 3);
        ld.fl = has_flag ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(flagr, kl * 2, 0, 0) : 0u;
    } else if (npol == 1) {
        auto v = __builtin_amdgcn_raw_buffer_load_b64(visr, kl * 8, 0, 0);
        ld.vr[0] = fel(v, 0); ld.vi[0] = fel(v, 1);
        ld.fl = has_flag ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b8(flagr, kl, 0, 0) : 0u;
    } else {
        auto v = __builtin_amdgcn_raw_buffer_load_b128(visr, kl * 32, 0, 0);
        auto u = __builtin_amdgcn_raw_buffer_load_b128(visr, kl * 32 + 16, 0, 0);
        ld.vr[0] = fel(v, 0); ld.vi[0] = fel(v, 1);
        ld.vr[1] = fel(v, 2); ld.vi[1] = fel(v, 3);
        if (NPOL != 2 && NPOL != 1) {
            ld.vr[2] = fel(u, 0); ld.vi[2] = fel(u, 1);
            ld.vr[3] = fel(u, 2); ld.vi[3] = fel(u, 3);
        }
        ld.fl = has_flag ? (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(flagr, kl * 4, 0, 0) : 0u;
    }
    if (NPOL == 0 && T.weight_per_chan) {
        for (int p = 0; p < 4; ++p)
            if (p < npol) {
                const uint32_t x = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(wchr, (kl * npol + p) * 4, 0, 0);
                ld.wc[p] = __builtin_bit_cast(float, x);
            } else {
                ld.wc[p] = 0.f;
            }
    }
}

// Accumulation of one (uv tile, rest-channel block) unit per workgroup iteration.
//   MODE == kModeAtomic : waves take the unit's records round-robin and add into the
//                         shared LDS cells with LDS float atomics.
//   MODE == kModeOrdered: every wave walks all records in order but only adds into its
//                         own slice of rest channels, so each cell has one writer; lanes
//                         that could share a cell add in separate phases.  The order of
//                         every addition is fixed: results are bit-identical from run to
//                         run, and KAHAN compensates each addition.
// NPOL == 2 is the path specialised for two polarisations and row weights; NPOL == 0
// handles any polarisation count and per-channel weights.
template <int TU, int TV, int JC, int MODE, bool KAHAN, int NPOL>
__global__ void __launch_bounds__(1024, 4) k_accum(const LaunchDesc* __restrict__ Lp,
                                                   const uint64_t* __restrict__ order,
                                                   uint32_t* __restrict__ counter,
                                                   const uint32_t* __restrict__ unit_off,
                                                   const uint64_t* __restrict__ recs) {
    using Sh = AccumShape<TU, TV, JC, MODE, KAHAN>;
    constexpr int JP = Sh::JP;
    constexpr int NC = Sh::NC;
    using Acc = typename std::conditional<KAHAN, float, double>::type;
    __shared__ Acc s_re[NC], s_im[NC], s_w[NC];
    __shared__ uint32_t s_n[NC];
    __shared__ float c_re[KAHAN ? NC : 1], c_im[KAHAN ? NC : 1], c_w[KAHAN ? NC : 1];
    __shared__ uint32_t s_unit;

    const LaunchDesc& L = *Lp;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = sgpr(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const VISTA_GLOBAL uint64_t* grecs = gptr(recs);
    const VISTA_CONST DevTarget* tgts = cptr(L.targets);
    const VISTA_CONST int64_t* trb = cptr(L.target_row_base);
    const int phase_fp32 = L.phase_fp32;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t li = (uint32_t)sgpr((int32_t)s_unit);
        if (li >= L.nunits) break;
        const int64_t unit = (uint32_t)sgpr((int32_t)(uint32_t)gptr(order)[li]);
        const int32_t si = sgpr((int32_t)find_le_uniform(L.stack_unit_base, L.nstacks, unit));
        const VISTA_CONST DevStack& S = cptr(L.stacks)[si];
        const int64_t local = unit - S.unit_base;
        const int64_t tile = local / S.nblocks;
        const int32_t b = (int32_t)(local - tile * S.nblocks);
        const int32_t tu0 = (int32_t)(tile % S.tiles_u) * TU;
        const int32_t tv0 = (int32_t)(tile / S.tiles_u) * TV;
        const int32_t jb0 = b * JC;
        const int32_t jb1 = min(jb0 + JC, S.nchan);
        const int32_t cu = S.nu / 2 - tu0, cv = S.nv / 2 - tv0;
        const double inv_du = S.inv_du, inv_dv = S.inv_dv;

        for (int i = threadIdx.x; i < NC; i += blockDim.x) {
            s_re[i] = 0; s_im[i] = 0; s_w[i] = 0; s_n[i] = 0u;
            if (KAHAN) { c_re[i] = 0.f; c_im[i] = 0.f; c_w[i] = 0.f; }
        }
        __syncthreads();

        const uint32_t rb = (uint32_t)sgpr((int32_t)gptr(unit_off)[unit]);
        const uint32_t re = (uint32_t)sgpr((int32_t)gptr(unit_off)[unit + 1]);
        int32_t js0, js1, sbi;
        uint32_t r_first, r_step;
        if (MODE == kModeOrdered) {
            const int32_t jsub = L.jsub;
            js0 = jb0 + wave * jsub;
            js1 = min(js0 + jsub, jb1);
            sbi = jb0 / jsub + wave;
            r_first = rb;
            r_step = 1;
        } else {
            js0 = jb0;
            js1 = jb1;
            sbi = b;
            r_first = rb + wave;
            r_step = nw;
        }
        uint32_t st_flag = 0, st_bad = 0, st_used = 0;
        unsigned long long st_contrib = 0;

        // ---- the wave's work items: its records, cut into 64-channel pieces.  Records
        // come 64 at a time, one per lane, together with their rows' context (target,
        // row, u, v, Eq. 2 turns per unit a_k, weights), so no record waits on memory.
        const uint32_t nrec_w = (js0 < js1 && re > r_first) ? (re - r_first + r_step - 1) / r_step : 0;
        uint32_t ri = 0;                  // next record of this wave
        uint64_t rec_l = 0;               // this lane's record of the current batch
        int32_t ti_l = 0, r_l = 0;
        double U_l = 0.0, V_l = 0.0, T_l = 0.0;
        float w0_l = 0.f, w1_l = 0.f;
        int32_t kc = 0, kend = 0;         // rest of the current record
        Item row;

        auto load_batch = [&]() __attribute__((always_inline)) {
            const uint32_t my = r_first + (ri + lane) * r_step;
            const bool valid = my < re;
            rec_l = valid ? grecs[my] : 0ull;
            const int64_t g = (int64_t)(rec_l >> 32);
            const VISTA_GLOBAL int64_t* rbase = gptr(L.target_row_base);
            int32_t lo = 0, hi = L.ntargets;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (rbase[mid] <= g) lo = mid; else hi = mid;
            }
            ti_l = lo;
            const VISTA_GLOBAL DevTarget* Tl = gptr(L.targets) + lo;
            const int64_t r = valid ? g - rbase[lo] : 0;
            r_l = (int32_t)r;
            if (valid) {
                const VISTA_GLOBAL double* uvw = gptr(Tl->uvw) + 3 * r;
                const double Um = uvw[0], Vm = uvw[1], Wm = uvw[2];
                if (Tl->rotate) {                    // uv cells: Eq. 1's rotated baseline
                    U_l = Tl->rot[0] * Um + Tl->rot[1] * Vm + Tl->rot[2] * Wm;
                    V_l = Tl->rot[3] * Um + Tl->rot[4] * Vm + Tl->rot[5] * Wm;
                } else {
                    U_l = Um;
                    V_l = Vm;
                }
                // Eq. 2 turns per unit a_k from the original baseline (formed in FP32 under
                // the ablation)
                T_l = phase_fp32 ? (double)((float)Um * (float)Tl->l + (float)Vm * (float)Tl->m +
                                            (float)Wm * (float)Tl->nm1)
                                 : Um * Tl->l + Vm * Tl->m + Wm * Tl->nm1;
                const int np = Tl->npol;
                const VISTA_GLOBAL float* wp = gptr(Tl->weight) + (size_t)r * np;
                const bool rw = !Tl->weight_per_chan;
                w0_l = rw ? wp[0] : 0.f;
                w1_l = (rw && np > 1) ? wp[1] : 0.f;
            }
        };

        // advance to the next item; false when the wave has no more work
        auto next_item = [&](Item& nx) __attribute__((always_inline)) -> bool {
            while (kc >= kend) {
                if (ri >= nrec_w) return false;
                const int jl = (int)(ri & (kWave - 1));
                if (jl == 0) load_batch();
                ++ri;
                const uint64_t rec = readlane_u64(rec_l, jl);
                int32_t kin = (int32_t)((rec >> 16) & 0xffff), kout = (int32_t)(rec & 0xffff);
                const int32_t ti = __builtin_amdgcn_readlane(ti_l, jl);
                if (MODE == kModeOrdered) {
                    const VISTA_CONST DevTarget& T = tgts[ti];
                    kin = max(kin, cptr(T.sblk)[2 * sbi]);
                    kout = min(kout, cptr(T.sblk)[2 * sbi + 1]);
                }
                if (kin >= kout) continue;
                kc = kin;
                kend = kout;
                row.ti = ti;
                row.r = __builtin_amdgcn_readlane(r_l, jl);
                row.U = __builtin_bit_cast(double, readlane_u64(__builtin_bit_cast(uint64_t, U_l), jl));
                row.V = __builtin_bit_cast(double, readlane_u64(__builtin_bit_cast(uint64_t, V_l), jl));
                row.trow = __builtin_bit_cast(double, readlane_u64(__builtin_bit_cast(uint64_t, T_l), jl));
                row.w[0] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, w0_l), jl));
                row.w[1] = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, w1_l), jl));
            }
            nx = row;
            nx.k0 = kc;
            nx.k1 = min(kc + kWave, kend);
            kc += kWave;
            return true;
        };

        // ---- one item: cell, polarisation merge, rotation, rest-channel split
        auto process = [&](const Item& itv, const LaneLoad<NPOL>& ld) __attribute__((always_inline)) {
            const Item it = uniform(itv);
            const VISTA_CONST DevTarget& T = tgts[it.ti];
            const int npol = NPOL > 0 ? NPOL : T.npol;
            const uint32_t nj = ld.jn >> 24;
            const int32_t j0 = (int32_t)(ld.jn & kJMask);
            const bool act = (it.k0 + lane < it.k1) && nj > 0;     // idle lanes add nothing
            // cell within the tile (exact FP64 sequence of the definition)
            const double ru = cell_coord(it.U, ld.a, inv_du);
            const double rv = cell_coord(it.V, ld.a, inv_dv);
            const int32_t lu = (int32_t)ru + cu, lv = (int32_t)rv + cv;
            const bool in_tile = act && (uint32_t)lu < (uint32_t)TU && (uint32_t)lv < (uint32_t)TV;
            // polarisations: drop flagged and bad-weight samples, merge the rest
            float ar = 0.f, ai = 0.f, q = 0.f;
            uint32_t n = 0, nflag = 0, nbad = 0;
#pragma unroll
            for (int p = 0; p < (NPOL > 0 ? NPOL : 4); ++p) {
                const bool live = p < npol;
                float w;
                if (NPOL == 0 && T.weight_per_chan) w = ld.wc[NPOL > 0 ? 0 : p];
                else if (p < 2) w = it.w[p];
                else w = live ? cptr(T.weight)[(size_t)it.r * npol + (p < npol ? p : 0)] : 0.f;
                const bool flagged = live && ((ld.fl >> (8 * p)) & 0xffu) != 0u;
                const bool good = live && (w > 0.0f) && (w < __builtin_inff());
                nflag += flagged ? 1u : 0u;
                nbad += (live && !flagged && !good) ? 1u : 0u;
                const bool use = !flagged && good;
                const float wu = use ? w : 0.0f;
                n += use ? 1u : 0u;
                ar = fmaf(wu, ld.vr[p], ar);
                ai = fmaf(wu, ld.vi[p], ai);
                q += wu;
            }
            float c, s;
            if (phase_fp32) {
                const float t = (float)it.trow * (float)ld.a;
                sincos_turns(t - rintf(t), &s, &c);
            } else {
                phasor(it.trow, ld.a, &c, &s);
            }
            const float pr = ar * c - ai * s;
            const float pi = fmaf(ar, s, ai * c);
            // classification is counted once, in the block holding j0
            if (in_tile && j0 >= js0 && j0 < js1) {
                st_flag += nflag;
                st_bad += nbad;
                st_used += n;
            }
            const bool add = in_tile && n > 0;
            const int cell = (lv * TU + lu) * JP - jb0;
            const int nph = (MODE == kModeOrdered) ? T.nphase : 1;
            for (int ph = 0; ph < nph; ++ph) {
                const bool mine = add && (MODE != kModeOrdered || (lane % nph) == ph);
#pragma unroll
                for (int qq = 0; qq < 2; ++qq) {
                    const int32_t j = j0 + qq;
                    if (!(mine && qq < (int)nj && j >= js0 && j < js1)) continue;
                    const float f = qq == 0 ? ld.f0 : ld.f1;
                    const int cc = cell + j;
                    const float xr = f * pr, xi = f * pi, xw = f * q;
                    st_contrib += n;
                    if (MODE == kModeAtomic) {
                        atomicAdd(&s_re[cc], (double)f * (double)pr);   // exact products
                        atomicAdd(&s_im[cc], (double)f * (double)pi);
                        atomicAdd(&s_w[cc], (double)f * (double)q);
                        atomicAdd(&s_n[cc], n);
                    } else if (!KAHAN) {
                        s_re[cc] += (double)f * (double)pr;
                        s_im[cc] += (double)f * (double)pi;
                        s_w[cc] += (double)f * (double)q;
                        s_n[cc] += n;
                    } else {
                        float y, t;
                        y = xr - c_re[cc]; t = s_re[cc] + y; c_re[cc] = (t - s_re[cc]) - y; s_re[cc] = t;
                        y = xi - c_im[cc]; t = s_im[cc] + y; c_im[cc] = (t - s_im[cc]) - y; s_im[cc] = t;
                        y = xw - c_w[cc]; t = s_w[cc] + y; c_w[cc] = (t - s_w[cc]) - y; s_w[cc] = t;
                        s_n[cc] += n;
                    }
                }
                // more than two rest channels (rest grid finer than the channel): rare
                if (mine && nj > 2) {
                    const int32_t fo = gptr(T.foff)[it.k0 + lane];
                    for (int qq = 2; qq < (int)nj; ++qq) {
                        const int32_t j = j0 + qq;
                        if (j < js0 || j >= js1) continue;
                        const float f = gptr(T.fval)[fo + qq];
                        const int cc = cell + j;
                        const float xr = f * pr, xi = f * pi, xw = f * q;
                        st_contrib += n;
                        if (MODE == kModeAtomic) {
                            atomicAdd(&s_re[cc], (double)f * (double)pr);
                            atomicAdd(&s_im[cc], (double)f * (double)pi);
                            atomicAdd(&s_w[cc], (double)f * (double)q);
                            atomicAdd(&s_n[cc], n);
                        } else if (!KAHAN) {
                            s_re[cc] += (double)f * (double)pr;
                            s_im[cc] += (double)f * (double)pi;
                            s_w[cc] += (double)f * (double)q;
                            s_n[cc] += n;
                        } else {
                            float y, t;
                            y = xr - c_re[cc]; t = s_re[cc] + y; c_re[cc] = (t - s_re[cc]) - y; s_re[cc] = t;
                            y = xi - c_im[cc]; t = s_im[cc] + y; c_im[cc] = (t - s_im[cc]) - y; s_im[cc] = t;
                            y = xw - c_w[cc]; t = s_w[cc] + y; c_w[cc] = (t - s_w[cc]) - y; s_w[cc] = t;
                            s_n[cc] += n;
                        }
                    }
                }
            }
        };

        // ---- items processed with the loads of the next item already in flight
        Item it0, it1;
        LaneLoad<NPOL> ld0, ld1;
        bool have0 = next_item(it0);
        if (have0) issue_loads<NPOL>(tgts, it0, lane, ld0);
        while (have0) {
            const bool have1 = next_item(it1);
            if (have1) issue_loads<NPOL>(tgts, it1, lane, ld1);
            process(it0, ld0);
            if (!have1) break;
            have0 = next_item(it0);
            if (have0) issue_loads<NPOL>(tgts, it0, lane, ld0);
            process(it1, ld1);
        }

        // classification and contribution counts: one atomic per wave and unit
        unsigned long long t_flag = wave_sum_u64(st_flag);
        unsigned long long t_bad = wave_sum_u64(st_bad);
        unsigned long long t_used = wave_sum_u64(st_used);
        unsigned long long t_contrib = wave_sum_u64(st_contrib);
        if (lane == 0) {
            if (t_flag) atomicAdd(&S.stats[1], t_flag);
            if (t_bad) atomicAdd(&S.stats[2], t_bad);
            if (t_used) atomicAdd(&S.stats[5], t_used);
            if (t_contrib) atomicAdd(&S.stats[6], t_contrib);
            if (t_contrib > 0xffffffffull) atomicOr(&S.stats[7], 1ull);
        }
        __syncthreads();

        flush_unit<TU, TV, JP, Acc, KAHAN>(L, S, tu0, tv0, jb0, jb1, s_re, s_im, s_w, s_n, c_re, c_im, c_w);
        __syncthreads();
    }
}

// --------------------------------------------------------------------------- debug

__global__ void k_debug_indices(const DevTarget* __restrict__ Tp, const DevStack* __restrict__ Sp,
                                int32_t* iu, int32_t* iv, int32_t* j0, int32_t* nj, int64_t nrow,
                                int32_t nchan) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrow * nchan) return;
    const DevTarget& T = *Tp;
    const DevStack& S = *Sp;
    int64_t r = e / nchan;
    int32_t k = (int32_t)(e % nchan);
    DevChan ce = T.chan[k];
    double U, V;
    cell_uv(T, T.uvw[3 * r], T.uvw[3 * r + 1], T.uvw[3 * r + 2], &U, &V);
    double ru = cell_coord(U, ce.a, S.inv_du);
    double rv = cell_coord(V, ce.a, S.inv_dv);
    iu[e] = fabs(ru) < 2.0e9 ? (int32_t)ru + S.nu / 2 : INT32_MIN;
    iv[e] = fabs(rv) < 2.0e9 ? (int32_t)rv + S.nv / 2 : INT32_MIN;
    int32_t n = (int32_t)(ce.jn >> 24);
    j0[e] = n ? (int32_t)(ce.jn & kJMask) : -1;
    nj[e] = n;
}

__global__ void k_debug_rotate(const DevTarget* __restrict__ Tp, float2* out, int64_t nrow, int32_t nchan,
                               int32_t npol, int phase_fp32) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nrow * nchan) return;
    const DevTarget& T = *Tp;
    int64_t r = e / nchan;
    int32_t k = (int32_t)(e % nchan);
    double U = T.uvw[3 * r], V = T.uvw[3 * r + 1], Wm = T.uvw[3 * r + 2];
    double a = T.chan[k].a;
    float c, s;
    if (phase_fp32) {
        float a32 = (float)a;
        phasor_fp32((float)U * a32, (float)V * a32, (float)Wm * a32, (float)T.l, (float)T.m, (float)T.nm1,
                    &c, &s);
    } else {
        phasor(U * T.l + V * T.m + Wm * T.nm1, a, &c, &s);
    }
    for (int p = 0; p < npol; ++p) {
        float2 v = T.vis[e * npol + p];
        out[e * npol + p] = make_float2(v.x * c - v.y * s, fmaf(v.x, s, v.y * c));
    }
}

}  // namespace

// ---------------------------------------------------------------------------- launchers

hipError_t launch_track(int64_t rows_cap, const LaunchDesc* dL, uint32_t* seg_count, const uint32_t* seg_off,
                        uint32_t* keys, uint64_t* vals, int emit, hipStream_t stream) {
    if (rows_cap <= 0) return hipSuccess;
    int64_t blocks = (rows_cap + kTrackThreads - 1) / kTrackThreads;
    if (emit)
        hipLaunchKernelGGL(k_track<true>, dim3((unsigned)blocks), dim3(kTrackThreads), 0, stream, dL, seg_count,
                           seg_off, keys, vals);
    else
        hipLaunchKernelGGL(k_track<false>, dim3((unsigned)blocks), dim3(kTrackThreads), 0, stream, dL, seg_count,
                           seg_off, keys, vals);
    return hipGetLastError();
}

hipError_t launch_unit_offsets(const uint32_t* sorted_keys, const int64_t* nrec_dev, int64_t nrec_cap,
                               const int64_t* nunits_dev, uint32_t* unit_off, hipStream_t stream) {
    int64_t n = (nrec_cap + 1 + 3) / 4;     // threads: four record positions each
    hipLaunchKernelGGL(k_unit_offsets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sorted_keys,
                       nrec_dev, nrec_cap, nunits_dev, unit_off);
    return hipGetLastError();
}

hipError_t launch_copy16(void* dst, const void* src, int64_t n16, hipStream_t stream) {
    if (n16 <= 0) return hipSuccess;
    int64_t blocks = std::min<int64_t>((n16 + 255) / 256, 256 * 256);
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, stream, (const v4u32*)src, (v4u32*)dst, n16);
    return hipGetLastError();
}

hipError_t launch_diff_u32(const uint32_t* a, const uint32_t* b, int64_t n, uint32_t* flag, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 16);
    hipLaunchKernelGGL(k_diff_u32, dim3((unsigned)blocks), dim3(256), 0, stream, a, b, n, flag);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

// Supported shapes (tile_u, tile_v, jblock).  The autotuner chooses among these.
#define VISTA_SHAPES(X) \
    X(8, 8, 64)          \
    X(16, 4, 64)         \
    X(16, 8, 32)         \
    X(8, 4, 128)         \
    X(16, 2, 128)        \
    X(4, 4, 256)         \
    X(8, 2, 256)         \
    X(4, 2, 512)

template <int TU, int TV, int JC, int MODE, bool KAHAN, int NPOL>
static hipError_t launch_one(const LaunchDesc* dL, const uint64_t* order, uint32_t* counter,
                             const uint32_t* unit_off, const uint64_t* recs, int grid, int waves,
                             hipStream_t stream) {
    hipLaunchKernelGGL((k_accum<TU, TV, JC, MODE, KAHAN, NPOL>), dim3(grid), dim3(waves * kWave), 0, stream, dL,
                       order, counter, unit_off, recs);
    return hipGetLastError();
}

template <int TU, int TV, int JC, int MODE, bool KAHAN, int NPOL>
static int occ_one(int waves) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_accum<TU, TV, JC, MODE, KAHAN, NPOL>, waves * kWave,
                                                     0) != hipSuccess)
        return 0;
    return nb;
}

int accum_shape_list(int mode, int* tu, int* tv, int* jc, int cap) {
    if (mode == kModeAtomic) return accum_packed_shape_list(0, tu, tv, jc, cap);
    int n = 0;
#define X(a, b, c)            \
    if (n < cap) {            \
        tu[n] = a; tv[n] = b; jc[n] = c; \
    }                         \
    ++n;
    VISTA_SHAPES(X)
#undef X
    return n;
}

size_t accum_lds_bytes(int tu, int tv, int jc, int mode, int kahan) {
    return (size_t)tu * tv * (jc + 1) * 28;
}

bool accum_shape_supported(int tu, int tv, int jc, int waves, int mode, int kahan) {
    if (waves < 1 || waves > 16) return false;
    if (kahan && mode != kModeOrdered) return false;
    if (mode == kModeOrdered && (jc % waves) != 0) return false;
#define X(a, b, c) if (tu == a && tv == b && jc == c) return accum_lds_bytes(a, b, c, mode, kahan) <= 160 * 1024;
    VISTA_SHAPES(X)
#undef X
    return false;
}

// npol: 2 for launches whose targets all have two polarisations (the specialised path),
// anything else selects the generic path.
// (The atomic mode runs the packed kernel; callers pass ordered launches only.)
#define VISTA_DISPATCH(a, b, c, CALL)                                                    \
    if (L.tu == a && L.tv == b && L.jc == c) {                                           \
        if (L.kahan) {                                                                   \
            if (npol == 2) return CALL(a, b, c, kModeOrdered, true, 2);                  \
            return CALL(a, b, c, kModeOrdered, true, 0);                                 \
        }                                                                                \
        if (npol == 2) return CALL(a, b, c, kModeOrdered, false, 2);                     \
        return CALL(a, b, c, kModeOrdered, false, 0);                                    \
    }

hipError_t launch_accum_impl(const LaunchDesc& L, const LaunchDesc* dL, const uint64_t* order,
                             uint32_t* counter, const uint32_t* unit_off, const uint64_t* recs, int grid,
                             int waves, int npol, hipStream_t stream) {
    if (L.mode != kModeOrdered || !accum_shape_supported(L.tu, L.tv, L.jc, waves, L.mode, L.kahan))
        return hipErrorInvalidValue;
#define CALL(a, b, c, m, k, p) launch_one<a, b, c, m, k, p>(dL, order, counter, unit_off, recs, grid, waves, stream)
#define X(a, b, c) VISTA_DISPATCH(a, b, c, CALL)
    VISTA_SHAPES(X)
#undef X
#undef CALL
    return hipErrorInvalidValue;
}

int accum_max_blocks_per_cu(int tu, int tv, int jc, int waves, int mode, int kahan, int npol) {
    if (mode != kModeOrdered || !accum_shape_supported(tu, tv, jc, waves, mode, kahan)) return 0;
    LaunchDesc L;
    L.tu = tu; L.tv = tv; L.jc = jc; L.mode = mode; L.kahan = kahan;
#define CALL(a, b, c, m, k, p) occ_one<a, b, c, m, k, p>(waves)
#define X(a, b, c) VISTA_DISPATCH(a, b, c, CALL)
    VISTA_SHAPES(X)
#undef X
#undef CALL
    return 0;
}

hipError_t launch_debug_indices(const DevTarget* t, const DevStack* s, int32_t* iu, int32_t* iv, int32_t* j0,
                                int32_t* nj, int64_t nrow, int32_t nchan, hipStream_t stream) {
    int64_t n = nrow * nchan;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_indices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, t, s, iu, iv,
                       j0, nj, nrow, nchan);
    return hipGetLastError();
}

hipError_t launch_debug_rotate(const DevTarget* t, float2* out, int64_t nrow, int32_t nchan, int32_t npol,
                               int phase_fp32, hipStream_t stream) {
    int64_t n = nrow * nchan;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_debug_rotate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, t, out, nrow,
                       nchan, npol, phase_fp32);
    return hipGetLastError();
}

}  // namespace vista
