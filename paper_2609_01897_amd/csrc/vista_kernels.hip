// gfx950 kernels of the ViSta stacking hot path.
//
//   track (count / emit) -- binning: each row's channels, walked in frequency order,
//       trace a radial line in uv (u_lambda = u_m nu/c); the cells along it are monotone,
//       so the channels that fall in one uv tile form one contiguous run.  Each run is
//       cut at the rest-channel block boundaries; every piece becomes one record keyed by
//       its (tile, block) unit.
//   sort (vista_sort.hip) / unit offsets -- stable grouping of the records by unit.
//   The accumulation kernels, which own one (uv tile, rest-channel block) unit of the grid
//   state at a time, are in vista_accum.hip.
//
// Cell and channel indices follow the FP64 operation sequence of the definition exactly
// (this file is compiled with -ffp-contract=off, no fast-math): u = u_m * a_k,
// iu = rint(u * (1/du)) + nu/2.
#include <hip/hip_runtime.h>

#include <algorithm>

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
        if (!EMIT && L.row_target) L.row_target[g] = ti;
        if (!EMIT && L.rowctx) {
            // the row's context for the accumulation
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

// unit_off[u] = index of the first record of unit u, for u = 0 .. nunits (records sorted by
// unit, so unit_off[nunits] = nrec): one lower-bound search of the sorted keys per unit.
// Neighbouring units share the search's upper levels in cache, and a run of empty units
// costs no more than occupied ones (a pass over the records that filled the gaps between
// keys gave a whole run of empty units to one thread).  nunits <= units_cap.
__global__ void k_unit_offsets(const uint32_t* __restrict__ keys, const int64_t* __restrict__ nrec_dev,
                               int64_t nrec_cap, const int64_t* __restrict__ nunits_dev,
                               uint32_t* __restrict__ off) {
    const int64_t nunits = *nunits_dev;
    const int64_t nrec = nrec_dev ? *nrec_dev : nrec_cap;
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u > nunits) return;
    int64_t lo = 0, hi = nrec;
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)keys[mid] < u) lo = mid + 1;
        else hi = mid;
    }
    off[u] = (uint32_t)lo;
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
                               const int64_t* nunits_dev, int64_t units_cap, uint32_t* unit_off,
                               hipStream_t stream) {
    const int64_t n = units_cap + 1;        // threads: one per unit offset
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
