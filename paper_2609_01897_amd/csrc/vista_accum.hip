// The accumulation kernels (Eq. 2 rotation, Eq. 3-4 rest-frame rebinning): the packed
// kernel of the atomic mode, and below it the ordered kernel of the deterministic form.
//
// The binning pass leaves the records of every (uv tile, rest-channel block) unit
// contiguous; a record is a run [k_lo, k_hi) of channels of one row.  Concatenated, the
// unit's records form one stream of (row, channel) samples, and pre[] gives each record's
// start in it.  A workgroup owns one unit at a time: its cells live in LDS (three sums and a
// u32 count per cell), so every cell of the grid is written exactly once, from one place.
// The sums are FP64 (28 B of LDS per cell), or, in the plain FP32 form, FP32 (16 B per
// cell, so units hold 1.75 times as many cells); both are native LDS atomic adds.
// The unit's stream is split into equal sample ranges, one per wavefront, and a wavefront
// walks its range in chunks of 128 consecutive samples, two adjacent ones per lane (records
// are padded to whole pairs), whatever records they come from: no lane idles at record
// ends.  Each lane finds its record in a window of 64
// records held one per lane (the starts falling inside the chunk are few and are tested
// one by one), takes the record's context from that lane with ds_bpermute, and loads its
// own channel-table entry, visibilities and flags.  The loads of the next chunk are in
// flight while the current one is processed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "vista_device.h"

namespace vista {

namespace {

__device__ __forceinline__ uint32_t bperm(uint32_t v, int src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute(src << 2, (int)v);
}
__device__ __forceinline__ uint64_t bperm64(uint64_t v, int src) {
    return ((uint64_t)bperm((uint32_t)(v >> 32), src) << 32) | bperm((uint32_t)v, src);
}
__device__ __forceinline__ double bpermd(double v, int src) {
    return __builtin_bit_cast(double, bperm64(__builtin_bit_cast(uint64_t, v), src));
}
__device__ __forceinline__ float bpermf(float v, int src) {
    return __builtin_bit_cast(float, bperm(__builtin_bit_cast(uint32_t, v), src));
}
__device__ __forceinline__ uint64_t ufl64(uint64_t x) {
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
}

// A record's context with its addresses rebased to the window's stream positions: the
// sample at position p (relative to the window origin) of the record has its visibilities
// at vis + p * (npol * 8), its flags at flag + p * npol, its channel-table entry at index
// chan + p and (per-channel weights) its weights at wadj + p * wstride; positions from
// `end` on are the record's padding.
template <int NPOL>
struct RecCtx {
    double U, V, T;
    float w0, w1;              // NPOL == 2: the row weights
    uint64_t vis, flag;
    uint64_t wadj;             // NPOL == 0: weight base
    uint32_t info;             // NPOL == 0: npol | wstride << 8 (wstride 0: row weights)
    int32_t chan;
    uint32_t end;
};

// What one sample loaded.
template <int NPOL>
struct Loaded {
    double a;                  // nu_k / c
    uint32_t jn;               // j0 | nj << 24 (nj = 0: nothing to add)
    float f0, f1;              // overlap fractions of j0 and j0 + 1
    float vr[NPOL == 2 ? 2 : 4], vi[NPOL == 2 ? 2 : 4];
    uint32_t fl;               // flag bytes, polarisation p in byte p
    float wc[NPOL == 2 ? 1 : 4];
};

// One lane's pair of samples of a chunk: positions pos and pos + 1 of one record.  Only the
// record's window lane is carried while the loads are in flight; the record's coordinates
// and weights are gathered again when the pair is processed.
template <int NPOL>
struct Pair {
    int rec;                   // window lane of the record
    uint32_t pos;              // stream position relative to the window origin
    bool act;                  // the first sample is inside the wavefront's range
    bool two;                  // so is the second (not the padding of an odd record)
    Loaded<NPOL> s[2];
};

template <class T>
__device__ __forceinline__ T gload(uint64_t addr) {
    return *(const VISTA_GLOBAL T*)addr;
}

// Loads of one sample.  Nothing here looks at the loaded values: the loads of the next
// chunk stay in flight while the current one is processed.
// Addresses of a record's samples (see RecCtx), gathered for issuing a chunk's loads.
template <int NPOL>
struct Bases {
    uint64_t vis, flag, wadj;
    uint32_t info;
    int32_t chan;
};

template <int NPOL>
__device__ __forceinline__ void load_sample(const VISTA_GLOBAL DevChan* chan_all, const VISTA_GLOBAL float* f1_all,
                                            const Bases<NPOL>& c, uint32_t p, Loaded<NPOL>& x) {
    const int32_t ci = c.chan + (int32_t)p;
    const uint4 ch = *(const VISTA_GLOBAL uint4*)(chan_all + ci);
    x.a = __builtin_bit_cast(double, ((uint64_t)ch.y << 32) | ch.x);
    x.jn = ch.z;
    x.f0 = __builtin_bit_cast(float, ch.w);
    x.f1 = f1_all[ci];
    if constexpr (NPOL == 2) {
        const float4 v = gload<float4>(c.vis + (uint64_t)p * 16u);
        x.vr[0] = v.x; x.vi[0] = v.y; x.vr[1] = v.z; x.vi[1] = v.w;
        x.fl = gload<uint16_t>(c.flag + (uint64_t)p * 2u);
    } else {
        const uint32_t np = c.info & 0xffu, ws = c.info >> 8;
        for (int q = 0; q < 4; ++q) { x.vr[q] = 0.f; x.vi[q] = 0.f; x.wc[q] = 0.f; }
        if (np == 1) {
            const float2 v = gload<float2>(c.vis + (uint64_t)p * 8u);
            x.vr[0] = v.x; x.vi[0] = v.y;
            x.fl = gload<uint8_t>(c.flag + p);
        } else if (np == 2) {
            const float4 v = gload<float4>(c.vis + (uint64_t)p * 16u);
            x.vr[0] = v.x; x.vi[0] = v.y; x.vr[1] = v.z; x.vi[1] = v.w;
            x.fl = gload<uint16_t>(c.flag + (uint64_t)p * 2u);
        } else {
            const float4 v = gload<float4>(c.vis + (uint64_t)p * 32u);
            const float4 u = gload<float4>(c.vis + (uint64_t)p * 32u + 16u);
            x.vr[0] = v.x; x.vi[0] = v.y; x.vr[1] = v.z; x.vi[1] = v.w;
            x.vr[2] = u.x; x.vi[2] = u.y; x.vr[3] = u.z; x.vi[3] = u.w;
            x.fl = gload<uint32_t>(c.flag + (uint64_t)p * 4u);
        }
        const uint64_t wb = c.wadj + (uint64_t)p * ws;
        for (int q = 0; q < 4; ++q)
            if (q < (int)np) x.wc[q] = gload<float>(wb + 4u * q);
    }
}

// Mark every loaded value of a sample as used, at one point, before any branch: a load
// whose result some path never reads stays "pending" for the compiler, which then waits
// for all loads in flight before that register is next written.
template <int NPOL>
__device__ __forceinline__ void settle(const Loaded<NPOL>& x) {
    __asm__ volatile("" ::"v"(x.a), "v"(x.jn), "v"(x.f0), "v"(x.f1), "v"(x.fl));
#pragma unroll
    for (int q = 0; q < (NPOL == 2 ? 2 : 4); ++q) __asm__ volatile("" ::"v"(x.vr[q]), "v"(x.vi[q]));
    if constexpr (NPOL != 2) {
#pragma unroll
        for (int q = 0; q < 4; ++q) __asm__ volatile("" ::"v"(x.wc[q]));
    }
}

template <int NPOL>
__device__ __forceinline__ Bases<NPOL> gather_bases(const RecCtx<NPOL>& w, int src) {
    Bases<NPOL> c;
    c.vis = bperm64(w.vis, src);
    c.flag = bperm64(w.flag, src);
    c.chan = (int32_t)bperm((uint32_t)w.chan, src);
    if (NPOL != 2) {
        c.wadj = bperm64(w.wadj, src);
        c.info = bperm(w.info, src);
    }
    return c;
}

// Both samples of a lane's pair.  Every lane loads from inside its record: a lane past the
// wavefront's range reads the record's last sample, the padding of an odd record re-reads
// the first; process() ignores what they read.  Nothing here looks at loaded values.
template <int NPOL>
__device__ __forceinline__ void issue(const VISTA_GLOBAL DevChan* chan_all, const VISTA_GLOBAL float* f1_all,
                                      const RecCtx<NPOL>& w, Pair<NPOL>& x) {
    const Bases<NPOL> c = gather_bases<NPOL>(w, x.rec);
    const uint32_t end = bperm(w.end, x.rec);
    x.two = x.act && x.pos + 1u < end;
    const uint32_t p0 = x.act ? x.pos : end - 1u;
    const uint32_t p1 = x.two ? x.pos + 1u : p0;
    load_sample<NPOL>(chan_all, f1_all, c, p0, x.s[0]);
    load_sample<NPOL>(chan_all, f1_all, c, p1, x.s[1]);
}

// One slot of contributions from every lane of the wavefront (all lanes call it together):
// lane adds (re, im, w, n) to LDS cell `key` (key < 0: nothing).  Lanes hold consecutive
// stream positions, so lanes adding to one cell form contiguous runs -- long ones where many
// input channels fall in one rest channel and one uv cell (fine channels, short baselines),
// and there the cell's LDS address would take one atomic per lane, one after another.  When
// the runs are 4 lanes long or more on average, each run is first summed across its lanes
// (a segmented inclusive scan, the run's last lane ends with its total) and only that lane
// adds to LDS; otherwise every lane adds its own values.  Sums are in Acc either way.
//
// The scan moves values between lanes with DPP (a VALU operand modifier), not through LDS:
// dppu/dppd/dppf give each lane the value of the lane that DPP control CTRL selects, in the
// rows of 16 lanes that ROWS enables, and 0 where there is no such lane (or the row is off).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dppu(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dppd(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint64_t r = ((uint64_t)dppu<CTRL, ROWS>((uint32_t)(b >> 32)) << 32) | dppu<CTRL, ROWS>((uint32_t)b);
    return __builtin_bit_cast(double, r);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dppf(float v) {
    return __builtin_bit_cast(float, dppu<CTRL, ROWS>(__builtin_bit_cast(uint32_t, v)));
}
// One scan step: the source lane's partial sums, added where `take` (the source is in the run).
template <int CTRL, int ROWS, class Acc>
__device__ __forceinline__ void scan_dpp(Acc& re, Acc& im, Acc& w, uint32_t& n, bool take) {
    Acc r2, i2, w2;
    if constexpr (sizeof(Acc) == 8) {
        r2 = dppd<CTRL, ROWS>(re); i2 = dppd<CTRL, ROWS>(im); w2 = dppd<CTRL, ROWS>(w);
    } else {
        r2 = dppf<CTRL, ROWS>(re); i2 = dppf<CTRL, ROWS>(im); w2 = dppf<CTRL, ROWS>(w);
    }
    const uint32_t n2 = dppu<CTRL, ROWS>(n);
    if (take) {
        re += r2;
        im += i2;
        w += w2;
        n += n2;
    }
}

template <class Acc>
__device__ __forceinline__ void emit(Acc* s_re, Acc* s_im, Acc* s_w, uint32_t* s_n, int lane, int key, Acc re,
                                     Acc im, Acc w, uint32_t n) {
    const uint64_t act = __ballot(key >= 0);
    if (act == 0) return;
    const int prev = __shfl_up(key, 1, kWave);
    const bool head = key >= 0 && (lane == 0 || prev != key);
    const uint64_t heads = __ballot(head);
    if (__popcll(heads) * 4 <= __popcll(act)) {
        // the lane's run starts at the last head at or below it (an inactive lane ends a run,
        // the next active lane heads one); span = lanes of its run below it
        const uint64_t upto = heads & ((2ull << lane) - 1ull);      // lane 63: every bit
        const int start = upto ? 63 - (int)__clzll(upto) : lane;
        const int span = key >= 0 ? lane - start : -1;
        const int c16 = lane & 15;
        // segmented inclusive scan: within each row of 16 lanes, shifts of 1, 2, 4 and 8 lanes
        // (row_shr; a source before the row start reads 0), so that a lane holds its run's sum
        // from max(run start, row start); then across rows, lane 15 to row 1 and lane 47 to
        // row 3 (row_bcast:15), where the lane's run began before its row; then lane 31 (now
        // complete) to rows 2 and 3 (row_bcast:31), where the run began at lane 31 or before
        scan_dpp<0x111, 0xf>(re, im, w, n, span >= 1);
        scan_dpp<0x112, 0xf>(re, im, w, n, span >= 2);
        scan_dpp<0x114, 0xf>(re, im, w, n, span >= 4);
        scan_dpp<0x118, 0xf>(re, im, w, n, span >= 8);
        scan_dpp<0x142, 0xa>(re, im, w, n, span >= c16 + 1);
        scan_dpp<0x143, 0xc>(re, im, w, n, span >= lane - 31);
        // the run's last lane holds its total
        const uint64_t ends = heads | ~act;
        if (key >= 0 && (lane == kWave - 1 || ((ends >> (lane + 1)) & 1ull))) {
            atomicAdd(&s_re[key], re);
            atomicAdd(&s_im[key], im);
            atomicAdd(&s_w[key], w);
            atomicAdd(&s_n[key], n);
        }
    } else if (key >= 0) {
        atomicAdd(&s_re[key], re);
        atomicAdd(&s_im[key], im);
        atomicAdd(&s_w[key], w);
        atomicAdd(&s_n[key], n);
    }
}

// Per-wavefront classification and contribution counts, kept over many units and added to
// the stack's statistics when the stack changes, every 64 units, after a unit of more than
// 2^26 sample pairs, and at the end.  Each lane counts its own samples' live, flagged and
// used polarisations (bad ones are the rest); the wave sums them only when it flushes.
struct WaveStats {
    uint32_t live = 0, flag = 0, used = 0;    // per lane
    uint64_t contrib = 0;                     // wave-uniform
    int32_t stack = -1;
    uint32_t units = 0;
    __device__ void flush(const LaunchDesc& L, int lane) {
        const uint64_t tl = wave_sum_u64(live), tf = wave_sum_u64(flag), tu = wave_sum_u64(used);
        if (lane == 0 && stack >= 0) {
            unsigned long long* st = cptr(L.stacks)[stack].stats;
            const uint64_t tb = tl - tf - tu;
            if (tf) atomicAdd(&st[1], (unsigned long long)tf);
            if (tb) atomicAdd(&st[2], (unsigned long long)tb);
            if (tu) atomicAdd(&st[5], (unsigned long long)tu);
            if (contrib) atomicAdd(&st[6], (unsigned long long)contrib);
        }
        live = flag = used = 0;
        contrib = 0;
        units = 0;
    }
};

// Pairs of stream positions per slice of a wavefront's share of a unit (4096 samples).
constexpr uint64_t kSlicePairs = 2048;

template <int TU, int TV, int JC, int NPOL, class Acc, bool AGG>
__global__ void __launch_bounds__(1024, 4) k_accum_packed(const LaunchDesc* __restrict__ Lp,
                                                          const uint64_t* __restrict__ order,
                                                          uint32_t* __restrict__ counter,
                                                          const uint32_t* __restrict__ unit_off,
                                                          const uint64_t* __restrict__ recs,
                                                          const uint64_t* __restrict__ pre) {
    constexpr int JP = JC + 1;            // padded channel stride of a cell
    constexpr int NC = TU * TV * JP;
    constexpr uint32_t kChunk = 2 * kWave;
    __shared__ Acc s_re[NC], s_im[NC], s_w[NC];
    __shared__ uint32_t s_n[NC];
    __shared__ uint32_t s_unit;
    __shared__ unsigned long long s_contrib;

    const LaunchDesc& L = *Lp;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = sgpr(threadIdx.x / kWave);
    const int nw = blockDim.x / kWave;
    const VISTA_GLOBAL uint64_t* grecs = gptr(recs);
    const VISTA_GLOBAL uint64_t* gpre = gptr(pre);
    const VISTA_CONST uint64_t* cpre = cptr(pre);
    const VISTA_GLOBAL RowCtx* rctx = gptr((const RowCtx*)L.rowctx);
    const VISTA_GLOBAL DevChan* chan_all = gptr(L.chan_all);
    const VISTA_GLOBAL float* f1_all = gptr(L.f1_all);
    const int phase_fp32 = L.phase_fp32;
    WaveStats ws;

    // LDS starts zeroed; afterwards each unit's flush zeroes the cells it wrote
    for (int i = threadIdx.x; i < NC; i += blockDim.x) {
        s_re[i] = Acc(0); s_im[i] = Acc(0); s_w[i] = Acc(0); s_n[i] = 0u;
    }
    // the next unit is claimed while the current one is processed
    if (threadIdx.x == 0) {
        s_unit = atomicAdd(counter, 1u);
        s_contrib = 0ull;
    }
    __syncthreads();
    for (;;) {
        const uint32_t li = (uint32_t)sgpr((int32_t)s_unit);
        if (li >= L.nunits) break;
        const int64_t unit = (int64_t)ufl64(cptr(order)[li]);
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
        const uint32_t ntu = (uint32_t)min(TU, S.nu - tu0), ntv = (uint32_t)min(TV, S.nv - tv0);   // in-grid part
        const double inv_du = S.inv_du, inv_dv = S.inv_dv;
        if (si != ws.stack || ws.units >= 64) {
            ws.flush(L, lane);
            ws.stack = si;
        }
        ++ws.units;
        __syncthreads();                  // every thread has read s_unit
        uint32_t next = 0;
        if (threadIdx.x == 0) next = atomicAdd(counter, 1u);

        const uint32_t rb = (uint32_t)sgpr((int32_t)cptr(unit_off)[unit]);
        const uint32_t re = (uint32_t)sgpr((int32_t)cptr(unit_off)[unit + 1]);
        uint32_t u_contrib_l = 0;         // contributions of this lane's samples
        // the unit's stream, in pairs, dealt to the wavefronts in slices of kSlicePairs: wave
        // w takes slices w, w + nw, ... of every full round, then an even share of what the
        // full rounds leave, so that at any time the wavefronts work on nearby records (rows
        // of one target share channel-table entries and cache lines) and finish together
        uint64_t sp0 = 0, npairs = 0;
        if (rb < re) {
            sp0 = ufl64(cpre[rb]);
            npairs = (ufl64(cpre[re]) - sp0) >> 1;
        }
        const uint64_t round = (uint64_t)nw * kSlicePairs;
        const uint64_t nfull = npairs / round, rest = npairs - nfull * round;
        for (uint64_t rr = 0; rr <= nfull; ++rr) {
        uint64_t sw0, sw1;
        if (rr < nfull) {
            sw0 = sp0 + 2 * ((rr * nw + wave) * kSlicePairs);
            sw1 = sw0 + 2 * kSlicePairs;
        } else {
            sw0 = sp0 + 2 * (nfull * round + rest * (uint64_t)wave / (uint64_t)nw);
            sw1 = sp0 + 2 * (nfull * round + rest * (uint64_t)(wave + 1) / (uint64_t)nw);
        }
        if (sw0 < sw1) {
            // ---- the record holding sample sw0: largest i in [rb, re) with pre[i] <= sw0
            uint32_t lo = rb, hi = re;
            while (hi - lo > (uint32_t)kWave) {
                const uint32_t step = (hi - lo + kWave - 1) / kWave;
                const uint32_t idx = lo + (uint32_t)lane * step;
                const bool v = idx < hi;
                const uint64_t p = v ? gpre[idx] : ~0ull;
                const uint64_t m = __ballot(v && p <= sw0);        // lane 0 always set
                lo = lo + (uint32_t)(63 - __clzll(m)) * step;
                hi = min(lo + step, hi);
            }
            uint32_t first;
            {
                const uint32_t idx = lo + (uint32_t)lane;
                const bool v = idx < hi;
                const uint64_t p = v ? gpre[idx] : ~0ull;
                const uint64_t m = __ballot(v && p <= sw0);
                first = lo + (uint32_t)(63 - __clzll(m));
            }

            // ---- window of up to 64 records, one per lane.  Stream positions in the loops
            // below are 32-bit offsets from sw0 (a slice and a window span far less than 2^31)
            uint32_t wb = 0, nwin = 0, cur = 0;
            int32_t pw = 0, wend = 0;      // the window's first and end positions
            const uint32_t se = (uint32_t)(sw1 - sw0);
            uint32_t wrel = 0;             // this lane's record start, relative to pw
            RecCtx<NPOL> w;
            auto load_window = [&](uint32_t nb) __attribute__((always_inline)) {
                wb = nb;
                nwin = min((uint32_t)kWave, re - nb);
                const uint64_t pw64 = ufl64(cpre[nb]);
                pw = (int32_t)(int64_t)(pw64 - sw0);
                wend = (int32_t)(int64_t)(ufl64(cpre[nb + nwin]) - sw0);
                const bool v = (uint32_t)lane < nwin;
                const uint64_t rec = v ? grecs[nb + lane] : 0ull;
                const uint64_t pg = v ? gpre[nb + lane] : 0ull;
                wrel = v ? (uint32_t)(pg - pw64) : 0xffffffffu;
                const uint32_t g = (uint32_t)(rec >> 32);
                const uint32_t kin = (uint32_t)((rec >> 16) & 0xffffu), kout = (uint32_t)(rec & 0xffffu);
                const int64_t d = (int64_t)kin - (int64_t)wrel;         // channel - position
                const VISTA_GLOBAL RowCtx& rc = rctx[g];
                w.U = rc.U;
                w.V = rc.V;
                w.T = rc.T;
                const uint64_t vrow = rc.vis, frow = rc.flag;
                w.chan = rc.chan0 + (int32_t)d;
                w.end = wrel + (kout - kin);
                if (NPOL == 2) {
                    w.w0 = rc.w0;
                    w.w1 = rc.w1;
                    w.vis = vrow + (uint64_t)(d * 16);
                    w.flag = frow + (uint64_t)(d * 2);
                } else {
                    const uint32_t info = rc.info;
                    const int64_t np = info & 0xffu;
                    const bool wpc = (info >> 8) & 1u;
                    w.vis = vrow + (uint64_t)(d * np * 8);
                    w.flag = frow + (uint64_t)(d * np);
                    w.wadj = rc.wrow + (wpc ? (uint64_t)(d * np * 4) : 0ull);
                    w.info = (uint32_t)np | ((wpc ? (uint32_t)np * 4u : 0u) << 8);
                }
                // the first chunk needs the window anyway; waiting here also tells the
                // compiler that no window load is pending in the chunk loop, where it
                // would otherwise wait for every load in flight before each gather
                __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
            };
            // lanes of the chunk starting at s (two samples each): records and contexts.
            // live == false: an idle chunk (every lane inactive, the window cursor kept) whose
            // lanes load from the record at the cursor.
            auto map = [&](uint32_t s, Pair<NPOL>& x, bool live) __attribute__((always_inline)) {
                const uint32_t srel = (uint32_t)((int32_t)s - pw);
                const uint32_t pos = srel + 2u * (uint32_t)lane;
                // (an idle chunk may find the cursor one past the window: use its last record)
                int rec = live ? (int)cur : (int)min(cur, nwin - 1u);
                if (live) {
                    // records starting in (s, s + 128]: the last one at or before a lane's
                    // pair wins
                    const uint64_t B = __ballot(lane > (int)cur && wrel <= srel + kChunk);
                    uint64_t m = B;
                    while (m) {
                        const int i = __builtin_ctzll(m);
                        m &= m - 1;
                        const uint32_t pi = (uint32_t)__builtin_amdgcn_readlane((int)wrel, i);
                        rec = pos >= pi ? i : rec;
                    }
                    cur += (uint32_t)__popcll(B);
                }
                x.rec = rec;
                x.pos = pos;
                x.act = live && s + 2u * (uint32_t)lane < se;
            };

            // What one sample adds: its LDS cell row (cell + j is the cell of rest channel j),
            // rest channel j0, whether it adds to j0 and j0 + 1 in this unit's block, the
            // merged polarisations rotated (pr, pi), their weight q and count n, and the
            // overlap fractions.
            struct Contrib {
                int cell;
                int32_t j0;
                bool add0, add1;
                float pr, pi, q, f0, f1;
                uint32_t n;
            };
            // one sample: g0, g1 tell whether the record's row weights are usable (NPOL == 2);
            // the statistics are counted here, and the rare rest channels beyond j0 + 1 (a
            // rest grid finer than the channel) are added here; the rest is returned
            auto prepare = [&](const RecCtx<NPOL>& rc, const Loaded<NPOL>& x, bool valid, int32_t ci, bool g0,
                               bool g1) __attribute__((always_inline)) {
                Contrib o;
                const uint32_t nj = valid ? x.jn >> 24 : 0u;
                const int32_t j0 = (int32_t)(x.jn & kJMask);
                // cell within the tile (exact FP64 sequence of the definition)
                const double ru = cell_coord(rc.U, x.a, inv_du);
                const double rv = cell_coord(rc.V, x.a, inv_dv);
                const int32_t lu = (int32_t)ru + cu, lv = (int32_t)rv + cv;
                const bool in_tile = nj > 0 && (uint32_t)lu < ntu && (uint32_t)lv < ntv;
                const bool home = in_tile && j0 >= jb0 && j0 < jb1;    // counted once, in j0's block
                // polarisations: drop flagged and bad-weight samples, merge the rest
                float ar = 0.f, ai = 0.f, q = 0.f;
                uint32_t n = 0;
                const int np = NPOL == 2 ? 2 : (int)(rc.info & 0xffu);
                uint32_t nflag = 0;
#pragma unroll
                for (int p = 0; p < (NPOL == 2 ? 2 : 4); ++p) {
                    const bool live = NPOL == 2 || p < np;
                    const float wgt = NPOL == 2 ? (p == 0 ? rc.w0 : rc.w1) : x.wc[p];
                    const bool flagged = live && ((x.fl >> (8 * p)) & 0xffu) != 0u;
                    const bool good = NPOL == 2 ? (p == 0 ? g0 : g1)
                                                : (live && (wgt > 0.0f) && (wgt < __builtin_inff()));
                    nflag += flagged ? 1u : 0u;
                    const bool use = !flagged && good;
                    const float wu = use ? wgt : 0.0f;
                    n += use ? 1u : 0u;
                    ar = fmaf(wu, x.vr[p], ar);
                    ai = fmaf(wu, x.vi[p], ai);
                    q += wu;
                }
                // statistics of the sample's home unit: live polarisations, flagged, used
                ws.live += home ? (uint32_t)np : 0u;
                ws.flag += home ? nflag : 0u;
                ws.used += home ? n : 0u;
                float c, sn;
                if (phase_fp32) {
                    const float t = (float)rc.T * (float)x.a;
                    sincos_turns(t - rintf(t), &sn, &c);
                } else {
                    phasor(rc.T, x.a, &c, &sn);
                }
                o.pr = ar * c - ai * sn;
                o.pi = fmaf(ar, sn, ai * c);
                o.q = q;
                o.n = n;
                o.f0 = x.f0;
                o.f1 = x.f1;
                o.j0 = j0;
                // rest channels j0 and j0 + 1 of this unit's block (counted before any lane leaves)
                const bool live_add = in_tile && n > 0;
                o.add0 = live_add && j0 >= jb0 && j0 < jb1;
                o.add1 = live_add && nj > 1 && j0 + 1 >= jb0 && j0 + 1 < jb1;
                u_contrib_l += (o.add0 ? n : 0u) + (o.add1 ? n : 0u);
                o.cell = (lv * TU + lu) * JP - jb0;
                // more than two rest channels (rest grid finer than the channel): rare
                if (live_add && nj > 2) {
                    const Acc dr = (Acc)o.pr, di = (Acc)o.pi, dq = (Acc)q;
                    const int32_t fo = gptr(L.foff_all)[ci];
                    for (int qq = 2; qq < (int)nj; ++qq) {
                        const int32_t j = j0 + qq;
                        if (j < jb0 || j >= jb1) continue;
                        const Acc f = (Acc)gptr(L.fval_all)[fo + qq];
                        const int cc = o.cell + j;
                        atomicAdd(&s_re[cc], f * dr);
                        atomicAdd(&s_im[cc], f * di);
                        atomicAdd(&s_w[cc], f * dq);
                        atomicAdd(&s_n[cc], n);
                        u_contrib_l += n;
                    }
                }
                return o;
            };
            auto process_pair = [&](const Pair<NPOL>& x) __attribute__((always_inline)) {
                settle<NPOL>(x.s[0]);
                settle<NPOL>(x.s[1]);
                RecCtx<NPOL> rc;
                rc.U = bpermd(w.U, x.rec);
                rc.V = bpermd(w.V, x.rec);
                rc.T = bpermd(w.T, x.rec);
                bool g0 = false, g1 = false;
                if (NPOL == 2) {
                    rc.w0 = bpermf(w.w0, x.rec);
                    rc.w1 = bpermf(w.w1, x.rec);
                    g0 = (rc.w0 > 0.0f) && (rc.w0 < __builtin_inff());
                    g1 = (rc.w1 > 0.0f) && (rc.w1 < __builtin_inff());
                } else {
                    rc.info = bperm(w.info, x.rec);
                }
                const int32_t ci = (int32_t)bperm((uint32_t)w.chan, x.rec) + (int32_t)x.pos;
                if constexpr (AGG) {
                    // fine channels: the pair's samples mostly add to the same cell of rest
                    // channel j0 -- one set of values for both there (the FP64 products are
                    // exact, their sum rounds once), each on its own otherwise
                    const Contrib a = prepare(rc, x.s[0], x.act, ci, g0, g1);
                    const Contrib b = prepare(rc, x.s[1], x.two, ci + 1, g0, g1);
                    const bool comb = a.add0 && b.add0 && a.cell + a.j0 == b.cell + b.j0;
                    const Acc fa = (Acc)a.f0, fb = (Acc)b.f0;
                    Acc re = fa * (Acc)a.pr, im = fa * (Acc)a.pi, wq = fa * (Acc)a.q;
                    uint32_t n = a.n;
                    if (comb) {
                        re += fb * (Acc)b.pr;
                        im += fb * (Acc)b.pi;
                        wq += fb * (Acc)b.q;
                        n += b.n;
                    }
                    emit<Acc>(s_re, s_im, s_w, s_n, lane, a.add0 ? a.cell + a.j0 : -1, re, im, wq, n);
                    // the rest is rare on fine channels (a run ends between the pair's samples,
                    // or a channel reaches a second rest channel): added directly
                    auto direct = [&](int key, Acc f, const Contrib& c) __attribute__((always_inline)) {
                        atomicAdd(&s_re[key], f * (Acc)c.pr);
                        atomicAdd(&s_im[key], f * (Acc)c.pi);
                        atomicAdd(&s_w[key], f * (Acc)c.q);
                        atomicAdd(&s_n[key], c.n);
                    };
                    if (b.add0 && !comb) direct(b.cell + b.j0, fb, b);
                    if (a.add1) direct(a.cell + a.j0 + 1, (Acc)a.f1, a);
                    if (b.add1) direct(b.cell + b.j0 + 1, (Acc)b.f1, b);
                } else {
                    // coarse channels: the pair's second channel mostly starts in the rest
                    // channel where the first one ends (or shares the first's), so its first
                    // contribution joins one of the first channel's in registers (the FP64
                    // products are exact, their sum rounds once) and three sets of LDS
                    // updates serve the pair instead of four
                    const Contrib a = prepare(rc, x.s[0], x.act, ci, g0, g1);
                    const Contrib b = prepare(rc, x.s[1], x.two, ci + 1, g0, g1);
                    const int ka0 = a.add0 ? a.cell + a.j0 : -1, ka1 = a.add1 ? a.cell + a.j0 + 1 : -1;
                    const int kb0 = b.add0 ? b.cell + b.j0 : -1, kb1 = b.add1 ? b.cell + b.j0 + 1 : -1;
                    const Acc fa0 = (Acc)a.f0, fa1 = (Acc)a.f1, fb0 = (Acc)b.f0, fb1 = (Acc)b.f1;
                    const bool m1 = kb0 >= 0 && kb0 == ka1;                 // b's first = a's second
                    const bool m0 = kb0 >= 0 && !m1 && kb0 == ka0;          // b's first = a's first
                    auto add = [&](int key, Acc re, Acc im, Acc w, uint32_t n) __attribute__((always_inline)) {
                        if (key >= 0) {
                            atomicAdd(&s_re[key], re);
                            atomicAdd(&s_im[key], im);
                            atomicAdd(&s_w[key], w);
                            atomicAdd(&s_n[key], n);
                        }
                    };
                    const Acc br = fb0 * (Acc)b.pr, bi = fb0 * (Acc)b.pi, bw = fb0 * (Acc)b.q;
                    add(ka0, fa0 * (Acc)a.pr + (m0 ? br : Acc(0)), fa0 * (Acc)a.pi + (m0 ? bi : Acc(0)),
                        fa0 * (Acc)a.q + (m0 ? bw : Acc(0)), a.n + (m0 ? b.n : 0u));
                    add(ka1, fa1 * (Acc)a.pr + (m1 ? br : Acc(0)), fa1 * (Acc)a.pi + (m1 ? bi : Acc(0)),
                        fa1 * (Acc)a.q + (m1 ? bw : Acc(0)), a.n + (m1 ? b.n : 0u));
                    add(m0 || m1 ? -1 : kb0, br, bi, bw, b.n);
                    add(kb1, fb1 * (Acc)b.pr, fb1 * (Acc)b.pi, fb1 * (Acc)b.q, b.n);
                }
            };

            // ---- chunks, the next one's loads in flight while one is processed.  A chunk is
            // mapped only when the window holds all of its records; the window is reloaded
            // between runs of chunks, so no other load sits among the chunks' loads.
            // (After a reload at the record holding s, the window reaches at least 128
            // positions past s: records take whole pairs and s is even.)
            auto fits = [&](uint32_t t) __attribute__((always_inline)) {
                return t < se && (int32_t)min(t + kChunk, se) <= wend;
            };
            load_window(first);
            cur = 0;
            uint32_t s = 0;
            // the next chunks, or, at the end of a run, idle ones: the loads are issued on
            // every path, so the wait before processing a chunk is for its own loads only
            auto next = [&](bool live, uint32_t t, Pair<NPOL>& x) __attribute__((always_inline)) {
                map(live ? t : (uint32_t)(wend - 2), x, live);
                issue<NPOL>(chan_all, f1_all, w, x);
            };
            for (;;) {
                // two chunks in the pipeline: one processed while the next one's loads fly
                Pair<NPOL> x0, x1;
                next(true, s, x0);
                for (;;) {
                    const bool l1 = fits(s + kChunk);
                    next(l1, s + kChunk, x1);
                    process_pair(x0);
                    s += kChunk;
                    if (!l1) break;
                    const bool l0 = fits(s + kChunk);
                    next(l0, s + kChunk, x0);
                    process_pair(x1);
                    s += kChunk;
                    if (!l0) break;
                }
                if (s >= se) break;
                // the record holding s and the 63 after it.  The cursor is the window's last
                // record starting at or before s; when s is the window's end, that record ends
                // at s and the one holding s is the first past the window.
                load_window((int32_t)s >= wend ? wb + nwin : wb + cur);
                cur = 0;
            }
        }
        }

        // a cell count can wrap only if the unit's contributions reach 2^32
        const unsigned long long t_contrib = wave_sum_u64(u_contrib_l);
        ws.contrib += t_contrib;
        if (npairs > (1ull << 26)) ws.units = 64;      // keep the lanes' 32-bit counts far from wrapping
        if (lane == 0 && t_contrib) atomicAdd(&s_contrib, t_contrib);
        __syncthreads();
        if (threadIdx.x == 0) {
            if (s_contrib > 0xffffffffull) atomicOr(&S.stats[7], 1ull);
            s_contrib = 0ull;
            s_unit = next;
        }
        flush_unit<TU, TV, JP, Acc, false, true>(L, S, tu0, tv0, jb0, jb1, s_re, s_im, s_w, s_n, nullptr,
                                                 nullptr, nullptr);
        __syncthreads();
    }
    ws.flush(L, lane);
}

// ------------------------------------------------------------- ordered accumulation

// The deterministic form: results are bit-identical from run to run.  A workgroup owns one
// unit at a time, as above, but each wavefront owns a slice of jsub rest channels of the
// unit's block and walks every record of the unit, keeping the channels that reach its
// slice (its target's sub-block range): no cell has two writers.  The clipped records of
// a window of 64 form one stream that the wavefront takes 64 positions (one channel with
// all its polarisations per lane) at a time, whatever records they come from, so lanes do
// not idle at record ends.  The lanes of a chunk add in phases: channels of one row that
// are nphase or more apart never share a rest channel, so with P phases (the window's
// largest nphase, at least two) phase p takes the lanes whose channel plus record index is
// congruent to p modulo P, which also puts the same channel of consecutive records (rows
// of one baseline, which often share a cell) in different phases.  Lanes of one phase from
// different rows can still meet in a cell; they take turns: every waiting lane bids for
// its cells with an LDS max of a stamp (the wavefront's turn count, then its lane id), the
// lanes that hold every cell they bid for add, the others bid again.  A turn's stamps
// exceed every earlier turn's, so stale bids lose without being cleared, and a turn reads
// the bids and the cells' state together (a winner holds its cells alone that turn, so
// what it read is current): one LDS round trip a turn.  Where channels are fine (long runs
// of lanes with the same cells), each run is summed first in lane order and only its last
// lane bids, in one phase.  The order of the additions to a cell thus depends on the
// records and lane ids only.  Sums are FP32 with a Kahan
// compensation per addition (KAHAN) or FP64, read and written plainly.

// Keeps the compiler from moving LDS accesses across this point: the lanes of a wavefront
// read what other lanes of it wrote just before (the LDS serves one wavefront's
// instructions in order).
__device__ __forceinline__ void lds_order() { __asm__ volatile("" ::: "memory"); }

// Fewest addition phases per chunk of the ordered kernel.
constexpr int32_t kOrdPhases = 2;

// One lane's sample of a chunk: window lane of its record, stream position (relative to
// the window), whether it is inside the stream.
template <int NPOL>
struct OrdSample {
    int rec;
    uint32_t pos;
    bool act;
    Loaded<NPOL> s;
};

template <int TU, int TV, int JC, int NPOL, bool KAHAN>
__global__ void __launch_bounds__(1024, 4) k_accum_ordered(const LaunchDesc* __restrict__ Lp,
                                                           const uint64_t* __restrict__ order,
                                                           uint32_t* __restrict__ counter,
                                                           const uint32_t* __restrict__ unit_off,
                                                           const uint64_t* __restrict__ recs) {
    constexpr int JP = JC + 1;            // padded channel stride of a cell
    constexpr int NC = TU * TV * JP;
    // a cell's state, a lane's few LDS accesses: KAHAN, (re, its compensation, im, its
    // compensation) and (w, its compensation) in FP32; else (re, im) and w in FP64
    using Sri = typename std::conditional<KAHAN, float4, double2>::type;
    using Sw = typename std::conditional<KAHAN, float2, double>::type;
    // a lane's terms: FP32 products (KAHAN), else exact FP64 products
    using AccR = typename std::conditional<KAHAN, float, double>::type;
    static_assert(NC < (1 << 13) - 1, "two cell indices form one run key");
    // the rest of a cell's state in one 16-byte access: w, the count, and the highest stamp
    // bid for the cell (0 at a unit's start)
    struct alignas(16) Cw {
        Sw w;
        uint32_t n, bid;
    };
    static_assert(sizeof(Cw) == 16, "one 16-byte LDS access per cell");
    __shared__ Sri s_ri[NC];
    __shared__ Cw s_c[NC];
    __shared__ uint32_t s_unit;

    const LaunchDesc& L = *Lp;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = sgpr(threadIdx.x / kWave);
    const VISTA_GLOBAL uint64_t* grecs = gptr(recs);
    const VISTA_GLOBAL RowCtx* rctx = gptr((const RowCtx*)L.rowctx);
    const VISTA_GLOBAL int32_t* rtgt = gptr((const int32_t*)L.row_target);
    const VISTA_GLOBAL DevTarget* gtgts = gptr(L.targets);
    const VISTA_GLOBAL DevChan* chan_all = gptr(L.chan_all);
    const VISTA_GLOBAL float* f1_all = gptr(L.f1_all);
    const int phase_fp32 = L.phase_fp32;
    const int32_t jsub = L.jsub;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t li = (uint32_t)sgpr((int32_t)s_unit);
        if (li >= L.nunits) break;
        const int64_t unit = (int64_t)ufl64(cptr(order)[li]);
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
        const uint32_t ntu = (uint32_t)min(TU, S.nu - tu0), ntv = (uint32_t)min(TV, S.nv - tv0);   // in-grid part
        const double inv_du = S.inv_du, inv_dv = S.inv_dv;

        for (int i = threadIdx.x; i < NC; i += blockDim.x) {
            s_ri[i] = Sri{};
            s_c[i] = Cw{};
        }
        __syncthreads();

        const uint32_t rb = (uint32_t)sgpr((int32_t)cptr(unit_off)[unit]);
        const uint32_t re = (uint32_t)sgpr((int32_t)cptr(unit_off)[unit + 1]);
        // this wavefront's slice of rest channels and its index among the stack's sub-blocks
        const int32_t js0 = jb0 + wave * jsub;
        const int32_t js1 = min(js0 + jsub, jb1);
        const int32_t sbi = jb0 / jsub + wave;
        // this lane's statistics of the unit: live, flagged and used polarisations of the
        // samples whose first rest channel is in the slice, and contributions added
        uint32_t st_live = 0, st_flag = 0, st_used = 0, st_contrib = 0;
        // turns of this wavefront in this unit: a turn's bids carry (turn << 6 | lane) + 1,
        // above every earlier turn's, so that earlier bids need no clearing
        uint32_t turns = 0;

        // one addition of (f pr, f pi, f q) and count n to a cell's state in registers
        auto accum = [&](Sri& ri, Sw& w, uint32_t& cnt, float f, float pr, float pi, float q, uint32_t n)
                         __attribute__((always_inline)) {
            if constexpr (KAHAN) {
                auto kadd = [](float& sum, float& comp, float x) __attribute__((always_inline)) {
                    const float y = x - comp, t = sum + y;
                    comp = (t - sum) - y;
                    sum = t;
                };
                kadd(ri.x, ri.y, f * pr);
                kadd(ri.z, ri.w, f * pi);
                kadd(w.x, w.y, f * q);
            } else {
                ri.x += (double)f * (double)pr;     // exact products, one rounding each
                ri.y += (double)f * (double)pi;
                w += (double)f * (double)q;
            }
            cnt += n;
        };
        // one addition of precomputed terms (vr, vi, vq) and count n to a cell's state
        auto accumv = [&](Sri& ri, Sw& w, uint32_t& cnt, AccR vr, AccR vi, AccR vq, uint32_t n)
                          __attribute__((always_inline)) {
            if constexpr (KAHAN) {
                auto kadd = [](float& sum, float& comp, float x) __attribute__((always_inline)) {
                    const float y = x - comp, t = sum + y;
                    comp = (t - sum) - y;
                    sum = t;
                };
                kadd(ri.x, ri.y, vr);
                kadd(ri.z, ri.w, vi);
                kadd(w.x, w.y, vq);
            } else {
                ri.x += vr;
                ri.y += vi;
                w += vq;
            }
            cnt += n;
        };
        // one addition to cell cc; no other lane writes cc meanwhile
        auto add = [&](int cc, float f, float pr, float pi, float q, uint32_t n) __attribute__((always_inline)) {
            Sri ri = s_ri[cc];
            Cw c = s_c[cc];
            accum(ri, c.w, c.n, f, pr, pi, q, n);
            s_ri[cc] = ri;
            s_c[cc] = c;
            st_contrib += n;
        };

        for (uint32_t wb = rb; js0 < js1 && wb < re; wb += (uint32_t)kWave) {
            // ---- window: records wb .. wb + 63, one per lane, clipped to the slice
            const uint32_t nwin = min((uint32_t)kWave, re - wb);
            const bool v = (uint32_t)lane < nwin;
            // a full window is taken in the order 25 q mod 64, so that records next to each
            // other in row order (often one baseline at consecutive times, in one cell) fall
            // in different chunks
            const uint32_t q = nwin == (uint32_t)kWave ? (uint32_t)(lane * 25) & (kWave - 1) : (uint32_t)lane;
            const uint64_t rec = v ? grecs[wb + q] : 0ull;
            const uint32_t g = (uint32_t)(rec >> 32);
            int32_t kin = (int32_t)((rec >> 16) & 0xffffu), kout = (int32_t)(rec & 0xffffu);
            int32_t len = 0, nph = 1;
            RecCtx<NPOL> w;
            w.U = 0.0; w.V = 0.0; w.T = 0.0; w.w0 = 0.f; w.w1 = 0.f;
            w.vis = 0; w.flag = 0; w.wadj = 0; w.info = 0; w.chan = 0; w.end = 0;
            if (v) {
                const VISTA_GLOBAL DevTarget& T = gtgts[rtgt[g]];
                const VISTA_GLOBAL int32_t* sb = gptr(T.sblk);
                kin = max(kin, sb[2 * sbi]);
                kout = min(kout, sb[2 * sbi + 1]);
                len = max(0, kout - kin);
                nph = max(1, T.nphase);
            }
            // stream position of each clipped record: exclusive prefix sum of the lengths
            uint32_t incl = (uint32_t)len;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) {
                const uint32_t t = (uint32_t)__shfl_up((int)incl, d, kWave);
                if (lane >= d) incl += t;
            }
            const uint32_t P = incl - (uint32_t)len;
            const uint32_t ltot = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
            if (ltot == 0) continue;
            // phases of this window: the largest nphase of its records, at least kOrdPhases
            int32_t nphw = len > 0 ? max(nph, kOrdPhases) : kOrdPhases;
#pragma unroll
            for (int d = 1; d < kWave; d <<= 1) nphw = max(nphw, __shfl_xor(nphw, d, kWave));
            nphw = sgpr(nphw);
            if (len > 0) {
                // the record's context, its addresses rebased to stream positions
                const VISTA_GLOBAL RowCtx& rc = rctx[g];
                const int64_t d = (int64_t)kin - (int64_t)P;      // channel minus position
                w.U = rc.U;
                w.V = rc.V;
                w.T = rc.T;
                w.chan = rc.chan0 + (int32_t)d;
                if (NPOL == 2) {
                    w.w0 = rc.w0;
                    w.w1 = rc.w1;
                    w.vis = rc.vis + (uint64_t)(d * 16);
                    w.flag = rc.flag + (uint64_t)(d * 2);
                } else {
                    const uint32_t info = rc.info;
                    const int64_t np = info & 0xffu;
                    const bool wpc = (info >> 8) & 1u;
                    w.vis = rc.vis + (uint64_t)(d * np * 8);
                    w.flag = rc.flag + (uint64_t)(d * np);
                    w.wadj = rc.wrow + (wpc ? (uint64_t)(d * np * 4) : 0ull);
                    w.info = (uint32_t)np | ((wpc ? (uint32_t)np * 4u : 0u) << 8);
                }
            }
            __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0): no window load stays pending below

            // ---- chunks of 64 positions; live == false: an idle chunk at c0 (no lane active)
            auto map = [&](uint32_t c0, OrdSample<NPOL>& x, bool live) __attribute__((always_inline)) {
                // the record holding position c0, then those starting inside the chunk
                const uint64_t m0 = __ballot(len > 0 && P <= c0);
                const int r0 = 63 - (int)__clzll(m0);
                const uint32_t p = c0 + (uint32_t)lane;
                int r = r0;
                uint64_t bm = __ballot(len > 0 && P > c0 && P < c0 + (uint32_t)kWave);
                while (bm) {
                    const int i = (int)__builtin_ctzll(bm);
                    bm &= bm - 1;
                    const uint32_t pi = (uint32_t)__builtin_amdgcn_readlane((int)P, i);
                    r = p >= pi ? i : r;
                }
                x.act = live && p < ltot;
                x.rec = x.act ? r : r0;
                x.pos = x.act ? p : c0;
            };
            auto issue = [&](OrdSample<NPOL>& x) __attribute__((always_inline)) {
                const Bases<NPOL> c = gather_bases<NPOL>(w, x.rec);
                load_sample<NPOL>(chan_all, f1_all, c, x.pos, x.s);
            };
            auto process = [&](const OrdSample<NPOL>& x) __attribute__((always_inline)) {
                settle<NPOL>(x.s);
                const Loaded<NPOL>& s = x.s;
                const double U = bpermd(w.U, x.rec), V = bpermd(w.V, x.rec), T = bpermd(w.T, x.rec);
                float w0 = 0.f, w1 = 0.f;
                uint32_t info = 2u;
                if (NPOL == 2) {
                    w0 = bpermf(w.w0, x.rec);
                    w1 = bpermf(w.w1, x.rec);
                } else {
                    info = bperm(w.info, x.rec);
                }
                const int32_t ci = (int32_t)bperm((uint32_t)w.chan, x.rec) + (int32_t)x.pos;
                const uint32_t nj = x.act ? s.jn >> 24 : 0u;
                const int32_t j0 = (int32_t)(s.jn & kJMask);
                // cell within the tile (exact FP64 sequence of the definition)
                const double ru = cell_coord(U, s.a, inv_du);
                const double rv = cell_coord(V, s.a, inv_dv);
                const int32_t lu = (int32_t)ru + cu, lv = (int32_t)rv + cv;
                const bool in_tile = nj > 0 && (uint32_t)lu < ntu && (uint32_t)lv < ntv;
                // polarisations: drop flagged and bad-weight samples, merge the rest
                float ar = 0.f, ai = 0.f, q = 0.f;
                uint32_t n = 0, nflag = 0;
                const int np = NPOL == 2 ? 2 : (int)(info & 0xffu);
#pragma unroll
                for (int p = 0; p < (NPOL == 2 ? 2 : 4); ++p) {
                    const bool live = NPOL == 2 || p < np;
                    const float wgt = NPOL == 2 ? (p == 0 ? w0 : w1) : s.wc[p];
                    const bool flagged = live && ((s.fl >> (8 * p)) & 0xffu) != 0u;
                    const bool good = live && (wgt > 0.0f) && (wgt < __builtin_inff());
                    nflag += flagged ? 1u : 0u;
                    const bool use = !flagged && good;
                    const float wu = use ? wgt : 0.0f;
                    n += use ? 1u : 0u;
                    ar = fmaf(wu, s.vr[p], ar);
                    ai = fmaf(wu, s.vi[p], ai);
                    q += wu;
                }
                // classification, counted once: in the slice holding j0
                const bool home = in_tile && j0 >= js0 && j0 < js1;
                st_live += home ? (uint32_t)np : 0u;
                st_flag += home ? nflag : 0u;
                st_used += home ? n : 0u;
                float c, sn;
                if (phase_fp32) {
                    const float t = (float)T * (float)s.a;
                    sincos_turns(t - rintf(t), &sn, &c);
                } else {
                    phasor(T, s.a, &c, &sn);
                }
                const float pr = ar * c - ai * sn;
                const float pi = fmaf(ar, sn, ai * c);
                const bool live_add = in_tile && n > 0;
                const int cell = (lv * TU + lu) * JP - jb0;
                const int a0 = (live_add && j0 >= js0 && j0 < js1) ? cell + j0 : -1;
                const int a1 = (live_add && nj > 1 && j0 + 1 >= js0 && j0 + 1 < js1) ? cell + j0 + 1 : -1;
                // the lane's terms for its two cells
                AccR r0 = 0, i0 = 0, q0 = 0, r1 = 0, i1 = 0, q1 = 0;
                uint32_t nn = n;
                if (a0 >= 0) { r0 = (AccR)s.f0 * (AccR)pr; i0 = (AccR)s.f0 * (AccR)pi; q0 = (AccR)s.f0 * (AccR)q; }
                if (a1 >= 0) { r1 = (AccR)s.f1 * (AccR)pr; i1 = (AccR)s.f1 * (AccR)pi; q1 = (AccR)s.f1 * (AccR)q; }
                bool mine = a0 >= 0 || a1 >= 0;
                // phase: channel plus window lane of the record, modulo nphw.  Channels of one
                // record fewer than nphw apart get different phases; so do the same channel
                // of consecutive records (rows of one baseline often share a cell)
                int32_t ph_l = (ci + x.rec) % nphw, nph_c = nphw;
                // fine channels: neighbouring lanes share cells in long runs, which phases
                // would take one lane at a time.  Where the window has more than four phases
                // and the chunk's runs of lanes with the same two cells are 4 lanes long or
                // more on average (a choice uniform over the wavefront), each run is summed first, in lane order (a segmented scan: the
                // run's last lane ends with its total), and only that lane bids, in one phase;
                // the bids order runs that share a cell
                const int key = mine ? ((a0 + 1) << 13 | (a1 + 1)) : -1;
                uint64_t act = 0, heads = 0;
                if (nphw > 4) {
                    const int prev = __shfl_up(key, 1, kWave);
                    act = __ballot(key >= 0);
                    heads = __ballot(key >= 0 && (lane == 0 || prev != key));
                }
                if (act != 0 && __popcll(heads) * 4 <= __popcll(act)) {
                    const uint64_t upto = heads & ((2ull << lane) - 1ull);
                    const int start = upto ? 63 - (int)__clzll(upto) : lane;
                    const int span = key >= 0 ? lane - start : -1;
                    const int c16 = lane & 15;
                    uint32_t nx = 0u;
                    scan_dpp<0x111, 0xf>(r0, i0, q0, nn, span >= 1);
                    scan_dpp<0x111, 0xf>(r1, i1, q1, nx, span >= 1);
                    scan_dpp<0x112, 0xf>(r0, i0, q0, nn, span >= 2);
                    scan_dpp<0x112, 0xf>(r1, i1, q1, nx, span >= 2);
                    scan_dpp<0x114, 0xf>(r0, i0, q0, nn, span >= 4);
                    scan_dpp<0x114, 0xf>(r1, i1, q1, nx, span >= 4);
                    scan_dpp<0x118, 0xf>(r0, i0, q0, nn, span >= 8);
                    scan_dpp<0x118, 0xf>(r1, i1, q1, nx, span >= 8);
                    scan_dpp<0x142, 0xa>(r0, i0, q0, nn, span >= c16 + 1);
                    scan_dpp<0x142, 0xa>(r1, i1, q1, nx, span >= c16 + 1);
                    scan_dpp<0x143, 0xc>(r0, i0, q0, nn, span >= lane - 31);
                    scan_dpp<0x143, 0xc>(r1, i1, q1, nx, span >= lane - 31);
                    const uint64_t ends = heads | ~act;
                    mine = key >= 0 && (lane == kWave - 1 || ((ends >> (lane + 1)) & 1ull));
                    ph_l = 0;
                    nph_c = 1;
                }
                // a lane with one cell bids for it twice (a max with the same stamp changes
                // nothing); a lane with none reads cell 0 and never bids
                const int b0 = a0 >= 0 ? a0 : max(a1, 0), b1 = a1 >= 0 ? a1 : max(a0, 0);
                for (int32_t ph = 0; ph < nph_c; ++ph) {
                    bool pend = mine && ph_l == ph;
                    if (turns >= (1u << 25)) {
                        // the stamps would wrap within this phase's 64 turns: clear this
                        // wavefront's bids and start again
                        for (int c = lane; c < NC; c += kWave) {
                            const int j = c % JP + jb0;
                            if (j >= js0 && j < js1) s_c[c].bid = 0u;
                        }
                        lds_order();
                        turns = 0;
                    }
                    // each turn the highest waiting lane adds, so 64 turns always suffice
                    for (int turn = 0; turn < kWave && __ballot(pend); ++turn) {
                        ++turns;
                        const uint32_t id = (turns << 6 | (uint32_t)lane) + 1u;
                        if (pend) {
                            atomicMax(&s_c[b0].bid, id);
                            atomicMax(&s_c[b1].bid, id);
                        }
                        lds_order();
                        // the cells' state is read with the bids: a winner holds its cells
                        // alone this turn, so what it read is current
                        Sri ri0 = s_ri[b0], ri1 = s_ri[b1];
                        Cw c0 = s_c[b0], c1 = s_c[b1];
                        const bool win = pend && c0.bid == id && c1.bid == id;
                        lds_order();
                        if (win) {
                            const bool h0 = a0 >= 0, h1 = a1 >= 0;
                            if (h0) {
                                accumv(ri0, c0.w, c0.n, r0, i0, q0, nn);
                                s_ri[a0] = ri0; s_c[a0] = c0;
                            }
                            if (h1) {
                                accumv(ri1, c1.w, c1.n, r1, i1, q1, nn);
                                s_ri[a1] = ri1; s_c[a1] = c1;
                            }
                            st_contrib += (h0 ? nn : 0u) + (h1 ? nn : 0u);
                        }
                        pend = pend && !win;
                        lds_order();
                    }
                    if (__ballot(pend) && lane == 0) atomicOr(&S.stats[7], 2ull);
                }
                // rest channels beyond j0 + 1 (a rest grid finer than the channel): rare, one
                // lane at a time in lane order
                uint64_t xm = __ballot(live_add && nj > 2);
                while (xm) {
                    const int i = (int)__builtin_ctzll(xm);
                    xm &= xm - 1;
                    if (lane == i) {
                        const int32_t fo = gptr(L.foff_all)[ci];
                        for (int qq = 2; qq < (int)nj; ++qq) {
                            const int32_t j = j0 + qq;
                            if (j < js0 || j >= js1) continue;
                            add(cell + j, gptr(L.fval_all)[fo + qq], pr, pi, q, n);
                        }
                    }
                }
            };

            // two chunks in the pipeline: one processed while the next one's loads fly (an
            // idle chunk's loads at the end, so that every path issues the same loads)
            OrdSample<NPOL> x0, x1;
            uint32_t c0 = 0;
            map(0u, x0, true);
            issue(x0);
            for (;;) {
                const bool l1 = c0 + (uint32_t)kWave < ltot;
                map(l1 ? c0 + (uint32_t)kWave : c0, x1, l1);
                issue(x1);
                process(x0);
                c0 += (uint32_t)kWave;
                if (!l1) break;
                const bool l0 = c0 + (uint32_t)kWave < ltot;
                map(l0 ? c0 + (uint32_t)kWave : c0, x0, l0);
                issue(x0);
                process(x1);
                c0 += (uint32_t)kWave;
                if (!l0) break;
            }
        }

        // statistics: one set of atomics per wavefront and unit; bad = live - flagged - used
        const unsigned long long t_live = wave_sum_u64(st_live), t_flag = wave_sum_u64(st_flag);
        const unsigned long long t_used = wave_sum_u64(st_used), t_contrib = wave_sum_u64(st_contrib);
        if (lane == 0) {
            const unsigned long long t_bad = t_live - t_flag - t_used;
            if (t_flag) atomicAdd(&S.stats[1], t_flag);
            if (t_bad) atomicAdd(&S.stats[2], t_bad);
            if (t_used) atomicAdd(&S.stats[5], t_used);
            if (t_contrib) atomicAdd(&S.stats[6], t_contrib);
            if (t_contrib > 0xffffffffull) atomicOr(&S.stats[7], 1ull);   // a cell count may have wrapped
        }
        __syncthreads();

        flush_cells<TU, TV, JP>(L, S, tu0, tv0, jb0, jb1,
                                [&](int c, double& dre, double& dim, double& dw, uint32_t& n)
                                    __attribute__((always_inline)) {
            const Sri ri = s_ri[c];
            const Sw w = s_c[c].w;
            if constexpr (KAHAN) {
                dre = (double)ri.x - (double)ri.y;
                dim = (double)ri.z - (double)ri.w;
                dw = (double)w.x - (double)w.y;
            } else {
                dre = ri.x; dim = ri.y; dw = w;
            }
            n = s_c[c].n;
        });
        __syncthreads();
    }
}

// ---------------------------------------------------------------- record prefix, order

__global__ void k_record_lens(const uint64_t* __restrict__ recs, const int64_t* __restrict__ n_dev,
                              uint32_t* __restrict__ lens) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < *n_dev) {
        const uint64_t r = recs[i];
        const uint32_t len = (uint32_t)(r & 0xffffu) - (uint32_t)((r >> 16) & 0xffffu);
        lens[i] = (len + 1u) & ~1u;        // records take whole pairs of stream positions
    }
}

// Work order of the units (key ascending, stable, value: unit id).
// - A launch of one stack: units holding more than four times the mean sample count first,
//   largest first (they bound the end of the launch); every other unit after them in unit
//   order (uv tile by tile, rest-channel block fastest), so that units which share rows,
//   and the cache lines where a row's records meet, run close together in time.
//   key: 0x7fffffff - samples for the large units, 0x80000000 for the rest.
// - A launch of several stacks: every unit by decreasing sample count.  Such stacks differ
//   in size by orders of magnitude, most of their units are small, and balancing the end of
//   the launch with the smallest units matters more than locality.  key: ~samples.
__global__ void k_unit_keys(const LaunchDesc* __restrict__ Lp, const uint32_t* __restrict__ unit_off,
                            const uint64_t* __restrict__ pre, const int64_t* __restrict__ nunits_dev,
                            uint32_t* __restrict__ keys, uint64_t* __restrict__ vals) {
    const int64_t nun = *nunits_dev;
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < nun) {
        const uint64_t ns = pre[unit_off[u + 1]] - pre[unit_off[u]];
        if (Lp->nstacks > 1) {
            keys[u] = 0xffffffffu - (uint32_t)min(ns, (uint64_t)0xffffffffu);
        } else {
            const uint64_t tot = pre[unit_off[nun]] - pre[unit_off[0]];
            const bool large = (double)ns * (double)nun > 4.0 * (double)tot;
            keys[u] = large ? 0x7fffffffu - (uint32_t)min(ns, (uint64_t)0x7fffffffu) : 0x80000000u;
        }
        vals[u] = (uint64_t)u;
    }
}

}  // namespace

hipError_t launch_record_prefix(const uint64_t* recs, const int64_t* nrec_dev, int64_t nrec_cap, uint32_t* lens,
                                uint64_t* pre, uint64_t* sums, hipStream_t stream) {
    if (nrec_cap > 0)
        hipLaunchKernelGGL(k_record_lens, dim3((unsigned)((nrec_cap + 255) / 256)), dim3(256), 0, stream, recs,
                           nrec_dev, lens);
    return exclusive_scan_u32_to_u64(lens, nrec_dev, nrec_cap, pre, sums, stream);
}

hipError_t launch_unit_order(const LaunchDesc* dL, const uint32_t* unit_off, const uint64_t* pre,
                             const int64_t* nunits_dev, int64_t nunits_cap, uint32_t* keys, uint64_t* vals,
                             void* sort_temp, hipStream_t stream) {
    if (nunits_cap <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_unit_keys, dim3((unsigned)((nunits_cap + 255) / 256)), dim3(256), 0, stream, dL, unit_off,
                       pre, nunits_dev, keys, vals);
    return radix_sort_pairs(keys, vals, nunits_dev, nunits_cap, 32, sort_temp, stream);
}

// Launch shapes (tile_u, tile_v, jblock) of the FP64-sum form (28 B of LDS per cell) ...
#define VISTA_PACKED_SHAPES(X) \
    X(8, 8, 64)                \
    X(16, 4, 64)               \
    X(16, 8, 32)               \
    X(8, 4, 128)               \
    X(16, 2, 128)              \
    X(4, 4, 256)               \
    X(8, 2, 256)               \
    X(4, 2, 512)               \
    X(4, 4, 128)               \
    X(8, 4, 64)                \
    X(8, 2, 128)               \
    X(4, 2, 256)               \
    X(16, 2, 160)              \
    X(8, 2, 320)               \
    X(8, 4, 160)

// ... and of the plain FP32 form (16 B per cell): units up to 1.75 times larger, and
// smaller ones that let two workgroups share a compute unit.
#define VISTA_PACKED_SHAPES_F32(X) \
    X(8, 4, 288)                   \
    X(16, 4, 144)                  \
    X(8, 8, 144)                   \
    X(16, 2, 288)                  \
    X(4, 4, 576)                   \
    X(8, 2, 576)                   \
    X(16, 8, 64)                   \
    X(8, 4, 128)                   \
    X(8, 4, 144)                   \
    X(16, 4, 64)

static size_t packed_lds_bytes(int tu, int tv, int jc, int acc32) {
    return (size_t)tu * tv * (jc + 1) * (acc32 ? 16 : 28) + 16;
}

int accum_packed_shape_list(int acc32, int* tu, int* tv, int* jc, int cap) {
    int n = 0;
#define X(a, b, c)            \
    if (n < cap) {            \
        tu[n] = a; tv[n] = b; jc[n] = c; \
    }                         \
    ++n;
    if (acc32) {
        VISTA_PACKED_SHAPES_F32(X)
    } else {
        VISTA_PACKED_SHAPES(X)
    }
#undef X
    return n;
}

size_t accum_packed_lds_bytes(int tu, int tv, int jc, int acc32) { return packed_lds_bytes(tu, tv, jc, acc32); }

bool accum_packed_shape_supported(int tu, int tv, int jc, int waves, int acc32) {
    if (waves < 1 || waves > 16) return false;
#define X(a, b, c) \
    if (tu == a && tv == b && jc == c) return packed_lds_bytes(a, b, c, acc32) <= 160 * 1024;
    if (acc32) {
        VISTA_PACKED_SHAPES_F32(X)
    } else {
        VISTA_PACKED_SHAPES(X)
    }
#undef X
    return false;
}

hipError_t launch_accum_packed(const LaunchDesc& L, const LaunchDesc* dL, const uint64_t* order, uint32_t* counter,
                               const uint32_t* unit_off, const uint64_t* recs, const uint64_t* pre, int grid, int waves,
                               int npol, int acc32, int agg, hipStream_t stream) {
    if (!accum_packed_shape_supported(L.tu, L.tv, L.jc, waves, acc32)) return hipErrorInvalidValue;
#define X_LAUNCH(a, b, c, P, ACC, G)                                                                             \
    hipLaunchKernelGGL((k_accum_packed<a, b, c, P, ACC, G>), dim3(grid), dim3(waves * kWave), 0, stream, dL,   \
                       order, counter, unit_off, recs, pre)
#define X_ACC(a, b, c, ACC)                                                                                     \
    if (L.tu == a && L.tv == b && L.jc == c) {                                                                  \
        if (npol == 2) {                                                                                        \
            if (agg) X_LAUNCH(a, b, c, 2, ACC, true);                                                           \
            else X_LAUNCH(a, b, c, 2, ACC, false);                                                              \
        } else {                                                                                                \
            if (agg) X_LAUNCH(a, b, c, 0, ACC, true);                                                           \
            else X_LAUNCH(a, b, c, 0, ACC, false);                                                              \
        }                                                                                                       \
        return hipGetLastError();                                                                               \
    }
#define X64(a, b, c) X_ACC(a, b, c, double)
#define X32(a, b, c) X_ACC(a, b, c, float)
    if (acc32) {
        VISTA_PACKED_SHAPES_F32(X32)
    } else {
        VISTA_PACKED_SHAPES(X64)
    }
#undef X64
#undef X32
#undef X_ACC
#undef X_LAUNCH
    return hipErrorInvalidValue;
}

int accum_packed_max_blocks_per_cu(int tu, int tv, int jc, int waves, int npol, int acc32, int agg) {
    if (!accum_packed_shape_supported(tu, tv, jc, waves, acc32)) return 0;
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define X_OCC(a, b, c, P, ACC, G) \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_accum_packed<a, b, c, P, ACC, G>, waves * kWave, 0)
#define X_ACC(a, b, c, ACC)                                           \
    if (tu == a && tv == b && jc == c) {                              \
        if (npol == 2) {                                              \
            if (agg) X_OCC(a, b, c, 2, ACC, true);                    \
            else X_OCC(a, b, c, 2, ACC, false);                       \
        } else {                                                      \
            if (agg) X_OCC(a, b, c, 0, ACC, true);                    \
            else X_OCC(a, b, c, 0, ACC, false);                       \
        }                                                             \
        return e == hipSuccess ? nb : 0;                              \
    }
#define X64(a, b, c) X_ACC(a, b, c, double)
#define X32(a, b, c) X_ACC(a, b, c, float)
    if (acc32) {
        VISTA_PACKED_SHAPES_F32(X32)
    } else {
        VISTA_PACKED_SHAPES(X64)
    }
#undef X64
#undef X32
#undef X_ACC
#undef X_OCC
    return 0;
}

// Launch shapes (tile_u, tile_v, jblock) of the ordered kernel: 32 B of LDS per cell (FP64
// sums, or FP32 sums with their compensations; a count; a bid slot).
// Small tiles first: at 32 B a cell, 2 x 2 x 64 and the other 8 KB shapes let sixteen
// one-wavefront workgroups share a compute unit, each wavefront owning a whole block (no
// wavefront walks records for channels another one adds); the larger shapes serve wider
// workgroups.
#define VISTA_ORDERED_SHAPES(X) \
    X(2, 2, 64)                 \
    X(2, 1, 128)                \
    X(1, 2, 128)                \
    X(1, 1, 256)                \
    X(2, 2, 128)                \
    X(2, 1, 256)                \
    X(2, 2, 256)                \
    X(4, 2, 256)                \
    X(2, 2, 512)                \
    X(4, 2, 512)                \
    X(8, 4, 128)                \
    X(8, 8, 64)

static size_t ordered_lds_bytes(int tu, int tv, int jc) { return (size_t)tu * tv * (jc + 1) * 32 + 16; }

int accum_shape_list(int mode, int* tu, int* tv, int* jc, int cap) {
    if (mode == kModeAtomic) return accum_packed_shape_list(0, tu, tv, jc, cap);
    int n = 0;
#define X(a, b, c)            \
    if (n < cap) {            \
        tu[n] = a; tv[n] = b; jc[n] = c; \
    }                         \
    ++n;
    VISTA_ORDERED_SHAPES(X)
#undef X
    return n;
}

size_t accum_lds_bytes(int tu, int tv, int jc, int mode, int kahan) { return ordered_lds_bytes(tu, tv, jc); }

bool accum_shape_supported(int tu, int tv, int jc, int waves, int mode, int kahan) {
    if (mode != kModeOrdered || waves < 1 || waves > 16 || (jc % waves) != 0) return false;
#define X(a, b, c) \
    if (tu == a && tv == b && jc == c) return ordered_lds_bytes(a, b, c) <= 160 * 1024;
    VISTA_ORDERED_SHAPES(X)
#undef X
    return false;
}

// npol: 2 for launches whose targets all have two polarisations and row weights (the
// specialised path); anything else selects the generic path.
hipError_t launch_accum_impl(const LaunchDesc& L, const LaunchDesc* dL, const uint64_t* order,
                             uint32_t* counter, const uint32_t* unit_off, const uint64_t* recs, int grid,
                             int waves, int npol, hipStream_t stream) {
    if (!accum_shape_supported(L.tu, L.tv, L.jc, waves, L.mode, L.kahan)) return hipErrorInvalidValue;
#define X_LAUNCH(a, b, c, P, K)                                                                               \
    hipLaunchKernelGGL((k_accum_ordered<a, b, c, P, K>), dim3(grid), dim3(waves * kWave), 0, stream, dL,     \
                       order, counter, unit_off, recs)
#define X(a, b, c)                                                                                            \
    if (L.tu == a && L.tv == b && L.jc == c) {                                                                \
        if (L.kahan) {                                                                                        \
            if (npol == 2) X_LAUNCH(a, b, c, 2, true);                                                        \
            else X_LAUNCH(a, b, c, 0, true);                                                                  \
        } else {                                                                                              \
            if (npol == 2) X_LAUNCH(a, b, c, 2, false);                                                       \
            else X_LAUNCH(a, b, c, 0, false);                                                                 \
        }                                                                                                     \
        return hipGetLastError();                                                                             \
    }
    VISTA_ORDERED_SHAPES(X)
#undef X
#undef X_LAUNCH
    return hipErrorInvalidValue;
}

int accum_max_blocks_per_cu(int tu, int tv, int jc, int waves, int mode, int kahan, int npol) {
    if (!accum_shape_supported(tu, tv, jc, waves, mode, kahan)) return 0;
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
#define X_OCC(a, b, c, P, K) \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_accum_ordered<a, b, c, P, K>, waves * kWave, 0)
#define X(a, b, c)                                     \
    if (tu == a && tv == b && jc == c) {               \
        if (kahan) {                                   \
            if (npol == 2) X_OCC(a, b, c, 2, true);    \
            else X_OCC(a, b, c, 0, true);              \
        } else {                                       \
            if (npol == 2) X_OCC(a, b, c, 2, false);   \
            else X_OCC(a, b, c, 0, false);             \
        }                                              \
        return e == hipSuccess ? nb : 0;               \
    }
    VISTA_ORDERED_SHAPES(X)
#undef X
#undef X_OCC
    return 0;
}

}  // namespace vista
