// gfx950 kernels of the ViSta stacking hot path.
//
//   track_count / track_emit  -- binning: each row's channels, walked in frequency
//       order, trace a radial line in uv (u_lambda = u_m nu/c); the cells along it are
//       monotone, so the channels that fall in one uv tile form one contiguous range.
//       Each (row, tile) range becomes one record, keyed by the tile.
//   sort / tile_offsets       -- stable grouping of the records by tile.
//   accum                     -- one workgroup owns one (uv tile, rest-channel block) of
//       the grid state in LDS at a time, streams the tile's records (contiguous channel
//       runs of one row), applies the Eq. 2 phase shift with the phase argument formed
//       and range-reduced in FP64, splits every sample over the rest channels with the
//       Eq. 3-4 fractions, accumulates in LDS, and writes its cells once.
//
// Cell and channel indices follow the FP64 operation sequence of the definition exactly
// (this file is compiled with -ffp-contract=off, no fast-math): u = u_m * a_k,
// iu = rint(u * (1/du)) + nu/2.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "vista_internal.h"

namespace vista {

namespace {

constexpr int kWave = 64;

__device__ __forceinline__ int64_t find_le(const int64_t* base, int32_t n, int64_t x) {
    // largest i in [0, n) with base[i] <= x (base non-decreasing, base[0] <= x)
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        int32_t mid = (lo + hi) >> 1;
        if (base[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

// rint((c * a) * inv): the nearest-cell coordinate of the definition (two roundings,
// then round half to even).
__device__ __forceinline__ double cell_coord(double c, double a, double inv) {
    double x = c * a;
    return rint(x * inv);
}

// First k in [lo, hi) with s * rint((c * a_k) * inv) >= A, or hi.  The key is
// non-decreasing in k for the given orientation s.
__device__ int32_t first_at_least(const DevChan* ch, int32_t lo, int32_t hi, double c, double inv,
                                  double s, double A) {
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        double key = s * cell_coord(c, ch[mid].a, inv);
        if (key >= A) hi = mid; else lo = mid + 1;
    }
    return lo;
}

struct Track {
    int32_t ga, gb;     // in-grid channel interval
    double su, sv;      // orientation of the u and v cell sequences
};

// In-grid interval of row (U, V) over channels [klo, khi).
__device__ Track in_grid(const DevChan* ch, int32_t klo, int32_t khi, double U, double V,
                         double inv_du, double inv_dv, int32_t nu, int32_t nv) {
    Track t;
    double u0 = cell_coord(U, ch[klo].a, inv_du), u1 = cell_coord(U, ch[khi - 1].a, inv_du);
    double v0 = cell_coord(V, ch[klo].a, inv_dv), v1 = cell_coord(V, ch[khi - 1].a, inv_dv);
    t.su = (u1 >= u0) ? 1.0 : -1.0;
    t.sv = (v1 >= v0) ? 1.0 : -1.0;
    // inside: -(n/2) <= r < n - n/2.  With key = s r: s>0 -> [lo_b, hi_b);
    // s<0 -> key in (-hi_b, -lo_b] = [1 - hi_b, 1 - lo_b) for integer-valued keys.
    double lob_u = -(double)(nu / 2), hib_u = (double)(nu - nu / 2);
    double lob_v = -(double)(nv / 2), hib_v = (double)(nv - nv / 2);
    double Au = t.su > 0 ? lob_u : 1.0 - hib_u, Bu = t.su > 0 ? hib_u : 1.0 - lob_u;
    double Av = t.sv > 0 ? lob_v : 1.0 - hib_v, Bv = t.sv > 0 ? hib_v : 1.0 - lob_v;
    int32_t a1 = first_at_least(ch, klo, khi, U, inv_du, t.su, Au);
    int32_t b1 = first_at_least(ch, a1, khi, U, inv_du, t.su, Bu);
    int32_t a2 = first_at_least(ch, klo, khi, V, inv_dv, t.sv, Av);
    int32_t b2 = first_at_least(ch, a2, khi, V, inv_dv, t.sv, Bv);
    t.ga = max(a1, a2);
    t.gb = min(b1, b2);
    if (t.gb < t.ga) t.gb = t.ga;
    return t;
}

// End (exclusive) of the run of channels starting at k that stay in k's uv tile.
__device__ int32_t tile_run_end(const DevChan* ch, int32_t k, int32_t gb, double U, double V,
                                double inv_du, double inv_dv, int32_t nu, int32_t nv, int32_t TU,
                                int32_t TV, const Track& tr, int32_t* tile_u, int32_t* tile_v) {
    double ru = cell_coord(U, ch[k].a, inv_du), rv = cell_coord(V, ch[k].a, inv_dv);
    int32_t iu = (int32_t)ru + nu / 2, iv = (int32_t)rv + nv / 2;
    int32_t tu = iu / TU, tv = iv / TV;
    *tile_u = tu;
    *tile_v = tv;
    // leave the tile upward: r >= (t+1) T - n/2; downward: r < t T - n/2, i.e.
    // -r >= -(t T - n/2) + 1.
    double Au = tr.su > 0 ? (double)((tu + 1) * TU - nu / 2) : (double)(-(tu * TU - nu / 2) + 1);
    double Av = tr.sv > 0 ? (double)((tv + 1) * TV - nv / 2) : (double)(-(tv * TV - nv / 2) + 1);
    int32_t nu_k = first_at_least(ch, k + 1, gb, U, inv_du, tr.su, Au);
    int32_t nv_k = first_at_least(ch, k + 1, gb, V, inv_dv, tr.sv, Av);
    return min(nu_k, nv_k);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// ----------------------------------------------------------------------------- binning

__global__ void __launch_bounds__(256) k_track(const LaunchDesc* __restrict__ Lp,
                                               uint64_t* __restrict__ seg_count,
                                               const uint64_t* __restrict__ seg_off,
                                               uint32_t* __restrict__ keys,
                                               uint64_t* __restrict__ vals, int emit) {
    const LaunchDesc& L = *Lp;
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long outside = 0;
    int32_t stack_id = -1;
    if (g < L.nrows) {
        int32_t ti = (int32_t)find_le(L.target_row_base, L.ntargets, g);
        const DevTarget& T = L.targets[ti];
        const DevStack& S = L.stacks[T.stack];
        stack_id = T.stack;
        int64_t r = g - T.row_base;
        uint64_t n = 0;
        if (T.kin_lo < T.kin_hi) {
            double U = T.uvw[3 * r], V = T.uvw[3 * r + 1];
            Track tr = in_grid(T.chan, T.kin_lo, T.kin_hi, U, V, S.inv_du, S.inv_dv, S.nu, S.nv);
            int32_t inb_all = T.inband[T.kin_hi] - T.inband[T.kin_lo];
            int32_t inb_in = T.inband[tr.gb] - T.inband[tr.ga];
            outside = (unsigned long long)(inb_all - inb_in) * (unsigned long long)T.npol;
            uint64_t base = emit ? seg_off[g] : 0;
            int32_t k = tr.ga;
            while (k < tr.gb) {
                int32_t tu, tv;
                int32_t k1 = tile_run_end(T.chan, k, tr.gb, U, V, S.inv_du, S.inv_dv, S.nu, S.nv, L.tu,
                                          L.tv, tr, &tu, &tv);
                if (emit) {
                    keys[base + n] = (uint32_t)(S.tile_base + (int64_t)tv * S.tiles_u + tu);
                    vals[base + n] = ((uint64_t)g << 32) | ((uint64_t)k << 16) | (uint64_t)k1;
                }
                ++n;
                k = k1;
            }
        }
        if (!emit) seg_count[g] = n;
    }
    if (!emit) {
        // outside-uv samples: one atomic per wave and stack run (waves rarely straddle
        // two stacks; lanes of another stack add their own share)
        int32_t first = __shfl(stack_id, 0, kWave);
        unsigned long long mine = (stack_id == first) ? outside : 0ull;
        unsigned long long tot = wave_sum_u64(mine);
        if ((threadIdx.x & (kWave - 1)) == 0 && first >= 0 && tot) atomicAdd(&L.stacks[first].stats[3], tot);
        if (stack_id >= 0 && stack_id != first && outside) atomicAdd(&L.stacks[stack_id].stats[3], outside);
    }
}

__global__ void k_tile_offsets(const uint32_t* __restrict__ keys, int64_t nrec, int64_t ntiles,
                               uint32_t* __restrict__ off, uint64_t* __restrict__ cost,
                               const uint64_t* __restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > nrec) return;
    int64_t prev = (i == 0) ? -1 : (int64_t)keys[i - 1];
    int64_t cur = (i == nrec) ? ntiles : (int64_t)keys[i];
    for (int64_t t = prev + 1; t <= cur && t <= ntiles; ++t) off[t] = (uint32_t)i;
    if (i < nrec && cost) {
        uint64_t v = vals[i];
        atomicAdd((unsigned long long*)&cost[cur], (unsigned long long)((v & 0xffff) - ((v >> 16) & 0xffff)));
    }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, unsigned long long v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------------ accumulation

// Phase of one channel: the Eq. 2 turns t = (u l + v m + w (n-1)) = trow * a, reduced
// to [-1/2, 1/2] in FP64, then sin/cos of 2 pi r in FP32.
__device__ __forceinline__ void phasor(double trow, double a, float* c, float* s) {
    double t = trow * a;
    double r = t - rint(t);
    float x = (float)r;
    sincospif(2.0f * x, s, c);
}

__device__ __forceinline__ void phasor_fp32(float u, float v, float w, float l, float m, float nm1,
                                            float* c, float* s) {
    float t = u * l + v * m + w * nm1;
    sincosf(6.2831853071795864769f * t, s, c);
}

struct Sample {
    float pr, pi, q;    // sum_p w_p V'_p (rotated), sum_p w_p
    uint32_t n;         // used polarisations
    uint32_t nflag, nbad;
    int32_t lu, lv;     // cell within the tile
    int32_t j0, nj, foff;
};

// Load, rotate and merge the polarisations of channel k of row r.
__device__ __forceinline__ void load_sample(const DevTarget& T, int64_t r, int32_t k, double U, double V,
                                            double Wm, double trow, double inv_du, double inv_dv,
                                            int32_t nu, int32_t nv, int32_t tu0, int32_t tv0,
                                            const float* wrow, int phase_fp32, Sample& sm) {
    DevChan ce = T.chan[k];
    sm.j0 = ce.j0;
    sm.nj = ce.nj;
    sm.foff = ce.foff;
    double ru = cell_coord(U, ce.a, inv_du), rv = cell_coord(V, ce.a, inv_dv);
    sm.lu = (int32_t)ru + nu / 2 - tu0;
    sm.lv = (int32_t)rv + nv / 2 - tv0;
    const int npol = T.npol;
    size_t e = ((size_t)r * T.nchan + k) * npol;
    float vr[4], vi[4], wt[4];
    uint32_t fl = 0;
    if (npol == 2) {
        float4 x = *(const float4*)(T.vis + e);
        vr[0] = x.x; vi[0] = x.y; vr[1] = x.z; vi[1] = x.w;
        if (T.flag) fl = *(const uint16_t*)(T.flag + e);
    } else if (npol == 1) {
        float2 x = T.vis[e];
        vr[0] = x.x; vi[0] = x.y;
        if (T.flag) fl = T.flag[e];
    } else {
        float4 x = *(const float4*)(T.vis + e);
        float4 y = *(const float4*)(T.vis + e + 2);
        vr[0] = x.x; vi[0] = x.y; vr[1] = x.z; vi[1] = x.w;
        vr[2] = y.x; vi[2] = y.y; vr[3] = y.z; vi[3] = y.w;
        if (T.flag) fl = *(const uint32_t*)(T.flag + e);
    }
    if (T.weight_per_chan) {
        for (int p = 0; p < npol; ++p) wt[p] = T.weight[e + p];
    } else {
        for (int p = 0; p < npol; ++p) wt[p] = wrow[p];
    }
    float ar = 0.f, ai = 0.f, q = 0.f;
    uint32_t n = 0, nflag = 0, nbad = 0;
    for (int p = 0; p < npol; ++p) {
        bool flagged = ((fl >> (8 * p)) & 0xffu) != 0u;
        float w = wt[p];
        bool good = (w > 0.0f) && (w < __builtin_inff());
        if (flagged) { ++nflag; continue; }
        if (!good) { ++nbad; continue; }
        ar = fmaf(w, vr[p], ar);
        ai = fmaf(w, vi[p], ai);
        q += w;
        ++n;
    }
    float c, s;
    if (phase_fp32) {
        float a32 = (float)ce.a;
        phasor_fp32((float)U * a32, (float)V * a32, (float)Wm * a32, (float)T.l, (float)T.m, (float)T.nm1,
                    &c, &s);
    } else {
        phasor(trow, ce.a, &c, &s);
    }
    sm.pr = ar * c - ai * s;
    sm.pi = fmaf(ar, s, ai * c);
    sm.q = q;
    sm.n = n;
    sm.nflag = nflag;
    sm.nbad = nbad;
}

template <int TU, int TV, int JC, int MODE, bool KAHAN>
struct AccumShape {
    static constexpr int JP = JC + 1;                 // padded channel stride
    static constexpr int NC = TU * TV * JP;           // LDS cells
    static constexpr int NARR = KAHAN ? 7 : 4;
    static constexpr size_t LDS = (size_t)NC * NARR * 4;
};

template <int TU, int TV, int JC, int MODE, bool KAHAN>
__global__ void __launch_bounds__(512) k_accum(const LaunchDesc* __restrict__ Lp,
                                               const uint2* __restrict__ units, int64_t nunits,
                                               uint32_t* __restrict__ counter,
                                               const uint32_t* __restrict__ tile_off,
                                               const uint64_t* __restrict__ recs) {
    using Sh = AccumShape<TU, TV, JC, MODE, KAHAN>;
    constexpr int JP = Sh::JP;
    constexpr int NC = Sh::NC;
    __shared__ float s_re[NC], s_im[NC], s_w[NC];
    __shared__ uint32_t s_n[NC];
    __shared__ float c_re[KAHAN ? NC : 1], c_im[KAHAN ? NC : 1], c_w[KAHAN ? NC : 1];
    __shared__ uint32_t s_unit;

    const LaunchDesc& L = *Lp;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;

    for (;;) {
        if (threadIdx.x == 0) s_unit = atomicAdd(counter, 1u);
        __syncthreads();
        uint32_t ui = s_unit;
        if (ui >= nunits) break;
        uint2 un = units[ui];
        int64_t gtile = un.x;
        int32_t b = (int32_t)un.y;
        int32_t si = (int32_t)find_le(L.stack_tile_base, L.nstacks, gtile);
        const DevStack& S = L.stacks[si];
        int64_t tile = gtile - S.tile_base;
        int32_t tu0 = (int32_t)(tile % S.tiles_u) * TU;
        int32_t tv0 = (int32_t)(tile / S.tiles_u) * TV;
        int32_t jb0 = b * JC;
        int32_t jb1 = min(jb0 + JC, S.nchan);

        for (int i = threadIdx.x; i < NC; i += blockDim.x) {
            s_re[i] = 0.f; s_im[i] = 0.f; s_w[i] = 0.f; s_n[i] = 0u;
            if (KAHAN) { c_re[i] = 0.f; c_im[i] = 0.f; c_w[i] = 0.f; }
        }
        __syncthreads();

        uint32_t rb = tile_off[gtile], re = tile_off[gtile + 1];
        // channel sub-range this wave adds into: the whole block (atomic mode) or the
        // wave's own slice of it (ordered mode: cells are never shared between waves)
        int32_t js0, js1, bi;
        uint32_t r_first, r_step;
        if (MODE == kModeOrdered) {
            int32_t jsub = L.jsub;
            js0 = jb0 + wave * jsub;
            js1 = min(js0 + jsub, jb1);
            bi = jb0 / jsub + wave;
            r_first = rb;
            r_step = 1;
        } else {
            js0 = jb0;
            js1 = jb1;
            bi = b;
            r_first = rb + wave;
            r_step = nw;
        }
        unsigned long long st_flag = 0, st_bad = 0, st_used = 0, st_contrib = 0;
        if (js0 < js1) {
            for (uint32_t ri = r_first; ri < re; ri += r_step) {
                uint64_t rec = recs[ri];
                int64_t g = (int64_t)(rec >> 32);
                int32_t kin = (int32_t)((rec >> 16) & 0xffff), kout = (int32_t)(rec & 0xffff);
                int32_t ti = (int32_t)find_le(L.target_row_base, L.ntargets, g);
                const DevTarget& T = L.targets[ti];
                int32_t ka = max(kin, T.blk[2 * bi]), kb = min(kout, T.blk[2 * bi + 1]);
                if (ka >= kb) continue;
                int64_t r = g - T.row_base;
                double U = T.uvw[3 * r], V = T.uvw[3 * r + 1], Wm = T.uvw[3 * r + 2];
                double trow = U * T.l + V * T.m + Wm * T.nm1;
                float wrow[4] = {0.f, 0.f, 0.f, 0.f};
                if (!T.weight_per_chan)
                    for (int p = 0; p < T.npol; ++p) wrow[p] = T.weight[(size_t)r * T.npol + p];
                const int nph = (MODE == kModeOrdered) ? T.nphase : 1;
                for (int32_t k0 = ka; k0 < kb; k0 += kWave) {
                    int32_t k = k0 + lane;
                    bool act = k < kb;
                    Sample sm;
                    sm.nj = 0;
                    sm.n = 0;
                    if (act) {
                        load_sample(T, r, k, U, V, Wm, trow, S.inv_du, S.inv_dv, S.nu, S.nv, tu0, tv0, wrow,
                                    L.phase_fp32, sm);
                        // a record's channels all lie in this tile; anything else is a bug
                        if (sm.lu < 0 || sm.lu >= TU || sm.lv < 0 || sm.lv >= TV) { sm.nj = 0; sm.n = 0; }
                        // per-sample classification is counted in the block of j0
                        if (sm.nj > 0 && sm.j0 >= js0 && sm.j0 < js1) {
                            st_flag += sm.nflag;
                            st_bad += sm.nbad;
                            st_used += sm.n;
                        }
                    }
                    int32_t cell = (sm.lv * TU + sm.lu) * JP;
                    for (int ph = 0; ph < nph; ++ph) {
                        bool mine = act && sm.n > 0 && (MODE != kModeOrdered || ((k - k0) % nph) == ph);
                        if (mine) {
                            for (int q = 0; q < sm.nj; ++q) {
                                int32_t j = sm.j0 + q;
                                if (j < js0 || j >= js1) continue;
                                float f = T.fval[sm.foff + q];
                                int c = cell + (j - jb0);
                                float xr = f * sm.pr, xi = f * sm.pi, xw = f * sm.q;
                                st_contrib += sm.n;
                                if (MODE == kModeAtomic) {
                                    atomicAdd(&s_re[c], xr);
                                    atomicAdd(&s_im[c], xi);
                                    atomicAdd(&s_w[c], xw);
                                    atomicAdd(&s_n[c], sm.n);
                                } else if (!KAHAN) {
                                    s_re[c] += xr;
                                    s_im[c] += xi;
                                    s_w[c] += xw;
                                    s_n[c] += sm.n;
                                } else {
                                    float y, t;
                                    y = xr - c_re[c]; t = s_re[c] + y; c_re[c] = (t - s_re[c]) - y; s_re[c] = t;
                                    y = xi - c_im[c]; t = s_im[c] + y; c_im[c] = (t - s_im[c]) - y; s_im[c] = t;
                                    y = xw - c_w[c]; t = s_w[c] + y; c_w[c] = (t - s_w[c]) - y; s_w[c] = t;
                                    s_n[c] += sm.n;
                                }
                            }
                        }
                    }
                }
            }
        }
        // classification and contribution counts: one atomic per wave and unit
        st_flag = wave_sum_u64(st_flag);
        st_bad = wave_sum_u64(st_bad);
        st_used = wave_sum_u64(st_used);
        st_contrib = wave_sum_u64(st_contrib);
        if (lane == 0) {
            if (st_flag) atomicAdd(&S.stats[1], st_flag);
            if (st_bad) atomicAdd(&S.stats[2], st_bad);
            if (st_used) atomicAdd(&S.stats[5], st_used);
            if (st_contrib) atomicAdd(&S.stats[6], st_contrib);
            if (st_contrib > 0xffffffffull) atomicOr(&S.stats[7], 1ull);
        }
        __syncthreads();

        // write the (tile, block) cells: iu fastest, so stores are contiguous runs of TU
        const int ncv = (jb1 - jb0) * TV * TU;
        for (int i = threadIdx.x; i < ncv; i += blockDim.x) {
            int lu = i % TU;
            int lv = (i / TU) % TV;
            int jl = i / (TU * TV);
            int iu = tu0 + lu, iv = tv0 + lv;
            if (iu >= S.nu || iv >= S.nv) continue;
            int c = (lv * TU + lu) * JP + jl;
            size_t o = ((size_t)(jb0 + jl) * S.nv + iv) * S.nu + iu;
            double dre, dim, dw;
            if (KAHAN) {
                dre = (double)s_re[c] - (double)c_re[c];
                dim = (double)s_im[c] - (double)c_im[c];
                dw = (double)s_w[c] - (double)c_w[c];
            } else {
                dre = s_re[c]; dim = s_im[c]; dw = s_w[c];
            }
            uint32_t n = s_n[c];
            if (L.carry) {
                // merge into the state carried across waves (this unit owns the cells)
                size_t plane = (size_t)S.nchan * S.nv * S.nu;
                float* sp = S.st_s;
                float* cp = S.st_c;
                double vals3[3] = {dre, dim, dw};
                for (int q = 0; q < 3; ++q) {
                    float x = (float)vals3[q];
                    float sv = sp[q * plane + o];
                    if (L.kahan) {
                        float cc = cp[q * plane + o];
                        float xl = (float)(vals3[q] - (double)x);   // keep the part lost to FP32
                        float y = x - cc;
                        float t = sv + y;
                        cc = (t - sv) - y;
                        sv = t;
                        y = xl - cc; t = sv + y; cc = (t - sv) - y; sv = t;
                        cp[q * plane + o] = cc;
                        vals3[q] = (double)sv - (double)cc;
                    } else {
                        sv = sv + x;
                        vals3[q] = sv;
                    }
                    sp[q * plane + o] = sv;
                }
                uint64_t nn = (uint64_t)S.st_n[o] + n;
                if (nn > 0xffffffffull) atomicOr(&S.stats[7], 1ull);
                S.st_n[o] = (uint32_t)nn;
                if (!L.last_wave) continue;
                dre = vals3[0]; dim = vals3[1]; dw = vals3[2]; n = (uint32_t)nn;
            }
            if (S.out_vis) S.out_vis[o] = make_float2((float)dre, (float)dim);
            if (S.out_w) S.out_w[o] = (float)dw;
            if (S.out_cnt) S.out_cnt[o] = n;
            if (S.out_vis64) S.out_vis64[o] = make_double2(dre, dim);
            if (S.out_w64) S.out_w64[o] = dw;
        }
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
    double ru = cell_coord(T.uvw[3 * r], ce.a, S.inv_du);
    double rv = cell_coord(T.uvw[3 * r + 1], ce.a, S.inv_dv);
    iu[e] = fabs(ru) < 2.0e9 ? (int32_t)ru + S.nu / 2 : INT32_MIN;
    iv[e] = fabs(rv) < 2.0e9 ? (int32_t)rv + S.nv / 2 : INT32_MIN;
    j0[e] = ce.nj ? ce.j0 : -1;
    nj[e] = ce.nj;
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

hipError_t launch_track(const LaunchDesc& L, const LaunchDesc* dL, uint64_t* seg_count,
                        const uint64_t* seg_off, uint32_t* keys, uint64_t* vals, int emit,
                        hipStream_t stream) {
    if (L.nrows <= 0) return hipSuccess;
    int64_t blocks = (L.nrows + 255) / 256;
    hipLaunchKernelGGL(k_track, dim3((unsigned)blocks), dim3(256), 0, stream, dL, seg_count, seg_off, keys,
                       vals, emit);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, void* tmp,
                                     size_t* tmp_bytes, hipStream_t stream) {
    return hipcub::DeviceScan::ExclusiveSum(tmp, *tmp_bytes, in, out, (int)n, stream);
}

hipError_t launch_sort_pairs(const uint32_t* kin, uint32_t* kout, const uint64_t* vin, uint64_t* vout,
                             int64_t n, int end_bit, void* tmp, size_t* tmp_bytes, hipStream_t stream) {
    return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, kin, kout, vin, vout, (int)n, 0, end_bit,
                                              stream);
}

hipError_t launch_tile_offsets(const uint32_t* sorted_keys, int64_t nrec, int64_t ntiles, uint32_t* tile_off,
                               uint64_t* tile_cost, const uint64_t* vals, hipStream_t stream) {
    int64_t n = nrec + 1;
    hipLaunchKernelGGL(k_tile_offsets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, sorted_keys,
                       nrec, ntiles, tile_off, tile_cost, vals);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, unsigned long long v, int64_t n, hipStream_t stream) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, v, n);
    return hipGetLastError();
}

// Supported shapes (tile_u, tile_v, jblock).  The autotuner chooses among these.
#define VISTA_SHAPES(X) \
    X(8, 8, 64)          \
    X(16, 8, 32)         \
    X(16, 16, 16)        \
    X(8, 4, 128)         \
    X(4, 4, 256)

template <int TU, int TV, int JC, int MODE, bool KAHAN>
static hipError_t launch_one(const LaunchDesc* dL, const uint2* units, int64_t nunits, uint32_t* counter,
                             const uint32_t* tile_off, const uint64_t* recs, int grid, int waves,
                             hipStream_t stream) {
    hipLaunchKernelGGL((k_accum<TU, TV, JC, MODE, KAHAN>), dim3(grid), dim3(waves * kWave), 0, stream, dL,
                       units, nunits, counter, tile_off, recs);
    return hipGetLastError();
}

template <int TU, int TV, int JC, int MODE, bool KAHAN>
static int occ_one(int waves) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_accum<TU, TV, JC, MODE, KAHAN>, waves * kWave, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

size_t accum_lds_bytes(int tu, int tv, int jc, int mode, int kahan) {
    return (size_t)tu * tv * (jc + 1) * (kahan ? 7 : 4) * 4;
}

bool accum_shape_supported(int tu, int tv, int jc, int waves, int mode, int kahan) {
    if (waves < 1 || waves > 8) return false;
    if (kahan && mode != kModeOrdered) return false;
    if (mode == kModeOrdered && (jc % waves) != 0) return false;
#define X(a, b, c) if (tu == a && tv == b && jc == c) return accum_lds_bytes(a, b, c, mode, kahan) <= 160 * 1024;
    VISTA_SHAPES(X)
#undef X
    return false;
}

hipError_t launch_accum_impl(const LaunchDesc& L, const LaunchDesc* dL, const uint2* units, int64_t nunits,
                             uint32_t* counter, const uint32_t* tile_off, const uint64_t* recs, int grid,
                             int waves, hipStream_t stream) {
    if (!accum_shape_supported(L.tu, L.tv, L.jc, waves, L.mode, L.kahan)) return hipErrorInvalidValue;
#define X(a, b, c)                                                                                         \
    if (L.tu == a && L.tv == b && L.jc == c) {                                                             \
        if (L.mode == kModeAtomic)                                                                         \
            return launch_one<a, b, c, kModeAtomic, false>(dL, units, nunits, counter, tile_off, recs, grid, \
                                                           waves, stream);                                 \
        if (L.kahan)                                                                                       \
            return launch_one<a, b, c, kModeOrdered, true>(dL, units, nunits, counter, tile_off, recs, grid, \
                                                           waves, stream);                                 \
        return launch_one<a, b, c, kModeOrdered, false>(dL, units, nunits, counter, tile_off, recs, grid,   \
                                                        waves, stream);                                    \
    }
    VISTA_SHAPES(X)
#undef X
    return hipErrorInvalidValue;
}

int accum_max_blocks_per_cu(int tu, int tv, int jc, int waves, int mode, int kahan, int /*npol*/) {
    if (!accum_shape_supported(tu, tv, jc, waves, mode, kahan)) return 0;
#define X(a, b, c)                                                                   \
    if (tu == a && tv == b && jc == c) {                                             \
        if (mode == kModeAtomic) return occ_one<a, b, c, kModeAtomic, false>(waves); \
        if (kahan) return occ_one<a, b, c, kModeOrdered, true>(waves);               \
        return occ_one<a, b, c, kModeOrdered, false>(waves);                         \
    }
    VISTA_SHAPES(X)
#undef X
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
