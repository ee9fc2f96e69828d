// Per-row rebinned product: the paper's per-row kernel output (Sec. 3.2).
//
// Every row of every target is shifted to the target's position (Eq. 2) and rebinned onto
// the target's own output window (Sec. 3.1) by Eq. 3 with the Eq. 4 weights, normalised
// per row, output channel and polarisation; flagged inputs are left out.  The work is a
// plain stream over HBM -- each input row is read once and each output row written once --
// so the kernel is laid out for coalescing, not for the matrix cores: a workgroup takes a
// few consecutive rows of one target, and its threads take consecutive output channels, so
// the stores of a wavefront are one contiguous run and its loads (the few input channels
// overlapping 64 consecutive output channels) are too.  The per-output-channel lists of
// (input channel, fraction) are small per-target tables that stay in cache.
#include <hip/hip_runtime.h>

#include "vista_device.h"

namespace vista {

namespace {

// Loads of one input sample (row r, channel k): visibilities and flag bytes.
template <int NPOL>
struct Sample {
    float vr[NPOL], vi[NPOL];
    uint32_t fl;
};

template <int NPOL>
__device__ __forceinline__ void load_sample(const RebinTarget& T, size_t idx, Sample<NPOL>& x) {
    x.fl = 0;
    if constexpr (NPOL == 1) {
        const float2 v = gptr(T.vis)[idx];
        x.vr[0] = v.x; x.vi[0] = v.y;
        if (T.flag) x.fl = gptr(T.flag)[idx];
    } else if constexpr (NPOL == 2) {
        const float4 v = gptr((const float4*)T.vis)[idx];
        x.vr[0] = v.x; x.vi[0] = v.y; x.vr[1] = v.z; x.vi[1] = v.w;
        if (T.flag) x.fl = gptr((const uint16_t*)T.flag)[idx];
    } else {
        const float4 v0 = gptr((const float4*)T.vis)[2 * idx];
        const float4 v1 = gptr((const float4*)T.vis)[2 * idx + 1];
        x.vr[0] = v0.x; x.vi[0] = v0.y; x.vr[1] = v0.z; x.vi[1] = v0.w;
        x.vr[2] = v1.x; x.vi[2] = v1.y; x.vr[3] = v1.z; x.vi[3] = v1.w;
        if (T.flag) x.fl = gptr((const uint32_t*)T.flag)[idx];
    }
}

typedef float v2f32 __attribute__((ext_vector_type(2)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// Output (row r, channel j) from the Eq. 3 sums.  Outputs are written once and not read
// again here: streaming (nontemporal) stores keep them from displacing the inputs that
// neighbouring output channels still read from cache.
template <int NPOL>
__device__ __forceinline__ void store_out(const RebinTarget& T, int64_t r, int32_t j, const float* nr,
                                          const float* ni, const float* dn) {
    const size_t o = ((size_t)r * T.nout + j) * NPOL;
    float ovr[NPOL], ovi[NPOL];
    uint32_t ofl = 0;
#pragma unroll
    for (int p = 0; p < NPOL; ++p) {
        const bool ok = dn[p] > 0.f;
        ovr[p] = ok ? nr[p] / dn[p] : 0.f;
        ovi[p] = ok ? ni[p] / dn[p] : 0.f;
        ofl |= (ok ? 0u : 1u) << (8 * p);
    }
    if constexpr (NPOL == 1) {
        const v2f32 v = {ovr[0], ovi[0]};
        __builtin_nontemporal_store(v, (v2f32*)T.out_vis + o);
        if (T.out_flag) __builtin_nontemporal_store((uint8_t)ofl, T.out_flag + o);
        if (T.out_wsum) __builtin_nontemporal_store(dn[0], T.out_wsum + o);
    } else if constexpr (NPOL == 2) {
        const v4f32 v = {ovr[0], ovi[0], ovr[1], ovi[1]};
        __builtin_nontemporal_store(v, (v4f32*)T.out_vis + o / 2);
        if (T.out_flag) __builtin_nontemporal_store((uint16_t)ofl, (uint16_t*)T.out_flag + o / 2);
        const v2f32 w = {dn[0], dn[1]};
        if (T.out_wsum) __builtin_nontemporal_store(w, (v2f32*)T.out_wsum + o / 2);
    } else {
        const v4f32 v0 = {ovr[0], ovi[0], ovr[1], ovi[1]}, v1 = {ovr[2], ovi[2], ovr[3], ovi[3]};
        __builtin_nontemporal_store(v0, (v4f32*)T.out_vis + o / 2);
        __builtin_nontemporal_store(v1, (v4f32*)T.out_vis + o / 2 + 1);
        if (T.out_flag) __builtin_nontemporal_store(ofl, (uint32_t*)T.out_flag + o / 4);
        const v4f32 w = {dn[0], dn[1], dn[2], dn[3]};
        if (T.out_wsum) __builtin_nontemporal_store(w, (v4f32*)T.out_wsum + o / 4);
    }
}

// rows whose loads a thread issues together (fewer with four polarisations: registers)
template <int NPOL>
constexpr int kRowsInFlight = NPOL == 4 ? 4 : 8;

// One workgroup per block of consecutive rows of one target (every target of the launch
// has NPOL polarisations).  Its 256 threads form `ng` groups of J = min(nout, 256) threads;
// thread (group g, lane jl) takes output channels j = jl, jl + J, ... and, for each, rows
// row0 + g, row0 + g + ng, ...: it reads output channel j's list of (input channel,
// fraction) once and then walks the rows kRowsInFlight at a time, their loads issued
// together.
template <int NPOL>
__global__ void __launch_bounds__(256) k_rebin_rows(const RebinTarget* __restrict__ targets,
                                                    const RebinBlock* __restrict__ blocks) {
    const RebinBlock B = cptr(blocks)[blockIdx.x];
    const RebinTarget& T = cptr(targets)[B.target];
    const int32_t nout = T.nout;
    const int32_t J = min(nout, 256), ng = 256 / J;
    const int32_t g = (int32_t)threadIdx.x / J, jl = (int32_t)threadIdx.x - g * J;
    if (g >= ng) return;
    const VISTA_GLOBAL double* uvw = gptr(T.uvw);
    for (int32_t j = jl; j < nout; j += J) {
        const int32_t e0 = gptr(T.jstart)[j], e1 = gptr(T.jstart)[j + 1];
        for (int32_t rb = g; rb < B.nrows; rb += kRowsInFlight<NPOL> * ng) {
            double trow[kRowsInFlight<NPOL>];
            int64_t r[kRowsInFlight<NPOL>];
            bool live[kRowsInFlight<NPOL>];
#pragma unroll
            for (int q = 0; q < kRowsInFlight<NPOL>; ++q) {
                const int32_t rr = rb + q * ng;
                live[q] = rr < B.nrows;
                r[q] = (int64_t)B.row0 + (live[q] ? rr : rb);
                const double U = uvw[3 * r[q]], V = uvw[3 * r[q] + 1], W = uvw[3 * r[q] + 2];
                trow[q] = U * T.l + V * T.m + W * T.nm1;     // Eq. 2 turns per unit a_k
                if (T.out_uvw && j == 0 && live[q]) {         // Eq. 1: R (u, v, w) / (1 + z)
                    VISTA_GLOBAL double* ou = (VISTA_GLOBAL double*)T.out_uvw;
                    if (T.rotate) {
                        for (int i = 0; i < 3; ++i)
                            ou[3 * r[q] + i] = (T.R[3 * i] * U + T.R[3 * i + 1] * V + T.R[3 * i + 2] * W) / T.opz;
                    } else {
                        ou[3 * r[q]] = U / T.opz;
                        ou[3 * r[q] + 1] = V / T.opz;
                        ou[3 * r[q] + 2] = W / T.opz;
                    }
                }
            }
            float nr[kRowsInFlight<NPOL>][NPOL], ni[kRowsInFlight<NPOL>][NPOL], dn[kRowsInFlight<NPOL>][NPOL];
#pragma unroll
            for (int q = 0; q < kRowsInFlight<NPOL>; ++q)
#pragma unroll
                for (int p = 0; p < NPOL; ++p) { nr[q][p] = 0.f; ni[q][p] = 0.f; dn[q][p] = 0.f; }
            for (int32_t e = e0; e < e1; ++e) {
                const int32_t k = gptr(T.ek)[e];
                const float f = gptr(T.ef)[e];
                const double a = gptr(T.a)[k];
                Sample<NPOL> x[kRowsInFlight<NPOL>];
#pragma unroll
                for (int q = 0; q < kRowsInFlight<NPOL>; ++q) load_sample<NPOL>(T, (size_t)r[q] * T.nchan + k, x[q]);
#pragma unroll
                for (int q = 0; q < kRowsInFlight<NPOL>; ++q) {
                    float c, s;
                    phasor(trow[q], a, &c, &s);
#pragma unroll
                    for (int p = 0; p < NPOL; ++p) {
                        if ((x[q].fl >> (8 * p)) & 0xffu) continue;
                        const float pr = x[q].vr[p] * c - x[q].vi[p] * s;
                        const float pi = x[q].vr[p] * s + x[q].vi[p] * c;
                        nr[q][p] = fmaf(f, pr, nr[q][p]);
                        ni[q][p] = fmaf(f, pi, ni[q][p]);
                        dn[q][p] += f;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kRowsInFlight<NPOL>; ++q)
                if (live[q]) store_out<NPOL>(T, r[q], j, nr[q], ni[q], dn[q]);
        }
    }
}

}  // namespace

hipError_t launch_rebin_rows(const RebinTarget* targets, const RebinBlock* blocks, int64_t nblocks, int npol,
                             hipStream_t stream) {
    if (nblocks <= 0) return hipSuccess;
    if (nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nblocks), block(256);
    if (npol == 1)
        hipLaunchKernelGGL(k_rebin_rows<1>, grid, block, 0, stream, targets, blocks);
    else if (npol == 2)
        hipLaunchKernelGGL(k_rebin_rows<2>, grid, block, 0, stream, targets, blocks);
    else if (npol == 4)
        hipLaunchKernelGGL(k_rebin_rows<4>, grid, block, 0, stream, targets, blocks);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace vista
