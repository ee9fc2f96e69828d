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

// One (row, output channel) of a target with NPOL polarisations.
template <int NPOL>
__device__ __forceinline__ void rebin_one(const RebinTarget& T, int64_t r, int32_t j, double trow) {
    const int32_t e0 = gptr(T.jstart)[j], e1 = gptr(T.jstart)[j + 1];
    float nr[NPOL], ni[NPOL], dn[NPOL];
#pragma unroll
    for (int p = 0; p < NPOL; ++p) { nr[p] = 0.f; ni[p] = 0.f; dn[p] = 0.f; }
    const size_t rowbase = (size_t)r * T.nchan;
    for (int32_t e = e0; e < e1; ++e) {
        const int32_t k = gptr(T.ek)[e];
        const float f = gptr(T.ef)[e];
        float c, s;
        phasor(trow, gptr(T.a)[k], &c, &s);
        float vr[NPOL], vi[NPOL];
        uint32_t fl = 0;
        const size_t idx = rowbase + (size_t)k;
        if constexpr (NPOL == 1) {
            const float2 v = gptr(T.vis)[idx];
            vr[0] = v.x; vi[0] = v.y;
            if (T.flag) fl = gptr(T.flag)[idx];
        } else if constexpr (NPOL == 2) {
            const float4 v = gptr((const float4*)T.vis)[idx];
            vr[0] = v.x; vi[0] = v.y; vr[1] = v.z; vi[1] = v.w;
            if (T.flag) fl = gptr((const uint16_t*)T.flag)[idx];
        } else {
            const float4 v0 = gptr((const float4*)T.vis)[2 * idx];
            const float4 v1 = gptr((const float4*)T.vis)[2 * idx + 1];
            vr[0] = v0.x; vi[0] = v0.y; vr[1] = v0.z; vi[1] = v0.w;
            vr[2] = v1.x; vi[2] = v1.y; vr[3] = v1.z; vi[3] = v1.w;
            if (T.flag) fl = gptr((const uint32_t*)T.flag)[idx];
        }
#pragma unroll
        for (int p = 0; p < NPOL; ++p) {
            if ((fl >> (8 * p)) & 0xffu) continue;
            const float pr = vr[p] * c - vi[p] * s;
            const float pi = vr[p] * s + vi[p] * c;
            nr[p] = fmaf(f, pr, nr[p]);
            ni[p] = fmaf(f, pi, ni[p]);
            dn[p] += f;
        }
    }
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
    VISTA_GLOBAL float* ov = (VISTA_GLOBAL float*)T.out_vis;
    if constexpr (NPOL == 1) {
        ((VISTA_GLOBAL float2*)ov)[o] = make_float2(ovr[0], ovi[0]);
        if (T.out_flag) ((VISTA_GLOBAL uint8_t*)T.out_flag)[o] = (uint8_t)ofl;
        if (T.out_wsum) ((VISTA_GLOBAL float*)T.out_wsum)[o] = dn[0];
    } else if constexpr (NPOL == 2) {
        ((VISTA_GLOBAL float4*)ov)[o / 2] = make_float4(ovr[0], ovi[0], ovr[1], ovi[1]);
        if (T.out_flag) ((VISTA_GLOBAL uint16_t*)T.out_flag)[o / 2] = (uint16_t)ofl;
        if (T.out_wsum) ((VISTA_GLOBAL float2*)T.out_wsum)[o / 2] = make_float2(dn[0], dn[1]);
    } else {
        ((VISTA_GLOBAL float4*)ov)[o / 2] = make_float4(ovr[0], ovi[0], ovr[1], ovi[1]);
        ((VISTA_GLOBAL float4*)ov)[o / 2 + 1] = make_float4(ovr[2], ovi[2], ovr[3], ovi[3]);
        if (T.out_flag) ((VISTA_GLOBAL uint32_t*)T.out_flag)[o / 4] = ofl;
        if (T.out_wsum) ((VISTA_GLOBAL float4*)T.out_wsum)[o / 4] = make_float4(dn[0], dn[1], dn[2], dn[3]);
    }
}

// One workgroup per block of consecutive rows of one target (every target of the launch
// has NPOL polarisations).  The block's (row, output channel) pairs are walked in order,
// output channel fastest, one per thread at a time, so narrow windows still fill the
// workgroup.
template <int NPOL>
__global__ void __launch_bounds__(256) k_rebin_rows(const RebinTarget* __restrict__ targets,
                                                    const RebinBlock* __restrict__ blocks) {
    const RebinBlock B = cptr(blocks)[blockIdx.x];
    const RebinTarget& T = cptr(targets)[B.target];
    const int32_t nout = T.nout;
    const VISTA_GLOBAL double* uvw = gptr(T.uvw);
    int32_t rr = (int32_t)threadIdx.x / nout, j = (int32_t)threadIdx.x - rr * nout;
    while (rr < B.nrows) {
        const int64_t r = (int64_t)B.row0 + rr;
        const double U = uvw[3 * r], V = uvw[3 * r + 1], W = uvw[3 * r + 2];
        const double trow = U * T.l + V * T.m + W * T.nm1;   // Eq. 2 turns per unit a_k
        if (T.out_uvw && j == 0) {                              // Eq. 1 without the rotation
            VISTA_GLOBAL double* ou = (VISTA_GLOBAL double*)T.out_uvw;
            ou[3 * r] = U / T.opz;
            ou[3 * r + 1] = V / T.opz;
            ou[3 * r + 2] = W / T.opz;
        }
        rebin_one<NPOL>(T, r, j, trow);
        j += (int32_t)blockDim.x;
        if (j >= nout) {
            const int32_t q = j / nout;
            rr += q;
            j -= q * nout;
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
