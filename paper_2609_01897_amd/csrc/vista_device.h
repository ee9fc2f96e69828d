// Device helpers shared by the binning and accumulation kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// (The host compilation pass only parses device code; address spaces exist on the device.)
#if defined(__HIP_DEVICE_COMPILE__)
#define VISTA_GLOBAL __attribute__((address_space(1)))
#define VISTA_CONST __attribute__((address_space(4)))
#else
#define VISTA_GLOBAL
#define VISTA_CONST
#endif

// A row's uv coordinates for cell assignment: the baseline rotated by Eq. 1's R when the
// target asks for it (the same FP64 operation sequence as the definition), else as given.
__device__ __forceinline__ void cell_uv(const DevTarget& T, double U, double V, double W, double* Ur,
                                        double* Vr) {
    if (T.rotate) {
        *Ur = T.rot[0] * U + T.rot[1] * V + T.rot[2] * W;
        *Vr = T.rot[3] * U + T.rot[4] * V + T.rot[5] * W;
    } else {
        *Ur = U;
        *Vr = V;
    }
}

// Pointers read from descriptors are generic; casting them to the global address space
// lets the compiler use global (not flat) memory instructions.
template <class T>
__device__ __forceinline__ const VISTA_GLOBAL T* gptr(const T* p) {
    return (const VISTA_GLOBAL T*)p;
}
// Read-only data addressed uniformly across the wave (descriptors, a row's uvw and
// weights): the constant address space lets the compiler use scalar loads.
template <class T>
__device__ __forceinline__ const VISTA_CONST T* cptr(const T* p) {
    return (const VISTA_CONST T*)p;
}

// find_le over a table read with scalar loads (a wave-uniform search).
__device__ __forceinline__ int64_t find_le_uniform(const int64_t* base, int32_t n, int64_t x) {
    const VISTA_CONST int64_t* b = cptr(base);
    int32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (b[mid] <= x) lo = mid; else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int32_t sgpr(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int j) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
    return ((uint64_t)hi << 32) | lo;
}

// sin and cos of 2 pi x for x in [-1/2, 1/2] (an already range-reduced phase in turns),
// from the hardware's FP32 sine and cosine, which take their argument in turns (measured
// maximum absolute error on this range: 1.3e-7).
__device__ __forceinline__ void sincos_turns(float x, float* sn, float* cs) {
    *sn = __builtin_amdgcn_sinf(x);
    *cs = __builtin_amdgcn_cosf(x);
}

// Phase of one channel: the Eq. 2 turns t = (u l + v m + w (n-1)) = trow * a_k formed and
// reduced to [-1/2, 1/2] in FP64; sin/cos of 2 pi r in FP32.
__device__ __forceinline__ void phasor(double trow, double a, float* c, float* s) {
    double t = trow * a;
    double r = t - rint(t);
    sincos_turns((float)r, s, c);
}

// Ablation: turns formed from FP32 coordinates and reduced in FP32, so large arguments
// lose their fractional part to FP32 rounding.
__device__ __forceinline__ void phasor_fp32(float u, float v, float w, float l, float m, float nm1,
                                            float* c, float* s) {
    float t = u * l + v * m + w * nm1;
    sincos_turns(t - rintf(t), s, c);
}

// Write one unit's cells [tu0, tu0 + TU) x [tv0, tv0 + TV) x [jb0, jb1) from the LDS
// state (cell c = (lv TU + lu) JP + j - jb0) to the outputs, iu fastest so that stores are
// contiguous runs of TU cells; with a carried state, merge into it instead (the unit owns
// its cells, so no other workgroup touches them).  Every field of the stack is read once,
// into registers, before the first store.  The cells' values come from
// read(c, re, im, w, n), which may also clear cell c (the next unit then starts from zero
// without a separate pass).
template <int TU, int TV, int JP, class Read>
__device__ __forceinline__ void flush_cells(const LaunchDesc& L, const VISTA_CONST DevStack& S, int32_t tu0,
                                            int32_t tv0, int32_t jb0, int32_t jb1, Read read) {
    const int32_t nu = S.nu, nv = S.nv;
    VISTA_GLOBAL float2* const o_vis = (VISTA_GLOBAL float2*)S.out_vis;
    VISTA_GLOBAL float* const o_w = (VISTA_GLOBAL float*)S.out_w;
    VISTA_GLOBAL uint32_t* const o_cnt = (VISTA_GLOBAL uint32_t*)S.out_cnt;
    VISTA_GLOBAL double2* const o_vis64 = (VISTA_GLOBAL double2*)S.out_vis64;
    VISTA_GLOBAL double* const o_w64 = (VISTA_GLOBAL double*)S.out_w64;
    VISTA_GLOBAL float* const st_s = (VISTA_GLOBAL float*)S.st_s;
    VISTA_GLOBAL float* const st_c = (VISTA_GLOBAL float*)S.st_c;
    VISTA_GLOBAL uint32_t* const st_n = (VISTA_GLOBAL uint32_t*)S.st_n;
    unsigned long long* const stats = S.stats;
    const int carry = S.carry, kahan = L.kahan, last = S.last;
    // the unit's block of the carried state: unit (tile, b) of this stack, TU x TV x jc cells
    const size_t splane = (size_t)S.st_plane;
    const size_t sbase = ((size_t)((tv0 / TV) * S.tiles_u + tu0 / TU) * (size_t)S.nblocks + (size_t)(jb0 / L.jc)) *
                         (size_t)(TU * TV * L.jc);
    const int ncv = (jb1 - jb0) * TV * TU;
    for (int i = threadIdx.x; i < ncv; i += blockDim.x) {
        const int lu = i % TU;
        const int lv = (i / TU) % TV;
        const int jl = i / (TU * TV);
        const int iu = tu0 + lu, iv = tv0 + lv;
        if (iu >= nu || iv >= nv) continue;
        const int c = (lv * TU + lu) * JP + jl;
        const size_t o = ((size_t)(jb0 + jl) * nv + iv) * nu + iu;
        double dre, dim, dw;
        uint32_t n;
        read(c, dre, dim, dw, n);
        if (carry) {
            // merge into the state carried across passes
            const size_t os = sbase + (size_t)i;        // the unit's state block, contiguous in i
            double vals3[3] = {dre, dim, dw};
            for (int q = 0; q < 3; ++q) {
                const float x = (float)vals3[q];
                float sv = st_s[q * splane + os];
                if (kahan) {
                    float cc = st_c[q * splane + os];
                    const float xl = (float)(vals3[q] - (double)x);   // the part lost to FP32
                    float y = x - cc;
                    float t = sv + y;
                    cc = (t - sv) - y;
                    sv = t;
                    y = xl - cc; t = sv + y; cc = (t - sv) - y; sv = t;
                    st_c[q * splane + os] = cc;
                    vals3[q] = (double)sv - (double)cc;
                } else {
                    sv = sv + x;
                    vals3[q] = sv;
                }
                st_s[q * splane + os] = sv;
            }
            const uint64_t nn = (uint64_t)st_n[os] + n;
            if (nn > 0xffffffffull) atomicOr(&stats[7], 1ull);
            st_n[os] = (uint32_t)nn;
            if (!last) continue;
            dre = vals3[0]; dim = vals3[1]; dw = vals3[2]; n = (uint32_t)nn;
        }
        if (o_vis) o_vis[o] = make_float2((float)dre, (float)dim);
        if (o_w) o_w[o] = (float)dw;
        if (o_cnt) o_cnt[o] = n;
        if (o_vis64) o_vis64[o] = make_double2(dre, dim);
        if (o_w64) o_w64[o] = dw;
    }
}

// flush_cells over per-cell arrays of sums (and, KAHAN, their compensations) and counts;
// ZERO: clear every cell read.
template <int TU, int TV, int JP, class Acc, bool KAHAN, bool ZERO = false>
__device__ __forceinline__ void flush_unit(const LaunchDesc& L, const VISTA_CONST DevStack& S, int32_t tu0,
                                           int32_t tv0, int32_t jb0, int32_t jb1, Acc* s_re,
                                           Acc* s_im, Acc* s_w, uint32_t* s_n,
                                           const float* c_re, const float* c_im, const float* c_w) {
    flush_cells<TU, TV, JP>(L, S, tu0, tv0, jb0, jb1,
                            [&](int c, double& dre, double& dim, double& dw, uint32_t& n)
                                __attribute__((always_inline)) {
        if (KAHAN) {
            dre = (double)s_re[c] - (double)c_re[c];
            dim = (double)s_im[c] - (double)c_im[c];
            dw = (double)s_w[c] - (double)c_w[c];
        } else {
            dre = (double)s_re[c]; dim = (double)s_im[c]; dw = (double)s_w[c];
        }
        n = s_n[c];
        if (ZERO) {
            s_re[c] = 0; s_im[c] = 0; s_w[c] = 0; s_n[c] = 0u;
        }
    });
}

}  // namespace
}  // namespace vista
