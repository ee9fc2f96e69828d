// Dirty image of each rest channel of a stacked grid: the imaging step on the stacked
// product (Sec. 3.4 proposes an FFT for it).
//
//   I_j(q, p) = Re sum_{iv, iu} S_j[iv][iu] exp(+2 pi i ((iu - nu/2)(p - nu/2) / nu +
//                                                        (iv - nv/2)(q - nv/2) / nv)) / W_j
//
// For power-of-two sizes the centring factors split off: multiply the input by
// (-1)^(iu + iv), take the unnormalised inverse FFT, multiply the output by (-1)^(p + q)
// and by a constant (-1 per axis of length 2, else 1).  The 2-D transform is done as row
// transforms then column transforms.  Transforms of 64 to 1024 points are held in registers
// (split into two shorter transforms with a twiddle, one exchange through LDS); other
// lengths use a Stockham (self-sorting) FFT in LDS.  Where both passes run in registers
// and 128 <= nv <= 2048, only the real part is formed: the row pass transforms the input's
// Hermitian part, of which rows 0 .. nv/2 are kept, and the column pass is a real
// transform from them (half the staging bytes).  The column passes work on tiles of
// adjacent columns so that their loads and stores are contiguous runs.  Nothing here is a
// matrix product: the work is a few passes over the grid in HBM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>

#include "vista_device.h"

namespace vista {

namespace {

constexpr int kSumThreads = 256;
constexpr int kRowThreads = 256;
constexpr int kColThreads = 1024;
constexpr int kRowElems = 1024;     // complex elements of one row tile, unless a row is longer
constexpr int kColElems = 4096;     // complex elements of one column tile
constexpr int kMaxSide = 4096;      // largest grid side; a tile is at least one whole row or column
constexpr int kColRegs = (kColElems > kMaxSide ? kColElems : kMaxSide) / kColThreads;

// Workgroup barrier ordering LDS only.  Every exchange between threads here goes through
// LDS, and a barrier that also orders global memory makes each wave wait for all of its
// outstanding global loads, including the next tile's, which are meant to stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// `cnt` inverse transforms (exp(+2 pi i ...)) of length n = 2^logn, transform t at
// x + t * n, ping-ponging between x and y; returns the buffer holding the result.  Stockham
// (self-sorting) stages of radix 4, after one radix-2 stage when logn is odd.  A stage of
// radix r, with m the product of the radices before it and l = n / (r m), maps the inputs
// c_p = x[k + j m + p l m] (p < r) to y[k + (r j + q) m] = w^(j q) sum_p c_p e^(2 pi i p q / r),
// w = e^(2 pi i / (r l)), for j < l and k < m.
__device__ float2* fft_inverse(float2* x, float2* y, int logn, int cnt) {
    const int n = 1 << logn;
    int lm = 0;                               // m = 2^lm
    if (logn & 1) {                           // radix 2: m = 1, l = n / 2
        const int half = n >> 1;
        const float inv = 1.f / (float)n;      // turns j / (2 l), exact: n is a power of two
        for (int b = threadIdx.x; b < cnt * half; b += blockDim.x) {
            const int t = b >> (logn - 1), j = b & (half - 1);
            const float2* xs = x + t * n;
            float2* ys = y + t * n;
            const float2 c0 = xs[j], c1 = xs[j + half];
            float sn, cs;
            sincos_turns((float)j * inv, &sn, &cs);
            ys[2 * j] = cadd(c0, c1);
            ys[2 * j + 1] = cmul(csub(c0, c1), make_float2(cs, sn));
        }
        lds_barrier();
        float2* t = x; x = y; y = t;
        lm = 1;
    }
    const int q4 = n >> 2;                    // l m of a radix-4 stage
    for (; lm < logn; lm += 2) {
        const int m = 1 << lm;
        const float inv4l = 1.f / (float)(n >> lm);    // 1 / (4 l), exact
        for (int b = threadIdx.x; b < cnt * q4; b += blockDim.x) {
            const int t = b >> (logn - 2), bb = b & (q4 - 1);
            const int j = bb >> lm, k = bb & (m - 1);
            const float2* xs = x + t * n + k + j * m;
            const float2 c0 = xs[0], c1 = xs[q4], c2 = xs[2 * q4], c3 = xs[3 * q4];
            const float2 a = cadd(c0, c2), bq = csub(c0, c2), c = cadd(c1, c3);
            const float2 e = csub(c1, c3), d = make_float2(-e.y, e.x);      // i (c1 - c3)
            float sn, cs;
            sincos_turns((float)j * inv4l, &sn, &cs);
            const float2 w1 = make_float2(cs, sn), w2 = cmul(w1, w1), w3 = cmul(w2, w1);
            float2* ys = y + t * n + k + 4 * j * m;
            ys[0] = cadd(a, c);
            ys[m] = cmul(cadd(bq, d), w1);
            ys[2 * m] = cmul(csub(a, c), w2);
            ys[3 * m] = cmul(csub(bq, d), w3);
        }
        lds_barrier();
        float2* t = x; x = y; y = t;
    }
    return x;
}

// Summed weight of every channel, in FP64.  VEC reads four weights per load (the plane is
// a multiple of 4; VEC needs the base 16-byte aligned).
template <bool VEC>
__global__ void __launch_bounds__(kSumThreads) k_image_wsum(const float* __restrict__ w, int64_t plane,
                                                            double* __restrict__ wsum) {
    __shared__ double part[kSumThreads];
    const VISTA_GLOBAL float* wj = gptr(w) + (size_t)blockIdx.x * plane;
    double acc = 0.0;
    if (VEC) {
        const VISTA_GLOBAL float4* w4 = (const VISTA_GLOBAL float4*)wj;
        const int64_t n4 = plane >> 2;
        double a1 = 0.0;
        int64_t i = threadIdx.x;
        for (; i + kSumThreads < n4; i += 2 * kSumThreads) {
            const float4 p = w4[i], q = w4[i + kSumThreads];
            acc += ((double)p.x + (double)p.y) + ((double)p.z + (double)p.w);
            a1 += ((double)q.x + (double)q.y) + ((double)q.z + (double)q.w);
        }
        if (i < n4) {
            const float4 p = w4[i];
            acc += ((double)p.x + (double)p.y) + ((double)p.z + (double)p.w);
        }
        acc += a1;
    } else {
        for (int64_t i = threadIdx.x; i < plane; i += blockDim.x) acc += (double)wj[i];
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kSumThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsum[blockIdx.x] = part[0];
}

// Row pass: block (j, row block) transforms `rows` consecutive rows of channel j.  The
// input is complex (S) or real (the weights, for the beam).
template <bool REAL>
__global__ void __launch_bounds__(kRowThreads) k_image_rows(const void* __restrict__ src, float2* __restrict__ tmp,
                                                            int lognu, int nv, int rows) {
    extern __shared__ float2 lds[];
    const int nu = 1 << lognu;
    const int j = blockIdx.y, iv0 = blockIdx.x * rows;
    const size_t base = ((size_t)j * nv + iv0) * nu;
    float2* x = lds;
    float2* y = lds + rows * nu;
    for (int i = threadIdx.x; i < rows * nu; i += blockDim.x) {
        const int iv = iv0 + (i >> lognu), iu = i & (nu - 1);
        float2 v;
        if (REAL) v = make_float2(gptr((const float*)src)[base + i], 0.f);
        else v = gptr((const float2*)src)[base + i];
        const float sg = ((iu + iv) & 1) ? -1.f : 1.f;            // centring (input side)
        x[i] = make_float2(sg * v.x, sg * v.y);
    }
    lds_barrier();
    const float2* r = fft_inverse(x, y, lognu, rows);
    for (int i = threadIdx.x; i < rows * nu; i += blockDim.x) tmp[base + i] = r[i];
}

// The column pass is persistent: a block walks tiles tile, tile + gridDim.x, ... and loads
// the next tile into registers before it transforms the current one, so that the loads
// are in flight while the block works in LDS.

// Column pass: tile t holds `cols` adjacent columns p0 = (t mod (nu / cols)) * cols, ...
// of channel t / (nu / cols); the block writes their real part, with the output centring
// and the channel's weight, to `out`.  FULL: every tile has exactly kColThreads * kColRegs
// elements.
template <bool FULL>
__global__ void __launch_bounds__(kColThreads) k_image_cols(const float2* __restrict__ tmp,
                                                            const double* __restrict__ wsum, float* __restrict__ out,
                                                            int lognu, int lognv, int logcols, int ntiles, float sign) {
    constexpr int E = kColRegs;
    extern __shared__ float2 lds[];
    const int nu = 1 << lognu, nv = 1 << lognv, cols = 1 << logcols, per = cols * nv;
    const int logtpc = lognu - logcols;                            // tiles per channel: nu / cols
    const size_t plane = (size_t)nu * nv;
    float2* x = lds;                                               // column c at x + c * nv
    float2* y = lds + per;
    float2 v[E];
    auto fetch = [&](int tile) {
        const size_t base = (size_t)(tile >> logtpc) * plane + ((size_t)(tile & ((1 << logtpc) - 1)) << logcols);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = threadIdx.x + e * kColThreads;           // c = i mod cols fastest: contiguous loads
            if (FULL || i < per) v[e] = gptr(tmp)[base + (size_t)(i >> logcols) * nu + (i & (cols - 1))];
        }
    };
    int tile = blockIdx.x;
    if (tile < ntiles) fetch(tile);
    for (; tile < ntiles; tile += gridDim.x) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = threadIdx.x + e * kColThreads;
            if (FULL || i < per) x[(i & (cols - 1)) * nv + (i >> logcols)] = v[e];
        }
        lds_barrier();
        if (tile + (int)gridDim.x < ntiles) fetch(tile + gridDim.x);
        const float2* r = fft_inverse(x, y, lognv, cols);
        const int j = tile >> logtpc, p0 = (tile & ((1 << logtpc) - 1)) << logcols;
        const double wt = wsum[j];
        const float inv = wt > 0.0 ? (float)(1.0 / wt) : 0.f;
        const size_t base = (size_t)j * plane;
        for (int i = threadIdx.x; i < per; i += blockDim.x) {
            const int q = i >> logcols, c = i & (cols - 1);
            const int p = p0 + c;
            const float sg = ((p + q) & 1) ? -sign : sign;        // centring (output side)
            ((VISTA_GLOBAL float*)out)[base + (size_t)q * nu + p] = sg * r[c * nv + q].x * inv;
        }
        lds_barrier();
    }
}

// e^{+2 pi i j / 64} for j < 32, rounded to FP32: the twiddles of every in-register
// transform below (lengths up to 64 take every 64/M-th entry).
__device__ constexpr float kCos64[32] = {
    1.000000000e+00f,  9.951847196e-01f,  9.807852507e-01f,  9.569403529e-01f,  9.238795042e-01f,
    8.819212914e-01f,  8.314695954e-01f,  7.730104327e-01f,  7.071067691e-01f,  6.343932748e-01f,
    5.555702448e-01f,  4.713967443e-01f,  3.826834261e-01f,  2.902846634e-01f,  1.950903237e-01f,
    9.801714122e-02f,  0.0f,              -9.801714122e-02f, -1.950903237e-01f, -2.902846634e-01f,
    -3.826834261e-01f, -4.713967443e-01f, -5.555702448e-01f, -6.343932748e-01f, -7.071067691e-01f,
    -7.730104327e-01f, -8.314695954e-01f, -8.819212914e-01f, -9.238795042e-01f, -9.569403529e-01f,
    -9.807852507e-01f, -9.951847196e-01f};
__device__ constexpr float kSin64[32] = {
    0.000000000e+00f, 9.801714122e-02f, 1.950903237e-01f, 2.902846634e-01f, 3.826834261e-01f,
    4.713967443e-01f, 5.555702448e-01f, 6.343932748e-01f, 7.071067691e-01f, 7.730104327e-01f,
    8.314695954e-01f, 8.819212914e-01f, 9.238795042e-01f, 9.569403529e-01f, 9.807852507e-01f,
    9.951847196e-01f, 1.000000000e+00f, 9.951847196e-01f, 9.807852507e-01f, 9.569403529e-01f,
    9.238795042e-01f, 8.819212914e-01f, 8.314695954e-01f, 7.730104327e-01f, 7.071067691e-01f,
    6.343932748e-01f, 5.555702448e-01f, 4.713967443e-01f, 3.826834261e-01f, 2.902846634e-01f,
    1.950903237e-01f, 9.801714122e-02f};

// a e^{+2 pi i j / 64}; j is a constant once the calling loops are unrolled, so the trivial
// factors (1 and i) cost nothing.
__device__ __forceinline__ float2 rot64(float2 a, int j) {
    if (j == 0) return a;
    if (j == 16) return make_float2(-a.y, a.x);
    return cmul(a, make_float2(kCos64[j], kSin64[j]));
}

template <int LOG>
__device__ constexpr int bitrev(int k) {
    int r = 0;
    for (int b = 0; b < LOG; ++b) r |= ((k >> b) & 1) << (LOG - 1 - b);
    return r;
}

// In-register inverse DFT of length M = 2^LOGM <= 64, Y[k] = sum_n v[n] e^{+2 pi i n k / M},
// radix-2 decimation in frequency: a stage of span h maps (a, b) = (v[i], v[i + h]) within
// each block of 2h to (a + b, (a - b) e^{2 pi i (i mod h) / (2h)}).  The input is in natural
// order and Y[k] ends in v[bitrev(k)].  Every index is a constant after unrolling, so v
// stays in registers.
template <int LOGM>
__device__ __forceinline__ void dft_regs(float2* v) {
    constexpr int M = 1 << LOGM;
#pragma unroll
    for (int h = M / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int b = 0; b < M; b += 2 * h) {
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const float2 a = v[b + i], c = v[b + i + h];
                v[b + i] = cadd(a, c);
                v[b + i + h] = rot64(csub(a, c), i * (32 / h));
            }
        }
    }
}

// Column pass held in registers, for nv = G R (G <= R, R <= 32): tile t is C adjacent
// columns of one channel, as in k_image_cols, and thread (c, g) = (tid mod C, tid / C)
// works on column c.  With input row n = g + G k and output row q = k' + R g',
//   X[q] = sum_g e^{2 pi i g g' / G} [ e^{2 pi i g k' / nv} sum_k x[g + G k] e^{2 pi i k k' / R} ]:
//   (1) thread (c, g) loads rows g + G k (k < R), takes their R-point transform in
//       registers and multiplies output k' by e^{2 pi i g k' / nv};
//   (2) the products cross the block once through LDS (cell (k' G + g) C + c), and thread
//       (c, g) takes, for each k' = g + G s (s < R / G), the G-point transform over the
//       block's g, which is output row k' + R g'.
// One LDS write and one read per element, two barriers per tile; loads are C-column runs of
// rows, stores C-float runs.  Persistent, with as many blocks as fit at once; the loads of
// a tile are all issued before its first use.
template <int LOGG, int LOGR, int LOGC>
__global__ void __launch_bounds__(1 << (LOGC + LOGG)) k_image_cols_reg(const float2* __restrict__ tmp,
                                                                        const double* __restrict__ wsum,
                                                                        float* __restrict__ out, int lognu,
                                                                        int ntiles, float sign) {
    constexpr int G = 1 << LOGG, R = 1 << LOGR, C = 1 << LOGC, NV = G * R, S = R / G;
    static_assert(G <= R && R <= 32, "tile split");
    __shared__ float2 lds[NV * C];
    const int c = threadIdx.x & (C - 1), g = threadIdx.x >> LOGC;
    const int nu = 1 << lognu, logtpc = lognu - LOGC;
    const size_t plane = (size_t)nu * NV;
    float2 v[R];
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const VISTA_GLOBAL float2* src = gptr(tmp) + (size_t)(tile >> logtpc) * plane +
                                         ((size_t)(tile & ((1 << logtpc) - 1)) << LOGC) + c;
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = src[(size_t)(g + G * k) * nu];
        dft_regs<LOGR>(v);
#pragma unroll
        for (int kp = 0; kp < R; ++kp) {
            float t = (float)((g * kp) & (NV - 1)) * (1.f / (float)NV);    // exact
            if (t > 0.5f) t -= 1.f;
            float sn, cs;
            sincos_turns(t, &sn, &cs);
            lds[(kp * G + g) * C + c] = cmul(v[bitrev<LOGR>(kp)], make_float2(cs, sn));
        }
        lds_barrier();
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int gg = 0; gg < G; ++gg) v[s * G + gg] = lds[((g + G * s) * G + gg) * C + c];
        }
        lds_barrier();
        const int j = tile >> logtpc, p = ((tile & ((1 << logtpc) - 1)) << LOGC) + c;
        const double wt = wsum[j];
        const float inv = wt > 0.0 ? (float)(1.0 / wt) : 0.f;
        VISTA_GLOBAL float* dst = (VISTA_GLOBAL float*)out + (size_t)j * plane + p;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            dft_regs<LOGG>(v + s * G);
#pragma unroll
            for (int gp = 0; gp < G; ++gp) {
                const int q = g + G * s + R * gp;
                const float sg = ((p + q) & 1) ? -sign : sign;                // centring (output side)
                dst[(size_t)q * nu] = sg * v[s * G + bitrev<LOGG>(gp)].x * inv;
            }
        }
    }
}

// Row pass held in registers, for nu = G R (G <= R, R <= 32): block (row tile, channel)
// transforms RT consecutive rows, thread (g, r) = (tid mod G, tid / G) working on row r of
// the tile, with the same split as the column pass along the row: input element n = g + G k
// (loads of G consecutive elements per row), output element q = k' + R g' (stores of G
// consecutive elements).  Row r's products sit at r (G (R + 1)) + g (R + 1) + k' in LDS (one
// padding element per g keeps the writes of consecutive g on distinct banks).  The input
// is complex (S) or real (the weights, for the beam), and takes the input-side centring.
template <int LOGG, int LOGR, int LOGRT, bool REAL>
__global__ void __launch_bounds__(1 << (LOGG + LOGRT)) k_image_rows_reg(const void* __restrict__ src,
                                                                         float2* __restrict__ tmp, int lognv) {
    constexpr int G = 1 << LOGG, R = 1 << LOGR, RT = 1 << LOGRT, NU = G * R, S = R / G, RP = R + 1;
    static_assert(G <= R && R <= 32 && G % 2 == 0, "tile split");
    __shared__ float2 lds[RT * G * RP];
    const int g = threadIdx.x & (G - 1), r = threadIdx.x >> LOGG;
    const int j = blockIdx.y, iv = blockIdx.x * RT + r;
    const size_t row = ((size_t)j << lognv) + iv;
    float2 v[R];
    const float sg = ((g + iv) & 1) ? -1.f : 1.f;          // (-1)^(iu + iv), iu = g + G k, G even
    if (REAL) {
        const VISTA_GLOBAL float* x = gptr((const float*)src) + row * NU + g;
#pragma unroll
        for (int k = 0; k < R; ++k) v[k] = make_float2(sg * x[G * k], 0.f);
    } else {
        const VISTA_GLOBAL float2* x = gptr((const float2*)src) + row * NU + g;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const float2 a = x[G * k];
            v[k] = make_float2(sg * a.x, sg * a.y);
        }
    }
    dft_regs<LOGR>(v);
    float2* mine = lds + r * (G * RP);
#pragma unroll
    for (int kp = 0; kp < R; ++kp) {
        float t = (float)((g * kp) & (NU - 1)) * (1.f / (float)NU);    // exact
        if (t > 0.5f) t -= 1.f;
        float sn, cs;
        sincos_turns(t, &sn, &cs);
        mine[g * RP + kp] = cmul(v[bitrev<LOGR>(kp)], make_float2(cs, sn));
    }
    lds_barrier();
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int gg = 0; gg < G; ++gg) v[s * G + gg] = mine[gg * RP + g + G * s];
    }
    float2* dst = tmp + row * NU + g;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        dft_regs<LOGG>(v + s * G);
#pragma unroll
        for (int gp = 0; gp < G; ++gp) dst[G * s + R * gp] = v[s * G + bitrev<LOGG>(gp)];
    }
}

// The Hermitian path (real output from half the staging).  With y the centred input, the
// image is Re F(y) = F(y_h), y_h(iu, iv) = (y(iu, iv) + conj(y(-iu, -iv))) / 2 (indices
// modulo the sides; the centring sign of (-iu, -iv) is that of (iu, iv), the sides being
// even).  y_h's row transforms T are Hermitian along each column, T(p, nv - k) =
// conj(T(p, k)), so rows 0 .. nv/2 of T determine the image and the column pass is a
// complex-to-real transform.
//
// Row pass: as k_image_rows_reg, for rows k = 0 .. nv/2 only, each loaded together with the
// mirror row (nv - k) mod nv read backwards ((nu - iu) mod nu) and folded into y_h before
// the transform.  Block x takes rows x RT .. x RT + RT - 1; rows past nv/2 (the last block)
// are transformed but not stored.
template <int LOGG, int LOGR, int LOGRT, bool REAL>
__global__ void __launch_bounds__(1 << (LOGG + LOGRT)) k_image_rows_herm(const void* __restrict__ src,
                                                                          float2* __restrict__ tmp, int lognv) {
    constexpr int G = 1 << LOGG, R = 1 << LOGR, RT = 1 << LOGRT, NU = G * R, S = R / G, RP = R + 1;
    static_assert(G <= R && R <= 32 && G % 2 == 0, "tile split");
    __shared__ float2 lds[RT * G * RP];
    const int g = threadIdx.x & (G - 1), r = threadIdx.x >> LOGG;
    const int nv = 1 << lognv;
    const int j = blockIdx.y, k = blockIdx.x * RT + r;
    const int kr = min(k, nv - 1);                         // (rows past nv/2 are not stored)
    const int km = (nv - kr) & (nv - 1);                   // the mirror row
    const size_t row = ((size_t)j << lognv) + kr, mrow = ((size_t)j << lognv) + km;
    float2 v[R];
    const float sg = ((g + kr) & 1) ? -0.5f : 0.5f;        // (-1)^(iu + k) / 2, iu = g + G kk, G even
    if (REAL) {
        const VISTA_GLOBAL float* x = gptr((const float*)src) + row * NU;
        const VISTA_GLOBAL float* xm = gptr((const float*)src) + mrow * NU;
#pragma unroll
        for (int kk = 0; kk < R; ++kk) {
            const int iu = g + G * kk;
            v[kk] = make_float2(sg * (x[iu] + xm[(NU - iu) & (NU - 1)]), 0.f);
        }
    } else {
        const VISTA_GLOBAL float2* x = gptr((const float2*)src) + row * NU;
        const VISTA_GLOBAL float2* xm = gptr((const float2*)src) + mrow * NU;
#pragma unroll
        for (int kk = 0; kk < R; ++kk) {
            const int iu = g + G * kk;
            const float2 a = x[iu], b = xm[(NU - iu) & (NU - 1)];
            v[kk] = make_float2(sg * (a.x + b.x), sg * (a.y - b.y));
        }
    }
    dft_regs<LOGR>(v);
    float2* mine = lds + r * (G * RP);
#pragma unroll
    for (int kp = 0; kp < R; ++kp) {
        float t = (float)((g * kp) & (NU - 1)) * (1.f / (float)NU);    // exact
        if (t > 0.5f) t -= 1.f;
        float sn, cs;
        sincos_turns(t, &sn, &cs);
        mine[g * RP + kp] = cmul(v[bitrev<LOGR>(kp)], make_float2(cs, sn));
    }
    lds_barrier();
#pragma unroll
    for (int s = 0; s < S; ++s) {
#pragma unroll
        for (int gg = 0; gg < G; ++gg) v[s * G + gg] = mine[gg * RP + g + G * s];
    }
    if (k > nv / 2) return;
    float2* dst = tmp + row * NU + g;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        dft_regs<LOGG>(v + s * G);
#pragma unroll
        for (int gp = 0; gp < G; ++gp) dst[G * s + R * gp] = v[s * G + bitrev<LOGG>(gp)];
    }
}

// Column pass of the Hermitian path: a real transform of length nv = 2 M from the rows
// H[0 .. M] of one column, as one complex transform of length M = G R.  Output row 2n is
// Re z[n] and row 2n + 1 is Im z[n], with z the length-M inverse transform of
//   Z[k] = E[k] + i O[k],  E[k] = H[k] + conj(H[M - k]),
//   O[k] = (H[k] - conj(H[M - k])) e^{2 pi i k / nv}    (k < M)
// (the even and the odd outputs are the length-M transforms of E and of O, both real).
// Tiles, threads and the two-step split of the length-M transform are those of
// k_image_cols_reg; thread (c, g) loads rows k = g + G kk and M - k of column c.
template <int LOGG, int LOGR, int LOGC>
__global__ void __launch_bounds__(1 << (LOGC + LOGG)) k_image_cols_herm(const float2* __restrict__ tmp,
                                                                         const double* __restrict__ wsum,
                                                                         float* __restrict__ out, int lognu,
                                                                         int ntiles, float sign) {
    constexpr int G = 1 << LOGG, R = 1 << LOGR, C = 1 << LOGC, M = G * R, NV = 2 * M, S = R / G;
    static_assert(G <= R && R <= 32, "tile split");
    __shared__ float2 lds[M * C];
    const int c = threadIdx.x & (C - 1), g = threadIdx.x >> LOGC;
    const int nu = 1 << lognu, logtpc = lognu - LOGC;
    const size_t plane = (size_t)nu * NV;
    float2 v[R];
    for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const VISTA_GLOBAL float2* src = gptr(tmp) + (size_t)(tile >> logtpc) * plane +
                                         ((size_t)(tile & ((1 << logtpc) - 1)) << LOGC) + c;
#pragma unroll
        for (int kk = 0; kk < R; ++kk) {
            const int k = g + G * kk;
            const float2 h = src[(size_t)k * nu], hm = src[(size_t)(M - k) * nu];
            const float2 e = make_float2(h.x + hm.x, h.y - hm.y);             // H[k] + conj(H[M - k])
            const float2 d = make_float2(h.x - hm.x, h.y + hm.y);             // H[k] - conj(H[M - k])
            float sn, cs;
            sincos_turns((float)k * (1.f / (float)NV), &sn, &cs);            // exact fraction, < 1/2
            const float2 o = cmul(d, make_float2(cs, sn));
            v[kk] = make_float2(e.x - o.y, e.y + o.x);                         // E + i O
        }
        dft_regs<LOGR>(v);
#pragma unroll
        for (int kp = 0; kp < R; ++kp) {
            float t = (float)((g * kp) & (M - 1)) * (1.f / (float)M);      // exact
            if (t > 0.5f) t -= 1.f;
            float sn, cs;
            sincos_turns(t, &sn, &cs);
            lds[(kp * G + g) * C + c] = cmul(v[bitrev<LOGR>(kp)], make_float2(cs, sn));
        }
        lds_barrier();
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
            for (int gg = 0; gg < G; ++gg) v[s * G + gg] = lds[((g + G * s) * G + gg) * C + c];
        }
        lds_barrier();
        const int j = tile >> logtpc, p = ((tile & ((1 << logtpc) - 1)) << LOGC) + c;
        const double wt = wsum[j];
        const float inv = wt > 0.0 ? (float)(1.0 / wt) : 0.f;
        VISTA_GLOBAL float* dst = (VISTA_GLOBAL float*)out + (size_t)j * plane + p;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            dft_regs<LOGG>(v + s * G);
#pragma unroll
            for (int gp = 0; gp < G; ++gp) {
                const int n = g + G * s + R * gp;
                const float2 z = v[s * G + bitrev<LOGG>(gp)];
                const float sg = ((p + 2 * n) & 1) ? -sign : sign;            // centring, row 2n
                dst[(size_t)(2 * n) * nu] = sg * z.x * inv;
                dst[(size_t)(2 * n + 1) * nu] = -sg * z.y * inv;              // row 2n + 1
            }
        }
    }
}

// Blocks of a persistent launch: as many as fit on the device at once, at most `ntiles`.
template <typename K>
int persistent_blocks(K kernel, int threads, size_t lds, int ntiles) {
    int dev = 0, cu = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0)
        cu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb <= 0) nb = 1;
    return (int)std::min<int64_t>(ntiles, (int64_t)nb * cu);
}

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

size_t image_temp_bytes(int nu, int nv, int nchan) { return (size_t)nu * nv * nchan * sizeof(float2); }

hipError_t launch_image(const void* sum_wvis, const float* sum_w, float* image, float* beam, int nu, int nv,
                        int nchan, float2* tmp, size_t tmp_bytes, double* wsum, hipStream_t stream) {
    if (nchan <= 0) return hipSuccess;
    const int lognu = log2i(nu), lognv = log2i(nv);
    if ((1 << lognu) != nu || (1 << lognv) != nv || nu < 2 || nv < 2 || nu > kMaxSide || nv > kMaxSide)
        return hipErrorInvalidValue;
    const size_t plane = (size_t)nu * nv;
    // channels per pass: as many staging planes as tmp holds (all of them when it holds the cube)
    const int64_t per_pass = std::min<int64_t>(nchan, (int64_t)(tmp_bytes / (plane * sizeof(float2))));
    if (per_pass < 1) return hipErrorInvalidValue;
    const int rows = std::min(nv, std::max(1, kRowElems / nu));
    const int cols = std::min(nu, std::max(1, kColElems / nv));
    const int logcols = log2i(cols);
    const size_t lrow = 2 * (size_t)rows * nu * sizeof(float2), lcol = 2 * (size_t)cols * nv * sizeof(float2);
    const float sign = (nu == 2 ? -1.f : 1.f) * (nv == 2 ? -1.f : 1.f);
    if (((uintptr_t)sum_w & 15) == 0)
        hipLaunchKernelGGL(k_image_wsum<true>, dim3(nchan), dim3(kSumThreads), 0, stream, sum_w, (int64_t)plane, wsum);
    else
        hipLaunchKernelGGL(k_image_wsum<false>, dim3(nchan), dim3(kSumThreads), 0, stream, sum_w, (int64_t)plane,
                           wsum);
    const bool cfull = cols * nv == kColThreads * kColRegs;
    auto cols_k = cfull ? k_image_cols<true> : k_image_cols<false>;
    // the in-register column pass, for 64 <= nv <= 1024 and at least one tile of columns:
    // tiles of 32 columns (256-byte row runs), 16 for nv = 1024 (a tile's LDS, nv C 8
    // bytes, stays within 128 KiB)
    void (*reg_k)(const float2*, const double*, float*, int, int, float) = nullptr;
    int reg_threads = 0, reg_cols = 0;
    switch (lognv) {
        case 6: reg_k = k_image_cols_reg<3, 3, 5>; reg_cols = 32; reg_threads = 32 << 3; break;
        case 7: reg_k = k_image_cols_reg<3, 4, 5>; reg_cols = 32; reg_threads = 32 << 3; break;
        case 8: reg_k = k_image_cols_reg<4, 4, 5>; reg_cols = 32; reg_threads = 32 << 4; break;
        case 9: reg_k = k_image_cols_reg<4, 5, 5>; reg_cols = 32; reg_threads = 32 << 4; break;
        case 10: reg_k = k_image_cols_reg<5, 5, 4>; reg_cols = 16; reg_threads = 16 << 5; break;
        default: break;
    }
    if (nu < reg_cols) reg_k = nullptr;
    // the in-register row pass, for 64 <= nu <= 1024 and at least one tile of rows
    void (*rrow_c)(const void*, float2*, int) = nullptr;
    void (*rrow_r)(const void*, float2*, int) = nullptr;
    int rrow_rows = 0;
    switch (lognu) {
        case 6: rrow_c = k_image_rows_reg<3, 3, 5, false>; rrow_r = k_image_rows_reg<3, 3, 5, true>; rrow_rows = 32; break;
        case 7: rrow_c = k_image_rows_reg<3, 4, 5, false>; rrow_r = k_image_rows_reg<3, 4, 5, true>; rrow_rows = 32; break;
        case 8: rrow_c = k_image_rows_reg<4, 4, 4, false>; rrow_r = k_image_rows_reg<4, 4, 4, true>; rrow_rows = 16; break;
        case 9: rrow_c = k_image_rows_reg<4, 5, 4, false>; rrow_r = k_image_rows_reg<4, 5, 4, true>; rrow_rows = 16; break;
        case 10: rrow_c = k_image_rows_reg<5, 5, 3, false>; rrow_r = k_image_rows_reg<5, 5, 3, true>; rrow_rows = 8; break;
        default: break;
    }
    if (nv < rrow_rows) rrow_c = rrow_r = nullptr;
    // the Hermitian path (rows 0 .. nv/2 staged, a real column transform), for register row
    // passes and 128 <= nv <= 2048: the same tiles, on the half-length column transform
    void (*hrow_c)(const void*, float2*, int) = nullptr;
    void (*hrow_r)(const void*, float2*, int) = nullptr;
    switch (lognu) {
        case 6: hrow_c = k_image_rows_herm<3, 3, 5, false>; hrow_r = k_image_rows_herm<3, 3, 5, true>; break;
        case 7: hrow_c = k_image_rows_herm<3, 4, 5, false>; hrow_r = k_image_rows_herm<3, 4, 5, true>; break;
        case 8: hrow_c = k_image_rows_herm<4, 4, 4, false>; hrow_r = k_image_rows_herm<4, 4, 4, true>; break;
        case 9: hrow_c = k_image_rows_herm<4, 5, 4, false>; hrow_r = k_image_rows_herm<4, 5, 4, true>; break;
        case 10: hrow_c = k_image_rows_herm<5, 5, 3, false>; hrow_r = k_image_rows_herm<5, 5, 3, true>; break;
        default: break;
    }
    void (*hcol_k)(const float2*, const double*, float*, int, int, float) = nullptr;
    int hcol_threads = 0, hcol_cols = 0;
    switch (lognv) {
        case 7: hcol_k = k_image_cols_herm<3, 3, 5>; hcol_cols = 32; hcol_threads = 32 << 3; break;
        case 8: hcol_k = k_image_cols_herm<3, 4, 5>; hcol_cols = 32; hcol_threads = 32 << 3; break;
        case 9: hcol_k = k_image_cols_herm<4, 4, 5>; hcol_cols = 32; hcol_threads = 32 << 4; break;
        case 10: hcol_k = k_image_cols_herm<4, 5, 5>; hcol_cols = 32; hcol_threads = 32 << 4; break;
        case 11: hcol_k = k_image_cols_herm<5, 5, 4>; hcol_cols = 16; hcol_threads = 16 << 5; break;
        default: break;
    }
    const bool herm = hrow_c && hcol_k && nu >= hcol_cols && nv / 2 >= rrow_rows;
    auto rows_pass = [&](const void* src, bool real, int nc) {
        if (herm) {
            hipLaunchKernelGGL(real ? hrow_r : hrow_c, dim3(nv / 2 / rrow_rows + 1, nc), dim3(kRowThreads), 0, stream,
                               src, tmp, lognv);
        } else if (rrow_c) {
            hipLaunchKernelGGL(real ? rrow_r : rrow_c, dim3(nv / rrow_rows, nc), dim3(kRowThreads), 0, stream, src, tmp,
                               lognv);
        } else if (real) {
            hipLaunchKernelGGL(k_image_rows<true>, dim3(nv / rows, nc), dim3(kRowThreads), lrow, stream, src, tmp,
                               lognu, nv, rows);
        } else {
            hipLaunchKernelGGL(k_image_rows<false>, dim3(nv / rows, nc), dim3(kRowThreads), lrow, stream, src, tmp,
                               lognu, nv, rows);
        }
    };
    auto columns = [&](const double* ws, float* dst, int nc) {
        if (herm) {
            const int nct = (int)((int64_t)nc * (nu / hcol_cols));
            hipLaunchKernelGGL(hcol_k, dim3(persistent_blocks(hcol_k, hcol_threads, 0, nct)), dim3(hcol_threads), 0,
                               stream, tmp, ws, dst, lognu, nct, sign);
        } else if (reg_k) {
            const int nct = (int)((int64_t)nc * (nu / reg_cols));
            hipLaunchKernelGGL(reg_k, dim3(persistent_blocks(reg_k, reg_threads, 0, nct)), dim3(reg_threads), 0,
                               stream, tmp, ws, dst, lognu, nct, sign);
        } else {
            const int nct = (int)((int64_t)nc * (nu / cols));
            hipLaunchKernelGGL(cols_k, dim3(persistent_blocks(cols_k, kColThreads, lcol, nct)), dim3(kColThreads),
                               lcol, stream, tmp, ws, dst, lognu, lognv, logcols, nct, sign);
        }
    };
    // channels [j0, j0 + nc): the kernels see the pass's slice of every array (planes are
    // multiples of 4 elements, so the slices keep the arrays' alignment)
    for (int64_t j0 = 0; j0 < nchan; j0 += per_pass) {
        const int nc = (int)std::min<int64_t>(per_pass, nchan - j0);
        const size_t off = (size_t)j0 * plane;
        rows_pass((const void*)((const float2*)sum_wvis + off), false, nc);
        columns(wsum + j0, image + off, nc);
        if (beam) {
            rows_pass((const void*)(sum_w + off), true, nc);
            columns(wsum + j0, beam + off, nc);
        }
    }
    return hipGetLastError();
}

// ------------------------------------------------------- scratch of the no-alloc entry point

// Device scratch of vista_image_noalloc: the complex staging planes of one pass and the
// channels' FP64 weight sums.  Each device that loads the library holds its own copy until
// the process ends; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device (the array's name is no device address on the host).
static __device__ __align__(256) unsigned char scratch[kNoAllocImageStaging + kNoAllocImageWsum];

void* image_noalloc_scratch(hipError_t* err) {
    static std::mutex m;
    static void* ptrs[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        *err = e != hipSuccess ? e : hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(m);
    if (!ptrs[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        ptrs[dev] = p;
    }
    *err = hipSuccess;
    return ptrs[dev];
}

}  // namespace vista
