// Dirty image of each rest channel of a stacked grid: the imaging step on the stacked
// product (Sec. 3.4 proposes an FFT for it).
//
//   I_j(q, p) = Re sum_{iv, iu} S_j[iv][iu] exp(+2 pi i ((iu - nu/2)(p - nu/2) / nu +
//                                                        (iv - nv/2)(q - nv/2) / nv)) / W_j
//
// For power-of-two sizes the centring factors split off: multiply the input by
// (-1)^(iu + iv), take the unnormalised inverse FFT, multiply the output by (-1)^(p + q)
// and by a constant (-1 per axis of length 2, else 1).  The 2-D transform is done as row
// transforms then column transforms, each a Stockham (self-sorting) FFT in LDS;
// the column pass stages a tile of adjacent columns so that its loads and stores are
// contiguous runs.  Nothing here is a matrix product: the work is a few passes over the
// grid in HBM.
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
    // channels [j0, j0 + nc): the kernels see the pass's slice of every array (planes are
    // multiples of 4 elements, so the slices keep the arrays' alignment)
    for (int64_t j0 = 0; j0 < nchan; j0 += per_pass) {
        const int nc = (int)std::min<int64_t>(per_pass, nchan - j0);
        const int nct = (int)((int64_t)nc * (nu / cols));
        const dim3 grow(nv / rows, nc), gcol(persistent_blocks(cols_k, kColThreads, lcol, nct));
        const size_t off = (size_t)j0 * plane;
        hipLaunchKernelGGL(k_image_rows<false>, grow, dim3(kRowThreads), lrow, stream,
                           (const void*)((const float2*)sum_wvis + off), tmp, lognu, nv, rows);
        hipLaunchKernelGGL(cols_k, gcol, dim3(kColThreads), lcol, stream, tmp, wsum + j0, image + off, lognu, lognv,
                           logcols, nct, sign);
        if (beam) {
            hipLaunchKernelGGL(k_image_rows<true>, grow, dim3(kRowThreads), lrow, stream,
                               (const void*)(sum_w + off), tmp, lognu, nv, rows);
            hipLaunchKernelGGL(cols_k, gcol, dim3(kColThreads), lcol, stream, tmp, wsum + j0, beam + off, lognu,
                               lognv, logcols, nct, sign);
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
