// Dirty image of each rest channel of a stacked grid: the imaging step on the stacked
// product (Sec. 3.4 proposes an FFT for it).
//
//   I_j(q, p) = Re sum_{iv, iu} S_j[iv][iu] exp(+2 pi i ((iu - nu/2)(p - nu/2) / nu +
//                                                        (iv - nv/2)(q - nv/2) / nv)) / W_j
//
// For power-of-two sizes the centring factors split off: multiply the input by
// (-1)^(iu + iv), take the unnormalised inverse FFT, multiply the output by (-1)^(p + q)
// and by a constant (-1 per axis of length 2, else 1).  The 2-D transform is done as row
// transforms then column transforms, each a radix-2 Stockham (self-sorting) FFT in LDS;
// the column pass stages a tile of adjacent columns so that its loads and stores are
// contiguous runs.  Nothing here is a matrix product: the work is a few passes over the
// grid in HBM.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "vista_device.h"

namespace vista {

namespace {

constexpr int kImgThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// `cnt` inverse transforms (exp(+2 pi i ...)) of length n = 2^logn, transform t at
// x + t * n, ping-ponging between x and y; returns the buffer holding the result.
__device__ float2* fft_inverse(float2* x, float2* y, int logn, int cnt) {
    const int n = 1 << logn, half = n >> 1;
    int l = half, lm = 0;                   // l = n / 2^(s+1); m = 2^s = 1 << lm
    for (int s = 0; s < logn; ++s, l >>= 1, ++lm) {
        const int m = 1 << lm;
        for (int b = threadIdx.x; b < cnt * half; b += blockDim.x) {
            const int t = b >> (logn - 1), bb = b & (half - 1);
            const int j = bb >> lm, k = bb & (m - 1);
            const float2* xs = x + t * n;
            float2* ys = y + t * n;
            const float2 c0 = xs[k + j * m], c1 = xs[k + j * m + l * m];
            float sn, cs;
            sincos_turns((float)j / (float)(2 * l), &sn, &cs);     // exp(+2 pi i j / (2 l))
            ys[k + 2 * j * m] = make_float2(c0.x + c1.x, c0.y + c1.y);
            ys[k + 2 * j * m + m] = cmul(make_float2(c0.x - c1.x, c0.y - c1.y), make_float2(cs, sn));
        }
        __syncthreads();
        float2* t = x; x = y; y = t;
    }
    return x;
}

// Summed weight of every channel, in FP64.
__global__ void __launch_bounds__(kImgThreads) k_image_wsum(const float* __restrict__ w, int64_t plane,
                                                            double* __restrict__ wsum) {
    __shared__ double part[kImgThreads];
    const VISTA_GLOBAL float* wj = gptr(w) + (size_t)blockIdx.x * plane;
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < plane; i += blockDim.x) acc += (double)wj[i];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int o = kImgThreads / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) wsum[blockIdx.x] = part[0];
}

// Row pass: block (j, row block) transforms `rows` consecutive rows of channel j.  The
// input is complex (S) or real (the weights, for the beam).
template <bool REAL>
__global__ void __launch_bounds__(kImgThreads) k_image_rows(const void* __restrict__ src, float2* __restrict__ tmp,
                                                            int lognu, int nv, int rows) {
    extern __shared__ float2 lds[];
    const int nu = 1 << lognu;
    const int j = blockIdx.y, iv0 = blockIdx.x * rows;
    const size_t base = ((size_t)j * nv + iv0) * nu;
    float2* x = lds;
    float2* y = lds + rows * nu;
    for (int i = threadIdx.x; i < rows * nu; i += blockDim.x) {
        const int iv = iv0 + i / nu, iu = i & (nu - 1);
        float2 v;
        if (REAL) v = make_float2(gptr((const float*)src)[base + i], 0.f);
        else v = gptr((const float2*)src)[base + i];
        const float sg = ((iu + iv) & 1) ? -1.f : 1.f;            // centring (input side)
        x[i] = make_float2(sg * v.x, sg * v.y);
    }
    __syncthreads();
    const float2* r = fft_inverse(x, y, lognu, rows);
    for (int i = threadIdx.x; i < rows * nu; i += blockDim.x) tmp[base + i] = r[i];
}

// Column pass: block (j, column tile) transforms `cols` adjacent columns of channel j and
// writes their real part, with the output centring and the channel's weight, to `out`.
__global__ void __launch_bounds__(kImgThreads) k_image_cols(const float2* __restrict__ tmp,
                                                            const double* __restrict__ wsum, float* __restrict__ out,
                                                            int lognu, int lognv, int cols, float sign) {
    extern __shared__ float2 lds[];
    const int nu = 1 << lognu, nv = 1 << lognv;
    const int j = blockIdx.y, p0 = blockIdx.x * cols;
    const size_t plane = (size_t)nu * nv, base = (size_t)j * plane;
    float2* x = lds;                       // column c at x + c * nv
    float2* y = lds + cols * nv;
    for (int i = threadIdx.x; i < cols * nv; i += blockDim.x) {
        const int iv = i / cols, c = i - iv * cols;                // c fastest: contiguous loads
        x[c * nv + iv] = gptr(tmp)[base + (size_t)iv * nu + p0 + c];
    }
    __syncthreads();
    const float2* r = fft_inverse(x, y, lognv, cols);
    const double wt = wsum[j];
    const float inv = wt > 0.0 ? (float)(1.0 / wt) : 0.f;
    for (int i = threadIdx.x; i < cols * nv; i += blockDim.x) {
        const int q = i / cols, c = i - q * cols;
        const int p = p0 + c;
        const float sg = ((p + q) & 1) ? -sign : sign;            // centring (output side)
        ((VISTA_GLOBAL float*)out)[base + (size_t)q * nu + p] = sg * r[c * nv + q].x * inv;
    }
}

int log2i(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

}  // namespace

size_t image_temp_bytes(int nu, int nv, int nchan) { return (size_t)nu * nv * nchan * sizeof(float2); }

hipError_t launch_image(const void* sum_wvis, const float* sum_w, float* image, float* beam, int nu, int nv,
                        int nchan, float2* tmp, double* wsum, hipStream_t stream) {
    if (nchan <= 0) return hipSuccess;
    const int lognu = log2i(nu), lognv = log2i(nv);
    if ((1 << lognu) != nu || (1 << lognv) != nv || nu < 2 || nv < 2 || nu > 4096 || nv > 4096)
        return hipErrorInvalidValue;
    const int rows = std::min(nv, std::max(1, 1024 / nu));
    const int cols = std::min(nu, std::max(1, 4096 / nv));
    const size_t lrow = 2 * (size_t)rows * nu * sizeof(float2), lcol = 2 * (size_t)cols * nv * sizeof(float2);
    const float sign = (nu == 2 ? -1.f : 1.f) * (nv == 2 ? -1.f : 1.f);
    hipLaunchKernelGGL(k_image_wsum, dim3(nchan), dim3(kImgThreads), 0, stream, sum_w, (int64_t)nu * nv, wsum);
    const dim3 grow(nv / rows, nchan), gcol(nu / cols, nchan);
    hipLaunchKernelGGL(k_image_rows<false>, grow, dim3(kImgThreads), lrow, stream, sum_wvis, tmp, lognu, nv, rows);
    hipLaunchKernelGGL(k_image_cols, gcol, dim3(kImgThreads), lcol, stream, tmp, wsum, image, lognu, lognv, cols,
                       sign);
    if (beam) {
        hipLaunchKernelGGL(k_image_rows<true>, grow, dim3(kImgThreads), lrow, stream, sum_w, tmp, lognu, nv, rows);
        hipLaunchKernelGGL(k_image_cols, gcol, dim3(kImgThreads), lcol, stream, tmp, wsum, beam, lognu, lognv, cols,
                           sign);
    }
    return hipGetLastError();
}

}  // namespace vista
