// Whitening front end: the filter bank's input is whitened strain; this is
// the step that makes it from raw detector data (the paper's SPIIR section
// takes noisy detector data as input, "SPIIR method"). Frames of N samples at
// hop H = N/2 with a periodic Hann window w[t] = sin^2(pi t / N):
//   PSD estimate : S[f] = mean over frames of |DFT(w . s_k)[f]|^2 / sum_t w[t]^2, f = 0..N/2
//   whitening    : y_k = IDFT(DFT(w . x_k) / sqrt(S)), overlap-added at hop H
// The stream is whitened with a delay of H samples (H zeros precede it).
// Each frame is one workgroup of 1,024 threads: a radix-2 FFT of N complex
// points in LDS (bit-reversed load, in-place butterflies taken two stages per
// pass, a bank swizzle on the frame buffer; the FP64-computed twiddle table
// is staged in LDS once per frame, so no stage waits on global memory); the
// inverse transform is the forward one applied to the conjugate.
#include "spiir_internal.h"

#include <atomic>

namespace spiir {
namespace {

constexpr int kThreads = 256;      // overlap-add and PSD launches
constexpr int kFftThreads = 1024;  // one frame per workgroup

__device__ inline int bitrev(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

// LDS position of frame element i: inside each aligned block of 16 elements,
// bits 4-5 of i are XORed into bits 0-1 and 2-3. The first two radix-2^2
// passes have 16 lanes touching elements 4 (s = 0) or 16 (s = 2) apart, which
// land on 4 bank groups unswizzled (4-way conflicts) and on 16 swizzled; the
// later passes touch 16 consecutive elements either way. A bijection on
// [0, n), applied to every access of the frame buffer.
__device__ inline int sw(int i) {
    const int m = (i >> 4) & 3;
    return i ^ (m | (m << 2));
}

__device__ inline float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place radix-2 decimation-in-time over bit-reversed input, two stages per
// pass: stage s combines pairs h = 2^s apart with exp(-2 pi i pos / 2h), stage
// s+1 pairs 2h apart with exp(-2 pi i pos' / 4h). The four elements
// b, b+h, b+2h, b+3h of a group (b = its 4h-block start + pos, pos < h) are
// closed under both stages, so each thread takes whole groups through both in
// registers: one LDS exchange and one barrier per two stages. An odd stage
// count ends with one plain radix-2 stage.
__device__ void fft_stages(float2 *buf, const float2 *tw, int n, int logn) {
    int s = 0;
    for (; s + 1 < logn; s += 2) {
        const int h = 1 << s;
        const int st1 = n >> (s + 1), st2 = n >> (s + 2);
        for (int q = threadIdx.x; q < n / 4; q += kFftThreads) {
            const int pos = q & (h - 1);
            const int b = ((q >> s) << (s + 2)) + pos;
            const float2 w1 = tw[pos * st1];
            const float2 w2a = tw[pos * st2], w2b = tw[(pos + h) * st2];
            const int e0 = sw(b), e1 = sw(b + h), e2 = sw(b + 2 * h), e3 = sw(b + 3 * h);
            const float2 a0 = buf[e0], a1 = cmul(buf[e1], w1), a2 = buf[e2], a3 = cmul(buf[e3], w1);
            const float2 b0 = make_float2(a0.x + a1.x, a0.y + a1.y), b1 = make_float2(a0.x - a1.x, a0.y - a1.y);
            const float2 c2 = cmul(make_float2(a2.x + a3.x, a2.y + a3.y), w2a);
            const float2 c3 = cmul(make_float2(a2.x - a3.x, a2.y - a3.y), w2b);
            buf[e0] = make_float2(b0.x + c2.x, b0.y + c2.y);
            buf[e2] = make_float2(b0.x - c2.x, b0.y - c2.y);
            buf[e1] = make_float2(b1.x + c3.x, b1.y + c3.y);
            buf[e3] = make_float2(b1.x - c3.x, b1.y - c3.y);
        }
        __syncthreads();
    }
    if (s < logn) {
        const int h = 1 << s;
        const int step = n >> (s + 1);
        for (int q = threadIdx.x; q < n / 2; q += kFftThreads) {
            const int pos = q & (h - 1);
            const int i0 = ((q >> s) << (s + 1)) + pos;
            const int p0 = sw(i0), p1 = sw(i0 + h);
            const float2 u = buf[p0], v = cmul(buf[p1], tw[pos * step]);
            buf[p0] = make_float2(u.x + v.x, u.y + v.y);
            buf[p1] = make_float2(u.x - v.x, u.y - v.y);
        }
        __syncthreads();
    }
}

// Frame j covers samples jH .. jH + N - 1 of the concatenation hist[0..hlen) ++ x.
// PSD mode: pw[j][f] = |X_j[f]|^2 for f = 0..H. Whitening mode: y[j][t] = the
// inverse DFT of X_j[f] * inv[min(f, N - f)], t = 0..N-1.
template <bool PSD>
__global__ __launch_bounds__(kFftThreads) void wh_frames_kernel(const float *__restrict__ hist, int64_t hlen,
                                                                const float *__restrict__ x,
                                                                const float *__restrict__ wtab,
                                                                const float2 *__restrict__ tw_g, int n, int logn,
                                                                const float *__restrict__ inv,
                                                                float *__restrict__ y, float *__restrict__ pw) {
    extern __shared__ float2 buf[];   // [n] data, then [n/2] twiddles
    float2 *tw = buf + n;
    const int H = n / 2;
    const int64_t base = (int64_t)blockIdx.x * H;
    for (int k = threadIdx.x; k < H; k += kFftThreads) tw[k] = tw_g[k];
    for (int i = threadIdx.x; i < n; i += kFftThreads) {
        const int64_t gi = base + i;
        const float v = gi < hlen ? hist[gi] : x[gi - hlen];
        buf[sw(bitrev(i, logn))] = make_float2(wtab[i] * v, 0.0f);
    }
    __syncthreads();
    fft_stages(buf, tw, n, logn);
    if (PSD) {
        for (int f = threadIdx.x; f <= H; f += kFftThreads) {
            const float2 X = buf[sw(f)];
            pw[(int64_t)blockIdx.x * (H + 1) + f] = X.x * X.x + X.y * X.y;
        }
        return;
    }
    // conj(X * inv), then bit-reversed order for the second forward transform
    for (int f = threadIdx.x; f < n; f += kFftThreads) {
        const float s = inv[min(f, n - f)];
        const float2 X = buf[sw(f)];
        buf[sw(f)] = make_float2(X.x * s, -X.y * s);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kFftThreads) {
        const int r = bitrev(i, logn);
        if (i < r) {
            const int pi = sw(i), pr = sw(r);
            const float2 t = buf[pi];
            buf[pi] = buf[pr];
            buf[pr] = t;
        }
    }
    __syncthreads();
    fft_stages(buf, tw, n, logn);
    const float scale = 1.0f / (float)n;
    for (int t = threadIdx.x; t < n; t += kFftThreads) y[(int64_t)blockIdx.x * n + t] = buf[sw(t)].x * scale;
}

// S[f] = sum_j pw[j][f] / (frames * wsum2) in FP64; inv[f] = 1 / sqrt(S[f]), 0 where S <= 0.
__global__ void wh_psd_reduce_kernel(const float *__restrict__ pw, int64_t frames, int H, double wsum2,
                                     double *__restrict__ S, float *__restrict__ inv) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > H) return;
    double acc = 0.0;
    for (int64_t j = 0; j < frames; ++j) acc += (double)pw[j * (H + 1) + f];
    const double v = acc / ((double)frames * wsum2);
    S[f] = v;
    inv[f] = v > 0.0 ? (float)(1.0 / sqrt(v)) : 0.0f;
}

// inv[f] from a given S (host-set PSD).
__global__ void wh_inv_kernel(const double *__restrict__ S, int H, float *__restrict__ inv) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f > H) return;
    const double v = S[f];
    inv[f] = v > 0.0 ? (float)(1.0 / sqrt(v)) : 0.0f;
}

// out[jH + t] = y[j][t] + (j == 0 ? pend[t] : y[j - 1][H + t]) for the nf frames;
// block 0 also stores the last frame's second half (pending for the next call)
// and the last H input samples (the next call's history).
__global__ __launch_bounds__(kThreads) void wh_ola_kernel(const float *__restrict__ y, int64_t nf, int n,
                                                          const float *__restrict__ pend,
                                                          float *__restrict__ pend_new,
                                                          const float *__restrict__ x, int64_t nx,
                                                          float *__restrict__ hist_new, float *__restrict__ out) {
    const int H = n / 2;
    const int64_t m = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (m < nf * H) {
        const int64_t j = m / H;
        const int t = (int)(m - j * H);
        const float prev = j == 0 ? pend[t] : y[(j - 1) * n + H + t];
        out[m] = y[j * n + t] + prev;
    }
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < H; t += kThreads) {
            pend_new[t] = y[(nf - 1) * n + H + t];
            hist_new[t] = x[nx - H + t];
        }
}

}  // namespace

hipError_t launch_wh_frames(bool psd, const float *hist, int64_t hlen, const float *x, const float *wtab,
                            const float2 *tw, int n, int logn, const float *inv, float *y, float *pw,
                            int64_t frames, hipStream_t st) {
    if (frames <= 0) return hipSuccess;
    const size_t lds = (size_t)n * sizeof(float2) + (size_t)(n / 2) * sizeof(float2);   // at most 96 KB
    // the frame kernels may use more than the default 64 KB of dynamic LDS:
    // raise their limit once per device
    static std::atomic<uint64_t> attr_done{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_done.load() & bit)) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&wh_frames_kernel<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(&wh_frames_kernel<false>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
        if (e != hipSuccess) return e;
        attr_done.fetch_or(bit);
    }
    if (psd)
        hipLaunchKernelGGL(wh_frames_kernel<true>, dim3((unsigned)frames), dim3(kFftThreads), lds, st, hist, hlen,
                           x, wtab, tw, n, logn, inv, y, pw);
    else
        hipLaunchKernelGGL(wh_frames_kernel<false>, dim3((unsigned)frames), dim3(kFftThreads), lds, st, hist, hlen,
                           x, wtab, tw, n, logn, inv, y, pw);
    return hipGetLastError();
}

hipError_t launch_wh_psd_reduce(const float *pw, int64_t frames, int H, double wsum2, double *S, float *inv,
                                hipStream_t st) {
    hipLaunchKernelGGL(wh_psd_reduce_kernel, dim3((unsigned)((H + 1 + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       st, pw, frames, H, wsum2, S, inv);
    return hipGetLastError();
}

hipError_t launch_wh_inv(const double *S, int H, float *inv, hipStream_t st) {
    hipLaunchKernelGGL(wh_inv_kernel, dim3((unsigned)((H + 1 + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, S,
                       H, inv);
    return hipGetLastError();
}

hipError_t launch_wh_ola(const float *y, int64_t nf, int n, const float *pend, float *pend_new, const float *x,
                         int64_t nx, float *hist_new, float *out, hipStream_t st) {
    const int64_t total = nf * (n / 2);
    const int64_t blocks = std::max<int64_t>(1, (total + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(wh_ola_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, y, nf, n, pend, pend_new, x, nx,
                       hist_new, out);
    return hipGetLastError();
}

}  // namespace spiir
