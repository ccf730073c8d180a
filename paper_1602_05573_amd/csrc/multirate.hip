// Multi-rate filter bank: the resampling and recombination around the
// per-level filter banks. The paper remarks that a slowly evolving chirp lets
// both the data and the templates run at a lower sampling rate (Sect.
// "Multimessenger astronomy"); this library's reading:
//   x_r[q]  = sum_i h[i] x_{r-1}[2q + 1 - i]                 (decimation, causal FIR)
//   z_r     = level-r template sums of filters run on x_r      (ordinary bank, z mode)
//   w_R     = z_R,  w_r[p] = z_r[p] + sum_q g[p - 2q] w_{r+1}[q]   (interpolation, causal FIR)
//   z       = w_0, then |z|^2 and the per-sample max / argmax over templates.
// All kernels here are streaming: each level keeps the last samples of its
// resampling input as history, so consecutive calls continue one stream.
#include "spiir_internal.h"

namespace spiir {
namespace {

constexpr int kThreads = 256;

int64_t nblk(int64_t n, int64_t b) { return (n + b - 1) / b; }

// dst[q] = sum_i h[i] v(2q + 1 - i) for q < n_src / 2, with v(m) = src[m] for
// m >= 0 and hist[lh - 1 + m] (the previous lh - 1 samples) for m < 0. Block 0
// also writes the next call's history (the last lh - 1 samples of v) to
// hist_new, a different buffer than hist.
__global__ __launch_bounds__(kThreads) void mr_decimate_kernel(const float *__restrict__ src, int64_t n_src,
                                                               const float *__restrict__ hist,
                                                               float *__restrict__ hist_new,
                                                               const float *__restrict__ h, int lh,
                                                               float *__restrict__ dst) {
    const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t nq = n_src / 2;
    if (q < nq) {
        float acc = 0.0f;
        for (int i = 0; i < lh; ++i) {
            const int64_t m = 2 * q + 1 - i;
            const float v = m >= 0 ? src[m] : hist[lh - 1 + m];
            acc = fmaf(h[i], v, acc);
        }
        dst[q] = acc;
    }
    if (blockIdx.x == 0 && threadIdx.x < lh - 1) {
        const int64_t m = n_src - (lh - 1) + threadIdx.x;
        hist_new[threadIdx.x] = m >= 0 ? src[m] : hist[lh - 1 + m];
    }
}

// One template row j per blockIdx.x / tiles, kOut = 1,024 output samples per
// block of 256 threads (two adjacent pairs per thread):
//   out[j][p] = Z(j, p) + sum_{i < lg, p - i even} g[i] W(j, (p - i) / 2)
// Z(j, p) = z[zrow[j]][p] (0 if z is NULL or zrow[j] < 0); W(j, q) =
// w[wrow(j)][q] for q >= 0 (wrow = identity if NULL; 0 if wrow[j] < 0) and
// whist[j][hh + q] for -hh <= q < 0, hh = lg / 2. w == NULL: no interpolation
// term. The block first stages the W samples its outputs need (at most
// kOut / 2 + hh + 1) and the taps in LDS, so the tap loop reads LDS only. The
// first block of a row writes the row's next history (the last hh samples of
// W) to whist_new.
constexpr int kMaxTaps = 64;
constexpr int kOut = 4 * kThreads;

__device__ inline float2 w_at(const float2 *wj, const float2 *hj, int hh, int64_t q) {
    if (q >= 0) return wj ? wj[q] : make_float2(0.0f, 0.0f);
    return hj[hh + q];
}

// Outputs t = 2m and 2m + 1 of a tile (t = p - p0) read the same W samples:
// out(2m) += sum_k g[2k] W(m' - k), out(2m + 1) += sum_k g[2k + 1] W(m' - k),
// m' = p0 / 2 + m, with s[sb + m - k] the staged W(m' - k). Each of the NU
// pairs of a lane accumulates its taps in ascending order, as the plain
// per-output sum does, so both forms give the same values.
template <int NU>
__device__ __forceinline__ void interp_pairs(const float2 *s, int sb, const float *sg, int lg, const int (&m)[NU],
                                             float2 (&ev)[NU], float2 (&od)[NU]) {
    for (int k = 0; 2 * k < lg; ++k) {
        const float ge = sg[2 * k];
        const bool odd = 2 * k + 1 < lg;   // uniform
        const float go = sg[2 * k + 1];    // inside the staged taps (lg <= kMaxTaps)
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const float2 x = s[sb + m[u] - k];
            ev[u].x = fmaf(ge, x.x, ev[u].x);
            ev[u].y = fmaf(ge, x.y, ev[u].y);
            if (odd) {
                od[u].x = fmaf(go, x.x, od[u].x);
                od[u].y = fmaf(go, x.y, od[u].y);
            }
        }
    }
}

__global__ __launch_bounds__(kThreads) void mr_upsample_add_kernel(
    const float2 *__restrict__ z, int64_t ld_z, const int32_t *__restrict__ zrow, const float2 *__restrict__ w,
    int64_t ld_w, const int32_t *__restrict__ wrow, int64_t n_w, const float2 *__restrict__ whist,
    float2 *__restrict__ whist_new, int hh, const float *__restrict__ g, int lg, float2 *__restrict__ out,
    int64_t ld_out, int64_t n_out, int64_t tiles) {
    __shared__ float2 sw[kOut / 2 + kMaxTaps / 2 + 2];
    __shared__ float sg[kMaxTaps];
    const int64_t j = blockIdx.x / tiles;
    const int64_t tile = blockIdx.x % tiles;
    const int64_t p0 = tile * kOut;
    const int zr = (z && zrow) ? zrow[j] : -1;
    const int wr = w ? (wrow ? wrow[j] : (int)j) : -1;
    const float2 *wj = wr >= 0 ? w + (int64_t)wr * ld_w : nullptr;
    const float2 *hj = whist ? whist + j * hh : nullptr;
    // staged W(j, q) for q in [q_lo, q_lo + cnt): q_lo = floor((p0 - lg + 1) / 2) >= -hh
    const int64_t v = p0 - lg + 1;
    const int64_t q_lo = v >= 0 ? v / 2 : -((-v + 1) / 2);
    const int cnt = (int)((p0 + kOut - 1) / 2 - q_lo + 1);
    if (w) {
        for (int k = threadIdx.x; k < cnt; k += kThreads) {
            const int64_t q = q_lo + k;
            sw[k] = q < n_w ? w_at(wj, hj, hh, q) : make_float2(0.0f, 0.0f);
        }
        if (threadIdx.x < lg) sg[threadIdx.x] = g[threadIdx.x];
    }
    __syncthreads();
    const float2 *zj = zr >= 0 ? z + (int64_t)zr * ld_z : nullptr;
    float2 *oj = out + j * ld_out;
    constexpr int NU = kOut / 2 / kThreads;
    int m[NU];
    float2 ev[NU], od[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        m[u] = u * kThreads + (int)threadIdx.x;   // pair m: tile offsets 2m, 2m + 1
        const int64_t p = p0 + 2 * m[u];
        ev[u] = zj && p < n_out ? zj[p] : make_float2(0.0f, 0.0f);
        od[u] = zj && p + 1 < n_out ? zj[p + 1] : make_float2(0.0f, 0.0f);
    }
    if (w) interp_pairs<NU>(sw, (int)(p0 / 2 - q_lo), sg, lg, m, ev, od);
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int64_t p = p0 + 2 * m[u];
        if (p < n_out) oj[p] = ev[u];
        if (p + 1 < n_out) oj[p + 1] = od[u];
    }
    if (w && tile == 0 && threadIdx.x < hh) whist_new[j * hh + threadIdx.x] = w_at(wj, hj, hh, n_w - hh + threadIdx.x);
}

// Templates per key chunk (rows folded into one per-sample key).
constexpr int kKeyChunk = 16;

// The last interpolation (into level 0) fused with the per-sample keys:
// block = one chunk of kKeyChunk template rows x kOut samples, one wave per
// row. Each wave stages its row's W samples in its own LDS slice, forms the
// full-rate z of its kOut / 64 samples per lane (8 adjacent pairs) as
// mr_upsample_add_kernel does, and folds its keys into the block's
// per-sample maximum (LDS atomics); the full-rate z itself is never stored.
// Tile 0 also writes every row's next interpolation history.
constexpr int kSw = kOut / 2 + kMaxTaps / 2 + 2;
constexpr int kFuseThreads = kKeyChunk * 64;

__global__ __launch_bounds__(kFuseThreads) void mr_interp_keys_kernel(
    const float2 *__restrict__ z, int64_t ld_z, const int32_t *__restrict__ zrow, const float2 *__restrict__ w,
    int64_t ld_w, const int32_t *__restrict__ wrow, int64_t n_w, const float2 *__restrict__ whist,
    float2 *__restrict__ whist_new, int hh, const float *__restrict__ g, int lg, int64_t n_out, int T,
    uint64_t *__restrict__ keys, int64_t ld_keys, int64_t tiles) {
    __shared__ float2 sw[kKeyChunk][kSw];
    __shared__ float sg[kMaxTaps];
    __shared__ unsigned long long kred[kOut];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t chunk = blockIdx.x / tiles;
    const int64_t tile = blockIdx.x % tiles;
    const int64_t p0 = tile * kOut;
    const int64_t j = chunk * kKeyChunk + wv;
    const bool live = j < T;
    const int zr = (live && z && zrow) ? zrow[j] : -1;
    const int wr = (live && w) ? (wrow ? wrow[j] : (int)j) : -1;
    const float2 *wj = wr >= 0 ? w + (int64_t)wr * ld_w : nullptr;
    const float2 *hj = (live && whist) ? whist + j * hh : nullptr;
    const int64_t v = p0 - lg + 1;
    const int64_t q_lo = v >= 0 ? v / 2 : -((-v + 1) / 2);
    const int cnt = (int)((p0 + kOut - 1) / 2 - q_lo + 1);
    for (int t = threadIdx.x; t < kOut; t += kFuseThreads) kred[t] = 0ull;
    if (threadIdx.x < lg) sg[threadIdx.x] = g[threadIdx.x];
    if (live && w)
        for (int k = lane; k < cnt; k += 64) {
            const int64_t q = q_lo + k;
            sw[wv][k] = q < n_w ? w_at(wj, hj, hh, q) : make_float2(0.0f, 0.0f);
        }
    __syncthreads();
    if (live) {
        const float2 *zj = zr >= 0 ? z + (int64_t)zr * ld_z : nullptr;
        const unsigned long long jkey = 0xFFFFFFFFu - (uint32_t)j;
        constexpr int NU = kOut / 2 / 64;
        int m[NU];
        float2 ev[NU], od[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            m[u] = u * 64 + lane;   // pair m: tile offsets 2m, 2m + 1
            const int64_t p = p0 + 2 * m[u];
            ev[u] = zj && p < n_out ? zj[p] : make_float2(0.0f, 0.0f);
            od[u] = zj && p + 1 < n_out ? zj[p + 1] : make_float2(0.0f, 0.0f);
        }
        if (w) interp_pairs<NU>(sw[wv], (int)(p0 / 2 - q_lo), sg, lg, m, ev, od);
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const int64_t p = p0 + 2 * m[u];
            const float se = ev[u].x * ev[u].x + ev[u].y * ev[u].y;
            const float so = od[u].x * od[u].x + od[u].y * od[u].y;
            if (p < n_out) atomicMax(&kred[2 * m[u]], ((unsigned long long)__float_as_uint(se) << 32) | jkey);
            if (p + 1 < n_out) atomicMax(&kred[2 * m[u] + 1], ((unsigned long long)__float_as_uint(so) << 32) | jkey);
        }
        if (w && tile == 0 && lane < hh) whist_new[j * hh + lane] = w_at(wj, hj, hh, n_w - hh + lane);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kOut; t += kFuseThreads) {
        const int64_t p = p0 + t;
        if (p < n_out) keys[chunk * ld_keys + p] = kred[t];
    }
}

}  // namespace

hipError_t launch_mr_interp_keys(const float2 *z, int64_t ld_z, const int32_t *zrow, const float2 *w, int64_t ld_w,
                                 const int32_t *wrow, int64_t n_w, const float2 *whist, float2 *whist_new, int hh,
                                 const float *g, int lg, int64_t n_out, int T, uint64_t *keys, int64_t ld_keys,
                                 hipStream_t st) {
    if (n_out <= 0) return hipSuccess;
    const int64_t tiles = nblk(n_out, kOut);
    hipLaunchKernelGGL(mr_interp_keys_kernel, dim3((unsigned)(tiles * mr_key_chunks(T))), dim3(kFuseThreads), 0,
                       st, z, ld_z, zrow, w, ld_w, wrow, n_w, whist, whist_new, hh, g, lg, n_out, T, keys, ld_keys,
                       tiles);
    return hipGetLastError();
}

hipError_t launch_mr_decimate(const float *src, int64_t n_src, const float *hist, float *hist_new,
                              const float *h, int lh, float *dst, hipStream_t st) {
    const int64_t nq = n_src / 2;
    const int64_t blocks = std::max<int64_t>(1, nblk(nq, kThreads));
    hipLaunchKernelGGL(mr_decimate_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, st, src, n_src, hist,
                       hist_new, h, lh, dst);
    return hipGetLastError();
}

hipError_t launch_mr_upsample_add(const float2 *z, int64_t ld_z, const int32_t *zrow, const float2 *w,
                                  int64_t ld_w, const int32_t *wrow, int64_t n_w, const float2 *whist,
                                  float2 *whist_new, int hh, const float *g, int lg, float2 *out,
                                  int64_t ld_out, int64_t n_out, int T, hipStream_t st) {
    const int64_t tiles = std::max<int64_t>(1, nblk(n_out, kOut));
    hipLaunchKernelGGL(mr_upsample_add_kernel, dim3((unsigned)(tiles * T)), dim3(kThreads), 0, st, z, ld_z, zrow,
                       w, ld_w, wrow, n_w, whist, whist_new, hh, g, lg, out, ld_out, n_out, tiles);
    return hipGetLastError();
}

int mr_key_chunks(int T) { return (T + kKeyChunk - 1) / kKeyChunk; }

}  // namespace spiir
