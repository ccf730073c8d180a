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

#include <algorithm>

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

constexpr int kMaxTaps = 64;

// Output pairs (2m, 2m + 1) read the same W samples:
// out(2m) += sum_k g[2k] W(m - k), out(2m + 1) += sum_k g[2k + 1] W(m - k),
// with s[sb + m[u] - k] the staged W(m - k). Each of the NU pairs of a lane
// accumulates its taps in ascending order, as the plain per-output sum does,
// so both forms give the same values.
template <int NU>
__device__ __forceinline__ void interp_pairs(const float2 *s, int sb, const float *sg, int lg, const int (&m)[NU],
                                             float2 (&ev)[NU], float2 (&od)[NU]) {
    // whole (even, odd) tap pairs, then an odd tap count's last even tap: the
    // loop body has no per-tap condition
    const int kp = lg >> 1;
    for (int k = 0; k < kp; ++k) {
        const float ge = sg[2 * k], go = sg[2 * k + 1];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const float2 x = s[sb + m[u] - k];
            ev[u].x = fmaf(ge, x.x, ev[u].x);
            ev[u].y = fmaf(ge, x.y, ev[u].y);
            od[u].x = fmaf(go, x.x, od[u].x);
            od[u].y = fmaf(go, x.y, od[u].y);
        }
    }
    if (lg & 1) {
        const float ge = sg[2 * kp];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            const float2 x = s[sb + m[u] - kp];
            ev[u].x = fmaf(ge, x.x, ev[u].x);
            ev[u].y = fmaf(ge, x.y, ev[u].y);
        }
    }
}

// Every decimation level of a piece in one launch: one workgroup, each level's
// samples kept in LDS (after the lh - 1 history samples of that level) as the
// input of the next; the full-rate input is staged in chunks. Level r
// (1 <= r <= top) is formed from level r - 1 with the taps in the same order
// as mr_decimate_kernel, so the values are those of the per-level launches;
// so are the histories written to hist_new.
constexpr int kPyrThreads = 1024;
constexpr int kPyrChunk = 1024;   // level-1 outputs per staged chunk of the input

// acc = sum_{i < lh} h[i] v(m0 - i), v(m0 - i) = s[-i], taps ascending.
__device__ __forceinline__ float fir_down(const float *sh, const float *s, int lh) {
    float acc = 0.0f;
    int i = 0;
    for (; i + 8 <= lh; i += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = fmaf(sh[i + u], s[-(i + u)], acc);
    }
    for (; i < lh; ++i) acc = fmaf(sh[i], s[-i], acc);
    return acc;
}

__global__ __launch_bounds__(kPyrThreads) void mr_pyramid_kernel(const float *__restrict__ x, int64_t n, int top,
                                                                 MrPyramid pm, const float *__restrict__ h, int lh,
                                                                 int cap0, int cap1) {
    // dynamic LDS: [cap0] level r < top with r odd, [cap1] r even (history, then
    // samples), [2 kPyrChunk + lh - 1] the staged chunk of the full-rate input
    extern __shared__ float pbuf[];
    __shared__ float sh[kMaxTaps];
    const int hl = lh - 1;
    float *xs = pbuf + cap0 + cap1;
    if (threadIdx.x < lh) sh[threadIdx.x] = h[threadIdx.x];
    for (int r = 1; r <= top; ++r) {
        const int64_t ns = n >> (r - 1);
        const int64_t nq = ns / 2;
        const float *hist = pm.hist[r];
        float *ldst = r < top ? pbuf + ((r - 1) & 1) * cap0 : nullptr;
        if (ldst)
            for (int i = threadIdx.x; i < hl; i += kPyrThreads) ldst[i] = pm.hist[r + 1][i];
        if (r == 1) {
            // chunks of kPyrChunk outputs: inputs 2 q0 + 1 - hl .. 2 q0 + 2 kPyrChunk - 1
            for (int64_t q0 = 0; q0 < nq; q0 += kPyrChunk) {
                const int64_t m0 = 2 * q0 + 1 - hl;
                const int cnt = (int)min((int64_t)(2 * kPyrChunk + hl), ns - m0);
                __syncthreads();   // the previous chunk's reads are done
                for (int k = threadIdx.x; k < cnt; k += kPyrThreads) {
                    const int64_t m = m0 + k;
                    xs[k] = m >= 0 ? x[m] : hist[hl + m];
                }
                __syncthreads();
                const int64_t q = q0 + threadIdx.x;
                if (threadIdx.x < kPyrChunk && q < nq) {
                    const float acc = fir_down(sh, xs + (2 * q + 1 - m0), lh);
                    pm.dst[1][q] = acc;
                    if (ldst) ldst[hl + q] = acc;
                }
            }
            for (int i = threadIdx.x; i < hl; i += kPyrThreads) {
                const int64_t m = ns - hl + i;
                pm.hist_new[1][i] = m >= 0 ? x[m] : hist[hl + m];
            }
        } else {
            const float *lsrc = pbuf + ((r - 2) & 1) * cap0;   // level r - 1: lsrc[hl + m] = sample m
            for (int64_t q = threadIdx.x; q < nq; q += kPyrThreads) {
                const float acc = fir_down(sh, lsrc + hl + 2 * q + 1, lh);
                pm.dst[r][q] = acc;
                if (ldst) ldst[hl + q] = acc;
            }
            for (int i = threadIdx.x; i < hl; i += kPyrThreads) pm.hist_new[r][i] = lsrc[hl + ns - hl + i];
        }
        __syncthreads();
    }
}

// Interpolation of every level back to the full rate, fused with the output:
//   W_top = z_top,  W_r(q) = Z_r(q) + sum_{i < lg, q - i even} g[i] W_{r+1}((q - i) / 2)  (r = top - 1 .. 0)
// with Z_r(q) = z[r][zrow[r][j]][q] (0 where the level or the row has no
// filters) and W_r(q) for -hh <= q < 0 taken from the previous call's history
// whist[r][j][hh + q]. Block = one chunk of kKeyChunk template rows x one
// tile of kTile full-rate samples, one wave per row. For the tile each wave
// forms, from the top level down, the window of every level that the tile's
// outputs depend on (level r + 1's window covers the taps of level r's,
// recomputed where tiles overlap) in two LDS buffers used in turn, then
// writes the full-rate z of the tile (Z mode) or its |z|^2 to LDS, from which
// every sample's largest key (|z|^2 bits << 32 | ~j) over the chunk's rows is
// formed (keys mode; plain LDS reads, no atomics). Outputs pair
// up (2m, 2m + 1), which read the same W samples with the even and the odd
// taps; each output adds its taps in ascending order onto Z_r, as the plain
// per-output sum does. The last tile writes every level's next history (the
// last hh samples of W_r) to whist_new.
constexpr int kKeyChunk = 16;
constexpr int kChainThreads = kKeyChunk * 64;
constexpr int kTile = 512;
constexpr int kChainLdsMax = 60 * 1024;   // dynamic LDS of mr_chain_kernel (static part: 384 bytes)

__device__ __forceinline__ int floor_half(int v) { return v >= 0 ? v / 2 : -((-v + 1) / 2); }

__device__ __forceinline__ float2 z_at(const float2 *zj, int q, int n) {
    return zj && q < n ? zj[q] : make_float2(0.0f, 0.0f);
}

// Indices inside a piece fit int32 (a piece has at most max_block samples).
template <bool KEYS>
__global__ __launch_bounds__(kChainThreads) void mr_chain_kernel(MrChain c, int top, int hh,
                                                                 const float *__restrict__ g, int lg, int n_out,
                                                                 int T, int capA, int capB, uint64_t *__restrict__ keys,
                                                                 int64_t ld_keys, float2 *__restrict__ out,
                                                                 int64_t ld_out, int tiles) {
    extern __shared__ __align__(16) float2 wbuf[];   // per wave: capA then capB samples
    __shared__ float sg[kMaxTaps];
    __shared__ int slo[kMaxLevels], shi[kMaxLevels];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int chunk = (int)blockIdx.x / tiles;
    const int tile = (int)blockIdx.x % tiles;
    const bool last = tile == tiles - 1;
    const int p0 = tile * kTile;
    const int j = chunk * kKeyChunk + wv;
    const bool live = j < T;
    float2 *bufA = wbuf + wv * (capA + capB);
    float2 *bufB = bufA + capA;
    if (threadIdx.x == 0) {
        // windows: level 0 = the tile; level r covers the taps of level r - 1's
        // computed part (its non-negative indices; the rest is history)
        slo[0] = p0;
        shi[0] = min(p0 + kTile, n_out) - 1;
        for (int r = 1; r <= top; ++r) {
            const int a = r == 1 ? slo[0] : max(slo[r - 1], 0);
            slo[r] = floor_half(a - lg + 1);
            shi[r] = shi[r - 1] / 2;
        }
    }
    if (threadIdx.x < lg) sg[threadIdx.x] = g[threadIdx.x];
    __syncthreads();
    auto zrow_of = [&](int r) -> const float2 * {
        if (!live || !c.z[r]) return nullptr;
        const int zr = c.zrow[r][j];
        return zr >= 0 ? c.z[r] + (int64_t)zr * c.ld_z[r] : nullptr;
    };
    auto write_hist = [&](int r, const float2 *win) {
        // the last hh samples of W_r lie inside the last tile's window of level r
        if (live && last && lane < hh) c.whist_new[r][j * hh + lane] = win[(n_out >> r) - hh + lane - slo[r]];
    };
    if (top > 0) {
        // top level: W_top = z_top, history below index 0
        float2 *win = (top & 1) ? bufA : bufB;
        const int lo = slo[top], hi = shi[top], nr = n_out >> top;
        const float2 *zj = zrow_of(top);
        if (live)
            for (int q = lo + lane; q <= hi; q += 64)
                win[q - lo] = q >= 0 ? z_at(zj, q, nr) : c.whist[top][j * hh + hh + q];
        __syncthreads();
        write_hist(top, win);
    }
    for (int r = top - 1; r >= 1; --r) {
        float2 *win = (r & 1) ? bufA : bufB;
        const float2 *src = (r & 1) ? bufB : bufA;   // W_{r+1}
        const int lo = slo[r], hi = shi[r], nr = n_out >> r, lo_src = slo[r + 1];
        const int qa = max(lo, 0);
        if (live) {
            for (int q = lo + lane; q < qa; q += 64) win[q - lo] = c.whist[r][j * hh + hh + q];
            const float2 *zj = zrow_of(r);
            const int mlo = qa / 2, mhi = hi / 2;
            for (int m0 = mlo; m0 <= mhi; m0 += 128) {
                int m[2];
                float2 ev[2], od[2];
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int mm = min(m0 + u * 64 + lane, mhi);   // past mhi: a repeat, not written
                    m[u] = mm - mlo;
                    ev[u] = z_at(zj, 2 * mm, nr);
                    od[u] = z_at(zj, 2 * mm + 1, nr);
                }
                interp_pairs<2>(src, mlo - lo_src, sg, lg, m, ev, od);
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    const int mm = m0 + u * 64 + lane;
                    if (mm > mhi) continue;
                    if (2 * mm >= qa) win[2 * mm - lo] = ev[u];
                    if (2 * mm + 1 <= hi) win[2 * mm + 1 - lo] = od[u];
                }
            }
        }
        __syncthreads();
        write_hist(r, win);
    }
    constexpr int NU = kTile / 2 / 64;
    float2 ev[NU], od[NU];
    if (live) {
        const float2 *zj = zrow_of(0);
        int m[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u) {
            m[u] = u * 64 + lane;   // pair m: tile offsets 2m, 2m + 1
            const int p = p0 + 2 * m[u];
            ev[u] = z_at(zj, p, n_out);
            od[u] = z_at(zj, p + 1, n_out);
        }
        if (top > 0) interp_pairs<NU>(bufA, p0 / 2 - slo[1], sg, lg, m, ev, od);
        if (!KEYS) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int p = p0 + 2 * m[u];
                if (p < n_out) out[j * ld_out + p] = ev[u];
                if (p + 1 < n_out) out[j * ld_out + p + 1] = od[u];
            }
        }
    }
    if (KEYS) {
        // |z|^2 of each row into its wave's first buffer (free once every wave
        // has read W_1), then per sample the largest key over the chunk's rows
        __syncthreads();
        float *sq = reinterpret_cast<float *>(bufA);
        if (live) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int t = 2 * (u * 64 + lane);
                sq[t] = ev[u].x * ev[u].x + ev[u].y * ev[u].y;
                sq[t + 1] = od[u].x * od[u].x + od[u].y * od[u].y;
            }
        }
        __syncthreads();
        const int nlive = min(kKeyChunk, T - chunk * kKeyChunk);
        const int wstride = (capA + capB) * 2;   // floats between the waves' buffers
        const float *sq0 = reinterpret_cast<const float *>(wbuf);
        for (int t = threadIdx.x; t < kTile; t += kChainThreads) {
            const int p = p0 + t;
            if (p >= n_out) continue;
            unsigned long long best = 0ull;
            for (int w = 0; w < nlive; ++w) {
                const unsigned long long key = ((unsigned long long)__float_as_uint(sq0[w * wstride + t]) << 32) |
                                               (unsigned long long)(0xFFFFFFFFu - (uint32_t)(chunk * kKeyChunk + w));
                best = key > best ? key : best;
            }
            keys[chunk * ld_keys + p] = best;
        }
    }
}

// The replayed piece's max / argmax out of the graph's buffers, one launch
// for both arrays.
__global__ __launch_bounds__(kThreads) void mr_copy_out_kernel(float *__restrict__ mx, const float *__restrict__ mxo,
                                                               int32_t *__restrict__ am,
                                                               const int32_t *__restrict__ amo, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) {
        mx[i] = mxo[i];
        am[i] = amo[i];
    }
}

}  // namespace

hipError_t launch_mr_copy_out(float *mx, const float *mxo, int32_t *am, const int32_t *amo, int64_t n,
                              hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(mr_copy_out_kernel, dim3((unsigned)nblk(n, kThreads)), dim3(kThreads), 0, st, mx, mxo, am, amo,
                       n);
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

void mr_chain_caps(int top, int lg, int *capA, int *capB) {
    // window lengths: level 1 at most (kTile + lg + 1) / 2, level r at most
    // (len_{r-1} + lg + 1) / 2 + 1; odd levels share buffer A, even ones B
    int cap = kTile;
    *capA = kTile / 2;   // at least the tile's |z|^2 (kTile floats) for the keys
    *capB = 0;
    for (int r = 1; r <= top; ++r) {
        cap = (cap + lg + 1) / 2 + 1;
        int &slot = (r & 1) ? *capA : *capB;
        slot = std::max(slot, cap);
    }
}

size_t mr_chain_lds(int top, int lg) {
    int capA = 0, capB = 0;
    mr_chain_caps(top, lg, &capA, &capB);
    return (size_t)kKeyChunk * (size_t)(capA + capB) * sizeof(float2);
}

hipError_t launch_mr_chain(const MrChain &c, int top, int hh, const float *g, int lg, int64_t n_out, int T,
                           uint64_t *keys, int64_t ld_keys, float2 *out, int64_t ld_out, hipStream_t st) {
    if (n_out <= 0) return hipSuccess;
    int capA = 0, capB = 0;
    mr_chain_caps(top, lg, &capA, &capB);
    const size_t lds = mr_chain_lds(top, lg);
    // at most 59,776 bytes (64 taps), within the default 64 KB with the static part
    if (lds > (size_t)kChainLdsMax) return hipErrorInvalidValue;
    if (n_out > INT32_MAX - kTile) return hipErrorInvalidValue;   // tile-local indices are int32
    const int tiles = (int)nblk(n_out, kTile);
    const unsigned grid = (unsigned)(tiles * mr_key_chunks(T));
    const int n = (int)n_out;
    if (keys)
        hipLaunchKernelGGL(mr_chain_kernel<true>, dim3(grid), dim3(kChainThreads), lds, st, c, top, hh, g, lg, n, T,
                           capA, capB, keys, ld_keys, out, ld_out, tiles);
    else
        hipLaunchKernelGGL(mr_chain_kernel<false>, dim3(grid), dim3(kChainThreads), lds, st, c, top, hh, g, lg, n, T,
                           capA, capB, keys, ld_keys, out, ld_out, tiles);
    return hipGetLastError();
}

size_t mr_pyramid_lds(int64_t B, int top, int lh) {
    // level buffers (levels 1..top-1) and the staged input chunk
    const int64_t hl = lh - 1;
    const int64_t cap0 = top >= 2 ? hl + (B >> 1) : 0, cap1 = top >= 3 ? hl + (B >> 2) : 0;
    return (size_t)(cap0 + cap1 + 2 * kPyrChunk + hl) * sizeof(float);
}

hipError_t launch_mr_pyramid(const float *x, int64_t n, int top, const MrPyramid &pm, const float *h, int lh,
                             int64_t B, hipStream_t st) {
    const int hl = lh - 1;
    const int cap0 = top >= 2 ? (int)(hl + (B >> 1)) : 0, cap1 = top >= 3 ? (int)(hl + (B >> 2)) : 0;
    hipLaunchKernelGGL(mr_pyramid_kernel, dim3(1), dim3(kPyrThreads), mr_pyramid_lds(B, top, lh), st, x, n, top, pm,
                       h, lh, cap0, cap1);
    return hipGetLastError();
}

int mr_key_chunks(int T) { return (T + kKeyChunk - 1) / kKeyChunk; }

}  // namespace spiir
