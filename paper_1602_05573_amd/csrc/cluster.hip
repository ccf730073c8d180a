// Trigger clustering over the fused per-sample maximum: the step after the
// filtering that turns the detection statistic into triggers (Sect. "GPU
// accelerated SPIIR method", subsection "SPIIR method": the SNR output is what
// identifies a signal; Sect. "Multimessenger astronomy": low-latency trigger
// generation). Reading of the clustering rule: sample m is a trigger when
//   max[m] >= threshold,
//   max[i] <  max[m] for every i in [m - W, m)        (earliest sample wins ties),
//   max[i] <= max[m] for every i in (m, m + W],
// windows clipped to the series. Triggers are therefore more than W apart and
// each is the peak of the samples within W of it.
//
// Four launches, all linear in n:
//   reduce : order-preserving 32-bit keys, maxima of 64-sample blocks (one wave)
//            and of 4,096-sample blocks (one workgroup)
//   find   : per sample, threshold test, then the two window maxima taken
//            nearest first from samples, 64-blocks and 4,096-blocks, stopping at
//            the first larger key; a 64-bit ballot mask per 64-block and a count
//            per 4,096-block
//   scan   : one workgroup, exclusive prefix of the 4,096-block counts
//   write  : triggers in increasing sample order, clipped to the capacity
// A 64-block whose maximum is below the threshold is skipped by find without
// reading its samples, so for a threshold well above the noise the only full
// pass over max[] is the reduce launch.
#include "spiir_internal.h"

namespace spiir {
namespace {

constexpr int kB1 = 64;     // level-1 block: one wave, one mask word
constexpr int kB2 = 4096;   // level-2 block: one workgroup
constexpr int kThreads = 256;

typedef float f4 __attribute__((ext_vector_type(4), aligned(4)));

// Order-preserving key: a < b  <=>  key(a) < key(b) for non-NaN floats, -0 and
// +0 share a key, every NaN maps above +inf and the smallest key (-inf) is
// above 0, so 0 is the maximum of an empty range.
__host__ __device__ inline uint32_t okey(float v) {
    uint32_t u;
    __builtin_memcpy(&u, &v, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0xffffffffu;
    if (u == 0x80000000u) u = 0;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ inline uint32_t max16(uint32_t k) {
    k = max(k, (uint32_t)__shfl_xor((int)k, 1));
    k = max(k, (uint32_t)__shfl_xor((int)k, 2));
    k = max(k, (uint32_t)__shfl_xor((int)k, 4));
    k = max(k, (uint32_t)__shfl_xor((int)k, 8));
    return k;
}

// One workgroup per 4,096-block c: thread t reads samples 4q..4q+3 of the block
// for q = t + 256 j (j = 0..3); the 16 lanes holding q/16 = b share a 64-block.
__global__ __launch_bounds__(kThreads) void clus_reduce_kernel(const float *__restrict__ M, int64_t n,
                                                               uint32_t *__restrict__ bm1,
                                                               uint32_t *__restrict__ bm2) {
    __shared__ uint32_t wmax[kThreads / 64];
    const int64_t c = blockIdx.x;
    const int64_t base = c * kB2;
    const int t = threadIdx.x;
    uint32_t kq[4];
    if (base + kB2 <= n) {
        f4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = *reinterpret_cast<const f4 *>(M + base + 4 * (t + kThreads * j));
#pragma unroll
        for (int j = 0; j < 4; ++j)
            kq[j] = max(max(okey(v[j].x), okey(v[j].y)), max(okey(v[j].z), okey(v[j].w)));
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint32_t k = 0;
            for (int e = 0; e < 4; ++e) {
                const int64_t i = base + 4 * (t + kThreads * j) + e;
                if (i < n) k = max(k, okey(M[i]));
            }
            kq[j] = k;
        }
    }
    const int64_t nb1 = (n + kB1 - 1) / kB1;
    uint32_t k2 = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const uint32_t k = max16(kq[j]);
        const int64_t b = c * (kB2 / kB1) + (t + kThreads * j) / 16;
        if ((t & 15) == 0 && b < nb1) bm1[b] = k;
        k2 = max(k2, k);
    }
    k2 = max(k2, (uint32_t)__shfl_xor((int)k2, 16));
    k2 = max(k2, (uint32_t)__shfl_xor((int)k2, 32));
    if ((t & 63) == 0) wmax[t >> 6] = k2;
    __syncthreads();
    if (t == 0) {
        uint32_t k = wmax[0];
        for (int w = 1; w < kThreads / 64; ++w) k = max(k, wmax[w]);
        bm2[c] = k;
    }
}

// True when no key in [lo, m) reaches km and no key in (m, e) exceeds km, with
// lo = max(0, m - W), e = min(n, m + W + 1). Every range is covered nearest
// first by samples up to a 64-block boundary, then 64-blocks up to a
// 4,096-block boundary, then 4,096-blocks, then 64-blocks and samples again;
// a block is only used when it lies wholly inside the range, so partial blocks
// at the end of the series are never read as blocks.
__device__ bool is_peak(const float *__restrict__ M, int64_t n, int64_t m, uint32_t km, int64_t W,
                        const uint32_t *__restrict__ bm1, const uint32_t *__restrict__ bm2) {
    const int64_t lo = m - W > 0 ? m - W : 0;
    const int64_t e = m + W + 1 < n ? m + W + 1 : n;
    // the direct neighbours first: a rising or falling edge fails here
    if (m - 1 >= lo && okey(M[m - 1]) >= km) return false;
    if (m + 1 < e && okey(M[m + 1]) > km) return false;

    int64_t p = m;
    const int64_t e1 = (m / kB1) * kB1 > lo ? (m / kB1) * kB1 : lo;
    for (; p > e1; --p)
        if (okey(M[p - 1]) >= km) return false;
    for (; p > lo && p % kB2 != 0 && p - kB1 >= lo; p -= kB1)
        if (bm1[p / kB1 - 1] >= km) return false;
    for (; p - kB2 >= lo; p -= kB2)
        if (bm2[p / kB2 - 1] >= km) return false;
    for (; p - kB1 >= lo; p -= kB1)
        if (bm1[p / kB1 - 1] >= km) return false;
    for (; p > lo; --p)
        if (okey(M[p - 1]) >= km) return false;

    p = m + 1;
    for (; p < e && p % kB1 != 0; ++p)
        if (okey(M[p]) > km) return false;
    for (; p % kB2 != 0 && p + kB1 <= e; p += kB1)
        if (bm1[p / kB1] > km) return false;
    for (; p + kB2 <= e; p += kB2)
        if (bm2[p / kB2] > km) return false;
    for (; p + kB1 <= e; p += kB1)
        if (bm1[p / kB1] > km) return false;
    for (; p < e; ++p)
        if (okey(M[p]) > km) return false;
    return true;
}

// One workgroup per 4,096-block c; wave w takes its 64-blocks c*64 + 16w .. +15,
// one sample per lane.
__global__ __launch_bounds__(kThreads) void clus_find_kernel(const float *__restrict__ M, int64_t n,
                                                             float thr, uint32_t kthr, int64_t W,
                                                             const uint32_t *__restrict__ bm1,
                                                             const uint32_t *__restrict__ bm2,
                                                             uint64_t *__restrict__ mask,
                                                             uint32_t *__restrict__ cnt2) {
    __shared__ uint32_t wc[kThreads / 64];
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nb1 = (n + kB1 - 1) / kB1;
    uint32_t cnt = 0;
    for (int it = 0; it < kB2 / kB1 / (kThreads / 64); ++it) {
        const int64_t b = c * (kB2 / kB1) + w * (kB2 / kB1 / (kThreads / 64)) + it;
        if (b >= nb1) break;
        uint64_t bits = 0;
        if (bm1[b] >= kthr) {
            const int64_t m = b * kB1 + lane;
            bool hit = false;
            if (m < n) {
                const float v = M[m];
                if (v >= thr) hit = is_peak(M, n, m, okey(v), W, bm1, bm2);
            }
            bits = __ballot(hit);
        }
        if (lane == 0) mask[b] = bits;
        cnt += (uint32_t)__popcll(bits);
    }
    if (lane == 0) wc[w] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int i = 0; i < kThreads / 64; ++i) s += wc[i];
        cnt2[c] = s;
    }
}

// Exclusive prefix of the nb2 block counts in one workgroup of 1,024 threads,
// each owning a contiguous run; the total goes to *count.
__global__ __launch_bounds__(1024) void clus_scan_kernel(const uint32_t *__restrict__ cnt2, int64_t nb2,
                                                         int64_t *__restrict__ off2,
                                                         int64_t *__restrict__ count) {
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb2 + 1023) / 1024;
    const int64_t s0 = min(nb2, (int64_t)t * per), s1 = min(nb2, s0 + per);
    int64_t sum = 0;
    for (int64_t i = s0; i < s1; ++i) sum += cnt2[i];
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const int64_t v = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = part[t] - sum;
    for (int64_t i = s0; i < s1; ++i) {
        off2[i] = run;
        run += cnt2[i];
    }
    if (t == 1023) *count = part[1023];
}

// One workgroup per 4,096-block with triggers: the first wave ranks the 64 mask
// words, then each wave writes whole words, lane = bit, so a word's triggers
// land in consecutive slots.
__global__ __launch_bounds__(kThreads) void clus_write_kernel(const float *__restrict__ M,
                                                              const int32_t *__restrict__ J, int64_t n,
                                                              const uint64_t *__restrict__ mask,
                                                              const uint32_t *__restrict__ cnt2,
                                                              const int64_t *__restrict__ off2, int64_t cap,
                                                              int64_t *__restrict__ idx,
                                                              int32_t *__restrict__ tpl,
                                                              float *__restrict__ val) {
    __shared__ uint64_t mk[kB2 / kB1];
    __shared__ uint32_t pre[kB2 / kB1];
    const int64_t c = blockIdx.x;
    if (cnt2[c] == 0) return;
    const int64_t off = off2[c];
    if (off >= cap) return;
    const int t = threadIdx.x;
    const int64_t nb1 = (n + kB1 - 1) / kB1;
    if (t < 64) {
        const int64_t b = c * (kB2 / kB1) + t;
        const uint64_t mm = b < nb1 ? mask[b] : 0;
        const uint32_t pc = (uint32_t)__popcll(mm);
        uint32_t s = pc;
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = (uint32_t)__shfl_up((int)s, d);
            if (t >= d) s += o;
        }
        mk[t] = mm;
        pre[t] = s - pc;
    }
    __syncthreads();
    const int lane = t & 63;
    for (int i = t >> 6; i < kB2 / kB1; i += kThreads / 64) {
        const uint64_t mm = mk[i];
        if (((mm >> lane) & 1) == 0) continue;
        const int64_t pos = off + pre[i] + __popcll(mm & ((1ull << lane) - 1));
        if (pos >= cap) continue;
        const int64_t m = (c * (kB2 / kB1) + i) * kB1 + lane;
        idx[pos] = m;
        tpl[pos] = J[m];
        val[pos] = M[m];
    }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct ClusterWs {
    uint32_t *bm1, *bm2, *cnt2;
    uint64_t *mask;
    int64_t *off2;
};

size_t carve(void *ws, int64_t n, ClusterWs *out) {
    const size_t nb1 = (size_t)((n + kB1 - 1) / kB1), nb2 = (size_t)((n + kB2 - 1) / kB2);
    char *p = static_cast<char *>(ws);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *q = p ? p + o : nullptr;
        o += align256(bytes);
        return q;
    };
    ClusterWs w;
    w.bm1 = reinterpret_cast<uint32_t *>(take(nb1 * 4));
    w.bm2 = reinterpret_cast<uint32_t *>(take(nb2 * 4));
    w.mask = reinterpret_cast<uint64_t *>(take(nb1 * 8));
    w.cnt2 = reinterpret_cast<uint32_t *>(take(nb2 * 4));
    w.off2 = reinterpret_cast<int64_t *>(take(nb2 * 8));
    if (out) *out = w;
    return o;
}

}  // namespace

size_t cluster_workspace_bytes(int64_t n) { return carve(nullptr, n, nullptr); }

hipError_t launch_cluster(const float *M, const int32_t *J, int64_t n, float thr, int64_t W, void *ws,
                          int64_t cap, int64_t *idx, int32_t *tpl, float *val, int64_t *count,
                          hipStream_t st) {
    ClusterWs w;
    carve(ws, n, &w);
    const int64_t nb2 = (n + kB2 - 1) / kB2;
    if (nb2 > 0) {
        hipLaunchKernelGGL(clus_reduce_kernel, dim3((unsigned)nb2), dim3(kThreads), 0, st, M, n, w.bm1, w.bm2);
        hipLaunchKernelGGL(clus_find_kernel, dim3((unsigned)nb2), dim3(kThreads), 0, st, M, n, thr, okey(thr), W,
                           w.bm1, w.bm2, w.mask, w.cnt2);
    }
    hipLaunchKernelGGL(clus_scan_kernel, dim3(1), dim3(1024), 0, st, w.cnt2, nb2, w.off2, count);
    if (nb2 > 0 && cap > 0)
        hipLaunchKernelGGL(clus_write_kernel, dim3((unsigned)nb2), dim3(kThreads), 0, st, M, J, n, w.mask,
                           w.cnt2, w.off2, cap, idx, tpl, val);
    return hipGetLastError();
}

}  // namespace spiir
