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
// Three launches (four for series of more than 8,192 4,096-blocks):
//   reduce : order-preserving 32-bit keys, maxima of 64-sample blocks (one wave)
//            and of 4,096-sample blocks (one workgroup)
//   find   : per sample, threshold and direct-neighbour tests, then the two
//            window maxima over samples, 64-blocks and 4,096-blocks (by the
//            whole wave for a few survivors, by each lane otherwise); a 64-bit
//            ballot mask per 64-block and a count per 4,096-block
//   (scan) : long series only: one workgroup, exclusive prefix of the counts
//   write  : triggers in increasing sample order, clipped to the capacity; for
//            short series each 4,096-block with triggers sums the counts before
//            it (the cost is the square of the block count, hence the limit)
//            and the last block writes the total
// A 64-block whose maximum is below the threshold is skipped by find without
// reading its samples, so for a threshold well above the noise the only full
// pass over max[] is the reduce launch.
#include "spiir_internal.h"

namespace spiir {
namespace {

constexpr int kB1 = 64;     // level-1 block: one wave, one mask word
constexpr int kB2 = 4096;   // level-2 block: one workgroup
constexpr int kThreads = 256;
constexpr int64_t kInlinePrefix = 8192;  // most 4,096-blocks whose offsets the write launch sums itself

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

// Per-lane test of sample m: no key in [lo, m) reaches km and no key in
// (m, e) exceeds km, with lo = max(0, m - W), e = min(n, m + W + 1). Each range
// is covered nearest first by samples up to a 64-block boundary, then 64-blocks
// up to a 4,096-block boundary, then 4,096-blocks, then 64-blocks and samples
// again, stopping at the first larger key; a block is only used when it lies
// wholly inside the range, so partial blocks at the end of the series are
// never read as blocks. Used when many lanes of a wave are candidates.
__device__ bool is_peak_lane(const float *__restrict__ M, int64_t n, int64_t m, uint32_t km, int64_t W,
                             const uint32_t *__restrict__ bm1, const uint32_t *__restrict__ bm2) {
    const int64_t lo = m - W > 0 ? m - W : 0;
    const int64_t e = m + W + 1 < n ? m + W + 1 : n;
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

// Exclusive prefix of the nb2 block counts in one workgroup of 1,024 threads,
// each owning a contiguous run; the total goes to *count. Used for long series
// (more than kInlinePrefix blocks).
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

// Count of an empty series.
__global__ void clus_zero_count_kernel(int64_t *count) { *count = 0; }

__device__ inline uint32_t wave_max(uint32_t k) {
    for (int o = 1; o < 64; o <<= 1) k = max(k, (uint32_t)__shfl_xor((int)k, o));
    return k;
}

// This lane's share of the maximum key over samples [a, z) (a, z uniform across
// the wave): samples up to the nearest 64-block boundaries, whole 64-blocks up
// to the nearest 4,096-block boundaries and whole 4,096-blocks in between, each
// piece one predicated load per lane, so the loads of every piece are in flight
// together. Blocks are only read when they lie wholly inside [a, z).
__device__ uint32_t range_max_part(const float *__restrict__ M, const uint32_t *__restrict__ bm1,
                                   const uint32_t *__restrict__ bm2, int64_t a, int64_t z, int lane) {
    uint32_t k = 0;
    if (a >= z) return k;
    const int64_t L1 = (a + kB1 - 1) / kB1 * kB1, H1 = z / kB1 * kB1;
    if (L1 >= H1) {
        // at most one 64-block boundary inside: fewer than 128 samples
        for (int64_t i = a + lane; i < z; i += 64) k = max(k, okey(M[i]));
        return k;
    }
    if (a + lane < L1) k = max(k, okey(M[a + lane]));
    if (H1 + lane < z) k = max(k, okey(M[H1 + lane]));
    const int64_t L2 = (a + kB2 - 1) / kB2 * kB2, H2 = z / kB2 * kB2;
    if (L2 <= H2) {
        if (L1 + kB1 * lane < L2) k = max(k, bm1[L1 / kB1 + lane]);
        if (H2 + kB1 * lane < H1) k = max(k, bm1[H2 / kB1 + lane]);
        for (int64_t j = L2 / kB2 + lane; j < H2 / kB2; j += 64) k = max(k, bm2[j]);
    } else if (L1 + kB1 * lane < H1) {
        // a and z in one 4,096-block: fewer than 64 whole 64-blocks
        k = max(k, bm1[L1 / kB1 + lane]);
    }
    return k;
}

// One workgroup of 16 waves per 4,096-block c. Every wave reads the 64 block
// maxima of c; blocks below the threshold are skipped without reading their
// samples, and the live blocks are dealt round robin by rank to the waves (the
// samples above a threshold come in runs, so neighbouring live blocks go to
// different waves). Only samples in [c_lo, c_hi) can trigger; the others serve
// as window neighbours. In a live block each lane tests one sample: threshold and
// the two direct neighbours (rising and falling edges fail there); the
// survivors are tested on their whole windows, one at a time by the whole wave
// when few, else each by its own lane.
constexpr int kFindThreads = 1024;
constexpr int kWaveTestMax = 4;

__global__ __launch_bounds__(kFindThreads) void clus_find_kernel(const float *__restrict__ M, int64_t n,
                                                                 float thr, uint32_t kthr, int64_t W,
                                                                 int64_t c_lo, int64_t c_hi,
                                                                 const uint32_t *__restrict__ bm1,
                                                                 const uint32_t *__restrict__ bm2,
                                                                 uint64_t *__restrict__ mask,
                                                                 uint32_t *__restrict__ cnt2) {
    constexpr int kWaves = kFindThreads / 64;
    __shared__ uint32_t wc[kWaves];
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t nb1 = (n + kB1 - 1) / kB1;
    const int64_t b0 = c * (kB2 / kB1);
    const bool own = b0 + lane < nb1;
    const bool live = own && bm1[b0 + lane] >= kthr;
    if (w == 0 && own && !live) mask[b0 + lane] = 0;
    uint64_t todo = __ballot(live);
    uint32_t cnt = 0;
    for (int r = 0; todo; ++r) {
        const int i = __builtin_ctzll(todo);
        todo &= todo - 1;
        if (r % kWaves != w) continue;
        const int64_t b = b0 + i;
        const int64_t m = b * kB1 + lane;
        float v = 0.0f;
        bool cand = false;
        if (m < n) {
            v = M[m];
            cand = m >= c_lo && m < c_hi && v >= thr;   // outside [c_lo, c_hi): neighbours only
        }
        if (cand && W >= 1) {
            const uint32_t km = okey(v);
            if (m >= 1 && okey(M[m - 1]) >= km) cand = false;
            if (m + 1 < n && okey(M[m + 1]) > km) cand = false;
        }
        uint64_t cm = __ballot(cand);
        uint64_t bits = 0;
        if (W == 0) {
            bits = cm;
        } else if (__popcll(cm) <= kWaveTestMax) {
            while (cm) {
                const int l = __builtin_ctzll(cm);
                cm &= cm - 1;
                const int64_t mm = b * kB1 + l;
                const uint32_t km = okey(__shfl(v, l));
                const int64_t lo = mm - W > 0 ? mm - W : 0;
                const int64_t e = mm + W + 1 < n ? mm + W + 1 : n;
                const uint32_t pl = range_max_part(M, bm1, bm2, lo, mm, lane);
                const uint32_t pr = range_max_part(M, bm1, bm2, mm + 1, e, lane);
                if (wave_max(pl) < km && wave_max(pr) <= km) bits |= 1ull << l;
            }
        } else {
            const bool hit = cand && is_peak_lane(M, n, m, okey(v), W, bm1, bm2);
            bits = __ballot(hit);
        }
        if (lane == 0) mask[b] = bits;
        cnt += (uint32_t)__popcll(bits);
    }
    if (lane == 0) wc[w] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int k = 0; k < kWaves; ++k) s += wc[k];
        cnt2[c] = s;
    }
}

// One workgroup per 4,096-block with triggers: the first wave ranks the 64 mask
// words, then each wave writes whole words, lane = bit, so a word's triggers
// land in consecutive slots. off2 = NULL: offsets and total summed here.
__global__ __launch_bounds__(kThreads) void clus_write_kernel(const float *__restrict__ M,
                                                              const int32_t *__restrict__ J, int64_t n,
                                                              const uint64_t *__restrict__ mask,
                                                              const uint32_t *__restrict__ cnt2,
                                                              const int64_t *__restrict__ off2, int64_t cap,
                                                              int64_t *__restrict__ count, int64_t index_base,
                                                              int64_t *__restrict__ idx,
                                                              int32_t *__restrict__ tpl,
                                                              float *__restrict__ val) {
    __shared__ uint64_t mk[kB2 / kB1];
    __shared__ uint32_t pre[kB2 / kB1];
    __shared__ uint64_t red[kThreads / 64];
    const int64_t c = blockIdx.x;
    const int64_t nb2 = gridDim.x;
    const int t = threadIdx.x;
    int64_t off;
    if (off2) {
        if (cnt2[c] == 0) return;
        off = off2[c];
    } else {
        // short series: this block's offset is the sum of the counts before it,
        // and the last block also writes the total
        const bool tail = c == nb2 - 1;
        if (cnt2[c] == 0 && !tail) return;
        const int64_t end = tail ? nb2 : c;
        uint64_t s = 0;
        for (int64_t i = t; i < end; i += kThreads) s += cnt2[i];
        for (int o = 1; o < 64; o <<= 1) s += (uint64_t)__shfl_xor((long long)s, o);
        if ((t & 63) == 0) red[t >> 6] = s;
        __syncthreads();
        s = 0;
        for (int k = 0; k < kThreads / 64; ++k) s += red[k];
        if (tail) {
            if (t == 0) *count = (int64_t)s;
            if (cnt2[c] == 0) return;
            s -= cnt2[c];
        }
        off = (int64_t)s;
    }
    if (off >= cap) return;
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
        idx[pos] = index_base + m;
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

// Next window of a trigger stream: dst = src[0..keep) ++ blk[0..n), the max
// and the argmax series together (one thread per window sample).
__global__ __launch_bounds__(256) void ts_compose_kernel(const float *__restrict__ sm,
                                                         const int32_t *__restrict__ sj, int64_t keep,
                                                         const float *__restrict__ bm,
                                                         const int32_t *__restrict__ bj, int64_t n,
                                                         float *__restrict__ dm, int32_t *__restrict__ dj) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= keep + n) return;
    if (i < keep) {
        dm[i] = sm[i];
        dj[i] = sj[i];
    } else {
        dm[i] = bm[i - keep];
        dj[i] = bj[i - keep];
    }
}

}  // namespace

size_t cluster_workspace_bytes(int64_t n) { return carve(nullptr, n, nullptr); }

hipError_t launch_cluster(const float *M, const int32_t *J, int64_t n, float thr, int64_t W, void *ws,
                          int64_t cap, int64_t *idx, int32_t *tpl, float *val, int64_t *count,
                          hipStream_t st, int64_t c_lo, int64_t c_hi, int64_t index_base) {
    ClusterWs w;
    carve(ws, n, &w);
    const int64_t nb2 = (n + kB2 - 1) / kB2;
    if (nb2 == 0) {
        hipLaunchKernelGGL(clus_zero_count_kernel, dim3(1), dim3(1), 0, st, count);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(clus_reduce_kernel, dim3((unsigned)nb2), dim3(kThreads), 0, st, M, n, w.bm1, w.bm2);
    hipLaunchKernelGGL(clus_find_kernel, dim3((unsigned)nb2), dim3(kFindThreads), 0, st, M, n, thr, okey(thr), W,
                       c_lo, c_hi < 0 ? n : c_hi, w.bm1, w.bm2, w.mask, w.cnt2);
    int64_t *off2 = nullptr;
    if (nb2 > kInlinePrefix) {
        hipLaunchKernelGGL(clus_scan_kernel, dim3(1), dim3(1024), 0, st, w.cnt2, nb2, w.off2, count);
        off2 = w.off2;
    }
    hipLaunchKernelGGL(clus_write_kernel, dim3((unsigned)nb2), dim3(kThreads), 0, st, M, J, n, w.mask, w.cnt2,
                       off2, cap, count, index_base, idx, tpl, val);
    return hipGetLastError();
}

hipError_t launch_ts_compose(const float *sm, const int32_t *sj, int64_t keep, const float *bm, const int32_t *bj,
                             int64_t n, float *dm, int32_t *dj, hipStream_t st) {
    const int64_t total = keep + n;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(ts_compose_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, sm, sj, keep, bm,
                       bj, n, dm, dj);
    return hipGetLastError();
}

}  // namespace spiir
