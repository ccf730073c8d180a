// Device kernels of libspiir (gfx950 / CDNA4).
//
// Forward path (Sect. "GPU accelerated SPIIR method", subsection "Optimized
// GPU implementation of SPIIR"): the per-template parameter arrays are loaded
// with coalesced accesses, each filter's output lives in registers across
// iterations, the strain window shared by all filters is staged once per
// workgroup, and the per-template sum of filter outputs is a parallel
// reduction. The MI355X mapping:
//   * one workgroup = up to 16 waves = a packed set of whole templates;
//     every lane holds FL filters of one template in registers;
//   * the delayed strain window x[m - d] of a whole block lives in LDS and is
//     read with immediate offsets (no address arithmetic in the hot loop);
//   * the template sum is done per tile of 8 time steps: an in-lane sum over
//     the lane's FL filters, a wave-local LDS transpose + 8-lane butterfly,
//     and a cross-wave sum by the template's first wave after one barrier;
//   * every L samples each filter's carried state gets its FP64 correction
//     (chunked time scan: the chunk-end state is a^L times the chunk-start
//     state plus the in-chunk response);
//   * epilogues: per-template SNR rows, z rows, or a fused per-sample
//     max/argmax encoded as a 64-bit key (SNR bits << 32 | ~template).
#include "spiir_internal.h"

namespace spiir {

namespace {

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 cpow64(double2 a, int e) {
    double2 r = make_double2(1.0, 0.0);
    while (e > 0) {
        if (e & 1) r = cmul64(r, a);
        a = cmul64(a, a);
        e >>= 1;
    }
    return r;
}

// LDS writes by one lane become visible to reads by other lanes of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int64_t slot_index(int g, int wpg, int wave, int f, int fl, int lane) {
    return ((int64_t)(g * wpg + wave) * fl + f) * 64 + lane;
}

// Per-lane register state of FL filter slots.
template <int FL>
struct Lane {
    float ar[FL], ai[FL], br[FL], bi[FL];
    int xo[FL], fl[FL];
    float yr[FL], yi[FL];     // running state (FP32)
    float y0r[FL], y0i[FL];   // state at the chunk start (hi part)
    float l0r[FL], l0i[FL];   // low part of the chunk-start carry
    int64_t slot[FL];
};

// One tile of time steps: FL filter updates per step and per lane, the lane's
// partial template sum written to the wave's LDS tile.
template <int FL, bool FULL, typename XP>
__device__ __forceinline__ void compute_tile(Lane<FL> &s, XP xw, int t0, int steps,
                                             float2 *wt, int lane) {
    XP xp[FL];
#pragma unroll
    for (int f = 0; f < FL; ++f) xp[f] = xw + (s.xo[f] + t0);
#pragma unroll
    for (int t = 0; t < kTile; ++t) {
        if (!FULL && t >= steps) break;
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int f = 0; f < FL; ++f) {
            const float xv = xp[f][t];
            const float nr = fmaf(-s.ai[f], s.yi[f], fmaf(s.ar[f], s.yr[f], s.br[f] * xv));
            const float ni = fmaf(s.ai[f], s.yr[f], fmaf(s.ar[f], s.yi[f], s.bi[f] * xv));
            s.yr[f] = nr;
            s.yi[f] = ni;
            if (f == 0) {
                pr = nr;
                pi = ni;
            } else {
                pr += nr;
                pi += ni;
            }
        }
        wt[t * 64 + lane] = make_float2(pr, pi);
    }
}

// Chunk-end correction of the carried state (len = samples in the chunk).
template <int FL>
__device__ __forceinline__ void carry_correct(Lane<FL> &s, const SlotArrays &sa, int prec,
                                              int len, int L) {
#pragma unroll
    for (int f = 0; f < FL; ++f) {
        float hr = s.yr[f], hi = s.yi[f], lr = 0.f, li = 0.f;
        if (prec != kPrecFp32) {
            double2 al, dl;
            if (len == L) {
                al = sa.aL[s.slot[f]];
                dl = sa.dL[s.slot[f]];
            } else {
                const double2 a = sa.a64[s.slot[f]];
                al = cpow64(a, len);
                const double2 ah = cpow64(make_double2((double)s.ar[f], (double)s.ai[f]), len);
                dl = make_double2(al.x - ah.x, al.y - ah.y);
            }
            if (prec == kPrecFp64 || (s.fl[f] & 1)) {
                // c_end = y_end + (a^l - fl(a)^l) * hi_start + a^l * lo_start, in FP64
                const double y0r = s.y0r[f], y0i = s.y0i[f], l0r = s.l0r[f], l0i = s.l0i[f];
                const double cr = (double)hr + (dl.x * y0r - dl.y * y0i) + (al.x * l0r - al.y * l0i);
                const double ci = (double)hi + (dl.x * y0i + dl.y * y0r) + (al.x * l0i + al.y * l0r);
                hr = (float)cr;
                hi = (float)ci;
                lr = (float)(cr - (double)hr);
                li = (float)(ci - (double)hi);
            } else {
                const float dr = (float)dl.x, di = (float)dl.y;
                hr = fmaf(dr, s.y0r[f], fmaf(-di, s.y0i[f], hr));
                hi = fmaf(dr, s.y0i[f], fmaf(di, s.y0r[f], hi));
            }
        }
        s.yr[f] = hr;
        s.yi[f] = hi;
        s.y0r[f] = hr;
        s.y0i[f] = hi;
        s.l0r[f] = lr;
        s.l0i[f] = li;
    }
}

// The whole forward pass of workgroup g over p.n samples.
template <int FL, int MODE, bool XLDS>
__device__ void fwd_group(const FwdArgs &p, int g, unsigned char *smem) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = p.wpg;
    const size_t win_bytes = XLDS ? (size_t)((p.dmax + p.nb + 3) & ~3) * 4 : 0;
    float *xs = reinterpret_cast<float *>(smem);
    float2 *wt = reinterpret_cast<float2 *>(smem + win_bytes) + wave * kTile * 64;
    float2 *wsum = reinterpret_cast<float2 *>(smem + win_bytes) + W * kTile * 64;  // [2][kTile][W]
    unsigned long long *kmax = reinterpret_cast<unsigned long long *>(wsum + 2 * kTile * W);

    const WaveInfo wi = p.waves[g * W + wave];
    const bool active = wi.tpl >= 0 && (p.only_tpl < 0 || wi.tpl == p.only_tpl);
    const bool leader = active && wi.w0 == wave;

    Lane<FL> s;
#pragma unroll
    for (int f = 0; f < FL; ++f) {
        s.slot[f] = slot_index(g, W, wave, f, FL, lane);
        if (active) {
            const float2 a = p.s.a32[s.slot[f]], b = p.s.b32[s.slot[f]];
            s.ar[f] = a.x; s.ai[f] = a.y; s.br[f] = b.x; s.bi[f] = b.y;
            s.xo[f] = p.s.xoff[s.slot[f]];
            s.fl[f] = p.s.flags[s.slot[f]];
            float4 st = make_float4(0.f, 0.f, 0.f, 0.f);
            if (p.state) st = p.state[s.slot[f]];
            s.yr[f] = st.x; s.yi[f] = st.y; s.l0r[f] = st.z; s.l0i[f] = st.w;
        } else {
            s.ar[f] = s.ai[f] = s.br[f] = s.bi[f] = 0.f;
            s.xo[f] = 0; s.fl[f] = 0;
            s.yr[f] = s.yi[f] = s.l0r[f] = s.l0i[f] = 0.f;
        }
        s.y0r[f] = s.yr[f];
        s.y0i[f] = s.yi[f];
    }
    if (MODE == kModeKeys && tid < 2 * kTile) kmax[tid] = 0ull;
    if (MODE == kModeZ && active && p.tape) {
#pragma unroll
        for (int f = 0; f < FL; ++f)
            p.tape[(int64_t)p.chunk0 * p.nslots + s.slot[f]] =
                make_float4(s.yr[f], s.yi[f], s.l0r[f], s.l0i[f]);
    }

    int64_t chunk_start = 0;
    int64_t chunk_idx = 0;
    int buf = 0;
    bool pending = false;
    int64_t pend_t = 0;
    int pend_steps = 0;

    for (int64_t s0 = 0; s0 < p.n; s0 += p.nb) {
        const int nbs = (int)min((int64_t)p.nb, p.n - s0);
        const float *xw;
        if (XLDS) {
            __syncthreads();
            const int cnt = p.dmax + nbs;
            const int64_t m0 = p.xbase + s0 - p.dmax;
            for (int i = tid; i < cnt; i += blockDim.x) {
                const int64_t m = m0 + i;
                xs[i] = m >= 0 ? p.x[m] : (p.hist ? p.hist[p.dmax + m] : 0.f);
            }
            __syncthreads();
            xw = xs;
        } else {
            xw = p.xwin + (p.xbase + s0);
        }

        for (int t0 = 0; t0 < nbs; t0 += kTile) {
            const int steps = min(kTile, nbs - t0);
            if (active) {
                if (steps == kTile)
                    compute_tile<FL, true>(s, xw, t0, steps, wt, lane);
                else
                    compute_tile<FL, false>(s, xw, t0, steps, wt, lane);
                wave_lds_sync();
                // wave-local transpose-reduce: lane (t, part) sums 8 lanes of step t
                const int t = lane >> 3, part = lane & 7;
                const float4 *src = reinterpret_cast<const float4 *>(wt + t * 64 + part * 8);
                const float4 v0 = src[0], v1 = src[1], v2 = src[2], v3 = src[3];
                float sr = ((v0.x + v0.z) + (v1.x + v1.z)) + ((v2.x + v2.z) + (v3.x + v3.z));
                float si = ((v0.y + v0.w) + (v1.y + v1.w)) + ((v2.y + v2.w) + (v3.y + v3.w));
                sr += __shfl_xor(sr, 1, 8);
                si += __shfl_xor(si, 1, 8);
                sr += __shfl_xor(sr, 2, 8);
                si += __shfl_xor(si, 2, 8);
                sr += __shfl_xor(sr, 4, 8);
                si += __shfl_xor(si, 4, 8);
                if (part == 0) wsum[(buf * kTile + t) * W + wave] = make_float2(sr, si);
            }
            __syncthreads();
            if (MODE == kModeKeys && pending && wave == 0 && lane < pend_steps) {
                const int pb = buf ^ 1;
                p.keys[(int64_t)g * p.ld + pend_t + lane] = kmax[pb * kTile + lane];
                kmax[pb * kTile + lane] = 0ull;
            }
            if (leader && lane < steps) {
                const float2 *ws = wsum + (buf * kTile + lane) * W;
                float zr = ws[wi.w0].x, zi = ws[wi.w0].y;
                for (int w = 1; w < wi.nw; ++w) {
                    zr += ws[wi.w0 + w].x;
                    zi += ws[wi.w0 + w].y;
                }
                const int64_t tl = s0 + t0 + lane;
                if (MODE == kModeSnr) {
                    p.snr[(int64_t)wi.tpl * p.ld + p.obase + tl] = zr * zr + zi * zi;
                } else if (MODE == kModeZ) {
                    p.z[(int64_t)wi.tpl * p.ld + p.obase + tl] = make_float2(zr, zi);
                } else {
                    const float sn = zr * zr + zi * zi;
                    const unsigned long long key =
                        ((unsigned long long)__float_as_uint(sn) << 32) |
                        (unsigned long long)(0xFFFFFFFFu - (uint32_t)wi.tpl);
                    atomicMax(&kmax[buf * kTile + lane], key);
                }
            }
            if (MODE == kModeKeys) {
                pending = true;
                pend_t = s0 + t0;
                pend_steps = steps;
            }
            const int64_t tend = s0 + t0 + steps;
            if (tend - chunk_start == p.L || tend == p.n) {
                if (active) {
                    carry_correct<FL>(s, p.s, p.prec, (int)(tend - chunk_start), p.L);
                    if (MODE == kModeZ && p.tape && tend < p.n) {
#pragma unroll
                        for (int f = 0; f < FL; ++f)
                            p.tape[(p.chunk0 + chunk_idx + 1) * p.nslots + s.slot[f]] =
                                make_float4(s.yr[f], s.yi[f], s.l0r[f], s.l0i[f]);
                    }
                }
                chunk_start = tend;
                ++chunk_idx;
            }
            buf ^= 1;
        }
    }
    if (MODE == kModeKeys) {
        __syncthreads();
        if (pending && wave == 0 && lane < pend_steps) {
            const int pb = buf ^ 1;
            p.keys[(int64_t)g * p.ld + pend_t + lane] = kmax[pb * kTile + lane];
            kmax[pb * kTile + lane] = 0ull;
        }
    }
    if (active && p.state) {
#pragma unroll
        for (int f = 0; f < FL; ++f)
            p.state[s.slot[f]] = make_float4(s.yr[f], s.yi[f], s.l0r[f], s.l0i[f]);
    }
}

template <int FL, int MODE, bool XLDS>
__global__ void __launch_bounds__(1024) fwd_kernel(FwdArgs p) {
    extern __shared__ __align__(16) unsigned char smem[];
    fwd_group<FL, MODE, XLDS>(p, p.gbase + blockIdx.x, smem);
}

// Persistent batch kernel: workgroups pop (stream, group) items until the list
// is exhausted; every item is one block of one stream for one group.
template <int FL>
__global__ void __launch_bounds__(1024) batch_kernel(const BatchStream *streams, const int2 *items,
                                                     int nitems, int *counter, const int64_t *pos,
                                                     int block_len) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int item_s;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) item_s = atomicAdd(counter, 1);
        __syncthreads();
        const int it = __builtin_amdgcn_readfirstlane(item_s);
        if (it >= nitems) break;
        const int2 item = items[it];
        const int sidx = __builtin_amdgcn_readfirstlane(item.x);
        const int g = __builtin_amdgcn_readfirstlane(item.y);
        const int64_t p0 = pos[sidx];
        const int64_t len = streams[sidx].len;
        if (p0 >= len) continue;
        FwdArgs a = streams[sidx].args;
        a.xbase = p0;
        a.n = min((int64_t)block_len, len - p0);
        a.ld = block_len;
        fwd_group<FL, kModeKeys, true>(a, g, smem);
    }
}

__global__ void finalize_keys_kernel(const uint64_t *keys, int groups, int64_t ld, int64_t n,
                                     float *mx, int32_t *am) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t k = 0;
    for (int g = 0; g < groups; ++g) {
        const uint64_t v = keys[(int64_t)g * ld + i];
        k = v > k ? v : k;
    }
    mx[i] = __uint_as_float((uint32_t)(k >> 32));
    am[i] = (int32_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
}

__global__ void rows_argmax_kernel(const float *snr, int T, int64_t ld, int64_t n, float *mx,
                                   int32_t *am) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float best = snr[i];
    int bj = 0;
    for (int j = 1; j < T; ++j) {
        const float v = snr[(int64_t)j * ld + i];
        if (v > best) {
            best = v;
            bj = j;
        }
    }
    mx[i] = best;
    am[i] = bj;
}

__global__ void hist_update_kernel(const float *old_h, float *new_h, const float *x, int64_t n,
                                   int dmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= dmax) return;
    const int64_t m = n - dmax + i;
    new_h[i] = m >= 0 ? x[m] : old_h[dmax + m];
}

__global__ void window_fill_kernel(float *xwin, const float *hist, const float *x, int64_t n,
                                   int dmax) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n + dmax) return;
    xwin[i] = i < dmax ? (hist ? hist[i] : 0.f) : x[i - dmax];
}

__global__ void fill_zero_kernel(uint32_t *p, int64_t words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0u;
}

__global__ void noise_fill_kernel(float *x, int64_t n, uint32_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // 64-bit mix (splitmix64 finaliser) of the index and seed -> uniform in [-1, 1)
    uint64_t z = (uint64_t)i + 0x9E3779B97F4A7C15ull * (uint64_t)(seed + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (float)((int64_t)(z >> 40) - (1ll << 23)) * (1.0f / 8388608.0f);
}

// ---------------------------------------------------------------------------
// Adjoint. Each lane owns FL filter slots and handles them one after another:
// chunks in reverse order; y is recomputed from the tape (chunk-start state),
// first over the whole chunk keeping every kSub-th state in scratch memory,
// then per sub-chunk into registers; lambda runs backwards with conj(a).
// ---------------------------------------------------------------------------
template <int FL>
__global__ void __launch_bounds__(256) bwd_kernel(BwdArgs p) {
    const int tid = threadIdx.x, lane = tid & 63, wave_in_block = tid >> 6;
    const int waves_per_block = blockDim.x >> 6;
    const int gw = blockIdx.x * waves_per_block + wave_in_block;  // global wave
    const int g = gw / p.wpg, wave = gw % p.wpg;
    const WaveInfo wi = p.waves[gw];
    if (wi.tpl < 0) return;
    const int64_t n = p.n;
    const int64_t nch = (n + p.L - 1) / p.L;
    const float2 *gz = p.gz + (int64_t)wi.tpl * n;
    for (int f = 0; f < FL; ++f) {
        const int64_t slot = slot_index(g, p.wpg, wave, f, FL, lane);
        const int k = p.slot_filter[slot];
        if (k < 0) continue;
        const float2 a = p.s.a32[slot], b = p.s.b32[slot];
        const float ar = a.x, ai = a.y, br = b.x, bi = b.y;
        const float *xw = p.xwin + p.s.xoff[slot];  // xw[m] = x[m - d]
        double gar = 0.0, gai = 0.0, gbr = 0.0, gbi = 0.0;
        float lr = 0.f, li = 0.f;  // lambda at the sample after the current chunk
        for (int64_t c = nch - 1; c >= 0; --c) {
            const int64_t c0 = c * p.L;
            const int l = (int)min((int64_t)p.L, n - c0);
            const int nq = (l + kSub - 1) / kSub;
            // pass 1: forward over the chunk, keep the state before every sub-chunk
            const float4 tp = p.tape[c * p.nslots + slot];
            float yr = tp.x, yi = tp.y;
            for (int q = 0; q < nq; ++q) {
                p.ysub[(int64_t)q * p.nslots + slot] = make_float2(yr, yi);
                const int qs = q * kSub, ql = min(kSub, l - qs);
#pragma unroll
                for (int t = 0; t < kSub; ++t) {
                    if (t < ql) {
                        const float xv = xw[c0 + qs + t];
                        const float nr = fmaf(-ai, yi, fmaf(ar, yr, br * xv));
                        const float ni = fmaf(ai, yr, fmaf(ar, yi, bi * xv));
                        yr = nr;
                        yi = ni;
                    }
                }
            }
            // pass 2: sub-chunks in reverse
            const float lin_r = lr, lin_i = li;
            float sar = 0.f, sai = 0.f, sbr = 0.f, sbi = 0.f;
            for (int q = nq - 1; q >= 0; --q) {
                const int qs = q * kSub, ql = min(kSub, l - qs);
                float hr[kSub + 1], hi[kSub + 1];  // hr[t] = y[m - 1] for m = c0 + qs + t
                const float2 y0 = p.ysub[(int64_t)q * p.nslots + slot];
                hr[0] = y0.x;
                hi[0] = y0.y;
#pragma unroll
                for (int t = 0; t < kSub; ++t) {
                    if (t < ql) {
                        const float xv = xw[c0 + qs + t];
                        hr[t + 1] = fmaf(-ai, hi[t], fmaf(ar, hr[t], br * xv));
                        hi[t + 1] = fmaf(ai, hr[t], fmaf(ar, hi[t], bi * xv));
                    }
                }
#pragma unroll
                for (int t = kSub - 1; t >= 0; --t) {
                    if (t < ql) {
                        const int64_t m = c0 + qs + t;
                        const float2 gm = gz[m];
                        // lambda[m] = G[m] + conj(a) lambda[m+1]
                        const float nr = gm.x + fmaf(ar, lr, ai * li);
                        const float ni = gm.y + fmaf(ar, li, -ai * lr);
                        lr = nr;
                        li = ni;
                        const float xv = xw[m];
                        sbr = fmaf(lr, xv, sbr);
                        sbi = fmaf(li, xv, sbi);
                        // lambda * conj(y[m-1])
                        sar = fmaf(lr, hr[t], fmaf(li, hi[t], sar));
                        sai = fmaf(li, hr[t], fmaf(-lr, hi[t], sai));
                    }
                }
            }
            if (p.prec != kPrecFp32) {
                // carry of lambda across the chunk used conj(fl32(a))^l; add conj(a^l - fl32(a)^l) lambda_in
                double2 dl;
                if (l == p.L) {
                    dl = p.s.dL[slot];
                } else {
                    const double2 al = cpow64(p.s.a64[slot], l);
                    const double2 ah = cpow64(make_double2((double)ar, (double)ai), l);
                    dl = make_double2(al.x - ah.x, al.y - ah.y);
                }
                const float dr = (float)dl.x, di = (float)dl.y;
                lr = fmaf(dr, lin_r, fmaf(di, lin_i, lr));
                li = fmaf(dr, lin_i, fmaf(-di, lin_r, li));
            }
            gar += (double)sar;
            gai += (double)sai;
            gbr += (double)sbr;
            gbi += (double)sbi;
        }
        p.grad_a[k] = make_float2((float)gar, (float)gai);
        p.grad_b[k] = make_float2((float)gbr, (float)gbi);
    }
}

// Batch bookkeeping.
__global__ void batch_finalize_kernel(const BatchStream *streams, const uint64_t *keys,
                                      int64_t key_stride, const int64_t *pos, int block_len) {
    const int sidx = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t p0 = pos[sidx];
    const int64_t len = streams[sidx].len;
    if (p0 >= len || i >= min((int64_t)block_len, len - p0)) return;
    const uint64_t *kk = keys + sidx * key_stride;
    const int groups = streams[sidx].groups;
    uint64_t k = 0;
    for (int g = 0; g < groups; ++g) {
        const uint64_t v = kk[(int64_t)g * block_len + i];
        k = v > k ? v : k;
    }
    streams[sidx].max_out[p0 + i] = __uint_as_float((uint32_t)(k >> 32));
    streams[sidx].arg_out[p0 + i] = (int32_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
}

__global__ void batch_advance_kernel(int64_t *pos, const BatchStream *streams, int nstreams,
                                     int *counter, int block_len) {
    const int i = threadIdx.x;
    if (i == 0) *counter = 0;
    if (i < nstreams) {
        const int64_t len = streams[i].len;
        pos[i] = min(len, pos[i] + (int64_t)block_len);
    }
}

template <int FL, int MODE, bool XLDS>
hipError_t launch_fwd_t(const FwdArgs &a, int groups, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((fwd_kernel<FL, MODE, XLDS>), dim3(groups), dim3(a.wpg * 64), lds, st, a);
    return hipGetLastError();
}

template <int MODE, bool XLDS>
hipError_t launch_fwd_m(const FwdArgs &a, int fl, int groups, size_t lds, hipStream_t st) {
    switch (fl) {
        case 1: return launch_fwd_t<1, MODE, XLDS>(a, groups, lds, st);
        case 2: return launch_fwd_t<2, MODE, XLDS>(a, groups, lds, st);
        case 3: return launch_fwd_t<3, MODE, XLDS>(a, groups, lds, st);
        case 4: return launch_fwd_t<4, MODE, XLDS>(a, groups, lds, st);
        default: return hipErrorInvalidValue;
    }
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

size_t fwd_lds_bytes(int wpg, int dmax, int nb, bool x_in_lds) {
    size_t win = x_in_lds ? (size_t)((dmax + nb + 3) & ~3) * 4 : 0;
    return win + (size_t)wpg * kTile * 64 * 8 + (size_t)2 * kTile * wpg * 8 + (size_t)2 * kTile * 8;
}

hipError_t launch_forward(const FwdArgs &a, int mode, int fl, bool x_in_lds, int groups,
                          size_t lds, hipStream_t st) {
    if (groups <= 0) return hipSuccess;
    if (x_in_lds) {
        switch (mode) {
            case kModeSnr: return launch_fwd_m<kModeSnr, true>(a, fl, groups, lds, st);
            case kModeKeys: return launch_fwd_m<kModeKeys, true>(a, fl, groups, lds, st);
            case kModeZ: return launch_fwd_m<kModeZ, true>(a, fl, groups, lds, st);
        }
    } else {
        switch (mode) {
            case kModeSnr: return launch_fwd_m<kModeSnr, false>(a, fl, groups, lds, st);
            case kModeKeys: return launch_fwd_m<kModeKeys, false>(a, fl, groups, lds, st);
            case kModeZ: return launch_fwd_m<kModeZ, false>(a, fl, groups, lds, st);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_finalize_keys(const uint64_t *keys, int groups, int64_t ld, int64_t n,
                                float *mx, int32_t *am, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_keys_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, keys, groups,
                       ld, n, mx, am);
    return hipGetLastError();
}

hipError_t launch_rows_argmax(const float *snr, int T, int64_t ld, int64_t n, float *mx,
                              int32_t *am, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(rows_argmax_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, snr, T, ld, n,
                       mx, am);
    return hipGetLastError();
}

hipError_t launch_hist_update(const float *old_h, float *new_h, const float *x, int64_t n,
                              int dmax, hipStream_t st) {
    if (dmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(hist_update_kernel, dim3(nblocks(dmax, 256)), dim3(256), 0, st, old_h,
                       new_h, x, n, dmax);
    return hipGetLastError();
}

hipError_t launch_window_fill(float *xwin, const float *hist, const float *x, int64_t n, int dmax,
                              hipStream_t st) {
    if (n + dmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(window_fill_kernel, dim3(nblocks(n + dmax, 256)), dim3(256), 0, st, xwin,
                       hist, x, n, dmax);
    return hipGetLastError();
}

int batch_occupancy(int fl, int wpg, size_t lds) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (fl) {
        case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<1>, wpg * 64, lds); break;
        case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<2>, wpg * 64, lds); break;
        case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<3>, wpg * 64, lds); break;
        case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<4>, wpg * 64, lds); break;
        default: break;
    }
    return e == hipSuccess ? nb : 0;
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t st) {
    const int64_t words = (int64_t)(bytes / 4);
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(nblocks(words, 256)), dim3(256), 0, st,
                       static_cast<uint32_t *>(p), words);
    return hipGetLastError();
}

hipError_t launch_noise_fill(float *x, int64_t n, uint32_t seed, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(noise_fill_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, x, n, seed);
    return hipGetLastError();
}

hipError_t launch_backward(const BwdArgs &a, int fl, int groups, hipStream_t st) {
    const int total_waves = groups * a.wpg;
    if (total_waves <= 0) return hipSuccess;
    // 4 waves per block; the wave count of a bank is a multiple of wpg, pad to 4
    const int wpb = (total_waves % 4 == 0) ? 4 : (total_waves % 2 == 0 ? 2 : 1);
    const dim3 grid(total_waves / wpb), block(64 * wpb);
    switch (fl) {
        case 1: hipLaunchKernelGGL(bwd_kernel<1>, grid, block, 0, st, a); break;
        case 2: hipLaunchKernelGGL(bwd_kernel<2>, grid, block, 0, st, a); break;
        case 3: hipLaunchKernelGGL(bwd_kernel<3>, grid, block, 0, st, a); break;
        case 4: hipLaunchKernelGGL(bwd_kernel<4>, grid, block, 0, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch(const BatchStream *streams, const int2 *items, int nitems, int *counter,
                        const int64_t *pos, int block_len, int fl, int grid, int wpg, size_t lds,
                        hipStream_t st) {
    const dim3 g(grid), b(wpg * 64);
    switch (fl) {
        case 1: hipLaunchKernelGGL(batch_kernel<1>, g, b, lds, st, streams, items, nitems, counter, pos, block_len); break;
        case 2: hipLaunchKernelGGL(batch_kernel<2>, g, b, lds, st, streams, items, nitems, counter, pos, block_len); break;
        case 3: hipLaunchKernelGGL(batch_kernel<3>, g, b, lds, st, streams, items, nitems, counter, pos, block_len); break;
        case 4: hipLaunchKernelGGL(batch_kernel<4>, g, b, lds, st, streams, items, nitems, counter, pos, block_len); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchStream *streams, int nstreams, const uint64_t *keys,
                                 int64_t key_stride, const int64_t *pos, int block_len,
                                 int max_groups, hipStream_t st) {
    (void)max_groups;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(nblocks(block_len, 256), nstreams), dim3(256), 0,
                       st, streams, keys, key_stride, pos, block_len);
    return hipGetLastError();
}

hipError_t launch_batch_advance(int64_t *pos, const BatchStream *streams, int nstreams,
                                int *counter, int block_len, hipStream_t st) {
    hipLaunchKernelGGL(batch_advance_kernel, dim3(1), dim3(((nstreams + 63) / 64) * 64), 0, st, pos,
                       streams, nstreams, counter, block_len);
    return hipGetLastError();
}

int forward_max_threads() { return kMaxWaves * 64; }

}  // namespace spiir
