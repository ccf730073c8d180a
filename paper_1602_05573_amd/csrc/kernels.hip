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
#include <hip/hip_ext.h>

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

__device__ __forceinline__ float dpp_swap_pairs(float v) {
    // quad_perm [1,0,3,2]: the value of lane ^ 1
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

__device__ __forceinline__ int64_t slot_index(int g, int wpg, int wave, int f, int fl, int lane) {
    return ((int64_t)(g * wpg + wave) * fl + f) * 64 + lane;
}

// Four floats at a 4-byte aligned address (global loads accept this alignment).
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));

// Per-lane register state of FL filter slots.
template <int FL>
struct Lane {
    float ar[FL], ai[FL], br[FL], bi[FL];
    int xo[FL];
    float yr[FL], yi[FL];     // running state (FP32)
    float y0r[FL], y0i[FL];   // state at the chunk start (hi part)
    float l0r[FL], l0i[FL];   // low part of the chunk-start carry
    unsigned flags;           // bit f: slot f carries in FP64 (hybrid mode)
    int64_t slot0;            // slot of filter f is slot0 + 64 f
    __device__ __forceinline__ int64_t slot(int f) const { return slot0 + 64 * f; }
};

// Steps of x[m - d] read ahead of their use: short for the LDS window, longer
// when the window stays in global memory (so more of the load latency is
// covered by the recursion itself).
template <bool XLDS, int TT>
struct Ahead {
    static constexpr int value = XLDS ? 2 : (TT >= 16 ? 8 : 4);
};

// x[m - d] of every filter for steps t0 .. t0 + AH - 1 of a tile. The window
// is padded by one tile, so reads past the sub-block end stay inside it (their
// values are never used).
template <int FL, int TT, int AH>
__device__ __forceinline__ void load_ahead(float (&xv)[TT][FL], const float *xw, const Lane<FL> &s, int t0) {
#pragma unroll
    for (int f = 0; f < FL; ++f) {
        const float *xp = xw + (s.xo[f] + t0);
#pragma unroll
        for (int t = 0; t < AH; ++t) xv[t][f] = xp[t];
    }
}

// Window in global memory: steps t0 .. t0 + AH - 1 as 16-byte loads.
template <int FL, int TT, int AH>
__device__ __forceinline__ void load_ahead_vec(float (&xv)[TT][FL], const float *xw, const Lane<FL> &s, int t0) {
#pragma unroll
    for (int f = 0; f < FL; ++f) {
#pragma unroll
        for (int u = 0; u < AH; u += 4) {
            const f4u q = *reinterpret_cast<const f4u *>(xw + (s.xo[f] + t0 + u));
            xv[u][f] = q.x;
            xv[u + 1][f] = q.y;
            xv[u + 2][f] = q.z;
            xv[u + 3][f] = q.w;
        }
    }
}

// One tile: FL filter updates per step and per lane, the lane's partial
// template sum of every step written to the wave's LDS tile [TT][64]. x for
// step t + AH is read while step t computes (xv[0..AH) arrive loaded).
// VEC (window in global memory): every 4 steps, 4 consecutive samples of each
// filter are read with one 16-byte load; reads for steps past the tile go to
// the slots of the next tile's first AH steps (already consumed here) when
// `more` says a next tile follows.
template <int FL, int TT, bool FULL, bool CARRY, int AH, bool VEC>
__device__ __forceinline__ void compute_tile(Lane<FL> &s, float (&xv)[TT][FL], const float *xw, int t0,
                                             int steps, float2 *wt, int lane, bool more) {
    static_assert(!VEC || (AH % 4 == 0 && TT % 4 == 0 && AH < TT), "vector read-ahead layout");
#pragma unroll
    for (int t = 0; t < TT; ++t) {
        if (!CARRY && VEC && t % 4 == 0) {
            const int u = t + AH;
            if (u < TT || more) {
                const int k = u < TT ? u : u - TT;
#pragma unroll
                for (int f = 0; f < FL; ++f) {
                    const f4u q = *reinterpret_cast<const f4u *>(xw + (s.xo[f] + t0 + u));
                    xv[k][f] = q.x;
                    xv[k + 1][f] = q.y;
                    xv[k + 2][f] = q.z;
                    xv[k + 3][f] = q.w;
                }
            }
        }
        if (!CARRY && !VEC && t + AH < TT) {
#pragma unroll
            for (int f = 0; f < FL; ++f) xv[t + AH][f] = xw[s.xo[f] + t0 + t + AH];
        }
        if (!FULL && t >= steps) continue;  // uniform; keeps every index static
        float pr = 0.f, pi = 0.f;
#pragma unroll
        for (int f = 0; f < FL; ++f) {
            float nr, ni;
            if (CARRY) {  // free response of the carried state: y <- a y
                nr = fmaf(-s.ai[f], s.yi[f], s.ar[f] * s.yr[f]);
                ni = fmaf(s.ai[f], s.yr[f], s.ar[f] * s.yi[f]);
            } else {
                const float xv_ = xv[t][f];
                nr = fmaf(-s.ai[f], s.yi[f], fmaf(s.ar[f], s.yr[f], s.br[f] * xv_));
                ni = fmaf(s.ai[f], s.yr[f], fmaf(s.ar[f], s.yi[f], s.bi[f] * xv_));
            }
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

// Row sums of a wave tile: wsum[t][4 * wave + r] = sum of the 16 lanes of row
// r at step t. Tile row k = 4 t + r is 128 bytes = four 32-byte units. Lanes
// 2p and 2p+1 read the two halves of one unit together (the LDS serves a
// ds_read_b128 per lane pair), and pair p walks its row's units in an order
// rotated by p / 2, so the 8 pairs served in one cycle hit distinct banks.
// Each lane sums its halves; one DPP swap adds the partner's half.
template <int TT>
struct RowSumPlan {
    static constexpr int kReads = TT == 16 ? 8 : 4;
    int off[kReads];   // byte offsets inside the wave tile, in read order
    int k0, k1;        // tile rows this pair sums (TT = 16: two rows; TT = 8: one)
};

template <int TT>
__device__ __forceinline__ RowSumPlan<TT> row_sum_plan(int lane) {
    RowSumPlan<TT> pl;
    const int p = lane >> 1, h = lane & 1;
    pl.k0 = p;
    pl.k1 = p + 32;
#pragma unroll
    for (int i = 0; i < pl.kReads; ++i) {
        const int k = (i < 4) ? pl.k0 : pl.k1;
        const int q = ((i & 3) + (p >> 1)) & 3;
        pl.off[i] = k * 128 + (2 * q + h) * 16;
    }
    return pl;
}

__device__ __forceinline__ float2 sum_chunks4(const float4 &a, const float4 &b, const float4 &c, const float4 &d) {
    return make_float2(((a.x + a.z) + (b.x + b.z)) + ((c.x + c.z) + (d.x + d.z)),
                       ((a.y + a.w) + (b.y + b.w)) + ((c.y + c.w) + (d.y + d.w)));
}

template <int TT>
__device__ __forceinline__ void row_sums(const float2 *wt, const RowSumPlan<TT> &pl, float2 *wsum_buf,
                                         int Rp, int wave, int lane) {
    const char *base = reinterpret_cast<const char *>(wt);
    const bool lo = (lane & 1) == 0;
    float4 v[RowSumPlan<TT>::kReads];
#pragma unroll
    for (int i = 0; i < RowSumPlan<TT>::kReads; ++i) v[i] = *reinterpret_cast<const float4 *>(base + pl.off[i]);
    const float2 s0 = sum_chunks4(v[0], v[1], v[2], v[3]);
    const float o0r = dpp_swap_pairs(s0.x), o0i = dpp_swap_pairs(s0.y);
    if (TT == 16) {
        const float2 s1 = sum_chunks4(v[4], v[5], v[6], v[7]);
        const float o1r = dpp_swap_pairs(s1.x), o1i = dpp_swap_pairs(s1.y);
        // the even lane writes row k0, the odd lane row k1; both as (even half) + (odd half)
        const int k = lo ? pl.k0 : pl.k1;
        const float2 tot = lo ? make_float2(s0.x + o0r, s0.y + o0i) : make_float2(o1r + s1.x, o1i + s1.y);
        wsum_buf[(k >> 2) * Rp + wave * 4 + (k & 3)] = tot;
    } else {
        if (lo) wsum_buf[(pl.k0 >> 2) * Rp + wave * 4 + (pl.k0 & 3)] = make_float2(s0.x + o0r, s0.y + o0i);
    }
}

// xs[i] = src[off + i] (0 if ZERO) for i in [i0, i1), by the whole workgroup:
// a scalar head up to a 16-byte LDS boundary, then 16-byte global loads (4-byte
// aligned) with four per thread in flight and 16-byte LDS stores, then a scalar
// tail. Indices off + i are in range for every i in [i0, i1).
template <bool ZERO>
__device__ __forceinline__ void stage_range(float *xs, const float *src, int64_t off, int i0, int i1) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int ia = min(i1, (i0 + 3) & ~3);
    for (int i = i0 + tid; i < ia; i += nt) xs[i] = ZERO ? 0.f : src[off + i];
    const int nv = (i1 - ia) >> 2;
    for (int v0 = tid; v0 < nv; v0 += 4 * nt) {
        float4 q[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int v = v0 + u * nt;
            q[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (!ZERO && v < nv) {
                const f4u w = *reinterpret_cast<const f4u *>(src + (off + ia + 4 * (int64_t)v));
                q[u] = make_float4(w.x, w.y, w.z, w.w);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int v = v0 + u * nt;
            if (v < nv) *reinterpret_cast<float4 *>(xs + ia + 4 * v) = q[u];
        }
    }
    for (int i = ia + 4 * nv + tid; i < i1; i += nt) xs[i] = ZERO ? 0.f : src[off + i];
}

// Template sum over its nr row sums of one step: N reads issued together
// (rows past nr read other rows or the buffer's slack and are zeroed), then a
// fixed pairwise tree; templates of more than 16 rows loop.
template <int N>
__device__ __forceinline__ void sum_rows(const float2 *ws, int nr, float &zr, float &zi) {
    float vr[N], vi[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const float2 v = ws[i];
        vr[i] = i < nr ? v.x : 0.f;
        vi[i] = i < nr ? v.y : 0.f;
    }
#pragma unroll
    for (int w = 1; w < N; w *= 2)
#pragma unroll
        for (int i = 0; i < N; i += 2 * w) {
            vr[i] += vr[i + w];
            vi[i] += vi[i + w];
        }
    zr = vr[0];
    zi = vi[0];
}

__device__ __forceinline__ void sum_rows_loop(const float2 *ws, int nr, float &zr, float &zi) {
    zr = 0.f;
    zi = 0.f;
    int r = 0;
    for (; r + 4 <= nr; r += 4) {
        const float2 v0 = ws[r], v1 = ws[r + 1], v2 = ws[r + 2], v3 = ws[r + 3];
        zr += (v0.x + v1.x) + (v2.x + v3.x);
        zi += (v0.y + v1.y) + (v2.y + v3.y);
    }
    for (; r < nr; ++r) {
        zr += ws[r].x;
        zi += ws[r].y;
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
                al = sa.aL[s.slot(f)];
                dl = sa.dL[s.slot(f)];
            } else {
                const double2 a = sa.a64[s.slot(f)];
                al = cpow64(a, len);
                const double2 ah = cpow64(make_double2((double)s.ar[f], (double)s.ai[f]), len);
                dl = make_double2(al.x - ah.x, al.y - ah.y);
            }
            if (prec == kPrecFp64 || ((s.flags >> f) & 1u)) {
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

// Time range and data routing of one workgroup item.
struct SegCtx {
    int64_t tb, tn;          // launch samples [tb, tb + tn)
    const float4 *st_in;     // initial state per slot (null: cold start), entry slot - in_off
    float4 *st_out;          // final state per slot (null: not stored), entry slot - out_off
    int64_t in_off, out_off;
    float2 *zl_out;          // local z goes here ([T][ld_zl]) instead of the mode's output
    const float2 *zl_in;     // added to z before the mode's output (carry pass)
    int64_t ld_zl;
};

// The whole forward pass of workgroup g over launch samples [sc.tb, sc.tb + sc.tn).
// CARRY: free response of the given state only (no input), z_local added.
// PARTS: the bank has templates split over workgroups (rows with part >= 0);
// banks without them run the variant that has no part branch.
template <int FL, int TT, int MODE, bool XLDS, bool CARRY, bool PARTS = false>
__device__ void fwd_group(const FwdArgs &p, int g, unsigned char *smem, const SegCtx &sc) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = p.wpg, R = 4 * W, Rp = R + 1;  // odd row stride of wsum: no bank aliasing over t
    // LDS window: x[m - d] for the group's delays d in [glo, glo + gw]; slot offsets are
    // max_delay - d, so a lane's window offset is that minus (max_delay - glo - gw)
    const int glo = XLDS && p.group_lo ? p.group_lo[g] : 0;
    const int gw = XLDS ? p.band_w : p.dmax;
    const int xshift = p.dmax - glo - gw;
    const size_t win_bytes = XLDS ? (size_t)((gw + p.nb + TT + 3) & ~3) * 4 : 0;
    float *xs = reinterpret_cast<float *>(smem);
    float2 *wt = reinterpret_cast<float2 *>(smem + win_bytes) + wave * TT * 64;
    float2 *wsum = reinterpret_cast<float2 *>(smem + win_bytes) + W * TT * 64;  // [2][TT][Rp]
    // [2][TT] after wsum and 16 float2 of slack (row-sum reads past a template's last row)
    unsigned long long *kmax = reinterpret_cast<unsigned long long *>(wsum + 2 * TT * Rp + 16);
    const RowSumPlan<TT> rsp = row_sum_plan<TT>(lane);
    constexpr int AH = Ahead<XLDS, TT>::value;

    const int row = wave * 4 + (lane >> 4);
    const RowInfo ri = p.rows[(int64_t)g * R + row];
    const bool ract = ri.tpl >= 0 && (p.only_tpl < 0 || ri.tpl == p.only_tpl);
    const bool wact = __ballot(ract) != 0;
    const int tl16 = lane & 15;
    const bool leader = ract && ri.r0 == row && tl16 < TT;

    Lane<FL> s;
    s.slot0 = slot_index(g, W, wave, 0, FL, lane);
    s.flags = 0u;
#pragma unroll
    for (int f = 0; f < FL; ++f) {
        if (ract) {
            const float2 a = p.s.a32[s.slot(f)], b = p.s.b32[s.slot(f)];
            s.ar[f] = a.x; s.ai[f] = a.y; s.br[f] = b.x; s.bi[f] = b.y;
            s.xo[f] = p.s.xoff[s.slot(f)] - xshift;
            s.flags |= (unsigned)(p.s.flags[s.slot(f)] & 1) << f;
            float4 st = make_float4(0.f, 0.f, 0.f, 0.f);
            if (sc.st_in) st = sc.st_in[s.slot(f) - sc.in_off];
            s.yr[f] = st.x; s.yi[f] = st.y; s.l0r[f] = st.z; s.l0i[f] = st.w;
        } else {
            s.ar[f] = s.ai[f] = s.br[f] = s.bi[f] = 0.f;
            s.xo[f] = 0;
            s.yr[f] = s.yi[f] = s.l0r[f] = s.l0i[f] = 0.f;
        }
        s.y0r[f] = s.yr[f];
        s.y0i[f] = s.yi[f];
    }
    const bool keys_out = MODE == kModeKeys && sc.zl_out == nullptr;
    const int64_t n = sc.tn;
    const int64_t xbase = p.xbase + sc.tb;
    if (keys_out && tid < 2 * TT) kmax[tid] = 0ull;

    int64_t chunk_start = 0;
    int buf = 0;
    bool pending = false;
    int64_t pend_t = 0;
    int pend_steps = 0;
    float xv[TT][FL];

    for (int64_t s0 = 0; s0 < n; s0 += p.nb) {
        const int nbs = (int)min((int64_t)p.nb, n - s0);
        const float *xw = nullptr;
        if (CARRY) {
            xw = nullptr;
        } else if (XLDS) {
            __syncthreads();
            const int cnt = gw + nbs;
            const int64_t m0 = xbase + s0 - glo - gw;   // xs[i] = x[m0 + i]; m < 0 from the history
            const int nneg = (int)min((int64_t)cnt, max((int64_t)0, -m0));
            // a band's window may reach past the largest delay (glo + gw > max_delay):
            // samples before the history (m < -max_delay) are read by no filter and
            // staged as zeros, so the history is only read at indices >= 0
            const int nz = (int)min((int64_t)nneg, max((int64_t)0, -(int64_t)p.dmax - m0));
            if (p.hist) {
                stage_range<true>(xs, nullptr, 0, 0, nz);
                stage_range<false>(xs, p.hist, p.dmax + m0, nz, nneg);
            } else {
                stage_range<true>(xs, nullptr, 0, 0, nneg);
            }
            stage_range<false>(xs, p.x, m0, nneg, cnt);
            __syncthreads();
            xw = xs;
        } else {
            xw = p.xwin + (xbase + s0);
        }
        if (!CARRY && wact) {
            if (XLDS)
                load_ahead<FL, TT, AH>(xv, xw, s, 0);
            else
                load_ahead_vec<FL, TT, AH>(xv, xw, s, 0);
        }

        for (int t0 = 0; t0 < nbs; t0 += TT) {
            const int steps = min(TT, nbs - t0);
            const bool more = t0 + TT < nbs;
            if (wact) {
                if (steps == TT)
                    compute_tile<FL, TT, true, CARRY, AH, !XLDS>(s, xv, xw, t0, steps, wt, lane, more);
                else
                    compute_tile<FL, TT, false, CARRY, AH, !XLDS>(s, xv, xw, t0, steps, wt, lane, more);
                wave_lds_sync();
                row_sums<TT>(wt, rsp, wsum + buf * TT * Rp, Rp, wave, lane);
                if (XLDS && !CARRY && more) load_ahead<FL, TT, AH>(xv, xw, s, t0 + TT);
            }
            __syncthreads();
            if (keys_out && pending && wave == 0 && lane < pend_steps) {
                const int pb = buf ^ 1;
                p.keys[(int64_t)g * p.ld + sc.tb + pend_t + lane] = kmax[pb * TT + lane];
                kmax[pb * TT + lane] = 0ull;
            }
            if (leader && tl16 < steps) {
                const float2 *ws = wsum + (buf * TT + tl16) * Rp + ri.r0;
                float zr, zi;
                if (ri.nr <= 8)
                    sum_rows<8>(ws, ri.nr, zr, zi);
                else if (ri.nr <= 16)
                    sum_rows<16>(ws, ri.nr, zr, zi);
                else
                    sum_rows_loop(ws, ri.nr, zr, zi);
                const int64_t tl = s0 + t0 + tl16;
                if (PARTS && ri.part >= 0) {
                    // one part of a template split over workgroups: its partial sum (the
                    // segment's local sum, completed in place by the carry pass) goes to the
                    // part's row; the parts are added before the mode's output
                    float2 *zp = p.zpart + (int64_t)ri.part * p.ld_part + sc.tb + tl;
                    if (sc.zl_in) {
                        const float2 zl = *zp;
                        zr += zl.x;
                        zi += zl.y;
                    }
                    *zp = make_float2(zr, zi);
                } else {
                    if (sc.zl_in) {
                        const float2 zl = sc.zl_in[(int64_t)ri.tpl * sc.ld_zl + tl];
                        zr += zl.x;
                        zi += zl.y;
                    }
                    if (sc.zl_out) {
                        sc.zl_out[(int64_t)ri.tpl * sc.ld_zl + tl] = make_float2(zr, zi);
                    } else if (MODE == kModeSnr) {
                        p.snr[(int64_t)ri.tpl * p.ld + p.obase + sc.tb + tl] = zr * zr + zi * zi;
                    } else if (MODE == kModeZ) {
                        p.z[(int64_t)ri.tpl * p.ld + p.obase + sc.tb + tl] = make_float2(zr, zi);
                    } else {
                        const float sn = zr * zr + zi * zi;
                        const unsigned long long key =
                            ((unsigned long long)__float_as_uint(sn) << 32) |
                            (unsigned long long)(0xFFFFFFFFu - (uint32_t)ri.tpl);
                        atomicMax(&kmax[buf * TT + tl16], key);
                    }
                }
            }
            if (keys_out) {
                pending = true;
                pend_t = s0 + t0;
                pend_steps = steps;
            }
            const int64_t tend = s0 + t0 + steps;
            if (tend - chunk_start == p.L || tend == n) {
                if (wact) carry_correct<FL>(s, p.s, p.prec, (int)(tend - chunk_start), p.L);
                chunk_start = tend;
            }
            buf ^= 1;
        }
    }
    if (keys_out) {
        __syncthreads();
        if (pending && wave == 0 && lane < pend_steps) {
            const int pb = buf ^ 1;
            p.keys[(int64_t)g * p.ld + sc.tb + pend_t + lane] = kmax[pb * TT + lane];
            kmax[pb * TT + lane] = 0ull;
        }
    }
    if (ract && sc.st_out) {
#pragma unroll
        for (int f = 0; f < FL; ++f)
            sc.st_out[s.slot(f) - sc.out_off] = make_float4(s.yr[f], s.yi[f], s.l0r[f], s.l0i[f]);
    }
}

__device__ __forceinline__ SegCtx whole_launch(const FwdArgs &p) {
    SegCtx sc;
    sc.tb = 0;
    sc.tn = p.n;
    sc.st_in = p.state;
    sc.st_out = p.state;
    sc.in_off = 0;
    sc.out_off = 0;
    sc.zl_out = nullptr;
    sc.zl_in = nullptr;
    sc.ld_zl = 0;
    return sc;
}

__device__ __forceinline__ void hist_copy_at(const HistCopy &hc, int i) {
    const int64_t m = hc.n - hc.dmax + i;
    hc.new_h[i] = m >= 0 ? hc.x[m] : hc.old_h[hc.dmax + m];
}

template <int FL, int TT, int MODE, bool XLDS, bool PARTS>
__global__ void __launch_bounds__(512) fwd_kernel(FwdArgs p) {
    extern __shared__ __align__(16) unsigned char smem[];
    if constexpr (MODE != kModeKeys) {
        // a streaming call's last launch also writes the next call's history
        // (hist_next.dmax > 0); it reads old_h and x only, which this launch
        // does not write
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.hist_next.dmax; i += gridDim.x * blockDim.x)
            hist_copy_at(p.hist_next, i);
    }
    const SegCtx sc = whole_launch(p);
    fwd_group<FL, TT, MODE, XLDS, false, PARTS>(p, p.gbase + blockIdx.x, smem, sc);
}

// Time split, local pass: item (segment, group). Segment 0 starts from the
// carried state and writes the mode's output; later segments start cold and
// keep their local z. Every item stores its end state.
template <int FL, int TT, int MODE, bool XLDS, bool PARTS>
__device__ __forceinline__ void seg_item(const FwdArgs &p, unsigned bid, unsigned char *smem) {
    const int g = p.gbase + bid % p.groups, seg = bid / p.groups;
    SegCtx sc;
    sc.tb = (int64_t)seg * p.seg_len;
    sc.tn = min(p.seg_len, p.n - sc.tb);
    sc.st_in = seg == 0 ? p.state : nullptr;
    sc.st_out = p.seg_end + (int64_t)seg * p.seg_stride;
    sc.in_off = 0;
    sc.out_off = p.seg_slot0;
    if (MODE == kModeZ) {  // the local z goes straight to the output rows; the carry pass adds to it
        sc.zl_out = seg == 0 ? nullptr : p.z + p.obase + sc.tb;
        sc.ld_zl = p.ld;
    } else {
        sc.zl_out = seg == 0 ? nullptr : p.zl + (int64_t)(seg - 1) * p.n_templates * p.seg_len;
        sc.ld_zl = p.seg_len;
    }
    sc.zl_in = nullptr;
    fwd_group<FL, TT, MODE, XLDS, false, PARTS>(p, g, smem, sc);
}

template <int FL, int TT, int MODE, bool XLDS, bool PARTS>
__global__ void __launch_bounds__(512) fwd_seg_kernel(FwdArgs p) {
    extern __shared__ __align__(16) unsigned char smem[];
    seg_item<FL, TT, MODE, XLDS, PARTS>(p, blockIdx.x, smem);
}

// Time split, carry pass over segments 1..: free response of the true
// segment-start state plus the local z, then the mode's output.
template <int FL, int TT, int MODE, bool PARTS>
__device__ __forceinline__ void carry_item(const FwdArgs &p, unsigned bid, unsigned char *smem) {
    const int g = p.gbase + bid % p.groups, seg = 1 + bid / p.groups;
    SegCtx sc;
    sc.tb = (int64_t)seg * p.seg_len;
    sc.tn = min(p.seg_len, p.n - sc.tb);
    sc.st_in = p.seg_start + (int64_t)seg * p.seg_stride;
    sc.st_out = nullptr;
    sc.in_off = p.seg_slot0;
    sc.out_off = 0;
    sc.zl_out = nullptr;
    if (MODE == kModeZ) {
        sc.zl_in = p.z + p.obase + sc.tb;
        sc.ld_zl = p.ld;
    } else {
        sc.zl_in = p.zl + (int64_t)(seg - 1) * p.n_templates * p.seg_len;
        sc.ld_zl = p.seg_len;
    }
    fwd_group<FL, TT, MODE, false, true, PARTS>(p, g, smem, sc);
}

template <int FL, int TT, int MODE, bool PARTS>
__global__ void __launch_bounds__(512) fwd_carry_kernel(FwdArgs p) {
    extern __shared__ __align__(16) unsigned char smem[];
    carry_item<FL, TT, MODE, PARTS>(p, blockIdx.x, smem);
}

// Carries of one slot across the segments of a launch: c holds the true end
// state of segment 0 on entry; for k >= 1 the true start of segment k is c,
// then c <- a^{len_k} c + e_k (e_k = segment k's end state from rest), in
// FP64. Full segments share one a^{seg_len}; the segment-end reads are issued
// eight at a time ahead of the dependent chain.
__device__ __forceinline__ void chain_segments(const float4 *seg_end, float4 *seg_start, int64_t nslots, int64_t sl,
                                               double2 a, int nseg, int64_t seg_len, int64_t n, double &cr,
                                               double &ci) {
    const double2 a_full = cpow64(a, (int)seg_len);
    for (int k0 = 1; k0 < nseg; k0 += 8) {
        float4 eb[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (k0 + u < nseg) eb[u] = seg_end[(int64_t)(k0 + u) * nslots + sl];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u;
            if (k >= nseg) break;
            const float hr = (float)cr, hi = (float)ci;
            seg_start[(int64_t)k * nslots + sl] =
                make_float4(hr, hi, (float)(cr - (double)hr), (float)(ci - (double)hi));
            const int64_t len = min(seg_len, n - (int64_t)k * seg_len);
            const double2 al = len == seg_len ? a_full : cpow64(a, (int)len);
            const float4 e = eb[u];
            const double er = (double)e.x + (double)e.z, ei = (double)e.y + (double)e.w;
            const double nr = al.x * cr - al.y * ci + er;
            const double ni = al.x * ci + al.y * cr + ei;
            cr = nr;
            ci = ni;
        }
    }
}

// Time split, carry chain: c_{s+1} = a^len_s c_s + e_s in FP64 per slot, from
// the true end of segment 0; writes every segment's true start state and the
// launch's final state. Covers slots [seg_slot0, seg_slot0 + seg_stride) of
// the segment buffers; with only_tpl >= 0 only that template's slots (the
// other slots' entries were not written by the segment pass).
__device__ __forceinline__ void chain_item(const FwdArgs &p, int fl, int nseg, unsigned chain_blocks, unsigned bid) {
    if (bid >= chain_blocks) {   // the history copy (hist_next.dmax > 0), 256 samples per block
        const int i = (int)(bid - chain_blocks) * 256 + (int)threadIdx.x;
        if (i < p.hist_next.dmax) hist_copy_at(p.hist_next, i);
        return;
    }
    const int64_t i = (int64_t)bid * blockDim.x + threadIdx.x;
    if (i >= p.seg_stride) return;  // every slot, padding included (its states stay zero)
    const int64_t sl = p.seg_slot0 + i;
    if (p.only_tpl >= 0) {
        // slot = ((group * wpg + wave) * fl + f) * 64 + lane; row = 4 (group * wpg + wave) + lane / 16
        const RowInfo ri = p.rows[((sl >> 6) / fl) * 4 + ((sl & 63) >> 4)];
        if (ri.tpl != p.only_tpl) return;
    }
    const float4 e0 = p.seg_end[i];
    double cr = (double)e0.x + (double)e0.z, ci = (double)e0.y + (double)e0.w;
    double2 a = p.s.a64[sl];
    if (p.prec == kPrecFp32) {  // the all-FP32 mode propagates with the rounded coefficient
        const float2 r = p.s.a32[sl];
        a = make_double2((double)r.x, (double)r.y);
    }
    chain_segments(p.seg_end, p.seg_start, p.seg_stride, i, a, nseg, p.seg_len, p.n, cr, ci);
    const float hr = (float)cr, hi = (float)ci;
    p.state[sl] = make_float4(hr, hi, (float)(cr - (double)hr), (float)(ci - (double)hi));
}

__global__ void seg_chain_kernel(FwdArgs p, int fl, int nseg, unsigned chain_blocks) {
    chain_item(p, fl, nseg, chain_blocks, blockIdx.x);
}

// Several banks' time-split passes, one launch per pass for all of them: the
// workgroups [first[b], first[b + 1]) of a pass run bank b's items (its own
// strain, segments, state and output rows) exactly as the one-bank kernels do.
__device__ __forceinline__ int multi_bank(const int32_t *first, int count) {
    int b = 0;
    while (b + 1 < count && (int)blockIdx.x >= first[b + 1]) ++b;
    return b;
}

template <int FL, int TT, int MODE>
__global__ void __launch_bounds__(512) fwd_seg_multi_kernel(MultiFwd m) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = multi_bank(m.seg_first, m.count);
    seg_item<FL, TT, MODE, true, false>(m.a[b], blockIdx.x - (unsigned)m.seg_first[b], smem);
}

template <int FL, int TT, int MODE>
__global__ void __launch_bounds__(512) fwd_carry_multi_kernel(MultiFwd m) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int b = multi_bank(m.carry_first, m.count);
    carry_item<FL, TT, MODE, false>(m.a[b], blockIdx.x - (unsigned)m.carry_first[b], smem);
}

__global__ void __launch_bounds__(256) seg_chain_multi_kernel(MultiFwd m, int fl) {
    const int b = multi_bank(m.chain_first, m.count);
    chain_item(m.a[b], fl, m.nseg[b], (unsigned)m.chain_blocks[b], blockIdx.x - (unsigned)m.chain_first[b]);
}

// Persistent batch kernel: workgroups pop (stream, group) items until the list
// is exhausted; every item is one block of one stream for one group.
template <int FL, int TT>
__global__ void __launch_bounds__(512) batch_kernel(const BatchStream *streams, const int2 *items,
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
        const SegCtx sc = whole_launch(a);
        fwd_group<FL, TT, kModeKeys, true, false>(a, g, smem, sc);
    }
}

// Batch with each live stream's block cut into time segments (used while the
// live streams alone cannot fill the device). Items are (stream, group << 4 |
// segment), one workgroup each; items of ended streams or of segments past the
// block's end exit at once. Per-stream segment buffers hang off the stream's
// FwdArgs (seg_end, seg_start, zl, seg_len).
__device__ __forceinline__ bool batch_item(const BatchStream *streams, const int2 *items, const int64_t *pos,
                                           int block_len, int &sidx, int &g, int &seg, int64_t &p0,
                                           int64_t &n) {
    const int2 item = items[blockIdx.x];
    sidx = __builtin_amdgcn_readfirstlane(item.x);
    g = __builtin_amdgcn_readfirstlane(item.y >> 4);
    seg = __builtin_amdgcn_readfirstlane(item.y & 15);
    p0 = pos[sidx];
    const int64_t len = streams[sidx].len;
    if (p0 >= len) return false;
    n = min((int64_t)block_len, len - p0);
    return (int64_t)seg * streams[sidx].args.seg_len < n;
}

template <int FL, int TT>
__global__ void __launch_bounds__(512) batch_seg_kernel(const BatchStream *streams, const int2 *items,
                                                        const int64_t *pos, int block_len) {
    extern __shared__ __align__(16) unsigned char smem[];
    int sidx, g, seg;
    int64_t p0, n;
    if (!batch_item(streams, items, pos, block_len, sidx, g, seg, p0, n)) return;
    FwdArgs a = streams[sidx].args;
    a.xbase = p0;
    a.n = n;
    a.ld = block_len;
    SegCtx sc;
    sc.tb = (int64_t)seg * a.seg_len;
    sc.tn = min(a.seg_len, n - sc.tb);
    sc.st_in = seg == 0 ? a.state : nullptr;
    sc.st_out = a.seg_end + (int64_t)seg * a.nslots;
    sc.in_off = 0;
    sc.out_off = 0;
    sc.zl_out = seg == 0 ? nullptr : a.zl + (int64_t)(seg - 1) * a.n_templates * a.seg_len;
    sc.zl_in = nullptr;
    sc.ld_zl = a.seg_len;
    fwd_group<FL, TT, kModeKeys, true, false>(a, g, smem, sc);
}

template <int FL, int TT>
__global__ void __launch_bounds__(512) batch_carry_kernel(const BatchStream *streams, const int2 *items,
                                                          const int64_t *pos, int block_len) {
    extern __shared__ __align__(16) unsigned char smem[];
    int sidx, g, seg;
    int64_t p0, n;
    if (!batch_item(streams, items, pos, block_len, sidx, g, seg, p0, n)) return;
    FwdArgs a = streams[sidx].args;
    a.xbase = p0;
    a.n = n;
    a.ld = block_len;
    SegCtx sc;
    sc.tb = (int64_t)seg * a.seg_len;
    sc.tn = min(a.seg_len, n - sc.tb);
    sc.st_in = a.seg_start + (int64_t)seg * a.nslots;
    sc.st_out = nullptr;
    sc.in_off = 0;
    sc.out_off = 0;
    sc.zl_out = nullptr;
    sc.zl_in = a.zl + (int64_t)(seg - 1) * a.n_templates * a.seg_len;
    sc.ld_zl = a.seg_len;
    fwd_group<FL, TT, kModeKeys, false, true>(a, g, smem, sc);
}

// FP64 carry chain of every live stream (grid.y = stream): the same
// composition as seg_chain_kernel over the segments the block actually has.
__global__ void __launch_bounds__(256) batch_chain_kernel(const BatchStream *streams, const int64_t *pos,
                                                          int block_len) {
    const int sidx = blockIdx.y;
    const FwdArgs &a = streams[sidx].args;
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= a.nslots) return;
    const int64_t p0 = pos[sidx], len = streams[sidx].len;
    if (p0 >= len) return;
    const int64_t n = min((int64_t)block_len, len - p0);
    const int nv = (int)((n + a.seg_len - 1) / a.seg_len);
    const float4 e0 = a.seg_end[sl];
    double cr = (double)e0.x + (double)e0.z, ci = (double)e0.y + (double)e0.w;
    double2 av = a.s.a64[sl];
    if (a.prec == kPrecFp32) {
        const float2 r = a.s.a32[sl];
        av = make_double2((double)r.x, (double)r.y);
    }
    chain_segments(a.seg_end, a.seg_start, a.nslots, sl, av, nv, a.seg_len, n, cr, ci);
    const float hr = (float)cr, hi = (float)ci;
    a.state[sl] = make_float4(hr, hi, (float)(cr - (double)hr), (float)(ci - (double)hi));
}

// Max over workgroup partial keys: 16 samples x 16 group slices per block.
// Blocks from key_blocks on write the history copy (hc.new_h set), 256
// samples each.
__global__ void __launch_bounds__(256) finalize_keys_kernel(const uint64_t *keys, int groups, int64_t ld,
                                                            int64_t n, float *mx, int32_t *am, HistCopy hc,
                                                            unsigned key_blocks) {
    if (blockIdx.x >= key_blocks) {   // uniform per block: no barrier below is reached
        const int i = (int)(blockIdx.x - key_blocks) * 256 + (int)threadIdx.x;
        if (i < hc.dmax) hist_copy_at(hc, i);
        return;
    }
    __shared__ uint64_t red[16][17];
    const int si = threadIdx.x & 15, q = threadIdx.x >> 4;
    const int64_t i = (int64_t)blockIdx.x * 16 + si;
    uint64_t k = 0;
    if (i < n)
        for (int g = q; g < groups; g += 16) {
            const uint64_t v = keys[(int64_t)g * ld + i];
            k = v > k ? v : k;
        }
    red[q][si] = k;
    __syncthreads();
    if (q == 0 && i < n) {
        for (int r = 1; r < 16; ++r) k = red[r][si] > k ? red[r][si] : k;
        mx[i] = __uint_as_float((uint32_t)(k >> 32));
        am[i] = (int32_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    }
}

// Templates split over workgroups: z_j = the sum of its parts' partial sums
// (in part order) for samples [0, n) of a piece, then the mode's output for
// those templates: SNR rows, z rows, or (keys) the per-sample maximum key over
// the split templates into key_row, which the key finalisation takes as one
// more workgroup.
__global__ void __launch_bounds__(256) combine_parts_kernel(const float2 *zpart, int64_t ld_part,
                                                            const int32_t *split_tpl, const int32_t *split_off,
                                                            int n_split, int64_t n, int mode, float *snr, float2 *z,
                                                            int64_t ld, int64_t obase, uint64_t *key_row) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    unsigned long long kbest = 0ull;
    for (int i = 0; i < n_split; ++i) {
        float zr = 0.f, zi = 0.f;
        for (int q = split_off[i]; q < split_off[i + 1]; ++q) {
            const float2 v = zpart[(int64_t)q * ld_part + t];
            zr += v.x;
            zi += v.y;
        }
        const int j = split_tpl[i];
        if (mode == kModeSnr) {
            snr[(int64_t)j * ld + obase + t] = zr * zr + zi * zi;
        } else if (mode == kModeZ) {
            z[(int64_t)j * ld + obase + t] = make_float2(zr, zi);
        } else {
            const float sn = zr * zr + zi * zi;
            const unsigned long long key = ((unsigned long long)__float_as_uint(sn) << 32) |
                                           (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
            kbest = key > kbest ? key : kbest;
        }
    }
    if (mode == kModeKeys) key_row[t] = kbest;
}

// Slot arrays from caller-order FP64 coefficients on the device (the same
// values the host plan computes: fl32 roundings, a^L and a^L - fl32(a)^L in
// FP64, the FP64-carry flag). Padding slots keep their zeros.
__global__ void __launch_bounds__(256) set_coeffs_kernel(const double2 *a, const double2 *b,
                                                         const int32_t *slot_filter, int64_t nslots, int L,
                                                         float2 *a32, float2 *b32, double2 *aL, double2 *dL,
                                                         double2 *a64, int32_t *flags) {
    const int64_t sl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (sl >= nslots) return;
    const int k = slot_filter[sl];
    if (k < 0) return;
    const double2 av = a[k], bv = b[k];
    const float2 af = make_float2((float)av.x, (float)av.y);
    a32[sl] = af;
    b32[sl] = make_float2((float)bv.x, (float)bv.y);
    const double2 p = cpow64(av, L), q = cpow64(make_double2((double)af.x, (double)af.y), L);
    aL[sl] = p;
    dL[sl] = make_double2(p.x - q.x, p.y - q.y);
    a64[sl] = av;
    flags[sl] = hypot(av.x, av.y) > 1.0 - 1e-5 ? 1 : 0;
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

__global__ void hist_update_kernel(HistCopy hc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < hc.dmax) hist_copy_at(hc, i);
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
// Adjoint. With lambda[m] = G[m] + conj(a) lambda[m+1] (lambda[n] = 0) the
// gradients of a real loss of z are
//     grad_b = sum_m lambda[m] x[m - d],
//     grad_a = sum_m lambda[m] conj(y[m - 1]).
// From a cold start y[m - 1] = sum_{k < m} a^(m-1-k) b x[k - d], so the second
// sum regroups exactly as
//     grad_a = conj(b) sum_k nu[k] x[k - d],
//     nu[k] = sum_{m > k} conj(a)^(m-1-k) lambda[m] = lambda[k+1] + conj(a) nu[k+1],
// a second reverse recursion driven by lambda. The backward therefore runs the
// pair (lambda, nu) from the end of the stream and never forms y: no forward
// recomputation and no stored filter states. Over s steps without input the
// pair moves by the Jordan block
//     lambda <- conj(a)^s lambda,   nu <- conj(a)^s nu + s conj(a)^(s-1) lambda.
// The pair recursion is linear, so the stream is cut into nseg segments of
// whole chunks: bwd_scan_kernel runs every segment but the first from a zero
// pair at its end (reading only G), bwd_chain_kernel composes the segments from
// the end in FP64 with the Jordan block, which gives the true pair entering
// each segment, and bwd_seg_kernel runs every segment from that pair with the
// gradient sums (FP32 within a chunk, FP64 across chunks). bwd_reduce_kernel
// adds the per-segment sums in FP64 in segment order and applies conj(b).
// Every L samples (a chunk) the pair carried into the chunk is corrected for
// the FP32 coefficient: lambda += conj(a^l - fl(a)^l) lambda_in,
// nu += conj(a^l - fl(a)^l) nu_in + l conj(a^(l-1) - fl(a)^(l-1)) lambda_in.
// ---------------------------------------------------------------------------


// v[t] = p[t] for t < ql, else 0; full runs use 16-byte loads (p is only
// 4-byte aligned, which global loads accept).
__device__ __forceinline__ void fetch_x(const float *p, int ql, float (&v)[kSub]) {
    if (ql == kSub) {
#pragma unroll
        for (int i = 0; i < kSub / 4; ++i) {
            const f4u q = *reinterpret_cast<const f4u *>(p + 4 * i);
            v[4 * i] = q.x;
            v[4 * i + 1] = q.y;
            v[4 * i + 2] = q.z;
            v[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < kSub; ++t) v[t] = t < ql ? p[t] : 0.f;
    }
}

__device__ __forceinline__ void fetch_g(const float2 *p, int ql, float (&gr)[kSub], float (&gi)[kSub]) {
    if (ql == kSub) {
#pragma unroll
        for (int i = 0; i < kSub / 2; ++i) {
            const f4u q = *reinterpret_cast<const f4u *>(p + 2 * i);
            gr[2 * i] = q.x;
            gi[2 * i] = q.y;
            gr[2 * i + 1] = q.z;
            gi[2 * i + 1] = q.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < kSub; ++t) {
            const float2 g = t < ql ? p[t] : make_float2(0.f, 0.f);
            gr[t] = g.x;
            gi[t] = g.y;
        }
    }
}

// G of one template for one sub-chunk when the address is the same for the
// whole wave: read through the constant address space, so the loads are
// scalar (one per wave, values in SGPRs) and never reach the texture path.
typedef const __attribute__((address_space(4))) float cfloat;

__device__ __forceinline__ void fetch_g_uniform(const float2 *p, int ql, float (&gr)[kSub], float (&gi)[kSub]) {
    cfloat *c = (cfloat *)p;
    if (ql == kSub) {
#pragma unroll
        for (int t = 0; t < kSub; ++t) {
            gr[t] = c[2 * t];
            gi[t] = c[2 * t + 1];
        }
    } else {
#pragma unroll
        for (int t = 0; t < kSub; ++t) {
            gr[t] = t < ql ? c[2 * t] : 0.f;
            gi[t] = t < ql ? c[2 * t + 1] : 0.f;
        }
    }
}

// A backward wave: the filters [k0, k1) of template tpl (at most 64, lane i
// takes filter k0 + i), so that G is the same for the whole wave.
struct BwdLane {
    int tpl;
    int64_t k0, k1, k;
};

__device__ __forceinline__ bool bwd_lane(const BwdArgs &p, BwdLane &bl) {
    const int w = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (w >= p.n_bwaves) return false;
    const int4 e = p.bwaves[w];
    bl.tpl = __builtin_amdgcn_readfirstlane(e.x);
    bl.k0 = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane(e.y);
    bl.k1 = (int64_t)(unsigned)__builtin_amdgcn_readfirstlane(e.z);
    bl.k = bl.k0 + (threadIdx.x & 63);
    return bl.k < bl.k1;
}

// The carried-pair corrections of an l-step chunk (see above), FP32:
// d1 = conj(a^l - fl(a)^l), d2 = l conj(a^(l-1) - fl(a)^(l-1)).
struct PairDrift {
    float d1r, d1i, d2r, d2i;
};

__device__ __forceinline__ PairDrift pair_drift(const SlotArrays &s, int64_t slot, int l, float ar, float ai) {
    const double2 a = s.a64[slot];
    const double2 af = make_double2((double)ar, (double)ai);
    const double2 p1 = cpow64(a, l - 1), q1 = cpow64(af, l - 1);
    const double2 p = cmul64(p1, a), q = cmul64(q1, af);
    PairDrift d;
    d.d1r = (float)(p.x - q.x);
    d.d1i = (float)-(p.y - q.y);
    d.d2r = (float)((double)l * (p1.x - q1.x));
    d.d2i = (float)-((double)l * (p1.y - q1.y));
    return d;
}

// lambda += d1 lambda_in; nu += d1 nu_in + d2 lambda_in (complex products).
__device__ __forceinline__ void pair_correct(float &lr, float &li, float &vr, float &vi, const PairDrift &d,
                                             float l0r, float l0i, float v0r, float v0i) {
    lr = fmaf(d.d1r, l0r, fmaf(-d.d1i, l0i, lr));
    li = fmaf(d.d1r, l0i, fmaf(d.d1i, l0r, li));
    vr = fmaf(d.d1r, v0r, fmaf(-d.d1i, v0i, fmaf(d.d2r, l0r, fmaf(-d.d2i, l0i, vr))));
    vi = fmaf(d.d1r, v0i, fmaf(d.d1i, v0r, fmaf(d.d2r, l0i, fmaf(d.d2i, l0r, vi))));
}

// One sub-chunk of the pair recursion, last step first: on entry (l, v) =
// (lambda[m+1], nu[m+1]); each step forms nu[m] = lambda[m+1] + conj(a) nu[m+1]
// and lambda[m] = G[m] + conj(a) lambda[m+1] (FULL: all kSub steps).
template <int FL, bool FULL>
__device__ __forceinline__ void pair_steps(float (&lr)[FL], float (&li)[FL], float (&vr)[FL], float (&vi)[FL],
                                           const float (&ar)[FL], const float (&ai)[FL], const float (&gr)[kSub],
                                           const float (&gi)[kSub], int ql) {
#pragma unroll
    for (int t = kSub - 1; t >= 0; --t) {
        if (FULL || t < ql) {
#pragma unroll
            for (int f = 0; f < FL; ++f) {
                const float nvr = fmaf(ar[f], vr[f], fmaf(ai[f], vi[f], lr[f]));
                const float nvi = fmaf(ar[f], vi[f], fmaf(-ai[f], vr[f], li[f]));
                const float nlr = fmaf(ar[f], lr[f], fmaf(ai[f], li[f], gr[t]));
                const float nli = fmaf(ar[f], li[f], fmaf(-ai[f], lr[f], gi[t]));
                vr[f] = nvr;
                vi[f] = nvi;
                lr[f] = nlr;
                li[f] = nli;
            }
        }
    }
}

// The same steps with the gradient sums sb += lambda[m] x[m - d],
// sa += nu[m] x[m - d] for one filter.
template <bool FULL>
__device__ __forceinline__ void grad_steps(float &lr, float &li, float &vr, float &vi, float ar, float ai,
                                           const float (&xv)[kSub], const float (&gr)[kSub], const float (&gi)[kSub],
                                           float &sar, float &sai, float &sbr, float &sbi, int ql) {
#pragma unroll
    for (int t = kSub - 1; t >= 0; --t) {
        if (FULL || t < ql) {
            const float nvr = fmaf(ar, vr, fmaf(ai, vi, lr));
            const float nvi = fmaf(ar, vi, fmaf(-ai, vr, li));
            const float nlr = fmaf(ar, lr, fmaf(ai, li, gr[t]));
            const float nli = fmaf(ar, li, fmaf(-ai, lr, gi[t]));
            vr = nvr;
            vi = nvi;
            lr = nlr;
            li = nli;
            sbr = fmaf(lr, xv[t], sbr);
            sbi = fmaf(li, xv[t], sbi);
            sar = fmaf(vr, xv[t], sar);
            sai = fmaf(vi, xv[t], sai);
        }
    }
}

// Segment-local pair at the start of segment blockIdx.y + 1, from a zero pair
// at its end (reads only G, by scalar loads). One filter per lane, one
// template per wave; the G of the next sub-chunk is loaded while the current
// one is computed.
__global__ void __launch_bounds__(256) bwd_scan_kernel(BwdArgs p) {
    BwdLane bl;
    if (!bwd_lane(p, bl)) return;
    const int64_t slot = p.filter_slot[bl.k];
    const int tpl = bl.tpl;
    const int seg = blockIdx.y + 1;
    const int64_t n = p.n, nch = (n + p.L - 1) / p.L;
    const int64_t cs = (int64_t)seg * p.seg_chunks, ce = min(nch, cs + p.seg_chunks);
    const float2 *gz = p.gz + (int64_t)tpl * n;
    const float2 a = p.s.a32[slot];
    float ar[1] = {a.x}, ai[1] = {a.y};
    PairDrift dfull;
    if (p.prec != kPrecFp32) dfull = pair_drift(p.s, slot, p.L, ar[0], ai[0]);
    float lr[1] = {0.f}, li[1] = {0.f}, vr[1] = {0.f}, vi[1] = {0.f};
    float l0r = 0.f, l0i = 0.f, v0r = 0.f, v0i = 0.f;
    auto nq_of = [&](int64_t c) { return (int)((min((int64_t)p.L, n - c * p.L) + kSub - 1) / kSub); };
    auto fetch = [&](float (&gr)[kSub], float (&gi)[kSub], int64_t c, int q) {
        const int64_t m0 = c * p.L + (int64_t)q * kSub;
        const int ql = (int)min((int64_t)kSub, min((int64_t)p.L, n - c * p.L) - (int64_t)q * kSub);
        fetch_g_uniform(gz + m0, ql, gr, gi);
    };
    auto run = [&](const float (&gr)[kSub], const float (&gi)[kSub], int64_t c, int q) {
        const int l = (int)min((int64_t)p.L, n - c * p.L);
        const int ql = min(kSub, l - q * kSub);
        if (q == nq_of(c) - 1) {
            l0r = lr[0];
            l0i = li[0];
            v0r = vr[0];
            v0i = vi[0];
        }
        if (ql == kSub)
            pair_steps<1, true>(lr, li, vr, vi, ar, ai, gr, gi, ql);
        else
            pair_steps<1, false>(lr, li, vr, vi, ar, ai, gr, gi, ql);
        if (q == 0 && p.prec != kPrecFp32) {
            const PairDrift d = l == p.L ? dfull : pair_drift(p.s, slot, l, ar[0], ai[0]);
            pair_correct(lr[0], li[0], vr[0], vi[0], d, l0r, l0i, v0r, v0i);
        }
    };
    auto step_back = [&](int64_t &c, int &q) {
        if (q > 0) {
            --q;
        } else {
            --c;
            q = c >= cs ? nq_of(c) - 1 : 0;
        }
    };
    if (ce > cs) {
        float agr[kSub], agi[kSub], bgr[kSub], bgi[kSub];
        int64_t c = ce - 1;
        int q = nq_of(c) - 1;
        fetch(agr, agi, c, q);
        while (true) {
            int64_t cb = c;
            int qb = q;
            step_back(cb, qb);
            if (cb >= cs) fetch(bgr, bgi, cb, qb);
            run(agr, agi, c, q);
            if (cb < cs) break;
            c = cb;
            q = qb;
            int64_t ca = c;
            int qa = q;
            step_back(ca, qa);
            if (ca >= cs) fetch(agr, agi, ca, qa);
            run(bgr, bgi, c, q);
            if (ca < cs) break;
            c = ca;
            q = qa;
        }
    }
    p.pair_loc[(int64_t)seg * p.nslots + slot] = make_float4(lr[0], li[0], vr[0], vi[0]);
}

// True pair entering every segment from the right (zero for the last one):
// pair[s0] = pair_loc[s0] + J^(e - s0) pair[e], J the Jordan block of conj(a),
// in FP64 (with fl32(a) in the all-FP32 mode).
__global__ void __launch_bounds__(256) bwd_chain_kernel(BwdArgs p) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= p.nslots) return;
    const int64_t n = p.n, nch = (n + p.L - 1) / p.L;
    double2 a = p.s.a64[slot];
    if (p.prec == kPrecFp32) {
        const float2 a32 = p.s.a32[slot];
        a = make_double2((double)a32.x, (double)a32.y);
    }
    double lr = 0.0, li = 0.0, vr = 0.0, vi = 0.0;
    for (int seg = p.nseg - 1; seg >= 0; --seg) {
        p.pair_in[(int64_t)seg * p.nslots + slot] = make_float4((float)lr, (float)li, (float)vr, (float)vi);
        if (seg == 0) break;
        const int64_t cs = (int64_t)seg * p.seg_chunks, ce = min(nch, cs + p.seg_chunks);
        const int64_t len = min(n, ce * p.L) - cs * p.L;
        const double2 a1 = cpow64(a, (int)(len - 1));   // conj(a)^k = conj(a^k)
        const double2 al = cmul64(a1, a);
        const double sr = (double)len * a1.x, si = (double)len * a1.y;
        const float4 loc = p.pair_loc[(int64_t)seg * p.nslots + slot];
        const double nvr = (double)loc.z + (al.x * vr + al.y * vi) + (sr * lr + si * li);
        const double nvi = (double)loc.w + (al.x * vi - al.y * vr) + (sr * li - si * lr);
        const double nlr = (double)loc.x + al.x * lr + al.y * li;
        const double nli = (double)loc.y + al.x * li - al.y * lr;
        lr = nlr;
        li = nli;
        vr = nvr;
        vi = nvi;
    }
}

// Strain and G of one sub-chunk of the backward.
struct SubBuf {
    float x[kSub], gr[kSub], gi[kSub];
};

// Full backward of segment blockIdx.y from its true incoming pair. One filter
// per lane; every wave holds filters of one template (G read by scalar loads).
// Sub-chunks are taken in reverse order through two register buffers: the
// next one is loaded while the current one is computed.
__global__ void __launch_bounds__(256) bwd_seg_kernel(BwdArgs p) {
    BwdLane bl;
    if (!bwd_lane(p, bl)) return;
    const int64_t slot = p.filter_slot[bl.k];
    const int tpl = bl.tpl;
    const int seg = blockIdx.y;
    const int64_t n = p.n, nch = (n + p.L - 1) / p.L;
    const int64_t cs = (int64_t)seg * p.seg_chunks, ce = min(nch, cs + p.seg_chunks);
    const float2 *gz = p.gz + (int64_t)tpl * n;
    const float2 a = p.s.a32[slot];
    const float ar = a.x, ai = a.y;
    const float *xw = p.xwin + p.s.xoff[slot];  // xw[m] = x[m - d]
    PairDrift dfull;
    if (p.prec != kPrecFp32) dfull = pair_drift(p.s, slot, p.L, ar, ai);
    double gar = 0.0, gai = 0.0, gbr = 0.0, gbi = 0.0;
    const float4 pin = p.pair_in[(int64_t)seg * p.nslots + slot];
    float lr = pin.x, li = pin.y, vr = pin.z, vi = pin.w;   // the pair after the current chunk
    float l0r = 0.f, l0i = 0.f, v0r = 0.f, v0i = 0.f;       // the pair entering the current chunk
    float sar = 0.f, sai = 0.f, sbr = 0.f, sbi = 0.f;
    auto nq_of = [&](int64_t c) { return (int)((min((int64_t)p.L, n - c * p.L) + kSub - 1) / kSub); };
    auto fetch = [&](SubBuf &b, int64_t c, int q) {
        const int64_t m0 = c * p.L + (int64_t)q * kSub;
        const int ql = (int)min((int64_t)kSub, min((int64_t)p.L, n - c * p.L) - (int64_t)q * kSub);
        fetch_x(xw + m0, ql, b.x);
        fetch_g_uniform(gz + m0, ql, b.gr, b.gi);
    };
    // one sub-chunk: chunk bookkeeping at its first (q = last) and last (q = 0) sub-chunk
    auto run = [&](const SubBuf &b, int64_t c, int q) {
        const int l = (int)min((int64_t)p.L, n - c * p.L);
        const int ql = min(kSub, l - q * kSub);
        if (q == nq_of(c) - 1) {
            l0r = lr;
            l0i = li;
            v0r = vr;
            v0i = vi;
            sar = sai = sbr = sbi = 0.f;
        }
        if (ql == kSub)
            grad_steps<true>(lr, li, vr, vi, ar, ai, b.x, b.gr, b.gi, sar, sai, sbr, sbi, ql);
        else
            grad_steps<false>(lr, li, vr, vi, ar, ai, b.x, b.gr, b.gi, sar, sai, sbr, sbi, ql);
        if (q == 0) {
            if (p.prec != kPrecFp32) {
                const PairDrift d = l == p.L ? dfull : pair_drift(p.s, slot, l, ar, ai);
                pair_correct(lr, li, vr, vi, d, l0r, l0i, v0r, v0i);
            }
            gar += (double)sar;
            gai += (double)sai;
            gbr += (double)sbr;
            gbi += (double)sbi;
        }
    };
    // reverse enumeration of the segment's sub-chunks
    auto step_back = [&](int64_t &c, int &q) {
        if (q > 0) {
            --q;
        } else {
            --c;
            q = c >= cs ? nq_of(c) - 1 : 0;
        }
    };
    if (ce > cs) {
        SubBuf A, B;
        int64_t c = ce - 1;
        int q = nq_of(c) - 1;
        fetch(A, c, q);
        while (true) {
            int64_t cb = c;
            int qb = q;
            step_back(cb, qb);
            if (cb >= cs) fetch(B, cb, qb);
            run(A, c, q);
            if (cb < cs) break;
            c = cb;
            q = qb;
            int64_t ca = c;
            int qa = q;
            step_back(ca, qa);
            if (ca >= cs) fetch(A, ca, qa);
            run(B, c, q);
            if (ca < cs) break;
            c = ca;
            q = qa;
        }
    }
    p.gpart[((int64_t)seg * 2 + 0) * p.nslots + slot] = make_double2(gar, gai);
    p.gpart[((int64_t)seg * 2 + 1) * p.nslots + slot] = make_double2(gbr, gbi);
}

// Sum over segments in FP64, then grad_a = conj(fl32(b)) * sum nu x.
__global__ void __launch_bounds__(256) bwd_reduce_kernel(BwdArgs p) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= p.nslots) return;
    const int k = p.slot_filter[slot];
    if (k < 0) return;
    double gar = 0.0, gai = 0.0, gbr = 0.0, gbi = 0.0;
    for (int seg = 0; seg < p.nseg; ++seg) {
        const double2 ga = p.gpart[((int64_t)seg * 2 + 0) * p.nslots + slot];
        const double2 gb = p.gpart[((int64_t)seg * 2 + 1) * p.nslots + slot];
        gar += ga.x;
        gai += ga.y;
        gbr += gb.x;
        gbi += gb.y;
    }
    const float2 b = p.s.b32[slot];
    const double br = (double)b.x, bi = (double)b.y;
    p.grad_a[k] = make_float2((float)(br * gar + bi * gai), (float)(br * gai - bi * gar));
    p.grad_b[k] = make_float2((float)gbr, (float)gbi);
}

// Batch bookkeeping.
__global__ void __launch_bounds__(256) batch_finalize_kernel(const BatchStream *streams, const uint64_t *keys,
                                                             int64_t key_stride, const int64_t *pos,
                                                             int block_len) {
    __shared__ uint64_t red[16][17];
    const int sidx = blockIdx.y;
    const int si = threadIdx.x & 15, q = threadIdx.x >> 4;
    const int64_t i = (int64_t)blockIdx.x * 16 + si;
    const int64_t p0 = pos[sidx];
    const int64_t len = streams[sidx].len;
    const bool live = p0 < len && i < min((int64_t)block_len, len - p0);
    const uint64_t *kk = keys + sidx * key_stride;
    const int groups = streams[sidx].groups;
    uint64_t k = 0;
    if (live)
        for (int g = q; g < groups; g += 16) {
            const uint64_t v = kk[(int64_t)g * block_len + i];
            k = v > k ? v : k;
        }
    red[q][si] = k;
    __syncthreads();
    if (q == 0 && live) {
        for (int r = 1; r < 16; ++r) k = red[r][si] > k ? red[r][si] : k;
        streams[sidx].max_out[p0 + i] = __uint_as_float((uint32_t)(k >> 32));
        streams[sidx].arg_out[p0 + i] = (int32_t)(0xFFFFFFFFu - (uint32_t)(k & 0xFFFFFFFFull));
    }
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

template <int FL, int TT, int MODE, bool XLDS>
hipError_t launch_fwd_t(const FwdArgs &a, int groups, size_t lds, hipStream_t st, KernelEvents ev) {
    if (a.zpart)
        hipExtLaunchKernelGGL((fwd_kernel<FL, TT, MODE, XLDS, true>), dim3(groups), dim3(a.wpg * 64), (uint32_t)lds,
                              st, ev.start, ev.stop, 0u, a);
    else
        hipExtLaunchKernelGGL((fwd_kernel<FL, TT, MODE, XLDS, false>), dim3(groups), dim3(a.wpg * 64), (uint32_t)lds,
                              st, ev.start, ev.stop, 0u, a);
    return hipGetLastError();
}

template <int TT, int MODE, bool XLDS>
hipError_t launch_fwd_m(const FwdArgs &a, int fl, int groups, size_t lds, hipStream_t st, KernelEvents ev) {
    switch (fl) {
        case 1: return launch_fwd_t<1, TT, MODE, XLDS>(a, groups, lds, st, ev);
        case 2: return launch_fwd_t<2, TT, MODE, XLDS>(a, groups, lds, st, ev);
        case 3: return launch_fwd_t<3, TT, MODE, XLDS>(a, groups, lds, st, ev);
        case 4: return launch_fwd_t<4, TT, MODE, XLDS>(a, groups, lds, st, ev);
        default: return hipErrorInvalidValue;
    }
}

template <int TT, bool XLDS>
hipError_t launch_fwd_x(const FwdArgs &a, int mode, int fl, int groups, size_t lds, hipStream_t st,
                        KernelEvents ev) {
    switch (mode) {
        case kModeSnr: return launch_fwd_m<TT, kModeSnr, XLDS>(a, fl, groups, lds, st, ev);
        case kModeKeys: return launch_fwd_m<TT, kModeKeys, XLDS>(a, fl, groups, lds, st, ev);
        case kModeZ: return launch_fwd_m<TT, kModeZ, XLDS>(a, fl, groups, lds, st, ev);
        default: return hipErrorInvalidValue;
    }
}

template <int FL, int TT, int MODE, bool XLDS>
hipError_t launch_split_t(const FwdArgs &a, int nseg, size_t lds, size_t lds_carry, const int32_t *slot_filter,
                          hipStream_t st, KernelEvents ev) {
    if (a.zpart)
        hipExtLaunchKernelGGL((fwd_seg_kernel<FL, TT, MODE, XLDS, true>), dim3(a.groups * nseg), dim3(a.wpg * 64),
                              (uint32_t)lds, st, ev.start, (hipEvent_t) nullptr, 0u, a);
    else
        hipExtLaunchKernelGGL((fwd_seg_kernel<FL, TT, MODE, XLDS, false>), dim3(a.groups * nseg), dim3(a.wpg * 64),
                              (uint32_t)lds, st, ev.start, (hipEvent_t) nullptr, 0u, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned nb = (unsigned)((a.seg_stride + 255) / 256);
    const unsigned hb = a.hist_next.dmax > 0 ? (unsigned)((a.hist_next.dmax + 255) / 256) : 0u;
    (void)slot_filter;
    hipLaunchKernelGGL(seg_chain_kernel, dim3(nb + hb), dim3(256), 0, st, a, FL, nseg, nb);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (a.zpart)
        hipExtLaunchKernelGGL((fwd_carry_kernel<FL, TT, MODE, true>), dim3(a.groups * (nseg - 1)), dim3(a.wpg * 64),
                              (uint32_t)lds_carry, st, (hipEvent_t) nullptr, ev.stop, 0u, a);
    else
        hipExtLaunchKernelGGL((fwd_carry_kernel<FL, TT, MODE, false>), dim3(a.groups * (nseg - 1)), dim3(a.wpg * 64),
                              (uint32_t)lds_carry, st, (hipEvent_t) nullptr, ev.stop, 0u, a);
    return hipGetLastError();
}

template <int TT, int MODE, bool XLDS>
hipError_t launch_split_m(const FwdArgs &a, int fl, int nseg, size_t lds, size_t ldc, const int32_t *sf,
                          hipStream_t st, KernelEvents ev) {
    switch (fl) {
        case 1: return launch_split_t<1, TT, MODE, XLDS>(a, nseg, lds, ldc, sf, st, ev);
        case 2: return launch_split_t<2, TT, MODE, XLDS>(a, nseg, lds, ldc, sf, st, ev);
        case 3: return launch_split_t<3, TT, MODE, XLDS>(a, nseg, lds, ldc, sf, st, ev);
        case 4: return launch_split_t<4, TT, MODE, XLDS>(a, nseg, lds, ldc, sf, st, ev);
        default: return hipErrorInvalidValue;
    }
}

template <int TT, bool XLDS>
hipError_t launch_split_x(const FwdArgs &a, int mode, int fl, int nseg, size_t lds, size_t ldc, const int32_t *sf,
                          hipStream_t st, KernelEvents ev) {
    if (mode == kModeSnr) return launch_split_m<TT, kModeSnr, XLDS>(a, fl, nseg, lds, ldc, sf, st, ev);
    if (mode == kModeKeys) return launch_split_m<TT, kModeKeys, XLDS>(a, fl, nseg, lds, ldc, sf, st, ev);
    if (mode == kModeZ) return launch_split_m<TT, kModeZ, XLDS>(a, fl, nseg, lds, ldc, sf, st, ev);
    return hipErrorInvalidValue;
}

template <int FL, int TT>
int occ_t(int wpg, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwd_kernel<FL, TT, kModeKeys, true, false>, wpg * 64, lds) !=
        hipSuccess)
        return 0;
    return nb;
}

inline unsigned nblocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_forward(const FwdArgs &a, int mode, int fl, int tt, bool x_in_lds, int groups,
                          size_t lds, hipStream_t st, KernelEvents ev) {
    if (groups <= 0) return hipSuccess;
    if (tt == 16)
        return x_in_lds ? launch_fwd_x<16, true>(a, mode, fl, groups, lds, st, ev)
                        : launch_fwd_x<16, false>(a, mode, fl, groups, lds, st, ev);
    if (tt == 8)
        return x_in_lds ? launch_fwd_x<8, true>(a, mode, fl, groups, lds, st, ev)
                        : launch_fwd_x<8, false>(a, mode, fl, groups, lds, st, ev);
    return hipErrorInvalidValue;
}

hipError_t launch_forward_split(const FwdArgs &a, int mode, int fl, int tt, bool x_in_lds, int nseg, size_t lds,
                                size_t lds_carry, const int32_t *slot_filter, hipStream_t st,
                                KernelEvents ev) {
    if (a.groups <= 0 || nseg < 2) return hipErrorInvalidValue;
    if (tt == 16)
        return x_in_lds ? launch_split_x<16, true>(a, mode, fl, nseg, lds, lds_carry, slot_filter, st, ev)
                        : launch_split_x<16, false>(a, mode, fl, nseg, lds, lds_carry, slot_filter, st, ev);
    if (tt == 8)
        return x_in_lds ? launch_split_x<8, true>(a, mode, fl, nseg, lds, lds_carry, slot_filter, st, ev)
                        : launch_split_x<8, false>(a, mode, fl, nseg, lds, lds_carry, slot_filter, st, ev);
    return hipErrorInvalidValue;
}

namespace {

template <int FL, int TT>
hipError_t launch_multi_t(const MultiFwd &m, int wpg, size_t lds, size_t lds_carry, hipStream_t st) {
    const int n = m.count;
    hipLaunchKernelGGL((fwd_seg_multi_kernel<FL, TT, kModeZ>), dim3((unsigned)m.seg_first[n]), dim3(wpg * 64), lds,
                       st, m);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(seg_chain_multi_kernel, dim3((unsigned)m.chain_first[n]), dim3(256), 0, st, m, FL);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((fwd_carry_multi_kernel<FL, TT, kModeZ>), dim3((unsigned)m.carry_first[n]), dim3(wpg * 64),
                       lds_carry, st, m);
    return hipGetLastError();
}

template <int TT>
hipError_t launch_multi_f(const MultiFwd &m, int fl, int wpg, size_t lds, size_t lds_carry, hipStream_t st) {
    switch (fl) {
        case 1: return launch_multi_t<1, TT>(m, wpg, lds, lds_carry, st);
        case 2: return launch_multi_t<2, TT>(m, wpg, lds, lds_carry, st);
        case 3: return launch_multi_t<3, TT>(m, wpg, lds, lds_carry, st);
        case 4: return launch_multi_t<4, TT>(m, wpg, lds, lds_carry, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_forward_split_multi(const MultiFwd &m, int fl, int tt, int wpg, size_t lds, size_t lds_carry,
                                      hipStream_t st) {
    if (m.count < 1 || m.count > kMultiMax) return hipErrorInvalidValue;
    if (tt == 16) return launch_multi_f<16>(m, fl, wpg, lds, lds_carry, st);
    if (tt == 8) return launch_multi_f<8>(m, fl, wpg, lds, lds_carry, st);
    return hipErrorInvalidValue;
}

int forward_occupancy(int fl, int tt, int wpg, size_t lds) {
    if (tt == 16) {
        switch (fl) {
            case 1: return occ_t<1, 16>(wpg, lds);
            case 2: return occ_t<2, 16>(wpg, lds);
            case 3: return occ_t<3, 16>(wpg, lds);
            case 4: return occ_t<4, 16>(wpg, lds);
        }
    } else {
        switch (fl) {
            case 1: return occ_t<1, 8>(wpg, lds);
            case 2: return occ_t<2, 8>(wpg, lds);
            case 3: return occ_t<3, 8>(wpg, lds);
            case 4: return occ_t<4, 8>(wpg, lds);
        }
    }
    return 0;
}

hipError_t launch_finalize_keys(const uint64_t *keys, int groups, int64_t ld, int64_t n,
                                float *mx, int32_t *am, hipStream_t st, const HistCopy *hc) {
    HistCopy h{nullptr, nullptr, nullptr, 0, 0};
    if (hc && hc->dmax > 0) h = *hc;
    const unsigned kb = n > 0 ? nblocks(n, 16) : 0u;
    const unsigned hb = h.dmax > 0 ? nblocks(h.dmax, 256) : 0u;
    if (kb + hb == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_keys_kernel, dim3(kb + hb), dim3(256), 0, st, keys, groups, ld, n, mx, am, h,
                       kb);
    return hipGetLastError();
}

hipError_t launch_combine_parts(const float2 *zpart, int64_t ld_part, const int32_t *split_tpl,
                                const int32_t *split_off, int n_split, int64_t n, int mode, float *snr, float2 *z,
                                int64_t ld, int64_t obase, uint64_t *key_row, hipStream_t st) {
    if (n <= 0 || n_split <= 0) return hipSuccess;
    hipLaunchKernelGGL(combine_parts_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, zpart, ld_part, split_tpl,
                       split_off, n_split, n, mode, snr, z, ld, obase, key_row);
    return hipGetLastError();
}

hipError_t launch_set_coeffs(const double *a, const double *b, const int32_t *slot_filter, int64_t nslots, int L,
                             float2 *a32, float2 *b32, double2 *aL, double2 *dL, double2 *a64, int32_t *flags,
                             hipStream_t st) {
    if (nslots <= 0) return hipSuccess;
    hipLaunchKernelGGL(set_coeffs_kernel, dim3(nblocks(nslots, 256)), dim3(256), 0, st,
                       reinterpret_cast<const double2 *>(a), reinterpret_cast<const double2 *>(b), slot_filter,
                       nslots, L, a32, b32, aL, dL, a64, flags);
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
    const HistCopy hc{old_h, new_h, x, n, dmax};
    hipLaunchKernelGGL(hist_update_kernel, dim3(nblocks(dmax, 256)), dim3(256), 0, st, hc);
    return hipGetLastError();
}

hipError_t launch_window_fill(float *xwin, const float *hist, const float *x, int64_t n, int dmax,
                              hipStream_t st) {
    if (n + dmax <= 0) return hipSuccess;
    hipLaunchKernelGGL(window_fill_kernel, dim3(nblocks(n + dmax, 256)), dim3(256), 0, st, xwin,
                       hist, x, n, dmax);
    return hipGetLastError();
}

template <int FL, int TT>
int bocc_t(int wpg, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batch_kernel<FL, TT>, wpg * 64, lds) != hipSuccess)
        return 0;
    return nb;
}

int batch_occupancy(int fl, int tt, int wpg, size_t lds) {
    switch (fl * 100 + tt) {
        case 108: return bocc_t<1, 8>(wpg, lds);
        case 208: return bocc_t<2, 8>(wpg, lds);
        case 308: return bocc_t<3, 8>(wpg, lds);
        case 408: return bocc_t<4, 8>(wpg, lds);
        case 116: return bocc_t<1, 16>(wpg, lds);
        case 216: return bocc_t<2, 16>(wpg, lds);
        case 316: return bocc_t<3, 16>(wpg, lds);
        case 416: return bocc_t<4, 16>(wpg, lds);
        default: return 0;
    }
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

hipError_t launch_backward_t(const BwdArgs &a, hipStream_t st) {
    if (a.nseg > 1) {
        hipLaunchKernelGGL(bwd_scan_kernel, dim3(nblocks(a.n_bwaves, 4), a.nseg - 1), dim3(256), 0, st, a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(bwd_chain_kernel, dim3(nblocks(a.nslots, 256)), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bwd_seg_kernel, dim3(nblocks(a.n_bwaves, 4), a.nseg), dim3(256), 0, st, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bwd_reduce_kernel, dim3(nblocks(a.nslots, 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_backward(const BwdArgs &a, hipStream_t st) {
    if (a.n_bwaves <= 0) return hipSuccess;
    if (a.nseg < 1 || a.nseg > 65535 || a.seg_chunks < 1) return hipErrorInvalidValue;
    return launch_backward_t(a, st);
}

template <int FL, int TT>
hipError_t launch_batch_t(const BatchStream *streams, const int2 *items, int nitems, int *counter,
                          const int64_t *pos, int block_len, int grid, int wpg, size_t lds, hipStream_t st) {
    hipLaunchKernelGGL((batch_kernel<FL, TT>), dim3(grid), dim3(wpg * 64), lds, st, streams, items, nitems,
                       counter, pos, block_len);
    return hipGetLastError();
}

hipError_t launch_batch(const BatchStream *streams, const int2 *items, int nitems, int *counter,
                        const int64_t *pos, int block_len, int fl, int tt, int grid, int wpg, size_t lds,
                        hipStream_t st) {
    switch (fl * 100 + tt) {
        case 108: return launch_batch_t<1, 8>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 208: return launch_batch_t<2, 8>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 308: return launch_batch_t<3, 8>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 408: return launch_batch_t<4, 8>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 116: return launch_batch_t<1, 16>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 216: return launch_batch_t<2, 16>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 316: return launch_batch_t<3, 16>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        case 416: return launch_batch_t<4, 16>(streams, items, nitems, counter, pos, block_len, grid, wpg, lds, st);
        default: return hipErrorInvalidValue;
    }
}

template <int FL, int TT>
hipError_t launch_batch_split_t(const BatchStream *streams, const int2 *seg_items, int n_seg_items,
                                const int2 *carry_items, int n_carry_items, const int64_t *pos, int block_len,
                                int nstreams, int64_t max_slots, int wpg, size_t lds, size_t lds_carry,
                                hipStream_t st) {
    hipLaunchKernelGGL((batch_seg_kernel<FL, TT>), dim3(n_seg_items), dim3(wpg * 64), lds, st, streams, seg_items,
                       pos, block_len);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_chain_kernel, dim3(nblocks(max_slots, 256), nstreams), dim3(256), 0, st, streams, pos,
                       block_len);
    e = hipGetLastError();
    if (e != hipSuccess || n_carry_items == 0) return e;
    hipLaunchKernelGGL((batch_carry_kernel<FL, TT>), dim3(n_carry_items), dim3(wpg * 64), lds_carry, st, streams,
                       carry_items, pos, block_len);
    return hipGetLastError();
}

hipError_t launch_batch_split(const BatchStream *streams, const int2 *seg_items, int n_seg_items,
                              const int2 *carry_items, int n_carry_items, const int64_t *pos, int block_len,
                              int nstreams, int64_t max_slots, int fl, int tt, int wpg, size_t lds,
                              size_t lds_carry, hipStream_t st) {
#define SPIIR_SPLIT_ARGS streams, seg_items, n_seg_items, carry_items, n_carry_items, pos, block_len, nstreams, \
                         max_slots, wpg, lds, lds_carry, st
    switch (fl * 100 + tt) {
        case 108: return launch_batch_split_t<1, 8>(SPIIR_SPLIT_ARGS);
        case 208: return launch_batch_split_t<2, 8>(SPIIR_SPLIT_ARGS);
        case 308: return launch_batch_split_t<3, 8>(SPIIR_SPLIT_ARGS);
        case 408: return launch_batch_split_t<4, 8>(SPIIR_SPLIT_ARGS);
        case 116: return launch_batch_split_t<1, 16>(SPIIR_SPLIT_ARGS);
        case 216: return launch_batch_split_t<2, 16>(SPIIR_SPLIT_ARGS);
        case 316: return launch_batch_split_t<3, 16>(SPIIR_SPLIT_ARGS);
        case 416: return launch_batch_split_t<4, 16>(SPIIR_SPLIT_ARGS);
        default: return hipErrorInvalidValue;
    }
#undef SPIIR_SPLIT_ARGS
}

hipError_t launch_batch_finalize(const BatchStream *streams, int nstreams, const uint64_t *keys,
                                 int64_t key_stride, const int64_t *pos, int block_len,
                                 int max_groups, hipStream_t st) {
    (void)max_groups;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(nblocks(block_len, 16), nstreams), dim3(256), 0,
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
