// Host side of the multi-rate bank (spiir_multirate_*): the level banks,
// their streams and graphs, and the resampling launches. Declared in
// include/spiir.h.
#include "host_common.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

using namespace spiir;
using namespace spiir::host;

struct spiir_multirate {
    int device = 0;
    int T = 0, R = 0, top = 0;  // levels 0..R; top = highest level holding filters
    int lh = 0, lg = 0, hh = 0;  // decimation / interpolation taps, interpolation history
    int64_t B = 0;               // most full-rate samples per piece (a multiple of 2^R)
    std::vector<spiir_bank *> bank;      // per level; NULL where the level holds no filters
    std::vector<int32_t *> zrow;         // per level, device [T]: row of template j in z, or -1
    std::vector<float *> xbuf;           // per level >= 1: the decimated stream [B >> r]
    std::vector<float *> dh[2];          // per level >= 1: decimation history [lh - 1] (double-buffered)
    std::vector<float2 *> z;             // per level with filters: template sums [T_r][B >> r]
    std::vector<float2 *> wh[2];         // 1 <= r <= top: interpolation history of W_r [T][hh]
    bool pyramid = false;                // every decimation level in one launch (fits in LDS)
    std::vector<int> multi;              // levels whose banks share one launch per time-split pass
    int cur = 0;
    uint64_t *keys = nullptr;            // [chunks][B]
    float *h = nullptr, *g = nullptr;
    // the level banks run concurrently: each on its own stream, forked from the
    // caller's stream after the decimation and joined before the interpolation
    std::vector<hipStream_t> lstream;
    std::vector<hipEvent_t> lfork, ldone;
    // trigger calls in pieces of exactly B samples replay a captured graph of
    // the whole piece (one per history parity): the block is copied into xin,
    // the max / argmax out of mxo / amo
    bool use_graph = true;
    bool graph_failed = false;
    int64_t eager_pieces = 0;
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    float *xin = nullptr, *mxo = nullptr;
    int32_t *amo = nullptr;
};

namespace {

void mr_free_graphs(spiir_multirate *mr) {
    for (auto &g : mr->gexec)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
}

void mr_free(spiir_multirate *mr) {
    mr_free_graphs(mr);
    if (mr->cap) (void)hipStreamDestroy(mr->cap);
    mr->cap = nullptr;
    dfree(mr->xin);
    dfree(mr->mxo);
    dfree(mr->amo);
    for (auto s : mr->lstream)
        if (s) (void)hipStreamDestroy(s);
    for (auto e : mr->ldone)
        if (e) (void)hipEventDestroy(e);
    for (auto e : mr->lfork)
        if (e) (void)hipEventDestroy(e);
    mr->lstream.clear();
    mr->ldone.clear();
    mr->lfork.clear();
    for (auto *bk : mr->bank)
        if (bk) spiir_bank_destroy(bk);
    for (auto *p : mr->zrow) dfree(p);
    for (auto *p : mr->xbuf) dfree(p);
    for (int c = 0; c < 2; ++c) {
        for (auto *p : mr->dh[c]) dfree(p);
        for (auto *p : mr->wh[c]) dfree(p);
    }
    for (auto *p : mr->z) dfree(p);
    dfree(mr->keys);
    dfree(mr->h);
    dfree(mr->g);
}

int mr_clear_history(spiir_multirate *mr, hipStream_t st) {
    for (int c = 0; c < 2; ++c)
        for (int r = 1; r <= mr->top; ++r) {
            HIPCHK(launch_fill_zero(mr->dh[c][r], (size_t)std::max(1, mr->lh - 1) * sizeof(float), st));
            HIPCHK(launch_fill_zero(mr->wh[c][r], (size_t)mr->T * std::max(1, mr->hh) * sizeof(float2), st));
        }
    mr->cur = 0;
    return SPIIR_OK;
}

// One piece (np <= B samples) of the multi-rate bank: decimation, the level
// banks forked onto their streams, then one launch that interpolates every
// level back to the full rate and writes the full-rate z (out0, row stride
// ld0) or the per-sample keys for the max / argmax (mx, am).
int mr_piece(spiir_multirate *mr, const float *x0, int64_t np, float2 *out0, int64_t ld0, float *mx, int32_t *am,
             hipStream_t st) {
    const int top = mr->top;
    const int c = mr->cur;
    // the small levels' banks as one group of time-split launches, on the
    // stream of the group's first level once the group's last input exists
    bool grouped[kMaxLevels] = {};
    int g0 = -1, g1 = -1;
    std::vector<spiir_bank *> gb;
    std::vector<const float *> gx;
    std::vector<int64_t> gn, gld;
    std::vector<float *> gz;
    if (!mr->multi.empty()) {
        for (int r : mr->multi) {
            gb.push_back(mr->bank[r]);
            gx.push_back(r == 0 ? x0 : mr->xbuf[r]);
            gn.push_back(np >> r);
            gz.push_back(reinterpret_cast<float *>(mr->z[r]));
            gld.push_back(mr->B >> r);
        }
        if (banks_multi_ok(gb.data(), (int)gb.size(), gn.data())) {
            for (int r : mr->multi) grouped[r] = true;
            g0 = mr->multi.front();
            g1 = mr->multi.back();
        }
    }
    // each level's bank is forked onto its stream as soon as its input exists
    auto fork = [&](int r, const float *xr) -> int {
        if (!mr->bank[r]) return SPIIR_OK;
        if (grouped[r]) {
            if (r != g1) return SPIIR_OK;
            HIPCHK(hipEventRecord(mr->lfork[g0], st));
            HIPCHK(hipStreamWaitEvent(mr->lstream[g0], mr->lfork[g0], 0));
            const int rc = banks_stream_z_multi(gb.data(), (int)gb.size(), gx.data(), gn.data(), gz.data(),
                                                gld.data(), mr->lstream[g0]);
            if (rc) return rc;
            HIPCHK(hipEventRecord(mr->ldone[g0], mr->lstream[g0]));
            return SPIIR_OK;
        }
        HIPCHK(hipEventRecord(mr->lfork[r], st));
        HIPCHK(hipStreamWaitEvent(mr->lstream[r], mr->lfork[r], 0));
        const int rc = bank_stream_z(mr->bank[r], xr, np >> r, reinterpret_cast<float *>(mr->z[r]), mr->B >> r,
                                     mr->lstream[r]);
        if (rc) return rc;
        HIPCHK(hipEventRecord(mr->ldone[r], mr->lstream[r]));
        return SPIIR_OK;
    };
    int rc = fork(0, x0);
    if (rc) return rc;
    if (top > 0 && mr->pyramid) {
        MrPyramid pm;
        std::memset(&pm, 0, sizeof pm);
        for (int r = 1; r <= top; ++r) {
            pm.hist[r] = mr->dh[c][r];
            pm.hist_new[r] = mr->dh[c ^ 1][r];
            pm.dst[r] = mr->xbuf[r];
        }
        HIPCHK(launch_mr_pyramid(x0, np, top, pm, mr->h, mr->lh, mr->B, st));
        for (int r = 1; r <= top; ++r)
            if ((rc = fork(r, mr->xbuf[r]))) return rc;
    } else {
        for (int r = 1; r <= top; ++r) {
            HIPCHK(launch_mr_decimate(r == 1 ? x0 : mr->xbuf[r - 1], np >> (r - 1), mr->dh[c][r], mr->dh[c ^ 1][r],
                                      mr->h, mr->lh, mr->xbuf[r], st));
            if ((rc = fork(r, mr->xbuf[r]))) return rc;
        }
    }
    for (int r = 0; r <= top; ++r)
        if (mr->bank[r] && (!grouped[r] || r == g0)) HIPCHK(hipStreamWaitEvent(st, mr->ldone[r], 0));
    MrChain ch;
    std::memset(&ch, 0, sizeof ch);
    for (int r = 0; r <= top; ++r) {
        ch.z[r] = mr->bank[r] ? mr->z[r] : nullptr;
        ch.ld_z[r] = mr->B >> r;
        ch.zrow[r] = mr->zrow[r];
        if (r >= 1) {
            ch.whist[r] = mr->wh[c][r];
            ch.whist_new[r] = mr->wh[c ^ 1][r];
        }
    }
    if (mx) {
        HIPCHK(launch_mr_chain(ch, top, mr->hh, mr->g, mr->lg, np, mr->T, mr->keys, mr->B, nullptr, 0, st));
        HIPCHK(launch_finalize_keys(mr->keys, mr_key_chunks(mr->T), mr->B, np, mx, am, st));
    } else {
        if (!out0) return fail(SPIIR_EINVAL, "multi-rate piece without an output");
        HIPCHK(launch_mr_chain(ch, top, mr->hh, mr->g, mr->lg, np, mr->T, nullptr, 0, out0, ld0, st));
    }
    mr->cur ^= 1;
    return SPIIR_OK;
}

bool mr_timing_on(const spiir_multirate *mr) {
    for (auto *bk : mr->bank)
        if (bk && bank_timing_on(bk)) return true;
    return false;
}

// Captures a trigger piece of B samples for each history parity. The host-side
// parity flags (mr->cur and every level bank's history index) toggle once per
// captured piece, so after the two captures they are back where they were;
// on failure they are restored and graphs stay off.
int mr_build_graphs(spiir_multirate *mr) {
    std::vector<int> hc;
    for (auto *bk : mr->bank) hc.push_back(bk ? bank_hist_cur(bk) : 0);
    const int cur0 = mr->cur;
    auto restore = [&]() {
        mr->cur = cur0;
        for (size_t r = 0; r < mr->bank.size(); ++r)
            if (mr->bank[r]) bank_set_hist_cur(mr->bank[r], hc[r]);
        mr_free_graphs(mr);
        mr->graph_failed = true;
    };
    hipError_t e = hipSuccess;
    if (!mr->cap) e = hipStreamCreateWithFlags(&mr->cap, hipStreamNonBlocking);
    if (e == hipSuccess && !mr->xin) e = dalloc(&mr->xin, (size_t)mr->B);
    if (e == hipSuccess && !mr->mxo) e = dalloc(&mr->mxo, (size_t)mr->B);
    if (e == hipSuccess && !mr->amo) e = dalloc(&mr->amo, (size_t)mr->B);
    if (e != hipSuccess) {
        restore();
        return fail(SPIIR_EHIP, "graph set-up: %s", hipGetErrorString(e));
    }
    for (int k = 0; k < 2; ++k) {
        const int parity = mr->cur;
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(mr->cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            restore();
            return fail(SPIIR_EHIP, "graph capture: %s", hipGetErrorString(e));
        }
        const int rc = mr_piece(mr, mr->xin, mr->B, nullptr, 0, mr->mxo, mr->amo, mr->cap);
        e = hipStreamEndCapture(mr->cap, &g);
        if (rc == SPIIR_OK && e == hipSuccess) e = hipGraphInstantiate(&mr->gexec[parity], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (rc || e != hipSuccess) {
            restore();
            return rc ? rc : fail(SPIIR_EHIP, "graph capture: %s", hipGetErrorString(e));
        }
    }
    return SPIIR_OK;
}

// One pass of the multi-rate bank over x[0..n), written as the full-rate z
// (zout, row stride ldz) or as max / argmax.
int mr_run(spiir_multirate *mr, const float *x, int64_t n, float2 *zout, int64_t ldz, float *mx, int32_t *am,
           hipStream_t st) {
    DeviceGuard guard(mr->device);
    for (int64_t P = 0; P < n; P += mr->B) {
        const int64_t np = std::min<int64_t>(mr->B, n - P);
        const bool graph = mx && np == mr->B && mr->use_graph && !mr->graph_failed && mr->eager_pieces > 0 &&
                           !mr_timing_on(mr);
        if (graph && !mr->gexec[mr->cur]) {
            const int rc = mr_build_graphs(mr);
            if (rc) return rc;
        }
        if (graph) {
            HIPCHK(hipMemcpyAsync(mr->xin, x + P, (size_t)np * sizeof(float), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipGraphLaunch(mr->gexec[mr->cur], st));
            HIPCHK(launch_mr_copy_out(mx + P, mr->mxo, am + P, mr->amo, np, st));
            mr->cur ^= 1;
            for (auto *bk : mr->bank)
                if (bk) bank_set_hist_cur(bk, bank_hist_cur(bk) ^ 1);   // as the captured stream calls did
            continue;
        }
        const int rc = mr_piece(mr, x + P, np, zout ? zout + P : nullptr, ldz, mx ? mx + P : nullptr,
                                am ? am + P : nullptr, st);
        if (rc) return rc;
        ++mr->eager_pieces;
    }
    return SPIIR_OK;
}

}  // namespace

extern "C" {

int spiir_multirate_create(spiir_multirate **out, int32_t n_levels, int32_t n_templates,
                           const int64_t *const *filter_offsets, const double *const *a, const double *const *b,
                           const int32_t *const *d, const double *decim_taps, int32_t n_decim_taps,
                           const double *interp_taps, int32_t n_interp_taps, const spiir_bank_opts *opts) {
    if (!out) return fail(SPIIR_EINVAL, "out is null");
    *out = nullptr;
    if (n_levels < 1 || n_levels > 8) return fail(SPIIR_EINVAL, "n_levels must be 1..8 (got %d)", n_levels);
    const int T = n_templates;
    if (T < 1) return fail(SPIIR_EINVAL, "n_templates must be >= 1 (got %d)", T);
    if (!filter_offsets || !a || !b || !d) return fail(SPIIR_EINVAL, "null per-level array");
    if (!decim_taps || !interp_taps) return fail(SPIIR_EINVAL, "null taps");
    if (n_decim_taps < 1 || n_decim_taps > 64 || n_interp_taps < 1 || n_interp_taps > 64)
        return fail(SPIIR_EINVAL, "taps: counts must be 1..64 (got %d, %d)", n_decim_taps, n_interp_taps);
    for (int i = 0; i < n_decim_taps; ++i)
        if (!std::isfinite(decim_taps[i])) return fail(SPIIR_EINVAL, "non-finite decimation tap");
    for (int i = 0; i < n_interp_taps; ++i)
        if (!std::isfinite(interp_taps[i])) return fail(SPIIR_EINVAL, "non-finite interpolation tap");
    const int R = n_levels - 1;
    int top = -1;
    for (int r = 0; r <= R; ++r) {
        const int64_t *off = filter_offsets[r];
        if (!off) return fail(SPIIR_EINVAL, "level %d: null filter_offsets", r);
        if (off[0] != 0) return fail(SPIIR_EINVAL, "level %d: filter_offsets[0] must be 0", r);
        for (int j = 0; j < T; ++j)
            if (off[j + 1] < off[j]) return fail(SPIIR_EINVAL, "level %d: filter_offsets decrease at %d", r, j);
        if (off[T] > 0) {
            if (!a[r] || !b[r] || !d[r]) return fail(SPIIR_EINVAL, "level %d: null coefficient / delay array", r);
            top = r;
        }
    }
    if (top < 0) return fail(SPIIR_EINVAL, "no level holds a filter");
    spiir_bank_opts o;
    spiir_bank_opts_default(&o);
    if (opts) o = *opts;
    if (o.max_block < 0) return fail(SPIIR_EINVAL, "max_block must be >= 0");
    int64_t B = o.max_block ? o.max_block : 16384;
    B = std::max<int64_t>((B >> R) << R, (int64_t)1 << R);
    // the interpolation launch: ceil(B / 512) x ceil(T / 16) workgroups of 1,024 threads
    if (((B + 511) / 512) * (((int64_t)T + 15) / 16) * 1024 > (int64_t)UINT32_MAX)
        return fail(SPIIR_EINVAL, "n_templates x max_block too large (%d x %lld)", T, (long long)B);
    int dev = o.device;
    if (dev < 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(SPIIR_ENODEV, "no HIP device available");
        HIPCHK(hipGetDevice(&dev));
    }
    DeviceFacts df;
    int rc = device_facts(dev, df);
    if (rc) return rc;
    DeviceGuard guard(dev);

    spiir_multirate *mr = new (std::nothrow) spiir_multirate();
    if (!mr) return fail(SPIIR_ENOMEM, "out of host memory");
    mr->device = dev;
    mr->T = T;
    mr->R = R;
    mr->top = top;
    mr->lh = n_decim_taps;
    mr->lg = n_interp_taps;
    mr->hh = n_interp_taps / 2;
    mr->B = B;
    mr->pyramid = mr_pyramid_lds(B, top, n_decim_taps) <= 64 * 1024;
    mr->bank.assign(R + 1, nullptr);
    mr->zrow.assign(R + 1, nullptr);
    mr->xbuf.assign(R + 1, nullptr);
    mr->z.assign(R + 1, nullptr);
    for (int c = 0; c < 2; ++c) {
        mr->dh[c].assign(R + 1, nullptr);
        mr->wh[c].assign(R + 1, nullptr);
    }
    auto bail = [&](int code) {
        (void)hipDeviceSynchronize();
        mr_free(mr);
        delete mr;
        return code;
    };
    auto alloc_fail = [&](hipError_t e) {
        const int code = fail(SPIIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
        return bail(code);
    };
    auto hip_fail = [&](hipError_t e, const char *what) {
        const int code = fail(SPIIR_EHIP, "%s: %s", what, hipGetErrorString(e));
        return bail(code);
    };
    std::vector<std::vector<int64_t>> offc(R + 1);
    // a level whose filters leave most of the device idle ("small") is a short
    // serial recursion per call: the automatic time split may cut it into up
    // to 32 segments. Two or more small levels run as one group of launches
    // (below) and keep chunk_len; a small level on its own takes 64-sample
    // chunks so that its segments can be that short. On the 1,024-template
    // chirp bank the group with 256-sample chunks replayed a block in 139 us,
    // with 128 in 143-145 and with 64 in 151 (16-32 segments at most).
    std::vector<bool> small(R + 1, false);
    int n_small = 0;
    for (int r = 0; r <= R; ++r) {
        const int64_t nf = filter_offsets[r][T];
        small[r] = nf > 0 && o.time_split == 0 && nf <= 128 * (int64_t)df.n_cu;
        n_small += small[r] ? 1 : 0;
    }
    const bool group_small = n_small >= 2 && n_small <= kMultiMax;
    auto make_bank = [&](int r, int wpg) -> int {
        spiir_bank_opts orr = o;
        orr.device = dev;
        orr.max_block = (int32_t)std::max<int64_t>(8, B >> r);
        if (wpg > 0) orr.waves_per_group = wpg;
        if (small[r] && !group_small) orr.chunk_len = 64;
        spiir_bank *bk = nullptr;
        const int n_rows = (int32_t)(offc[r].size() - 1);
        const int code = orr.autotune
                             ? spiir_bank_create(&bk, n_rows, offc[r].data(), a[r], b[r], d[r], &orr)
                             : bank_create_capped(&bk, n_rows, offc[r].data(), a[r], b[r], d[r], orr, small[r] ? 32 : 8);
        if (code) {
            g_err = "level " + std::to_string(r) + ": " + g_err;
            return code;
        }
        mr->bank[r] = bk;
        return SPIIR_OK;
    };
    for (int r = 0; r <= R; ++r) {
        const int64_t *off = filter_offsets[r];
        std::vector<int32_t> row(T, -1);
        offc[r].assign(1, 0);
        for (int j = 0; j < T; ++j)
            if (off[j + 1] > off[j]) {
                row[j] = (int32_t)(offc[r].size() - 1);
                offc[r].push_back(off[j + 1]);
            }
        hipError_t e = dalloc(&mr->zrow[r], (size_t)T);
        if (e != hipSuccess) return alloc_fail(e);
        e = hipMemcpy(mr->zrow[r], row.data(), T * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "row map upload");
        if (off[T] == 0) continue;
        if ((rc = make_bank(r, 0))) return bail(rc);
        e = dalloc(&mr->z[r], (size_t)(offc[r].size() - 1) * (size_t)(B >> r));
        if (e != hipSuccess) return alloc_fail(e);
    }
    // the small levels share one launch per time-split pass (one stream, three
    // launches in place of three per level) when their banks agree in
    // workgroup size: with the automatic choice, rebuild the ones below the
    // largest with that size, and with at least 4 waves (one per SIMD). On the
    // 1,024-template chirp bank with 64-sample chunks a replayed block took
    // 152 us with 4-wave workgroups for the group, 156.5 with 2 (the largest
    // automatic size there), 180 with 1 and 172 with 8; with 256-sample chunks
    // 139.0 with 4, 138.6 with 2 and 145 with 8.
    for (int r = 0; r <= R; ++r)
        if (mr->bank[r] && small[r]) mr->multi.push_back(r);
    if (mr->multi.size() < 2 || mr->multi.size() > (size_t)kMultiMax) {
        mr->multi.clear();
    } else if (o.waves_per_group == 0) {
        int wmax = 4;
        for (int r : mr->multi) wmax = std::max(wmax, bank_wpg(mr->bank[r]));
        for (int r : mr->multi)
            if (bank_wpg(mr->bank[r]) != wmax) {
                spiir_bank_destroy(mr->bank[r]);
                mr->bank[r] = nullptr;
                if ((rc = make_bank(r, wmax))) return bail(rc);
            }
    }
    for (int r = 1; r <= top; ++r) {
        hipError_t e = dalloc(&mr->xbuf[r], (size_t)(B >> r));
        for (int c = 0; c < 2 && e == hipSuccess; ++c) {
            e = dalloc(&mr->dh[c][r], (size_t)std::max(1, mr->lh - 1));
            if (e == hipSuccess) e = dalloc(&mr->wh[c][r], (size_t)T * std::max(1, mr->hh));
        }
        if (e != hipSuccess) return alloc_fail(e);
    }
    {
        hipError_t e = dalloc(&mr->keys, (size_t)mr_key_chunks(T) * (size_t)B);
        if (e == hipSuccess) e = dalloc(&mr->h, (size_t)mr->lh);
        if (e == hipSuccess) e = dalloc(&mr->g, (size_t)mr->lg);
        if (e != hipSuccess) return alloc_fail(e);
    }
    mr->lstream.assign(R + 1, nullptr);
    mr->lfork.assign(R + 1, nullptr);
    mr->ldone.assign(R + 1, nullptr);
    {
        hipError_t e = hipSuccess;
        for (int r = 0; r <= R && e == hipSuccess; ++r)
            if (mr->bank[r]) {
                e = hipStreamCreateWithFlags(&mr->lstream[r], hipStreamNonBlocking);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&mr->lfork[r], hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventCreateWithFlags(&mr->ldone[r], hipEventDisableTiming);
            }
        if (e != hipSuccess) return hip_fail(e, "level streams");
    }
    std::vector<float> hf(decim_taps, decim_taps + mr->lh), gf(interp_taps, interp_taps + mr->lg);
    hipError_t e = hipMemcpy(mr->h, hf.data(), hf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(mr->g, gf.data(), gf.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "taps upload");
    rc = mr_clear_history(mr, nullptr);
    if (rc) return bail(rc);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "multi-rate bank set-up");
    *out = mr;
    return SPIIR_OK;
}

int spiir_multirate_destroy(spiir_multirate *mr) {
    if (!mr) return SPIIR_OK;
    {
        DeviceGuard guard(mr->device);
        (void)hipDeviceSynchronize();
        mr_free(mr);
    }
    delete mr;
    return SPIIR_OK;
}

int spiir_multirate_reset(spiir_multirate *mr, void *stream) {
    if (!mr) return fail(SPIIR_EINVAL, "multi-rate bank is null");
    DeviceGuard guard(mr->device);
    for (auto *bk : mr->bank)
        if (bk) {
            const int rc = spiir_bank_reset(bk, stream);
            if (rc) return rc;
            // every piece toggles the object's parity and each level bank's history
            // index together, so they stay equal; the captured graphs rely on it
            bank_set_hist_cur(bk, 0);
        }
    return mr_clear_history(mr, as_stream(stream));   // sets mr->cur = 0
}

static int mr_check_call(const spiir_multirate *mr, const float *x, int64_t n) {
    if (!mr) return fail(SPIIR_EINVAL, "multi-rate bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n % ((int64_t)1 << mr->R))
        return fail(SPIIR_EINVAL, "n (%lld) must be a multiple of 2^%d", (long long)n, mr->R);
    if (n > 0 && !x) return fail(SPIIR_EINVAL, "null device pointer");
    return SPIIR_OK;
}

int spiir_multirate_filter_block_z(spiir_multirate *mr, const float *x, int64_t n, float *z, int64_t ld,
                                   void *stream) {
    int rc = mr_check_call(mr, x, n);
    if (rc || n == 0) return rc;
    if (!z) return fail(SPIIR_EINVAL, "null device pointer");
    if (ld < n) return fail(SPIIR_EINVAL, "ld_z (%lld) < n (%lld)", (long long)ld, (long long)n);
    return mr_run(mr, x, n, reinterpret_cast<float2 *>(z), ld, nullptr, nullptr, as_stream(stream));
}

int spiir_multirate_trigger_max(spiir_multirate *mr, const float *x, int64_t n, float *mx, int32_t *am,
                                void *stream) {
    int rc = mr_check_call(mr, x, n);
    if (rc || n == 0) return rc;
    if (!mx || !am) return fail(SPIIR_EINVAL, "null device pointer");
    return mr_run(mr, x, n, nullptr, 0, mx, am, as_stream(stream));
}

int spiir_multirate_set_graph(spiir_multirate *mr, int32_t enable) {
    if (!mr) return fail(SPIIR_EINVAL, "multi-rate bank is null");
    mr->use_graph = enable != 0;
    return SPIIR_OK;
}

int spiir_multirate_level_bank(spiir_multirate *mr, int32_t level, spiir_bank **bank) {
    if (!mr || !bank) return fail(SPIIR_EINVAL, "null argument");
    if (level < 0 || level > mr->R) return fail(SPIIR_EINVAL, "level %d out of range 0..%d", level, mr->R);
    *bank = mr->bank[level];
    return SPIIR_OK;
}

}  // extern "C"
