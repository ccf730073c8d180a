// Host side of libspiir's filter banks: device buffers and upload of the
// bank plan (argument checks, slot layout, LDS geometry and FP64
// precomputation come from layout.cpp), launches, streaming state, the
// adjoint tape, batches in a HIP graph and the autotuner; also the shared
// error and device helpers of host_common.h. The multi-rate bank, the whitener and the clustering objects
// have their own host sources. Declared in include/spiir.h.
#include "host_common.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace spiir;
using namespace spiir::host;

namespace spiir {
namespace host {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int device_facts(int dev, DeviceFacts &f) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(SPIIR_ENODEV, "no HIP device available");
    if (dev < 0 || dev >= count) return fail(SPIIR_ENODEV, "device %d out of range (%d devices)", dev, count);
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(SPIIR_ENODEV, "device %d is %s; this library is built for gfx950 only", dev,
                    prop.gcnArchName);
    f.n_cu = prop.multiProcessorCount;
    f.lds_cap = prop.sharedMemPerBlock;
    return SPIIR_OK;
}

}  // namespace host
}  // namespace spiir

namespace {

using layout::Layout;
using layout::Plan;
using layout::Geometry;
using layout::plan_rows;
using layout::auto_wpg;
using layout::choose_fl;
using layout::plan_geometry;
using layout::fwd_lds_bytes;

static_assert(sizeof(layout::F2) == sizeof(float2) && sizeof(layout::D2) == sizeof(double2) &&
                  sizeof(RowInfo) == 16,
              "host slot arrays must match the device vector types");

int build_layout(int T, const int64_t *off, const int32_t *d, int fl, int wpg, int band, Layout &lay) {
    std::string err;
    const int rc = layout::build_layout(T, off, d, fl, wpg, band, lay, err);
    return rc ? fail(rc, "%s", err.c_str()) : SPIIR_OK;
}

int check_bank_args(int32_t T, const int64_t *off, const double *a, const double *b, const int32_t *d,
                    const spiir_bank_opts &o, int &dmax_out) {
    std::string err;
    const int rc = layout::check_bank_args(T, off, a, b, d, o, dmax_out, err);
    return rc ? fail(rc, "%s", err.c_str()) : SPIIR_OK;
}

}  // namespace

struct spiir_bank {
    int device = 0;
    int T = 0;
    int64_t F = 0;
    int dmax = 0, L = 256, prec = 0, max_block = 16384;
    DeviceFacts dev;
    std::vector<int64_t> off;
    std::vector<double> a, b;
    std::vector<int32_t> d;
    Layout lay;
    int nb = 0;
    bool xlds = true;
    size_t lds = 0;
    uint64_t coeff_version = 1;
    // device buffers
    float2 *a32 = nullptr, *b32 = nullptr;
    int32_t *xoff = nullptr, *flags = nullptr, *slot_filter = nullptr, *filter_slot = nullptr;
    int4 *bwaves = nullptr;       // backward waves: (template, first filter, end filter, 0)
    int n_bwaves = 0;
    double2 *aL = nullptr, *dL = nullptr, *a64 = nullptr;
    float4 *state = nullptr, *zstate = nullptr;
    RowInfo *rows = nullptr;
    int tt = 16;
    float *hist[2] = {nullptr, nullptr};
    int hist_cur = 0;
    uint64_t *keys = nullptr;     // [groups + (split templates ? 1 : 0)][max_block]
    float *xwin = nullptr;
    int64_t xwin_cap = 0;
    // templates split over workgroups (layout parts): partial sums [n_parts][max_block],
    // the split templates and their part ranges on the device
    float2 *zpart = nullptr;
    int32_t *split_tpl = nullptr, *split_off = nullptr;
    int n_split = 0;
    int band = 0;                  // delay band width (0: none); group_lo [groups] on the device
    int32_t *group_lo = nullptr;
    int nseg = 1;                 // time segments per streaming launch
    int64_t seg_len_max = 0;
    size_t lds_carry = 0;
    float4 *seg_end = nullptr, *seg_start = nullptr;
    float2 *zl = nullptr;
    // per-template comparator: segment states [pl_cap][one workgroup's slots], local z [pl_cap - 1][T][L]
    float4 *pl_seg_end = nullptr, *pl_seg_start = nullptr;
    float2 *pl_zl = nullptr;
    int pl_cap = 0;
    int tsplit_opt = 0;           // opts.time_split as given (the adjoint honours it too)
    // adjoint scratch, grown on demand: (lambda, nu) pairs [2][cap][S], gpart [cap][2][S]
    int bwd_cap = 0;
    float4 *bpair = nullptr;
    double2 *bgpart = nullptr;
    // optional kernel timing ring (spiir_bank_time_kernels)
    std::vector<hipEvent_t> tev0, tev1;
    std::vector<char> tpend;
    int tidx = 0;
    double tms = 0.0;
    int64_t tn = 0;

    SlotArrays slots() const { return SlotArrays{a32, b32, xoff, aL, dL, a64, flags}; }

    FwdArgs base_args() const {
        FwdArgs p;
        std::memset(&p, 0, sizeof p);
        p.s = slots();
        p.dmax = dmax;
        p.L = L;
        p.nb = nb;
        p.prec = prec;
        p.wpg = lay.wpg;
        p.only_tpl = -1;
        p.gbase = 0;
        p.rows = rows;
        p.nslots = lay.nslots;
        p.groups = lay.groups;
        p.n_templates = T;
        p.seg_end = seg_end;
        p.seg_start = seg_start;
        p.seg_slot0 = 0;
        p.seg_stride = lay.nslots;
        p.zpart = zpart;
        p.ld_part = max_block;
        p.band_w = band ? band - 1 : dmax;
        p.group_lo = band ? group_lo : nullptr;
        p.zl = zl;
        return p;
    }
};

// What the adjoint needs from a forward_z call: the strain window of the call
// (the backward reads x[m - d] for every filter) and the coefficient version
// the forward ran with. No filter state is kept: the a-gradient is formed from
// a second reverse recursion instead of the forward outputs.
struct spiir_tape {
    spiir_bank *bank = nullptr;
    uint64_t coeff_version = 0;
    int64_t n = 0;
    float *xwin = nullptr;
};

struct spiir_batch {
    int device = 0;
    int ns = 0, B = 0, fl = 1, tt = 16, wpg = 1, grid = 0, nitems = 0;
    size_t lds = 0;
    std::vector<spiir_bank *> banks;
    std::vector<int64_t> len;
    BatchStream *streams = nullptr;
    int2 *items = nullptr;
    int *counter = nullptr;
    int64_t *pos = nullptr;
    uint64_t *keys = nullptr;
    int64_t key_stride = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // time-split graph for steps where the live streams alone cannot fill the device
    // sgraph[k - 1]: the k longest streams live (streams end in order of length)
    std::vector<hipGraph_t> sgraph;
    std::vector<hipGraphExec_t> sexec;
    int2 *seg_items = nullptr, *carry_items = nullptr;
    std::vector<float4 *> seg_bufs;
    std::vector<float2 *> zl_bufs;
    std::vector<int> groups;
    int64_t slots_dev = 0;   // resident workgroups on the device
    int split_mode = 0;      // 0 auto, 1 never, 2 always
    int64_t host_step = 0;   // replays since creation / reset
};

namespace {

// Slot arrays on the host, then uploaded.
int upload_coeffs(spiir_bank *bk) {
    const int64_t S = bk->lay.nslots;
    layout::SlotHost h;
    layout::slot_arrays(bk->lay, bk->a.data(), bk->b.data(), bk->d.data(), bk->dmax, bk->L, h);
    HIPCHK(hipMemcpy(bk->a32, h.a32.data(), S * sizeof(float2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->b32, h.b32.data(), S * sizeof(float2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->xoff, h.xoff.data(), S * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->flags, h.flags.data(), S * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->aL, h.aL.data(), S * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->dL, h.dL.data(), S * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->a64, h.a64.data(), S * sizeof(double2), hipMemcpyHostToDevice));
    return SPIIR_OK;
}

constexpr int kTimerRing = 256;

hipError_t timer_collect(spiir_bank *bk, int i) {
    if (!bk->tpend[i]) return hipSuccess;
    hipError_t e = hipEventSynchronize(bk->tev1[i]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, bk->tev0[i], bk->tev1[i]);
    if (e != hipSuccess) return e;
    bk->tpend[i] = 0;
    bk->tms += ms;
    bk->tn += 1;
    return hipSuccess;
}

// Events for the next forward launch (none while timing is off).
hipError_t timer_next(spiir_bank *bk, KernelEvents *ev) {
    *ev = KernelEvents();
    if (bk->tev0.empty()) return hipSuccess;
    const int i = bk->tidx;
    hipError_t e = timer_collect(bk, i);
    if (e != hipSuccess) return e;
    ev->start = bk->tev0[i];
    ev->stop = bk->tev1[i];
    bk->tpend[i] = 1;
    bk->tidx = (i + 1) % kTimerRing;
    return hipSuccess;
}

void timer_free(spiir_bank *bk) {
    for (auto e : bk->tev0) (void)hipEventDestroy(e);
    for (auto e : bk->tev1) (void)hipEventDestroy(e);
    bk->tev0.clear();
    bk->tev1.clear();
    bk->tpend.clear();
    bk->tidx = 0;
}

void free_bank_buffers(spiir_bank *bk) {
    timer_free(bk);
    dfree(bk->a32); dfree(bk->b32); dfree(bk->xoff); dfree(bk->flags); dfree(bk->slot_filter);
    dfree(bk->filter_slot); dfree(bk->bwaves);
    dfree(bk->aL); dfree(bk->dL); dfree(bk->a64); dfree(bk->state); dfree(bk->zstate);
    dfree(bk->rows); dfree(bk->hist[0]); dfree(bk->hist[1]); dfree(bk->keys); dfree(bk->xwin);
    dfree(bk->zpart); dfree(bk->split_tpl); dfree(bk->split_off); dfree(bk->group_lo);
    dfree(bk->bpair); dfree(bk->bgpart); dfree(bk->seg_end); dfree(bk->seg_start); dfree(bk->zl);
    dfree(bk->pl_seg_end); dfree(bk->pl_seg_start); dfree(bk->pl_zl);
    bk->pl_cap = 0;
}

// Working memory of the allocation-free trigger call (spiir_trigger_max_noalloc):
// one array per device, held until the process ends. Host code never passes
// the array's name to a kernel (on the host it is only a stand-in): its device
// address is looked up once per device with that device current and kept.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kScratchDevices] = {};

// Device address of this device's scratch array; the device must be current.
int scratch_setup(int dev, unsigned char **out) {
    *out = nullptr;
    if (dev < 0 || dev >= kScratchDevices)
        return fail(SPIIR_ENODEV, "device %d: no allocation-free scratch slot (ordinals below %d)", dev,
                    kScratchDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(SPIIR_EHIP, "scratch symbol address on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return SPIIR_OK;
}

// seg_cap: most time segments the automatic time split may choose (8 for
// banks created through the ABI; the multi-rate object allows more for its
// small levels, whose calls are short serial recursions).
int create_bank(spiir_bank **out, int32_t T, const int64_t *off, const double *a, const double *b,
                const int32_t *d, const spiir_bank_opts &o, int seg_cap = 8) {
    int dmax = 0;
    int rc = check_bank_args(T, off, a, b, d, o, dmax);
    if (rc) return rc;
    int dev = o.device;
    if (dev < 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
            return fail(SPIIR_ENODEV, "no HIP device available");
        HIPCHK(hipGetDevice(&dev));
    }
    DeviceFacts df;
    rc = device_facts(dev, df);
    if (rc) return rc;
    DeviceGuard guard(dev);
    unsigned char *scr = nullptr;
    rc = scratch_setup(dev, &scr);
    if (rc) return rc;

    const int L = o.chunk_len ? o.chunk_len : 256;
    int max_block = o.max_block ? o.max_block : 16384;
    max_block = std::max(L, (max_block / L) * L);
    // Delay bands (an option): every workgroup takes filters of one band of delays and stages
    // only that band's window in LDS. Not chosen automatically: on the chirp-fit bank (delays
    // up to 65,535) the best banded layout only matched the strain window in global memory.
    const bool global_window = !plan_geometry(1, dmax, L, max_block, df.lds_cap).xlds;
    int band = 0;
    if (o.delay_band > 0) {
        band = o.delay_band;
        if (!plan_geometry(1, band - 1, L, max_block, df.lds_cap).xlds)
            return fail(SPIIR_EINVAL, "delay_band %d: its strain window does not fit LDS", band);
    }
    const int win_delay = band ? band - 1 : dmax;   // delays one workgroup's window covers
    // a banded window is refilled every band samples (at most), so that several workgroups
    // share a compute unit
    const int nb_cap = band ? std::max(L, std::min(max_block, (band + L - 1) / L * L)) : max_block;
    // A bank of more than 128 filters per compute unit that cannot fill the device with
    // the lane count the wave-count rule below picks (fewer than 7 waves per CU) is cut
    // into time segments anyway. With long pieces the cost per update then matters more
    // than the wave count: 4 filters per lane, 8-wave workgroups (two waves per SIMD,
    // several templates per workgroup) and up to 16 segments. On the 64 x 1,000-filter
    // precision bank this ran at 2.29e12 updates/s against 1.39e12 for the wave-count
    // rule's 2 filters per lane, one template per workgroup and 8 segments.
    bool seg_layout = false;
    if (!global_window && !band && o.filters_per_lane == 0 && o.waves_per_group == 0 && o.time_split == 0 &&
        max_block >= 8192 && off[T] > 128 * (int64_t)df.n_cu) {
        const Plan p4 = plan_rows(T, off, 4);
        const Plan pw = plan_rows(T, off, choose_fl(T, off, df.n_cu));
        seg_layout = p4.max_nr <= 4 * kMaxWaves && (pw.total_rows + 3) / 4 < (int64_t)7 * df.n_cu;
    }
    if (seg_layout) seg_cap = std::max(seg_cap, 16);
    int fl = o.filters_per_lane;
    if (fl == 0 && seg_layout) fl = 4;
    if (fl == 0) {
        // With the strain in global memory four filters per lane give each wave more
        // independent loads in flight, and the time split supplies the parallelism a small
        // bank lacks.
        fl = choose_fl(T, off, df.n_cu);
        if (global_window && !band && plan_rows(T, off, 4).max_nr <= 4 * kMaxWaves) fl = 4;
    }
    const Plan plan = plan_rows(T, off, fl);
    int wpg = o.waves_per_group;
    if (wpg == 0 && seg_layout) wpg = kMaxWaves;
    if (wpg == 0) {
        // smallest workgroup that packs the bank into one round of resident workgroups (a
        // template longer than the largest workgroup is split into parts)
        const int w0 = auto_wpg(plan.total_rows, std::min(plan.max_nr, 4 * kMaxWaves), df.n_cu);
        wpg = w0;
        for (int w = w0; w <= kMaxWaves; ++w) {
            const Geometry gm = plan_geometry(w, win_delay, L, nb_cap, df.lds_cap);
            const int occ = std::max(1, forward_occupancy(fl, gm.tt, w, gm.lds));
            Layout trial;
            if (build_layout(T, off, d, fl, w, band, trial)) continue;
            wpg = w;
            if (trial.groups <= (int64_t)df.n_cu * occ) break;
        }
    }

    spiir_bank *bk = new (std::nothrow) spiir_bank();
    if (!bk) return fail(SPIIR_ENOMEM, "out of host memory");
    bk->device = dev;
    bk->T = T;
    bk->F = off[T];
    bk->dmax = dmax;
    bk->L = L;
    bk->prec = o.precision;
    bk->max_block = max_block;
    bk->dev = df;
    bk->off.assign(off, off + T + 1);
    bk->a.assign(a, a + 2 * bk->F);
    bk->b.assign(b, b + 2 * bk->F);
    bk->d.assign(d, d + bk->F);
    rc = build_layout(T, off, d, fl, wpg, band, bk->lay);
    if (rc) {
        delete bk;
        return rc;
    }
    bk->band = band;
    const Geometry gm = plan_geometry(wpg, win_delay, L, nb_cap, df.lds_cap);
    if (L % gm.tt) {   // chunk ends are detected at tile ends only
        delete bk;
        return fail(SPIIR_EINVAL, "internal: tile length %d does not divide chunk_len %d", gm.tt, L);
    }
    bk->tt = gm.tt;
    bk->xlds = gm.xlds;
    bk->nb = gm.nb;
    bk->lds = gm.lds;
    bk->lds_carry = fwd_lds_bytes(wpg, 0, 0, false, gm.tt);
    bk->tsplit_opt = o.time_split;
    // time split: only when the bank's workgroups fill at most half the device
    if (o.time_split != 1) {
        if (o.time_split >= 2) {
            bk->nseg = o.time_split;
        } else {
            const int occ = std::max(1, forward_occupancy(fl, gm.tt, wpg, gm.lds));
            const int64_t slots_dev = (int64_t)df.n_cu * occ;
            // segments oversubscribe the resident workgroup slots twice: on the
            // 64 x 1,000-filter precision bank (64 groups, one resident per CU)
            // 8 segments ran 23% faster than 4, and 16 or 32 no faster than 8
            if (2 * (int64_t)bk->lay.groups <= slots_dev)
                bk->nseg = (int)std::min<int64_t>(seg_cap, 2 * slots_dev / std::max(1, bk->lay.groups));
        }
        bk->nseg = std::min(bk->nseg, std::max(1, max_block / L));
    }
    if (bk->nseg > 1) bk->seg_len_max = ((max_block + bk->nseg - 1) / bk->nseg + L - 1) / L * L;

    const int64_t S = bk->lay.nslots;
    const int G = bk->lay.groups;
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    A(dalloc(&bk->a32, S)); A(dalloc(&bk->b32, S)); A(dalloc(&bk->xoff, S)); A(dalloc(&bk->flags, S));
    A(dalloc(&bk->slot_filter, S)); A(dalloc(&bk->filter_slot, (size_t)bk->F)); A(dalloc(&bk->aL, S)); A(dalloc(&bk->dL, S)); A(dalloc(&bk->a64, S));
    A(dalloc(&bk->state, S)); A(dalloc(&bk->zstate, S)); A(dalloc(&bk->rows, (size_t)G * wpg * 4));
    A(dalloc(&bk->hist[0], (size_t)dmax)); A(dalloc(&bk->hist[1], (size_t)dmax));
    bk->n_split = (int)bk->lay.split_tpl.size();
    A(dalloc(&bk->keys, (size_t)(G + (bk->n_split ? 1 : 0)) * max_block));
    if (bk->band) A(dalloc(&bk->group_lo, (size_t)G));
    if (bk->n_split) {
        A(dalloc(&bk->zpart, (size_t)bk->lay.n_parts * max_block));
        A(dalloc(&bk->split_tpl, bk->lay.split_tpl.size()));
        A(dalloc(&bk->split_off, bk->lay.split_off.size()));
    }
    if (bk->nseg > 1) {
        A(dalloc(&bk->seg_end, (size_t)bk->nseg * S));
        A(dalloc(&bk->seg_start, (size_t)bk->nseg * S));
        A(dalloc(&bk->zl, (size_t)(bk->nseg - 1) * T * bk->seg_len_max));
    }
    if (e != hipSuccess) {
        free_bank_buffers(bk);
        delete bk;
        return fail(SPIIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    rc = upload_coeffs(bk);
    if (!rc) {
        e = hipMemcpy(bk->slot_filter, bk->lay.slot_filter.data(), S * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            std::vector<int32_t> fs((size_t)bk->F, -1);
            for (int64_t sl = 0; sl < S; ++sl)
                if (bk->lay.slot_filter[(size_t)sl] >= 0) fs[(size_t)bk->lay.slot_filter[(size_t)sl]] = (int32_t)sl;
            e = hipMemcpy(bk->filter_slot, fs.data(), fs.size() * sizeof(int32_t), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) {
            // backward waves: each template's filters in runs of at most 64
            std::vector<int4> bw;
            for (int j = 0; j < T; ++j)
                for (int64_t k0 = off[j]; k0 < off[j + 1]; k0 += 64)
                    bw.push_back(make_int4(j, (int)k0, (int)std::min<int64_t>(off[j + 1], k0 + 64), 0));
            bk->n_bwaves = (int)bw.size();
            e = dalloc(&bk->bwaves, bw.size());
            if (e == hipSuccess)
                e = hipMemcpy(bk->bwaves, bw.data(), bw.size() * sizeof(int4), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess)
            e = hipMemcpy(bk->rows, bk->lay.rows.data(), bk->lay.rows.size() * sizeof(RowInfo),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(bk->state, 0, S * sizeof(float4));
        if (e == hipSuccess && bk->band)
            e = hipMemcpy(bk->group_lo, bk->lay.group_lo.data(), (size_t)G * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e == hipSuccess && bk->n_split)
            e = hipMemcpy(bk->split_tpl, bk->lay.split_tpl.data(), bk->lay.split_tpl.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess && bk->n_split)
            e = hipMemcpy(bk->split_off, bk->lay.split_off.data(), bk->lay.split_off.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess && bk->nseg > 1) e = hipMemset(bk->seg_end, 0, (size_t)bk->nseg * S * sizeof(float4));
        if (e == hipSuccess && bk->nseg > 1) e = hipMemset(bk->seg_start, 0, (size_t)bk->nseg * S * sizeof(float4));
        if (e == hipSuccess && dmax > 0) e = hipMemset(bk->hist[0], 0, (size_t)dmax * sizeof(float));
        if (e == hipSuccess && dmax > 0) e = hipMemset(bk->hist[1], 0, (size_t)dmax * sizeof(float));
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) rc = fail(SPIIR_EHIP, "bank upload: %s", hipGetErrorString(e));
    }
    if (rc) {
        free_bank_buffers(bk);
        delete bk;
        return rc;
    }
    *out = bk;
    return SPIIR_OK;
}


int ensure_xwin(spiir_bank *bk, int64_t need) {
    if (need <= bk->xwin_cap) return SPIIR_OK;
    HIPCHK(hipDeviceSynchronize());
    dfree(bk->xwin);
    bk->xwin_cap = 0;
    HIPCHK(dalloc(&bk->xwin, (size_t)need + 16));  // one tile of read-ahead padding
    bk->xwin_cap = need;
    return SPIIR_OK;
}

// Working buffers of one streaming call besides the bank's state and history:
// per-workgroup partial keys [groups][keys_ld], the time split's segment
// states and local z, and the strain window when it is not staged in LDS.
struct CallScratch {
    uint64_t *keys = nullptr;
    int64_t keys_ld = 0;
    int nseg = 0;   // time segments per launch for this call (0: the bank's)
    float4 *seg_end = nullptr, *seg_start = nullptr;
    float2 *zl = nullptr;
    float *xwin = nullptr;
};

// Shared driver of the streaming calls (snr rows or fused keys). cs = null:
// the bank's own buffers (the global strain window grown on demand).
int stream_call(spiir_bank *bk, const float *x, int64_t n, int mode, float *snr, int64_t ld,
                float *mx, int32_t *am, hipStream_t st, const CallScratch *cs = nullptr) {
    DeviceGuard guard(bk->device);
    const float *hist = bk->hist[bk->hist_cur];
    float *xwin = bk->xwin;
    if (!bk->xlds) {
        if (cs) {
            xwin = cs->xwin;
        } else {
            int rc = ensure_xwin(bk, n + bk->dmax);
            if (rc) return rc;
            xwin = bk->xwin;
        }
        HIPCHK(launch_window_fill(xwin, hist, x, n, bk->dmax, st));
    }
    uint64_t *keys = cs ? cs->keys : bk->keys;
    const int64_t keys_ld = cs ? cs->keys_ld : bk->max_block;
    bool hist_done = false;
    for (int64_t P = 0; P < n; P += bk->max_block) {
        const int64_t np = std::min<int64_t>(bk->max_block, n - P);
        FwdArgs a = bk->base_args();
        if (cs) {
            a.seg_end = cs->seg_end;
            a.seg_start = cs->seg_start;
            a.zl = cs->zl;
        }
        a.state = bk->state;
        a.x = x;
        a.hist = hist;
        a.xwin = xwin;
        a.xbase = P;
        a.n = np;
        a.obase = P;
        if (mode == kModeSnr) {
            a.snr = snr;
            a.ld = ld;
        } else if (mode == kModeZ) {
            a.z = reinterpret_cast<float2 *>(snr);
            a.ld = ld;
        } else {
            a.keys = keys;
            a.ld = keys_ld;
        }
        int nseg = 1;
        const int bn = (cs && cs->nseg > 0) ? cs->nseg : bk->nseg;
        if (bn > 1) {
            a.seg_len = ((np + bn - 1) / bn + bk->L - 1) / bk->L * bk->L;
            nseg = (int)((np + a.seg_len - 1) / a.seg_len);
        }
        // the next call's history is written by a launch that follows every
        // strain read of this call or by the last reading launch itself (it
        // goes to the other history buffer): the last key finalisation, else
        // the last piece's carry chain or its one forward launch
        const bool last = P + np >= n;
        const HistCopy hc{hist, bk->hist[bk->hist_cur ^ 1], x, n, bk->dmax};
        if (last && mode != kModeKeys) {
            a.hist_next = hc;
            hist_done = true;
        }
        KernelEvents ev;
        HIPCHK(timer_next(bk, &ev));
        if (nseg >= 2)
            HIPCHK(launch_forward_split(a, mode, bk->lay.fl, bk->tt, bk->xlds, nseg, bk->lds, bk->lds_carry,
                                        bk->slot_filter, st, ev));
        else
            HIPCHK(launch_forward(a, mode, bk->lay.fl, bk->tt, bk->xlds, bk->lay.groups, bk->lds, st, ev));
        if (bk->n_split)   // split templates: their parts' sums, then their SNR / z / keys
            HIPCHK(launch_combine_parts(bk->zpart, bk->max_block, bk->split_tpl, bk->split_off, bk->n_split, np,
                                        mode, a.snr, a.z, a.ld, a.obase, keys + (int64_t)bk->lay.groups * keys_ld,
                                        st));
        if (mode == kModeKeys) {
            HIPCHK(launch_finalize_keys(keys, bk->lay.groups + (bk->n_split ? 1 : 0), keys_ld, np, mx + P, am + P,
                                        st, last ? &hc : nullptr));
            hist_done = hist_done || last;
        }
    }
    if (!hist_done) HIPCHK(launch_hist_update(hist, bk->hist[bk->hist_cur ^ 1], x, n, bk->dmax, st));
    bk->hist_cur ^= 1;
    return SPIIR_OK;
}

}  // namespace

namespace spiir {
namespace host {

int bank_stream_z(spiir_bank *bk, const float *x, int64_t n, float *z, int64_t ld, hipStream_t st) {
    return stream_call(bk, x, n, kModeZ, z, ld, nullptr, nullptr, st);
}

int bank_create_capped(spiir_bank **out, int32_t T, const int64_t *off, const double *a, const double *b,
                       const int32_t *d, const spiir_bank_opts &o, int seg_cap) {
    return create_bank(out, T, off, a, b, d, o, seg_cap);
}

int bank_wpg(const spiir_bank *bk) { return bk->lay.wpg; }

bool banks_multi_ok(spiir_bank *const *bks, int nb, const int64_t *n) {
    if (nb < 1 || nb > kMultiMax) return false;
    const spiir_bank *b0 = bks[0];
    for (int b = 0; b < nb; ++b) {
        const spiir_bank *bk = bks[b];
        if (!bk || !bk->xlds || bk->n_split || bk->nseg < 2 || !bk->tev0.empty()) return false;
        if (bk->device != b0->device || bk->lay.fl != b0->lay.fl || bk->tt != b0->tt || bk->lay.wpg != b0->lay.wpg)
            return false;
        if (n[b] <= 0 || n[b] > bk->max_block) return false;
        const int64_t seg_len = ((n[b] + bk->nseg - 1) / bk->nseg + bk->L - 1) / bk->L * bk->L;
        if (n[b] <= seg_len) return false;   // one segment: the call would not be time-split
    }
    return true;
}

int banks_stream_z_multi(spiir_bank *const *bks, int nb, const float *const *x, const int64_t *n, float *const *z,
                         const int64_t *ld, hipStream_t st) {
    if (!banks_multi_ok(bks, nb, n)) return fail(SPIIR_EINVAL, "internal: the banks cannot share time-split launches");
    DeviceGuard guard(bks[0]->device);
    MultiFwd m;
    std::memset(&m, 0, sizeof m);
    m.count = nb;
    size_t lds = 0, lds_carry = 0;
    for (int b = 0; b < nb; ++b) {
        spiir_bank *bk = bks[b];
        const float *hist = bk->hist[bk->hist_cur];
        // the arguments of this bank's streaming z call as one time-split piece
        FwdArgs a = bk->base_args();
        a.state = bk->state;
        a.x = x[b];
        a.hist = hist;
        a.xwin = bk->xwin;
        a.xbase = 0;
        a.n = n[b];
        a.obase = 0;
        a.z = reinterpret_cast<float2 *>(z[b]);
        a.ld = ld[b];
        a.seg_len = ((n[b] + bk->nseg - 1) / bk->nseg + bk->L - 1) / bk->L * bk->L;
        a.hist_next = HistCopy{hist, bk->hist[bk->hist_cur ^ 1], x[b], n[b], bk->dmax};
        const int nseg = (int)((n[b] + a.seg_len - 1) / a.seg_len);
        const int cb = (int)((a.seg_stride + 255) / 256);
        const int hb = bk->dmax > 0 ? (bk->dmax + 255) / 256 : 0;
        m.a[b] = a;
        m.nseg[b] = nseg;
        m.chain_blocks[b] = cb;
        m.seg_first[b + 1] = m.seg_first[b] + bk->lay.groups * nseg;
        m.chain_first[b + 1] = m.chain_first[b] + cb + hb;
        m.carry_first[b + 1] = m.carry_first[b] + bk->lay.groups * (nseg - 1);
        lds = std::max(lds, bk->lds);
        lds_carry = std::max(lds_carry, bk->lds_carry);
    }
    HIPCHK(launch_forward_split_multi(m, bks[0]->lay.fl, bks[0]->tt, bks[0]->lay.wpg, lds, lds_carry, st));
    for (int b = 0; b < nb; ++b) bks[b]->hist_cur ^= 1;
    return SPIIR_OK;
}

int bank_hist_cur(const spiir_bank *bk) { return bk->hist_cur; }
void bank_set_hist_cur(spiir_bank *bk, int v) { bk->hist_cur = v; }
bool bank_timing_on(const spiir_bank *bk) { return !bk->tev0.empty(); }

// gfx950 check of a device, cached per ordinal for the process.
int resolve_device(int32_t device, int &dev) {
    static std::mutex mu;
    static std::map<int, int> checked;
    dev = device;
    if (dev < 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
            return fail(SPIIR_ENODEV, "no HIP device available");
        HIPCHK(hipGetDevice(&dev));
    }
    std::lock_guard<std::mutex> lk(mu);
    auto it = checked.find(dev);
    if (it != checked.end()) return it->second;
    DeviceFacts df;
    const int rc = device_facts(dev, df);
    if (rc != SPIIR_ENODEV) checked[dev] = rc;
    return rc;
}


}  // namespace host
}  // namespace spiir

extern "C" {

void spiir_bank_opts_default(spiir_bank_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->chunk_len = 256;
    o->filters_per_lane = 0;
    o->max_delay = 0;
    o->precision = SPIIR_PREC_HYBRID;
    o->device = -1;
    o->max_block = 16384;
    o->waves_per_group = 0;
    o->autotune = 0;
    o->time_split = 0;
    o->delay_band = 0;
}

int spiir_bank_create(spiir_bank **out, int32_t n_templates, const int64_t *filter_offsets,
                      const double *a, const double *b, const int32_t *d, const spiir_bank_opts *opts) {
    if (!out) return fail(SPIIR_EINVAL, "out is null");
    *out = nullptr;
    spiir_bank_opts o;
    spiir_bank_opts_default(&o);
    if (opts) o = *opts;
    if (o.autotune) {
        int dmax = 0;
        int rc = check_bank_args(n_templates, filter_offsets, a, b, d, o, dmax);
        if (rc) return rc;
        int32_t L = 0, F = 0;
        const int32_t block = o.max_block ? std::min(o.max_block, 4096) : 4096;
        rc = spiir_autotune(1, &n_templates, &filter_offsets, &a, &b, &d, o.max_delay, block, o.device,
                            &L, &F, nullptr);
        if (rc) return rc;
        o.chunk_len = L;
        o.filters_per_lane = F;
        o.autotune = 0;
    }
    return create_bank(out, n_templates, filter_offsets, a, b, d, o);
}

int spiir_bank_destroy(spiir_bank *bk) {
    if (!bk) return SPIIR_OK;
    {
        DeviceGuard guard(bk->device);
        (void)hipDeviceSynchronize();
        free_bank_buffers(bk);
    }
    delete bk;
    return SPIIR_OK;
}

int spiir_bank_time_kernels(spiir_bank *bk, int32_t enable) {
    if (!bk) return fail(SPIIR_EINVAL, "null bank");
    DeviceGuard guard(bk->device);
    if (!bk->tev0.empty()) {
        for (int i = 0; i < kTimerRing; ++i)
            if (bk->tpend[i]) (void)hipEventSynchronize(bk->tev1[i]);
        timer_free(bk);
    }
    bk->tms = 0.0;
    bk->tn = 0;
    if (!enable) return SPIIR_OK;
    bk->tev0.assign(kTimerRing, nullptr);
    bk->tev1.assign(kTimerRing, nullptr);
    bk->tpend.assign(kTimerRing, 0);
    for (int i = 0; i < kTimerRing; ++i) {
        hipError_t e = hipEventCreate(&bk->tev0[i]);
        if (e == hipSuccess) e = hipEventCreate(&bk->tev1[i]);
        if (e != hipSuccess) {
            timer_free(bk);
            return fail(SPIIR_EHIP, "hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    return SPIIR_OK;
}

int spiir_bank_kernel_time(spiir_bank *bk, double *total_ms, int64_t *launches) {
    if (!bk || !total_ms || !launches) return fail(SPIIR_EINVAL, "null argument");
    if (bk->tev0.empty()) return fail(SPIIR_ESTATE, "kernel timing is off (spiir_bank_time_kernels)");
    DeviceGuard guard(bk->device);
    for (int k = 0; k < kTimerRing; ++k) {
        const int i = (bk->tidx + k) % kTimerRing;  // oldest first
        hipError_t e = timer_collect(bk, i);
        if (e != hipSuccess) return fail(SPIIR_EHIP, "kernel timing: %s", hipGetErrorString(e));
    }
    *total_ms = bk->tms;
    *launches = bk->tn;
    bk->tms = 0.0;
    bk->tn = 0;
    return SPIIR_OK;
}

int spiir_bank_get_info(const spiir_bank *bk, spiir_bank_info *info) {
    if (!bk || !info) return fail(SPIIR_EINVAL, "null argument");
    info->n_templates = bk->T;
    info->n_filters = bk->F;
    info->max_delay = bk->dmax;
    info->chunk_len = bk->L;
    info->filters_per_lane = bk->lay.fl;
    info->waves_per_group = bk->lay.wpg;
    info->n_groups = bk->lay.groups;
    info->n_slots = bk->lay.nslots;
    info->lds_bytes = (int32_t)bk->lds;
    info->x_in_lds = bk->xlds ? 1 : 0;
    info->sub_block = bk->nb;
    info->precision = bk->prec;
    info->device = bk->device;
    info->n_cu = bk->dev.n_cu;
    info->time_split = bk->nseg;
    info->n_parts = bk->lay.n_parts;
    info->delay_band = bk->band;
    return SPIIR_OK;
}

int spiir_bank_reset(spiir_bank *bk, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    DeviceGuard guard(bk->device);
    hipStream_t st = as_stream(stream);
    HIPCHK(launch_fill_zero(bk->state, bk->lay.nslots * sizeof(float4), st));
    HIPCHK(launch_fill_zero(bk->hist[0], (size_t)bk->dmax * sizeof(float), st));
    HIPCHK(launch_fill_zero(bk->hist[1], (size_t)bk->dmax * sizeof(float), st));
    return SPIIR_OK;
}

int spiir_bank_set_coeffs(spiir_bank *bk, const double *a, const double *b) {
    if (!bk || !a || !b) return fail(SPIIR_EINVAL, "null argument");
    for (int64_t k = 0; k < bk->F; ++k) {
        const double ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
        if (!std::isfinite(ar) || !std::isfinite(ai) || !std::isfinite(br) || !std::isfinite(bi))
            return fail(SPIIR_EINVAL, "filter %lld has a non-finite coefficient", (long long)k);
        if (std::hypot(ar, ai) >= 1.0)
            return fail(SPIIR_EINVAL, "filter %lld is not stable: |a| >= 1", (long long)k);
    }
    DeviceGuard guard(bk->device);
    HIPCHK(hipDeviceSynchronize());
    std::copy(a, a + 2 * bk->F, bk->a.begin());
    std::copy(b, b + 2 * bk->F, bk->b.begin());
    int rc = upload_coeffs(bk);
    if (rc) return rc;
    ++bk->coeff_version;
    return SPIIR_OK;
}

int spiir_bank_set_coeffs_dev(spiir_bank *bk, const double *a, const double *b, void *stream) {
    if (!bk || !a || !b) return fail(SPIIR_EINVAL, "null argument");
    DeviceGuard guard(bk->device);
    HIPCHK(launch_set_coeffs(a, b, bk->slot_filter, bk->lay.nslots, bk->L, bk->a32, bk->b32, bk->aL, bk->dL,
                             bk->a64, bk->flags, as_stream(stream)));
    ++bk->coeff_version;
    return SPIIR_OK;
}

int spiir_bank_state_size(const spiir_bank *bk, size_t *nbytes) {
    if (!bk || !nbytes) return fail(SPIIR_EINVAL, "null argument");
    *nbytes = 32 + (size_t)bk->F * sizeof(float4) + (size_t)bk->dmax * sizeof(float);
    return SPIIR_OK;
}

// Checkpoint format: magic, version, F, dmax (4 x int64), then per filter in the
// caller's order (hi.re, hi.im, lo.re, lo.im) float32, then the history.
int spiir_bank_get_state(const spiir_bank *bk, void *buf, size_t nbytes) {
    if (!bk || !buf) return fail(SPIIR_EINVAL, "null argument");
    size_t need = 0;
    spiir_bank_state_size(bk, &need);
    if (nbytes < need) return fail(SPIIR_EINVAL, "buffer too small (%zu < %zu)", nbytes, need);
    DeviceGuard guard(bk->device);
    HIPCHK(hipDeviceSynchronize());
    std::vector<float4> st((size_t)bk->lay.nslots);
    HIPCHK(hipMemcpy(st.data(), bk->state, st.size() * sizeof(float4), hipMemcpyDeviceToHost));
    int64_t *h = static_cast<int64_t *>(buf);
    h[0] = 0x52494950535ll;  // "SPIIR"
    h[1] = 1;
    h[2] = bk->F;
    h[3] = bk->dmax;
    float4 *fs = reinterpret_cast<float4 *>(static_cast<char *>(buf) + 32);
    for (int64_t s = 0; s < bk->lay.nslots; ++s) {
        const int32_t k = bk->lay.slot_filter[(size_t)s];
        if (k >= 0) std::memcpy(&fs[k], &st[(size_t)s], sizeof(float4));
    }
    if (bk->dmax > 0)
        HIPCHK(hipMemcpy(static_cast<char *>(buf) + 32 + bk->F * sizeof(float4), bk->hist[bk->hist_cur],
                         (size_t)bk->dmax * sizeof(float), hipMemcpyDeviceToHost));
    return SPIIR_OK;
}

int spiir_bank_set_state(spiir_bank *bk, const void *buf, size_t nbytes) {
    if (!bk || !buf) return fail(SPIIR_EINVAL, "null argument");
    size_t need = 0;
    spiir_bank_state_size(bk, &need);
    if (nbytes < need) return fail(SPIIR_EINVAL, "buffer too small (%zu < %zu)", nbytes, need);
    const int64_t *h = static_cast<const int64_t *>(buf);
    if (h[0] != 0x52494950535ll || h[1] != 1 || h[2] != bk->F || h[3] != bk->dmax)
        return fail(SPIIR_ESTATE, "checkpoint does not belong to a bank of this shape");
    std::vector<float4> st((size_t)bk->lay.nslots, make_float4(0.f, 0.f, 0.f, 0.f));
    const float4 *fs = reinterpret_cast<const float4 *>(static_cast<const char *>(buf) + 32);
    for (int64_t s = 0; s < bk->lay.nslots; ++s) {
        const int32_t k = bk->lay.slot_filter[(size_t)s];
        if (k >= 0) std::memcpy(&st[(size_t)s], &fs[k], sizeof(float4));
    }
    DeviceGuard guard(bk->device);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(bk->state, st.data(), st.size() * sizeof(float4), hipMemcpyHostToDevice));
    if (bk->dmax > 0)
        HIPCHK(hipMemcpy(bk->hist[bk->hist_cur], static_cast<const char *>(buf) + 32 + bk->F * sizeof(float4),
                         (size_t)bk->dmax * sizeof(float), hipMemcpyHostToDevice));
    return SPIIR_OK;
}

int spiir_filter_block(spiir_bank *bk, const float *x, int64_t n, float *snr, int64_t ld, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n == 0) return SPIIR_OK;
    if (!x || !snr) return fail(SPIIR_EINVAL, "null device pointer");
    if (ld < n) return fail(SPIIR_EINVAL, "ld_snr (%lld) < n (%lld)", (long long)ld, (long long)n);
    return stream_call(bk, x, n, kModeSnr, snr, ld, nullptr, nullptr, as_stream(stream));
}

int spiir_filter_block_z(spiir_bank *bk, const float *x, int64_t n, float *z, int64_t ld, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n == 0) return SPIIR_OK;
    if (!x || !z) return fail(SPIIR_EINVAL, "null device pointer");
    if (ld < n) return fail(SPIIR_EINVAL, "ld_z (%lld) < n (%lld)", (long long)ld, (long long)n);
    return stream_call(bk, x, n, kModeZ, z, ld, nullptr, nullptr, as_stream(stream));
}

int spiir_trigger_max(spiir_bank *bk, const float *x, int64_t n, float *mx, int32_t *am, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n == 0) return SPIIR_OK;
    if (!x || !mx || !am) return fail(SPIIR_EINVAL, "null device pointer");
    return stream_call(bk, x, n, kModeKeys, nullptr, 0, mx, am, as_stream(stream));
}

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// The allocation-free call's buffers carved from the device's scratch array
// (scr = null: only the size). Bytes needed, or 0 with an error set.
// Carves the call's buffers out of scr (null: sizes only) for time segments
// of nseg per launch (at most the bank's count).
size_t plan_scratch(const spiir_bank *bk, int64_t n, int nseg, unsigned char *scr, CallScratch &cs) {
    size_t at = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = scr ? scr + at : nullptr;
        at += align256(bytes);
        return p;
    };
    const int64_t keys_ld = std::min<int64_t>(n, bk->max_block);
    cs.keys_ld = keys_ld;
    cs.nseg = nseg;
    cs.keys = reinterpret_cast<uint64_t *>(
        take((size_t)(bk->lay.groups + (bk->n_split ? 1 : 0)) * keys_ld * sizeof(uint64_t)));
    const size_t seg_bytes = (size_t)nseg * bk->lay.nslots * sizeof(float4);
    if (nseg > 1) {
        const int64_t seg_len = ((keys_ld + nseg - 1) / nseg + bk->L - 1) / bk->L * bk->L;
        cs.seg_end = reinterpret_cast<float4 *>(take(seg_bytes));
        cs.seg_start = reinterpret_cast<float4 *>(take(seg_bytes));
        cs.zl = reinterpret_cast<float2 *>(take((size_t)(nseg - 1) * bk->T * seg_len * sizeof(float2)));
    }
    if (!bk->xlds) cs.xwin = reinterpret_cast<float *>(take((size_t)(n + bk->dmax + 16) * sizeof(float)));
    return at;
}

}  // namespace

int spiir_trigger_max_noalloc(spiir_bank *bk, const float *x, int64_t n, float *mx, int32_t *am, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n == 0) return SPIIR_OK;
    if (!x || !mx || !am) return fail(SPIIR_EINVAL, "null device pointer");
    CallScratch cs;
    // the bank's time segments, or as many as the array holds (the per-segment
    // states grow with the segment count)
    int nseg = std::max(1, bk->nseg);
    size_t need = plan_scratch(bk, n, nseg, nullptr, cs);
    while (need > kScratchBytes && nseg > 1) need = plan_scratch(bk, n, --nseg, nullptr, cs);
    if (need > kScratchBytes)
        return fail(SPIIR_EINVAL,
                    "this call needs %zu bytes of working memory, more than the %zu bytes the allocation-free "
                    "call holds per device (fewer samples per call, or spiir_trigger_max)",
                    need, kScratchBytes);
    DeviceGuard guard(bk->device);
    unsigned char *scr = nullptr;
    const int rc = scratch_setup(bk->device, &scr);   // the address looked up when the bank was created
    if (rc) return rc;
    plan_scratch(bk, n, nseg, scr, cs);
    hipStream_t st = as_stream(stream);
    if (nseg > 1) {
        // slots outside every template are chained from these buffers; start them at zero as the bank's own
        const size_t seg_bytes = (size_t)nseg * bk->lay.nslots * sizeof(float4);
        HIPCHK(launch_fill_zero(cs.seg_end, seg_bytes, st));
        HIPCHK(launch_fill_zero(cs.seg_start, seg_bytes, st));
    }
    return stream_call(bk, x, n, kModeKeys, nullptr, 0, mx, am, st, &cs);
}

int spiir_trigger_max_per_template(spiir_bank *bk, const float *x, int64_t n, float *mx, int32_t *am,
                                   float *snr, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n == 0) return SPIIR_OK;
    if (!x || !mx || !am || !snr) return fail(SPIIR_EINVAL, "null device pointer");
    if (bk->n_split)
        return fail(SPIIR_EINVAL, "the per-template comparator needs every template inside one workgroup");
    DeviceGuard guard(bk->device);
    hipStream_t st = as_stream(stream);
    const float *hist = bk->hist[bk->hist_cur];
    // The strain window stays in global memory: a segment workgroup reads only
    // its template's delayed samples for one chunk instead of staging the
    // whole max_delay + chunk window in LDS.
    {
        int rc = ensure_xwin(bk, n + bk->dmax);
        if (rc) return rc;
        HIPCHK(launch_window_fill(bk->xwin, hist, x, n, bk->dmax, st));
    }
    // Each template's launch fills the device by itself: its block is cut into
    // segments of one chunk (L samples), one workgroup per segment, chained in
    // FP64 as in the bank's own time split, over that template's workgroup only.
    const int L = bk->L;
    const int64_t gslots = (int64_t)bk->lay.wpg * bk->lay.fl * 64;   // slots of one workgroup
    const int nseg_max = (int)((std::min<int64_t>(n, bk->max_block) + L - 1) / L);
    if (nseg_max >= 2 && bk->pl_cap < nseg_max) {
        HIPCHK(hipDeviceSynchronize());
        dfree(bk->pl_seg_end);
        dfree(bk->pl_seg_start);
        dfree(bk->pl_zl);
        bk->pl_cap = 0;
        hipError_t e = dalloc(&bk->pl_seg_end, (size_t)nseg_max * gslots);
        if (e == hipSuccess) e = dalloc(&bk->pl_seg_start, (size_t)nseg_max * gslots);
        if (e == hipSuccess) e = dalloc(&bk->pl_zl, (size_t)(nseg_max - 1) * bk->T * L);
        if (e == hipSuccess) e = launch_fill_zero(bk->pl_seg_end, (size_t)nseg_max * gslots * sizeof(float4), st);
        if (e == hipSuccess) e = launch_fill_zero(bk->pl_seg_start, (size_t)nseg_max * gslots * sizeof(float4), st);
        if (e != hipSuccess) {
            dfree(bk->pl_seg_end);
            dfree(bk->pl_seg_start);
            dfree(bk->pl_zl);
            return fail(SPIIR_ENOMEM, "per-template scratch allocation failed: %s", hipGetErrorString(e));
        }
        bk->pl_cap = nseg_max;
    }
    for (int64_t P = 0; P < n; P += bk->max_block) {
        const int64_t np = std::min<int64_t>(bk->max_block, n - P);
        const int nseg = (int)((np + L - 1) / L);
        for (int j = 0; j < bk->T; ++j) {
            FwdArgs a = bk->base_args();
            a.state = bk->state;
            a.x = x;
            a.hist = hist;
            a.xwin = bk->xwin;
            a.xbase = P;
            a.n = np;
            a.obase = P;
            a.snr = snr;
            a.ld = n;
            a.only_tpl = j;
            a.gbase = bk->lay.tpl_group[j];
            a.groups = 1;
            if (nseg >= 2) {
                a.seg_len = L;
                a.seg_end = bk->pl_seg_end;
                a.seg_start = bk->pl_seg_start;
                a.zl = bk->pl_zl;
                a.seg_slot0 = (int64_t)a.gbase * gslots;
                a.seg_stride = gslots;
                HIPCHK(launch_forward_split(a, kModeSnr, bk->lay.fl, bk->tt, false, nseg, bk->lds_carry, bk->lds_carry,
                                            bk->slot_filter, st, KernelEvents()));
            } else {
                HIPCHK(launch_forward(a, kModeSnr, bk->lay.fl, bk->tt, false, 1, bk->lds_carry, st));
            }
        }
    }
    HIPCHK(launch_rows_argmax(snr, bk->T, n, n, mx, am, st));
    HIPCHK(launch_hist_update(hist, bk->hist[bk->hist_cur ^ 1], x, n, bk->dmax, st));
    bk->hist_cur ^= 1;
    return SPIIR_OK;
}

int spiir_forward_z(spiir_bank *bk, const float *x, int64_t n, float *z, spiir_tape **tape_out, void *stream) {
    if (tape_out) *tape_out = nullptr;
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 1) return fail(SPIIR_EINVAL, "n must be >= 1");
    if (!x || !z) return fail(SPIIR_EINVAL, "null device pointer");
    DeviceGuard guard(bk->device);
    hipStream_t st = as_stream(stream);
    spiir_tape *tp = nullptr;
    float *xwin = nullptr;
    if (tape_out || !bk->xlds) {
        tp = new (std::nothrow) spiir_tape();
        if (!tp) return fail(SPIIR_ENOMEM, "out of host memory");
        tp->bank = bk;
        tp->coeff_version = bk->coeff_version;
        tp->n = n;
        hipError_t e = dalloc(&tp->xwin, (size_t)(n + bk->dmax) + 16);  // read-ahead padding
        if (e != hipSuccess) {
            dfree(tp->xwin);
            delete tp;
            return fail(SPIIR_ENOMEM, "tape allocation failed: %s", hipGetErrorString(e));
        }
        xwin = tp->xwin;
        hipError_t le = launch_window_fill(xwin, nullptr, x, n, bk->dmax, st);
        if (le != hipSuccess) {
            spiir_tape_destroy(tp);
            return fail(SPIIR_EHIP, "window fill: %s", hipGetErrorString(le));
        }
    }
    hipError_t e = launch_fill_zero(bk->zstate, bk->lay.nslots * sizeof(float4), st);
    for (int64_t P = 0; P < n && e == hipSuccess; P += bk->max_block) {
        const int64_t np = std::min<int64_t>(bk->max_block, n - P);
        FwdArgs a = bk->base_args();
        a.state = bk->zstate;
        a.x = x;
        a.hist = nullptr;
        a.xwin = xwin;
        a.xbase = P;
        a.n = np;
        a.obase = P;
        a.z = reinterpret_cast<float2 *>(z);
        a.ld = n;
        int nseg = 1;
        if (bk->nseg > 1) {
            a.seg_len = ((np + bk->nseg - 1) / bk->nseg + bk->L - 1) / bk->L * bk->L;
            nseg = (int)((np + a.seg_len - 1) / a.seg_len);
        }
        KernelEvents ev;
        e = timer_next(bk, &ev);
        if (e != hipSuccess) break;
        if (nseg >= 2)
            e = launch_forward_split(a, kModeZ, bk->lay.fl, bk->tt, bk->xlds, nseg, bk->lds, bk->lds_carry,
                                     bk->slot_filter, st, ev);
        else
            e = launch_forward(a, kModeZ, bk->lay.fl, bk->tt, bk->xlds, bk->lay.groups, bk->lds, st, ev);
        if (e == hipSuccess && bk->n_split)
            e = launch_combine_parts(bk->zpart, bk->max_block, bk->split_tpl, bk->split_off, bk->n_split, np, kModeZ,
                                     nullptr, a.z, a.ld, a.obase, nullptr, st);
    }
    if (e != hipSuccess) {
        if (tp) {
            (void)hipDeviceSynchronize();
            spiir_tape_destroy(tp);
        }
        return fail(SPIIR_EHIP, "forward_z launch: %s", hipGetErrorString(e));
    }
    if (tape_out) {
        *tape_out = tp;
    } else if (tp) {
        (void)hipStreamSynchronize(st);
        spiir_tape_destroy(tp);
    }
    return SPIIR_OK;
}

int spiir_backward(spiir_bank *bk, const spiir_tape *tp, const float *gz, float *ga, float *gb, void *stream) {
    if (!bk || !tp) return fail(SPIIR_EINVAL, "null bank or tape");
    if (!gz || !ga || !gb) return fail(SPIIR_EINVAL, "null device pointer");
    if (tp->bank != bk) return fail(SPIIR_ESTATE, "tape was made by another bank");
    if (tp->coeff_version != bk->coeff_version)
        return fail(SPIIR_ESTATE, "bank coefficients changed since the tape was made");
    if (!tp->xwin) return fail(SPIIR_ESTATE, "tape holds no strain window");
    DeviceGuard guard(bk->device);
    BwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.s = bk->slots();
    a.rows = bk->rows;
    a.slot_filter = bk->slot_filter;
    a.filter_slot = bk->filter_slot;
    a.bwaves = bk->bwaves;
    a.n_bwaves = bk->n_bwaves;
    a.xwin = tp->xwin;
    a.gz = reinterpret_cast<const float2 *>(gz);
    // time segments only when the per-segment kernel (one filter per lane)
    // would leave SIMDs idle: segments add a G-only scan over all but the first
    const int64_t nch = (tp->n + bk->L - 1) / bk->L;
    int want = 1;
    if (bk->tsplit_opt >= 2) {
        want = bk->tsplit_opt;
    } else if (bk->tsplit_opt == 0) {
        const int64_t waves = std::max<int64_t>(1, bk->n_bwaves);
        const int64_t target = (int64_t)4 * bk->dev.n_cu;   // one wave per SIMD
        want = (int)std::min<int64_t>(16, (target + waves - 1) / waves);
    }
    want = (int)std::max<int64_t>(1, std::min<int64_t>(want, nch));
    const int64_t seg_chunks = (nch + want - 1) / want;
    const int nseg = (int)((nch + seg_chunks - 1) / seg_chunks);
    const int64_t S = bk->lay.nslots;
    if (bk->bwd_cap < nseg) {
        dfree(bk->bpair);
        dfree(bk->bgpart);
        bk->bwd_cap = 0;
        hipError_t e = dalloc(&bk->bpair, (size_t)2 * nseg * S);
        if (e == hipSuccess) e = dalloc(&bk->bgpart, (size_t)2 * nseg * S);
        if (e != hipSuccess) {
            dfree(bk->bpair);
            dfree(bk->bgpart);
            return fail(SPIIR_ENOMEM, "adjoint scratch allocation failed: %s", hipGetErrorString(e));
        }
        bk->bwd_cap = nseg;
    }
    a.pair_loc = bk->bpair;
    a.pair_in = bk->bpair + (size_t)nseg * S;
    a.gpart = bk->bgpart;
    a.nseg = nseg;
    a.seg_chunks = (int32_t)seg_chunks;
    a.grad_a = reinterpret_cast<float2 *>(ga);
    a.grad_b = reinterpret_cast<float2 *>(gb);
    a.n = tp->n;
    a.nslots = bk->lay.nslots;
    a.dmax = bk->dmax;
    a.L = bk->L;
    a.prec = bk->prec;
    a.wpg = bk->lay.wpg;
    HIPCHK(launch_backward(a, as_stream(stream)));
    return SPIIR_OK;
}

int spiir_tape_destroy(spiir_tape *tp) {
    if (!tp) return SPIIR_OK;
    dfree(tp->xwin);
    delete tp;
    return SPIIR_OK;
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------

int spiir_batch_create(spiir_batch **out, int32_t ns, spiir_bank *const *banks, const float *const *x,
                       const int64_t *lengths, float *const *mx, int32_t *const *am, int32_t B, void *stream) {
    if (!out) return fail(SPIIR_EINVAL, "out is null");
    *out = nullptr;
    if (ns < 1) return fail(SPIIR_EINVAL, "n_streams must be >= 1");
    if (!banks || !x || !lengths || !mx || !am) return fail(SPIIR_EINVAL, "null array argument");
    if (B < 8 || B % 8) return fail(SPIIR_EINVAL, "block_len must be a positive multiple of 8");
    for (int s = 0; s < ns; ++s) {
        if (!banks[s] || !x[s] || !mx[s] || !am[s]) return fail(SPIIR_EINVAL, "null entry for stream %d", s);
        if (lengths[s] < 1) return fail(SPIIR_EINVAL, "stream %d has length < 1", s);
        if (banks[s]->device != banks[0]->device) return fail(SPIIR_EINVAL, "banks on different devices");
        if (banks[s]->lay.fl != banks[0]->lay.fl || banks[s]->lay.wpg != banks[0]->lay.wpg ||
            banks[s]->tt != banks[0]->tt)
            return fail(SPIIR_EINVAL, "banks must share filters_per_lane, waves_per_group and tile length");
        if (!banks[s]->xlds) return fail(SPIIR_EINVAL, "bank %d keeps its strain window outside LDS", s);
        if (banks[s]->n_split)
            return fail(SPIIR_EINVAL, "bank %d has templates split over workgroups; a batch takes none", s);
        for (int t = 0; t < s; ++t)
            if (banks[t] == banks[s]) return fail(SPIIR_EINVAL, "a bank appears twice in the batch");
    }
    spiir_batch *bt = new (std::nothrow) spiir_batch();
    if (!bt) return fail(SPIIR_ENOMEM, "out of host memory");
    bt->device = banks[0]->device;
    DeviceGuard guard(bt->device);
    bt->ns = ns;
    bt->B = B;
    bt->fl = banks[0]->lay.fl;
    bt->wpg = banks[0]->lay.wpg;
    bt->tt = banks[0]->tt;
    bt->banks.assign(banks, banks + ns);
    bt->len.assign(lengths, lengths + ns);
    int max_groups = 0;
    for (int s = 0; s < ns; ++s) {
        bt->lds = std::max(bt->lds, banks[s]->lds);
        max_groups = std::max(max_groups, banks[s]->lay.groups);
    }
    bt->key_stride = (int64_t)max_groups * B;
    // work items, largest first: (stream length) x (filters in the group)
    std::vector<std::tuple<double, int, int>> it;
    for (int s = 0; s < ns; ++s) {
        const spiir_bank *bk = banks[s];
        std::vector<int64_t> gf(bk->lay.groups, 0);
        for (int j = 0; j < bk->T; ++j) gf[bk->lay.tpl_group[j]] += bk->off[j + 1] - bk->off[j];
        for (int g = 0; g < bk->lay.groups; ++g) it.emplace_back(-(double)lengths[s] * gf[g], s, g);
    }
    std::sort(it.begin(), it.end());
    std::vector<int2> items;
    for (auto &t : it) items.push_back(make_int2(std::get<1>(t), std::get<2>(t)));
    bt->nitems = (int)items.size();
    std::vector<BatchStream> hs(ns);
    for (int s = 0; s < ns; ++s) {
        std::memset(&hs[s], 0, sizeof(BatchStream));
        FwdArgs a = banks[s]->base_args();
        a.state = banks[s]->state;
        a.x = x[s];
        a.hist = nullptr;
        a.ld = B;
        hs[s].args = a;
        hs[s].len = lengths[s];
        hs[s].groups = banks[s]->lay.groups;
        hs[s].max_out = mx[s];
        hs[s].arg_out = am[s];
    }
    hipError_t e = hipSuccess;
    auto A = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    A(dalloc(&bt->streams, (size_t)ns));
    A(dalloc(&bt->items, items.size()));
    A(dalloc(&bt->counter, 1));
    A(dalloc(&bt->pos, (size_t)ns));
    A(dalloc(&bt->keys, (size_t)(bt->key_stride * ns)));
    if (e == hipSuccess) {
        for (int s = 0; s < ns; ++s) hs[s].args.keys = bt->keys + s * bt->key_stride;
        A(hipMemcpy(bt->streams, hs.data(), ns * sizeof(BatchStream), hipMemcpyHostToDevice));
        A(hipMemcpy(bt->items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
        A(hipMemset(bt->counter, 0, sizeof(int)));
        A(hipMemset(bt->pos, 0, ns * sizeof(int64_t)));
    }
    const int occ = std::max(1, batch_occupancy(bt->fl, bt->tt, bt->wpg, bt->lds));
    bt->grid = std::min(bt->nitems, banks[0]->dev.n_cu * occ);
    bt->slots_dev = (int64_t)banks[0]->dev.n_cu * occ;
    // time-split plan per stream: segments of whole chunks, enough to fill the
    // device with this stream alone (at most 8 and at most one per chunk)
    // Items of the time-split step are grouped by stream, longest stream first,
    // so that the items of the k live streams are a prefix of the list.
    std::vector<int> order(ns);
    for (int s = 0; s < ns; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int p, int q) { return lengths[p] > lengths[q]; });
    std::vector<int2> si, ci;
    std::vector<int> sp(ns + 1, 0), cp(ns + 1, 0);   // prefix item counts over `order`
    int64_t max_slots = 0;
    bool any_split = false;
    for (int s = 0; s < ns; ++s) bt->groups.push_back(banks[s]->lay.groups);
    for (int oi = 0; oi < ns; ++oi) {
        const int s = order[oi];
        const spiir_bank *bk = banks[s];
        max_slots = std::max(max_slots, bk->lay.nslots);
        const int L = bk->L;
        // as in a bank's automatic split: twice the resident slots over the workgroups, at most 8
        int want = (int)std::min<int64_t>(8, 2 * bt->slots_dev / std::max(1, bk->lay.groups));
        want = std::max(1, std::min(want, (B + L - 1) / L));
        const int64_t seg_len = ((B + want - 1) / want + L - 1) / L * L;
        const int nseg = (int)((B + seg_len - 1) / seg_len);
        hs[s].args.seg_len = seg_len;
        any_split = any_split || nseg >= 2;
        // every stream takes part in the split step (a single segment needs only its end state)
        float4 *se = nullptr, *ss = nullptr;
        float2 *zl = nullptr;
        A(dalloc(&se, (size_t)nseg * bk->lay.nslots));
        A(dalloc(&ss, (size_t)nseg * bk->lay.nslots));
        if (nseg >= 2) A(dalloc(&zl, (size_t)(nseg - 1) * bk->T * seg_len));
        bt->seg_bufs.push_back(se);
        bt->seg_bufs.push_back(ss);
        if (zl) bt->zl_bufs.push_back(zl);
        hs[s].args.seg_end = se;
        hs[s].args.seg_start = ss;
        hs[s].args.zl = zl;
        // this stream's items, largest workgroups first
        std::vector<int64_t> gf(bk->lay.groups, 0);
        for (int j = 0; j < bk->T; ++j) gf[bk->lay.tpl_group[j]] += bk->off[j + 1] - bk->off[j];
        std::vector<int> gord(bk->lay.groups);
        for (int g = 0; g < bk->lay.groups; ++g) gord[g] = g;
        std::stable_sort(gord.begin(), gord.end(), [&](int p, int q) { return gf[p] > gf[q]; });
        for (int k = 0; k < nseg; ++k)
            for (int g : gord) {
                si.push_back(make_int2(s, (g << 4) | k));
                if (k > 0) ci.push_back(make_int2(s, (g << 4) | k));
            }
        sp[oi + 1] = (int)si.size();
        cp[oi + 1] = (int)ci.size();
    }
    if (!any_split) {
        si.clear();
        ci.clear();
    }
    if (!si.empty() && e == hipSuccess) {
        A(dalloc(&bt->seg_items, si.size()));
        A(dalloc(&bt->carry_items, std::max<size_t>(1, ci.size())));
        if (e == hipSuccess) A(hipMemcpy(bt->seg_items, si.data(), si.size() * sizeof(int2), hipMemcpyHostToDevice));
        if (e == hipSuccess && !ci.empty())
            A(hipMemcpy(bt->carry_items, ci.data(), ci.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    // segment plans are part of the stream descriptors
    if (e == hipSuccess) A(hipMemcpy(bt->streams, hs.data(), ns * sizeof(BatchStream), hipMemcpyHostToDevice));
    hipStream_t cap = nullptr;
    if (e == hipSuccess) A(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    if (e == hipSuccess) {
        A(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        if (e == hipSuccess) {
            A(launch_batch(bt->streams, bt->items, bt->nitems, bt->counter, bt->pos, B, bt->fl, bt->tt,
                           bt->grid, bt->wpg, bt->lds, cap));
            A(launch_batch_finalize(bt->streams, ns, bt->keys, bt->key_stride, bt->pos, B, max_groups, cap));
            A(launch_batch_advance(bt->pos, bt->streams, ns, bt->counter, B, cap));
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(cap, &g);
            A(ee);
            bt->graph = g;
        }
        if (e == hipSuccess) A(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
    }
    for (int k = 1; k <= ns && e == hipSuccess && !si.empty(); ++k) {
        const size_t lds_carry = fwd_lds_bytes(bt->wpg, 0, 0, false, bt->tt);
        A(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
        if (e == hipSuccess) {
            A(launch_batch_split(bt->streams, bt->seg_items, sp[k], bt->carry_items, cp[k], bt->pos, B, ns,
                                 max_slots, bt->fl, bt->tt, bt->wpg, bt->lds, lds_carry, cap));
            A(launch_batch_finalize(bt->streams, ns, bt->keys, bt->key_stride, bt->pos, B, max_groups, cap));
            A(launch_batch_advance(bt->pos, bt->streams, ns, bt->counter, B, cap));
            hipGraph_t g = nullptr;
            hipError_t ee = hipStreamEndCapture(cap, &g);
            A(ee);
            bt->sgraph.push_back(g);
        }
        hipGraphExec_t x = nullptr;
        if (e == hipSuccess) A(hipGraphInstantiate(&x, bt->sgraph.back(), nullptr, nullptr, 0));
        bt->sexec.push_back(x);
    }
    if (cap) (void)hipStreamDestroy(cap);
    for (int s = 0; s < ns && e == hipSuccess; ++s) {
        A(launch_fill_zero(banks[s]->state, banks[s]->lay.nslots * sizeof(float4), as_stream(stream)));
    }
    if (e == hipSuccess) A(hipStreamSynchronize(as_stream(stream)));
    if (e != hipSuccess) {
        spiir_batch_destroy(bt);
        return fail(SPIIR_EHIP, "batch creation: %s", hipGetErrorString(e));
    }
    *out = bt;
    return SPIIR_OK;
}

int spiir_batch_step(spiir_batch *bt, void *stream) {
    if (!bt) return fail(SPIIR_EINVAL, "batch is null");
    DeviceGuard guard(bt->device);
    // the device positions follow the replay count, so the host knows which streams are live
    int nlive = 0;
    int64_t live = 0;
    for (int s = 0; s < bt->ns; ++s)
        if (bt->len[s] > bt->host_step * bt->B) {
            ++nlive;
            live += bt->groups[s];
        }
    bool split = false;
    if (!bt->sexec.empty() && nlive > 0 && bt->split_mode != 1)
        split = bt->split_mode == 2 || 2 * live <= bt->slots_dev;
    HIPCHK(hipGraphLaunch(split ? bt->sexec[nlive - 1] : bt->exec, as_stream(stream)));
    ++bt->host_step;
    return SPIIR_OK;
}

int spiir_batch_set_time_split(spiir_batch *bt, int32_t mode) {
    if (!bt) return fail(SPIIR_EINVAL, "batch is null");
    if (mode < 0 || mode > 2) return fail(SPIIR_EINVAL, "mode must be 0 (auto), 1 (never) or 2 (always)");
    if (mode == 2 && bt->sexec.empty())
        return fail(SPIIR_EINVAL, "this batch has no time-split step (blocks shorter than two chunks)");
    bt->split_mode = mode;
    return SPIIR_OK;
}

int spiir_batch_steps_total(const spiir_batch *bt, int64_t *steps) {
    if (!bt || !steps) return fail(SPIIR_EINVAL, "null argument");
    int64_t m = 0;
    for (int64_t l : bt->len) m = std::max(m, (l + bt->B - 1) / bt->B);
    *steps = m;
    return SPIIR_OK;
}

int spiir_batch_reset(spiir_batch *bt, void *stream) {
    if (!bt) return fail(SPIIR_EINVAL, "batch is null");
    DeviceGuard guard(bt->device);
    hipStream_t st = as_stream(stream);
    HIPCHK(launch_fill_zero(bt->pos, bt->ns * sizeof(int64_t), st));
    bt->host_step = 0;
    HIPCHK(launch_fill_zero(bt->counter, sizeof(int), st));
    for (spiir_bank *bk : bt->banks) HIPCHK(launch_fill_zero(bk->state, bk->lay.nslots * sizeof(float4), st));
    return SPIIR_OK;
}

int spiir_batch_destroy(spiir_batch *bt) {
    if (!bt) return SPIIR_OK;
    {
        DeviceGuard guard(bt->device);
        (void)hipDeviceSynchronize();
        if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
        if (bt->graph) (void)hipGraphDestroy(bt->graph);
        for (auto x : bt->sexec)
            if (x) (void)hipGraphExecDestroy(x);
        for (auto g : bt->sgraph)
            if (g) (void)hipGraphDestroy(g);
        dfree(bt->seg_items);
        dfree(bt->carry_items);
        for (auto &p : bt->seg_bufs) dfree(p);
        for (auto &p : bt->zl_bufs) dfree(p);
        dfree(bt->streams);
        dfree(bt->items);
        dfree(bt->counter);
        dfree(bt->pos);
        dfree(bt->keys);
    }
    delete bt;
    return SPIIR_OK;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------

int spiir_autotune(int32_t nbk, const int32_t *T, const int64_t *const *off, const double *const *a,
                   const double *const *b, const int32_t *const *d, int32_t max_delay, int32_t B,
                   int32_t device, int32_t *L_out, int32_t *F_out, float *table) {
    static std::mutex mu;
    static std::map<std::vector<int64_t>, std::pair<int32_t, int32_t>> cache;
    if (nbk < 1 || !T || !off || !a || !b || !d || !L_out || !F_out)
        return fail(SPIIR_EINVAL, "null or empty autotune argument");
    if (B < 8 || B % 8) return fail(SPIIR_EINVAL, "block_len must be a positive multiple of 8");
    spiir_bank_opts probe;
    spiir_bank_opts_default(&probe);
    probe.max_delay = max_delay;
    for (int i = 0; i < nbk; ++i) {
        int dm = 0;
        int rc = check_bank_args(T[i], off[i], a[i], b[i], d[i], probe, dm);
        if (rc) return rc;
    }
    int dev = device;
    if (dev < 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(SPIIR_ENODEV, "no HIP device available");
        HIPCHK(hipGetDevice(&dev));
    }
    DeviceFacts df;
    int rc = device_facts(dev, df);
    if (rc) return rc;
    std::vector<int64_t> key = {dev, nbk, max_delay, B};
    for (int i = 0; i < nbk; ++i) {
        key.push_back(T[i]);
        int64_t h = 0;
        for (int j = 0; j <= T[i]; ++j) h = h * 1000003 + off[i][j];
        key.push_back(h);
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        auto itc = cache.find(key);
        if (itc != cache.end() && !table) {
            *L_out = itc->second.first;
            *F_out = itc->second.second;
            return SPIIR_OK;
        }
    }
    DeviceGuard guard(dev);
    const int Ls[4] = {64, 128, 256, 512};
    float best = 1e30f;
    int bestL = 256, bestF = 1;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    {
        hipError_t ce = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (ce == hipSuccess) ce = hipEventCreate(&e0);
        if (ce == hipSuccess) ce = hipEventCreate(&e1);
        if (ce != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            if (st) (void)hipStreamDestroy(st);
            return fail(SPIIR_EHIP, "autotune stream/event: %s", hipGetErrorString(ce));
        }
    }
    const int warm = 2, iters = 6;
    const int64_t len = (int64_t)B * (warm + iters);
    std::vector<float *> xs(nbk, nullptr), ms(nbk, nullptr);
    std::vector<int32_t *> as(nbk, nullptr);
    hipError_t e = hipSuccess;
    for (int i = 0; i < nbk && e == hipSuccess; ++i) {
        e = dalloc(&xs[i], (size_t)len);
        if (e == hipSuccess) e = dalloc(&ms[i], (size_t)len);
        if (e == hipSuccess) e = dalloc(&as[i], (size_t)len);
        if (e == hipSuccess) e = launch_noise_fill(xs[i], len, 1602u + (uint32_t)i, st);
    }
    for (int li = 0; li < 4 && e == hipSuccess; ++li) {
        for (int fl = 1; fl <= 4; ++fl) {
            if (table) table[li * 4 + fl - 1] = -1.f;
            int64_t total = 0;
            int maxnr = 0;
            for (int i = 0; i < nbk; ++i) {
                const Plan p = plan_rows(T[i], off[i], fl);
                total += p.total_rows;
                maxnr = std::max(maxnr, p.max_nr);
            }
            if (maxnr > 4 * kMaxWaves) continue;
            spiir_bank_opts o;
            spiir_bank_opts_default(&o);
            o.chunk_len = Ls[li];
            o.filters_per_lane = fl;
            o.max_delay = max_delay;
            o.device = dev;
            o.waves_per_group = auto_wpg(total, maxnr, df.n_cu);
            std::vector<spiir_bank *> bks(nbk, nullptr);
            bool ok = true;
            for (int i = 0; i < nbk && ok; ++i)
                ok = create_bank(&bks[i], T[i], off[i], a[i], b[i], d[i], o) == SPIIR_OK && bks[i]->xlds;
            spiir_batch *bt = nullptr;
            std::vector<int64_t> lens(nbk, len);
            if (ok)
                ok = spiir_batch_create(&bt, nbk, bks.data(), xs.data(), lens.data(), ms.data(), as.data(), B, st) ==
                     SPIIR_OK;
            float ms_per = -1.f;
            if (ok) {
                for (int w = 0; w < warm && ok; ++w) ok = spiir_batch_step(bt, st) == SPIIR_OK;
                if (ok) ok = hipEventRecord(e0, st) == hipSuccess;
                for (int w = 0; w < iters && ok; ++w) ok = spiir_batch_step(bt, st) == SPIIR_OK;
                if (ok) ok = hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
                if (ok) ok = hipEventElapsedTime(&ms_per, e0, e1) == hipSuccess;
                if (ok) ms_per /= iters;
            }
            if (bt) spiir_batch_destroy(bt);
            for (spiir_bank *bk : bks) spiir_bank_destroy(bk);
            if (ok && ms_per > 0.f) {
                if (table) table[li * 4 + fl - 1] = ms_per * 1e6f;
                if (ms_per < best) {
                    best = ms_per;
                    bestL = Ls[li];
                    bestF = fl;
                }
            }
        }
    }
    for (int i = 0; i < nbk; ++i) {
        dfree(xs[i]);
        dfree(ms[i]);
        dfree(as[i]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(st);
    if (e != hipSuccess) return fail(SPIIR_EHIP, "autotune setup: %s", hipGetErrorString(e));
    if (best >= 1e30f) return fail(SPIIR_EINVAL, "no autotune candidate could run on this bank");
    {
        std::lock_guard<std::mutex> lk(mu);
        cache[key] = {bestL, bestF};
    }
    *L_out = bestL;
    *F_out = bestF;
    g_err.clear();
    return SPIIR_OK;
}

const char *spiir_last_error(void) { return g_err.c_str(); }

const char *spiir_version(void) { return "spiir-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
