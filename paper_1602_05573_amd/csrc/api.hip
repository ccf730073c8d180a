// Host side of libspiir: argument checking, bank layout, FP64 precomputation,
// launches, streaming state, the adjoint tape, batches in a HIP graph and the
// autotuner. Declared in include/spiir.h.
#include "spiir.h"
#include "spiir_internal.h"

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

namespace {

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

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(SPIIR_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

template <typename T>
hipError_t dalloc(T **p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

template <typename T>
void dfree(T *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

std::pair<double, double> cpow(double re, double im, long e) {
    double rr = 1.0, ri = 0.0;
    while (e > 0) {
        if (e & 1) {
            const double t = rr * re - ri * im;
            ri = rr * im + ri * re;
            rr = t;
        }
        const double t = re * re - im * im;
        im = 2.0 * re * im;
        re = t;
        e >>= 1;
    }
    return {rr, ri};
}

// Filter-to-slot layout of one bank.
struct Layout {
    int fl = 1, wpg = 1, groups = 0;
    int64_t nslots = 0;
    std::vector<RowInfo> rows;            // [groups * wpg * 4]
    std::vector<int32_t> slot_filter;     // [nslots], -1 = padding
    std::vector<int64_t> pad_src;         // [nslots], padding: slot whose window offset it reuses
    std::vector<int32_t> tpl_group;       // [T]
};

struct Plan {
    int64_t total_rows = 0;
    int max_nr = 0;
};

inline int rows_of(int64_t k, int fl) { return (int)((k + kRowLanes * fl - 1) / (kRowLanes * fl)); }

Plan plan_rows(int T, const int64_t *off, int fl) {
    Plan p;
    for (int j = 0; j < T; ++j) {
        const int nr = rows_of(off[j + 1] - off[j], fl);
        p.total_rows += nr;
        p.max_nr = std::max(p.max_nr, nr);
    }
    return p;
}

int auto_wpg(int64_t total_rows, int max_nr, int n_cu) {
    const int64_t waves = (total_rows + 3) / 4;
    int w = (int)((waves + n_cu - 1) / n_cu);
    return std::min(kMaxWaves, std::max(w, (max_nr + 3) / 4));
}

// First-fit decreasing packing of whole templates, in 16-lane rows, into
// workgroups of 4 * wpg rows; then the filter-to-slot assignment inside every
// template. A template has nr rows x fl slots = C columns of 16 lanes, and one
// ds_read_b32 of x[m - d] serves a column's 16 lanes in one LDS pass: filters
// sorted by d mod 32 are dealt round-robin over the C columns, so the lanes
// of a column have distinct d mod 32 (a residue class holds about K/32 < C
// filters) and read from distinct banks. Padding lanes take the window offset
// of a real lane of their column (same address: a broadcast, not a conflict).
// Places the filters [k0, k1) of one template into its rows r0 .. r0+nr-1 of
// workgroup g. A ds_read_b32 of the strain window x[m - d] is served 32 lanes
// per LDS cycle with bank = (dword address mod 32), i.e. by d mod 32; the 32
// lanes are the two rows 2q, 2q+1 of a wave at one filter column f. Where both
// rows of such a pair belong to this template, the pair is one 32-lane column
// that takes each residue class at most once while it can; a row whose partner
// row belongs to another template takes residues 0..15 (even row) or 16..31
// (odd row), so the two templates of the pair stay apart. Classes are placed
// in order of decreasing count; a filter that finds every allowed column
// already holding its class goes where its class is rarest, preferring
// columns that already hold a double, so that the unavoidable extra cycles
// gather in few passes. Padding lanes read the address of their row's first
// lane (a broadcast).
void deal_template(int64_t k0, int64_t k1, const int32_t *d, int g, int wpg, int fl, int r0, int nr, Layout &lay) {
    struct Col {
        int cap, lo, hi, rows[2], nparts, f, dbl;
        std::vector<int32_t> items;
        uint8_t has[32];
    };
    std::vector<Col> cols;
    for (int r = r0; r < r0 + nr; ++r) {
        const int p = r ^ 1;
        const bool internal = p >= r0 && p < r0 + nr;
        if (internal && p < r) continue;
        for (int f = 0; f < fl; ++f) {
            Col c{};
            c.f = f;
            c.rows[0] = r;
            if (internal) {
                c.cap = 2 * kRowLanes;
                c.lo = 0;
                c.hi = 32;
                c.rows[1] = p;
                c.nparts = 2;
            } else {
                c.cap = kRowLanes;
                c.lo = (r & 1) ? 16 : 0;
                c.hi = c.lo + 16;
                c.nparts = 1;
            }
            cols.push_back(c);
        }
    }
    std::vector<std::vector<int32_t>> bycls(32);
    for (int64_t k = k0; k < k1; ++k) bycls[d[k] & 31].push_back((int32_t)k);
    std::vector<int> corder(32);
    for (int c = 0; c < 32; ++c) corder[c] = c;
    std::stable_sort(corder.begin(), corder.end(),
                     [&](int a, int b) { return bycls[a].size() > bycls[b].size(); });
    // rank of a candidate column for a filter of class cls (lower is better): fewest of
    // the class already there; among columns that already hold it, one with a double;
    // then the least filled
    auto key = [](const Col &c, int cls) {
        const double fill = (double)c.items.size() / c.cap;
        const int again = c.has[cls] > 0 && c.dbl == 0 ? 1 : 0;
        return std::make_tuple((int)c.has[cls], again, fill);
    };
    for (int cls : corder) {
        for (int32_t k : bycls[cls]) {
            Col *best = nullptr;
            for (int pass = 0; pass < 2 && !best; ++pass)   // allowed classes first, then any room
                for (Col &c : cols) {
                    if ((int)c.items.size() >= c.cap) continue;
                    if (pass == 0 && (cls < c.lo || cls >= c.hi)) continue;
                    if (!best || key(c, cls) < key(*best, cls)) best = &c;
                }
            if (best->has[cls]) ++best->dbl;
            ++best->has[cls];
            best->items.push_back(k);
        }
    }
    for (const Col &c : cols) {
        if (c.items.empty()) continue;
        int64_t first = -1;   // slot of the column's first filter: padding lanes read its address
        for (int part = 0; part < c.nparts; ++part) {
            const int row = c.rows[part];
            const int64_t base = ((int64_t)(g * wpg + row / 4) * fl + c.f) * 64 + (row % 4) * kRowLanes;
            if (part == 0) first = base;
            const int n0 = part * kRowLanes;
            const int n = std::max(0, std::min<int>(kRowLanes, (int)c.items.size() - n0));
            for (int l = 0; l < n; ++l) lay.slot_filter[(size_t)(base + l)] = c.items[(size_t)(n0 + l)];
            for (int l = n; l < kRowLanes; ++l) lay.pad_src[(size_t)(base + l)] = first;
        }
    }
}

int build_layout(int T, const int64_t *off, const int32_t *d, int fl, int wpg, Layout &lay) {
    const int R = 4 * wpg;
    std::vector<int> nr(T);
    int max_nr = 0;
    for (int j = 0; j < T; ++j) {
        nr[j] = rows_of(off[j + 1] - off[j], fl);
        max_nr = std::max(max_nr, nr[j]);
    }
    if (max_nr > R)
        return fail(SPIIR_EINVAL, "a template needs %d rows of %d filters but a workgroup has %d",
                    max_nr, kRowLanes * fl, R);
    std::vector<int> order(T);
    for (int j = 0; j < T; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return nr[x] > nr[y]; });
    std::vector<int> room;                  // free rows per group
    std::vector<std::vector<int>> members;  // templates per group
    for (int j : order) {
        size_t g = 0;
        for (; g < room.size(); ++g)
            if (room[g] >= nr[j]) break;
        if (g == room.size()) {
            room.push_back(R);
            members.emplace_back();
        }
        room[g] -= nr[j];
        members[g].push_back(j);
    }
    lay.fl = fl;
    lay.wpg = wpg;
    lay.groups = (int)members.size();
    lay.nslots = (int64_t)lay.groups * wpg * fl * 64;
    lay.rows.assign((size_t)lay.groups * R, RowInfo{-1, 0, 0, 0});
    lay.slot_filter.assign((size_t)lay.nslots, -1);
    lay.pad_src.assign((size_t)lay.nslots, -1);
    lay.tpl_group.assign(T, -1);
    for (int g = 0; g < lay.groups; ++g) {
        std::vector<int> &mem = members[g];
        std::sort(mem.begin(), mem.end());
        int r0 = 0;
        for (int j : mem) {
            lay.tpl_group[j] = g;
            for (int r = 0; r < nr[j]; ++r) lay.rows[(size_t)g * R + r0 + r] = RowInfo{j, r0, nr[j], 0};
            deal_template(off[j], off[j + 1], d, g, wpg, fl, r0, nr[j], lay);
            r0 += nr[j];
        }
    }
    return SPIIR_OK;
}

struct DeviceFacts {
    int n_cu = 0;
    size_t lds_cap = 0;
};

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
    int32_t *xoff = nullptr, *flags = nullptr, *slot_filter = nullptr;
    double2 *aL = nullptr, *dL = nullptr, *a64 = nullptr;
    float4 *state = nullptr, *zstate = nullptr;
    RowInfo *rows = nullptr;
    int tt = 16;
    float *hist[2] = {nullptr, nullptr};
    int hist_cur = 0;
    uint64_t *keys = nullptr;
    float *xwin = nullptr;
    int64_t xwin_cap = 0;
    float2 *ysub = nullptr;
    int nseg = 1;                 // time segments per streaming launch
    int64_t seg_len_max = 0;
    size_t lds_carry = 0;
    float4 *seg_end = nullptr, *seg_start = nullptr;
    float2 *zl = nullptr;
    int tsplit_opt = 0;           // opts.time_split as given (the adjoint honours it too)
    // adjoint scratch, grown on demand: ysub [cap][ceil(L/kSub)][S], lam [2][cap][S], gpart [cap][2][S]
    int bwd_cap = 0;
    float2 *blam = nullptr;
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
        p.zl = zl;
        return p;
    }
};

struct spiir_tape {
    spiir_bank *bank = nullptr;
    uint64_t coeff_version = 0;
    int64_t n = 0, nchunks = 0;
    float4 *tape = nullptr;
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

// Host-side checks of create arguments; no HIP call is made here.
int check_bank_args(int32_t T, const int64_t *off, const double *a, const double *b, const int32_t *d,
                    const spiir_bank_opts &o, int &dmax_out) {
    if (T < 1) return fail(SPIIR_EINVAL, "n_templates must be >= 1 (got %d)", T);
    if (!off || !a || !b || !d) return fail(SPIIR_EINVAL, "null coefficient / offset / delay array");
    if (off[0] != 0) return fail(SPIIR_EINVAL, "filter_offsets[0] must be 0");
    for (int j = 0; j < T; ++j)
        if (off[j + 1] <= off[j])
            return fail(SPIIR_EINVAL, "template %d has no filters (offsets must strictly increase)", j);
    const int64_t F = off[T];
    if (F > (int64_t)INT32_MAX) return fail(SPIIR_EINVAL, "too many filters (%lld)", (long long)F);
    int dm = 0;
    for (int64_t k = 0; k < F; ++k) {
        const double ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
        if (!std::isfinite(ar) || !std::isfinite(ai) || !std::isfinite(br) || !std::isfinite(bi))
            return fail(SPIIR_EINVAL, "filter %lld has a non-finite coefficient", (long long)k);
        if (std::hypot(ar, ai) >= 1.0)
            return fail(SPIIR_EINVAL, "filter %lld is not stable: |a| = %.17g >= 1", (long long)k, std::hypot(ar, ai));
        if (d[k] < 0) return fail(SPIIR_EINVAL, "filter %lld has a negative delay", (long long)k);
        dm = std::max(dm, d[k]);
    }
    if (o.max_delay < 0) return fail(SPIIR_EINVAL, "max_delay must be >= 0");
    if (o.max_delay > 0 && dm > o.max_delay)
        return fail(SPIIR_EINVAL, "a delay (%d) exceeds max_delay (%d)", dm, o.max_delay);
    const int dmax = o.max_delay > 0 ? o.max_delay : dm;
    if (dmax > (1 << 26)) return fail(SPIIR_EINVAL, "max_delay %d too large", dmax);
    if (o.chunk_len != 0 && (o.chunk_len < 8 || o.chunk_len > 4096 || o.chunk_len % 8))
        return fail(SPIIR_EINVAL, "chunk_len must be a multiple of 8 in [8, 4096] (got %d)", o.chunk_len);
    if (o.filters_per_lane < 0 || o.filters_per_lane > 4)
        return fail(SPIIR_EINVAL, "filters_per_lane must be 0..4 (got %d)", o.filters_per_lane);
    if (o.precision < 0 || o.precision > 2) return fail(SPIIR_EINVAL, "precision must be 0, 1 or 2");
    if (o.max_block < 0) return fail(SPIIR_EINVAL, "max_block must be >= 0");
    if (o.waves_per_group < 0 || o.waves_per_group > kMaxWaves)
        return fail(SPIIR_EINVAL, "waves_per_group must be 0..%d", kMaxWaves);
    if (o.time_split < 0 || o.time_split > 32) return fail(SPIIR_EINVAL, "time_split must be 0..32");
    dmax_out = dmax;
    return SPIIR_OK;
}

// Slot arrays on the host, then uploaded.
int upload_coeffs(spiir_bank *bk) {
    const int64_t S = bk->lay.nslots;
    std::vector<float2> a32((size_t)S, make_float2(0.f, 0.f)), b32((size_t)S, make_float2(0.f, 0.f));
    std::vector<int32_t> xo((size_t)S, 0), fl((size_t)S, 0);
    std::vector<double2> aL((size_t)S, make_double2(0, 0)), dL((size_t)S, make_double2(0, 0)),
        a64((size_t)S, make_double2(0, 0));
    for (int64_t s = 0; s < S; ++s) {
        const int32_t k = bk->lay.slot_filter[(size_t)s];
        if (k < 0) {
            const int64_t src = bk->lay.pad_src[(size_t)s];
            if (src >= 0) xo[(size_t)s] = bk->dmax - bk->d[(size_t)bk->lay.slot_filter[(size_t)src]];
            continue;
        }
        const double ar = bk->a[2 * (size_t)k], ai = bk->a[2 * (size_t)k + 1];
        const float far = (float)ar, fai = (float)ai;
        a32[(size_t)s] = make_float2(far, fai);
        b32[(size_t)s] = make_float2((float)bk->b[2 * (size_t)k], (float)bk->b[2 * (size_t)k + 1]);
        xo[(size_t)s] = bk->dmax - bk->d[(size_t)k];
        const auto p = cpow(ar, ai, bk->L);
        const auto q = cpow((double)far, (double)fai, bk->L);
        aL[(size_t)s] = make_double2(p.first, p.second);
        dL[(size_t)s] = make_double2(p.first - q.first, p.second - q.second);
        a64[(size_t)s] = make_double2(ar, ai);
        fl[(size_t)s] = std::hypot(ar, ai) > 1.0 - 1e-5 ? 1 : 0;
    }
    HIPCHK(hipMemcpy(bk->a32, a32.data(), S * sizeof(float2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->b32, b32.data(), S * sizeof(float2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->xoff, xo.data(), S * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->flags, fl.data(), S * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->aL, aL.data(), S * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->dL, dL.data(), S * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(bk->a64, a64.data(), S * sizeof(double2), hipMemcpyHostToDevice));
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
    dfree(bk->aL); dfree(bk->dL); dfree(bk->a64); dfree(bk->state); dfree(bk->zstate);
    dfree(bk->rows); dfree(bk->hist[0]); dfree(bk->hist[1]); dfree(bk->keys); dfree(bk->xwin);
    dfree(bk->ysub); dfree(bk->blam); dfree(bk->bgpart); dfree(bk->seg_end); dfree(bk->seg_start); dfree(bk->zl);
}

// Filters per lane: the largest count that still gives every SIMD about two
// waves (more filters per lane amortise the template sums over more updates);
// banks too small for that get one filter per lane.
int choose_fl(int T, const int64_t *off, int n_cu) {
    for (int fl = 4; fl >= 1; --fl) {
        const Plan p = plan_rows(T, off, fl);
        if (p.max_nr > 4 * kMaxWaves) return std::min(4, fl + 1);
        if ((p.total_rows + 3) / 4 >= (int64_t)7 * n_cu) return fl;
    }
    return 1;
}

struct Geometry {
    int tt = 16, nb = 0;
    bool xlds = true;
    size_t lds = 0;
};

// LDS plan for a workgroup of wpg waves: the strain window (max_delay + nb
// samples) when it fits, and 16-step tiles when they fit beside it.
Geometry plan_geometry(int wpg, int dmax, int L, int max_block, size_t lds_cap) {
    Geometry best;
    for (int tt : {16, 8}) {
        Geometry g;
        g.tt = tt;
        const int64_t fixed = (int64_t)fwd_lds_bytes(wpg, 0, 0, false, tt);
        int64_t nb = ((int64_t)lds_cap - fixed - 4 * (int64_t)(dmax + tt) - 64) / (4 * L) * L;
        nb = std::min<int64_t>(nb, max_block);
        g.xlds = nb >= L;
        g.nb = g.xlds ? (int)nb : max_block;
        g.lds = fwd_lds_bytes(wpg, dmax, g.nb, g.xlds, tt);
        if (tt == 16) {
            best = g;
            if (!g.xlds || g.nb >= std::min(max_block, 2048)) return g;
        } else if (g.xlds && (!best.xlds || g.nb > best.nb)) {
            return g;
        }
    }
    return best;
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

    const int L = o.chunk_len ? o.chunk_len : 256;
    int max_block = o.max_block ? o.max_block : 16384;
    max_block = std::max(L, (max_block / L) * L);
    int fl = o.filters_per_lane;
    if (fl == 0) {
        // A delay window too long for LDS (even beside a single wave's tiles) leaves the strain
        // in global memory; there four filters per lane give each wave more independent loads
        // in flight, and the time split supplies the parallelism a small bank lacks.
        const bool global_window = !plan_geometry(1, dmax, L, max_block, df.lds_cap).xlds;
        fl = choose_fl(T, off, df.n_cu);
        if (global_window && plan_rows(T, off, 4).max_nr <= 4 * kMaxWaves) fl = 4;
    }
    const Plan plan = plan_rows(T, off, fl);
    if (plan.max_nr > 4 * kMaxWaves)
        return fail(SPIIR_EINVAL, "a template has more than %d filters; use more filters per lane",
                    4 * kMaxWaves * kRowLanes * fl);
    int wpg = o.waves_per_group;
    if (wpg == 0) {
        // smallest workgroup that packs the bank into one round of resident workgroups
        const int w0 = auto_wpg(plan.total_rows, plan.max_nr, df.n_cu);
        wpg = w0;
        for (int w = w0; w <= kMaxWaves; ++w) {
            const Geometry gm = plan_geometry(w, dmax, L, max_block, df.lds_cap);
            const int occ = std::max(1, forward_occupancy(fl, gm.tt, w, gm.lds));
            Layout trial;
            if (build_layout(T, off, d, fl, w, trial)) continue;
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
    rc = build_layout(T, off, d, fl, wpg, bk->lay);
    if (rc) {
        delete bk;
        return rc;
    }
    const Geometry gm = plan_geometry(wpg, dmax, L, max_block, df.lds_cap);
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
    A(dalloc(&bk->slot_filter, S)); A(dalloc(&bk->aL, S)); A(dalloc(&bk->dL, S)); A(dalloc(&bk->a64, S));
    A(dalloc(&bk->state, S)); A(dalloc(&bk->zstate, S)); A(dalloc(&bk->rows, (size_t)G * wpg * 4));
    A(dalloc(&bk->hist[0], (size_t)dmax)); A(dalloc(&bk->hist[1], (size_t)dmax));
    A(dalloc(&bk->keys, (size_t)G * max_block));
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
        if (e == hipSuccess)
            e = hipMemcpy(bk->rows, bk->lay.rows.data(), bk->lay.rows.size() * sizeof(RowInfo),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(bk->state, 0, S * sizeof(float4));
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

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

int ensure_xwin(spiir_bank *bk, int64_t need) {
    if (need <= bk->xwin_cap) return SPIIR_OK;
    HIPCHK(hipDeviceSynchronize());
    dfree(bk->xwin);
    bk->xwin_cap = 0;
    HIPCHK(dalloc(&bk->xwin, (size_t)need + 16));  // one tile of read-ahead padding
    bk->xwin_cap = need;
    return SPIIR_OK;
}

// Shared driver of the streaming calls (snr rows or fused keys).
int stream_call(spiir_bank *bk, const float *x, int64_t n, int mode, float *snr, int64_t ld,
                float *mx, int32_t *am, hipStream_t st) {
    DeviceGuard guard(bk->device);
    const float *hist = bk->hist[bk->hist_cur];
    if (!bk->xlds) {
        int rc = ensure_xwin(bk, n + bk->dmax);
        if (rc) return rc;
        HIPCHK(launch_window_fill(bk->xwin, hist, x, n, bk->dmax, st));
    }
    for (int64_t P = 0; P < n; P += bk->max_block) {
        const int64_t np = std::min<int64_t>(bk->max_block, n - P);
        FwdArgs a = bk->base_args();
        a.state = bk->state;
        a.x = x;
        a.hist = hist;
        a.xwin = bk->xwin;
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
            a.keys = bk->keys;
            a.ld = bk->max_block;
        }
        int nseg = 1;
        if (bk->nseg > 1) {
            a.seg_len = ((np + bk->nseg - 1) / bk->nseg + bk->L - 1) / bk->L * bk->L;
            nseg = (int)((np + a.seg_len - 1) / a.seg_len);
        }
        KernelEvents ev;
        HIPCHK(timer_next(bk, &ev));
        if (nseg >= 2)
            HIPCHK(launch_forward_split(a, mode, bk->lay.fl, bk->tt, bk->xlds, nseg, bk->lds, bk->lds_carry,
                                        bk->slot_filter, st, ev));
        else
            HIPCHK(launch_forward(a, mode, bk->lay.fl, bk->tt, bk->xlds, bk->lay.groups, bk->lds, st, ev));
        if (mode == kModeKeys)
            HIPCHK(launch_finalize_keys(bk->keys, bk->lay.groups, bk->max_block, np, mx + P, am + P, st));
    }
    HIPCHK(launch_hist_update(hist, bk->hist[bk->hist_cur ^ 1], x, n, bk->dmax, st));
    bk->hist_cur ^= 1;
    return SPIIR_OK;
}

}  // namespace

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
    std::vector<float2 *> w;             // 1 <= r < top: w_r [T][B >> r]
    std::vector<float2 *> wh[2];         // 1 <= r <= top: interpolation history of w_r [T][hh]
    int cur = 0;
    float2 *w0 = nullptr;                // [T][B]: full-rate z for the max / argmax
    uint64_t *keys = nullptr;            // [chunks][B]
    float *h = nullptr, *g = nullptr;
    // the level banks run concurrently: each on its own stream, forked from the
    // caller's stream after the decimation and joined before the interpolation
    std::vector<hipStream_t> lstream;
    std::vector<hipEvent_t> ldone;
    hipEvent_t fork = nullptr;
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
    if (mr->fork) (void)hipEventDestroy(mr->fork);
    mr->lstream.clear();
    mr->ldone.clear();
    mr->fork = nullptr;
    for (auto *bk : mr->bank)
        if (bk) spiir_bank_destroy(bk);
    for (auto *p : mr->zrow) dfree(p);
    for (auto *p : mr->xbuf) dfree(p);
    for (int c = 0; c < 2; ++c) {
        for (auto *p : mr->dh[c]) dfree(p);
        for (auto *p : mr->wh[c]) dfree(p);
    }
    for (auto *p : mr->z) dfree(p);
    for (auto *p : mr->w) dfree(p);
    dfree(mr->w0);
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
// banks forked onto their streams, interpolation and sums, and the full-rate
// z (out0, row stride ld0) or the max / argmax (mx, am).
int mr_piece(spiir_multirate *mr, const float *x0, int64_t np, float2 *out0, int64_t ld0, float *mx, int32_t *am,
             hipStream_t st) {
    const int top = mr->top;
    const int c = mr->cur;
    std::vector<const float *> xs(top + 1);
    xs[0] = x0;
    for (int r = 1; r <= top; ++r) {
        HIPCHK(launch_mr_decimate(xs[r - 1], np >> (r - 1), mr->dh[c][r], mr->dh[c ^ 1][r], mr->h, mr->lh,
                                  mr->xbuf[r], st));
        xs[r] = mr->xbuf[r];
    }
    HIPCHK(hipEventRecord(mr->fork, st));
    for (int r = top; r >= 0; --r)   // the top level holds the most filters: start it first
        if (mr->bank[r]) {
            HIPCHK(hipStreamWaitEvent(mr->lstream[r], mr->fork, 0));
            const int rc = stream_call(mr->bank[r], xs[r], np >> r, kModeZ, reinterpret_cast<float *>(mr->z[r]),
                                       mr->B >> r, nullptr, nullptr, mr->lstream[r]);
            if (rc) return rc;
            HIPCHK(hipEventRecord(mr->ldone[r], mr->lstream[r]));
            HIPCHK(hipStreamWaitEvent(st, mr->ldone[r], 0));
        }
    if (!out0) {
        out0 = mr->w0;
        ld0 = mr->B;
    }
    if (top == 0) {
        HIPCHK(launch_mr_upsample_add(mr->z[0], mr->B, mr->zrow[0], nullptr, 0, nullptr, 0, nullptr, nullptr, 0,
                                      mr->g, mr->lg, out0, ld0, np, mr->T, st));
    } else {
        const float2 *src = mr->z[top];
        int64_t ld_src = mr->B >> top;
        const int32_t *srow = mr->zrow[top];
        for (int r = top - 1; r >= 0; --r) {
            float2 *dst = r == 0 ? out0 : mr->w[r];
            const int64_t ld_dst = r == 0 ? ld0 : (mr->B >> r);
            HIPCHK(launch_mr_upsample_add(mr->bank[r] ? mr->z[r] : nullptr, mr->B >> r, mr->zrow[r], src, ld_src,
                                          srow, np >> (r + 1), mr->wh[c][r + 1], mr->wh[c ^ 1][r + 1], mr->hh,
                                          mr->g, mr->lg, dst, ld_dst, np >> r, mr->T, st));
            src = dst;
            ld_src = ld_dst;
            srow = nullptr;
        }
    }
    if (mx) {
        HIPCHK(launch_mr_row_keys(mr->w0, mr->B, mr->T, np, mr->keys, mr->B, st));
        HIPCHK(launch_finalize_keys(mr->keys, mr_key_chunks(mr->T), mr->B, np, mx, am, st));
    }
    mr->cur ^= 1;
    return SPIIR_OK;
}

bool mr_timing_on(const spiir_multirate *mr) {
    for (auto *bk : mr->bank)
        if (bk && !bk->tev0.empty()) return true;
    return false;
}

// Captures a trigger piece of B samples for each history parity. The host-side
// parity flags (mr->cur and every level bank's history index) toggle once per
// captured piece, so after the two captures they are back where they were;
// on failure they are restored and graphs stay off.
int mr_build_graphs(spiir_multirate *mr) {
    std::vector<int> hc;
    for (auto *bk : mr->bank) hc.push_back(bk ? bk->hist_cur : 0);
    const int cur0 = mr->cur;
    auto restore = [&]() {
        mr->cur = cur0;
        for (size_t r = 0; r < mr->bank.size(); ++r)
            if (mr->bank[r]) mr->bank[r]->hist_cur = hc[r];
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
            HIPCHK(hipMemcpyAsync(mx + P, mr->mxo, (size_t)np * sizeof(float), hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(am + P, mr->amo, (size_t)np * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
            mr->cur ^= 1;
            for (auto *bk : mr->bank)
                if (bk) bk->hist_cur ^= 1;   // as the captured stream calls did
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

struct spiir_whitener {
    int device = 0;
    int N = 0, logN = 0, H = 0;
    int64_t B = 0;                 // most samples per piece (a multiple of H)
    double wsum2 = 0.0;            // sum of the squared window
    float *wtab = nullptr;         // [N] periodic Hann window
    float2 *tw = nullptr;          // [N/2] exp(-2 pi i k / N)
    double *S = nullptr;           // [H+1] PSD
    float *inv = nullptr;          // [H+1] 1 / sqrt(S)
    float *hist[2] = {nullptr, nullptr};  // last H input samples (double-buffered)
    float *pend[2] = {nullptr, nullptr};  // second half of the last frame's output
    int cur = 0;
    float *y = nullptr;            // [B/H][N] frame outputs
    float *pw = nullptr;           // [frames][H+1] power spectra of the PSD training frames
    int64_t pw_frames = 0;
    bool has_psd = false;
};

namespace {

void wh_free(spiir_whitener *wh) {
    dfree(wh->wtab);
    dfree(wh->tw);
    dfree(wh->S);
    dfree(wh->inv);
    for (int c = 0; c < 2; ++c) {
        dfree(wh->hist[c]);
        dfree(wh->pend[c]);
    }
    dfree(wh->y);
    dfree(wh->pw);
}

}  // namespace

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

int spiir_trigger_max_per_template(spiir_bank *bk, const float *x, int64_t n, float *mx, int32_t *am,
                                   float *snr, void *stream) {
    if (!bk) return fail(SPIIR_EINVAL, "bank is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n == 0) return SPIIR_OK;
    if (!x || !mx || !am || !snr) return fail(SPIIR_EINVAL, "null device pointer");
    DeviceGuard guard(bk->device);
    hipStream_t st = as_stream(stream);
    const float *hist = bk->hist[bk->hist_cur];
    if (!bk->xlds) {
        int rc = ensure_xwin(bk, n + bk->dmax);
        if (rc) return rc;
        HIPCHK(launch_window_fill(bk->xwin, hist, x, n, bk->dmax, st));
    }
    for (int64_t P = 0; P < n; P += bk->max_block) {
        const int64_t np = std::min<int64_t>(bk->max_block, n - P);
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
            HIPCHK(launch_forward(a, kModeSnr, bk->lay.fl, bk->tt, bk->xlds, 1, bk->lds, st));
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
        tp->nchunks = (n + bk->L - 1) / bk->L;
        hipError_t e = dalloc(&tp->xwin, (size_t)(n + bk->dmax) + 16);  // read-ahead padding
        if (e == hipSuccess && tape_out) e = dalloc(&tp->tape, (size_t)(tp->nchunks * bk->lay.nslots));
        if (e != hipSuccess) {
            dfree(tp->xwin);
            dfree(tp->tape);
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
        a.tape = tp ? tp->tape : nullptr;
        a.chunk0 = P / bk->L;
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
    if (!tp->tape) return fail(SPIIR_ESTATE, "tape holds no carries");
    DeviceGuard guard(bk->device);
    BwdArgs a;
    std::memset(&a, 0, sizeof a);
    a.s = bk->slots();
    a.rows = bk->rows;
    a.slot_filter = bk->slot_filter;
    a.tape = tp->tape;
    a.xwin = tp->xwin;
    a.gz = reinterpret_cast<const float2 *>(gz);
    // time segments: enough waves for about 8 per SIMD, at most 16 segments
    const int64_t nch = (tp->n + bk->L - 1) / bk->L;
    int want = 1;
    if (bk->tsplit_opt >= 2) {
        want = bk->tsplit_opt;
    } else if (bk->tsplit_opt == 0) {
        // counted in layout waves (the per-segment kernel runs FL times as many): on the
        // chirp-fit bank 16 segments of 4-filter lanes ran faster than 4
        const int64_t waves = std::max<int64_t>(1, (int64_t)bk->lay.groups * bk->lay.wpg);
        const int64_t target = (int64_t)32 * bk->dev.n_cu;
        want = (int)std::min<int64_t>(16, (target + waves - 1) / waves);
    }
    want = (int)std::max<int64_t>(1, std::min<int64_t>(want, nch));
    const int64_t seg_chunks = (nch + want - 1) / want;
    const int nseg = (int)((nch + seg_chunks - 1) / seg_chunks);
    const int64_t S = bk->lay.nslots;
    if (bk->bwd_cap < nseg) {
        dfree(bk->ysub);
        dfree(bk->blam);
        dfree(bk->bgpart);
        bk->bwd_cap = 0;
        hipError_t e = dalloc(&bk->ysub, (size_t)nseg * ((bk->L + kSub - 1) / kSub) * S);
        if (e == hipSuccess) e = dalloc(&bk->blam, (size_t)2 * nseg * S);
        if (e == hipSuccess) e = dalloc(&bk->bgpart, (size_t)2 * nseg * S);
        if (e != hipSuccess) {
            dfree(bk->ysub);
            dfree(bk->blam);
            dfree(bk->bgpart);
            return fail(SPIIR_ENOMEM, "adjoint scratch allocation failed: %s", hipGetErrorString(e));
        }
        bk->bwd_cap = nseg;
    }
    a.ysub = bk->ysub;
    a.lam_loc = bk->blam;
    a.lam_in = bk->blam + (size_t)nseg * S;
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
    HIPCHK(launch_backward(a, bk->lay.fl, bk->lay.groups, as_stream(stream)));
    return SPIIR_OK;
}

int spiir_tape_destroy(spiir_tape *tp) {
    if (!tp) return SPIIR_OK;
    dfree(tp->tape);
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

namespace {

constexpr int64_t kMaxClusterN = (int64_t)1 << 40;

// gfx950 check of a device, cached per ordinal for the process.
int cluster_device(int32_t device, int &dev) {
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

}  // namespace

}  // extern "C"

// Streaming trigger clustering: a window of the series, [base, base + len),
// holds the samples whose triggers are not final yet plus W samples before
// them; each push appends a block, clusters the window with candidates
// limited to the newly final samples [final_end, total - W) and keeps the
// last W samples before the new final_end (ping-pong buffers).
struct spiir_trigger_stream {
    int device = 0;
    float thr = 0.0f;
    int64_t W = 0, B = 0;
    float *wm[2] = {nullptr, nullptr};
    int32_t *wj[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t base = 0, len = 0, total = 0, final_end = 0;
    void *ws = nullptr;
    size_t ws_bytes = 0;
};

namespace {

void ts_free(spiir_trigger_stream *ts) {
    for (int c = 0; c < 2; ++c) {
        dfree(ts->wm[c]);
        dfree(ts->wj[c]);
    }
    if (ts->ws) (void)hipFree(ts->ws);
    ts->ws = nullptr;
}

// Clusters the window with candidates [final_end, new_end) and slides it.
int ts_step(spiir_trigger_stream *ts, int64_t new_end, int64_t *idx, int32_t *tpl, float *val, int64_t cap,
            int64_t *count, hipStream_t st) {
    const int c = ts->cur;
    HIPCHK(launch_cluster(ts->wm[c], ts->wj[c], ts->len, ts->thr, ts->W, ts->ws, cap, idx, tpl, val, count, st,
                          ts->final_end - ts->base, new_end - ts->base, ts->base));
    ts->final_end = new_end;
    const int64_t keep_from = std::max(ts->base, ts->final_end - ts->W) - ts->base;
    const int64_t keep = ts->len - keep_from;
    if (keep > 0) {
        HIPCHK(hipMemcpyAsync(ts->wm[c ^ 1], ts->wm[c] + keep_from, (size_t)keep * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(ts->wj[c ^ 1], ts->wj[c] + keep_from, (size_t)keep * sizeof(int32_t),
                              hipMemcpyDeviceToDevice, st));
    }
    ts->cur ^= 1;
    ts->base += keep_from;
    ts->len = keep;
    return SPIIR_OK;
}

}  // namespace

extern "C" {

int spiir_trigger_stream_create(spiir_trigger_stream **out, float threshold, int32_t window, int64_t max_block,
                                int32_t device) {
    if (!out) return fail(SPIIR_EINVAL, "out is null");
    *out = nullptr;
    if (window < 0) return fail(SPIIR_EINVAL, "window must be >= 0 (got %d)", window);
    if (max_block < 1 || max_block > ((int64_t)1 << 32))
        return fail(SPIIR_EINVAL, "max_block must be in [1, 2^32] (got %lld)", (long long)max_block);
    int dev = 0;
    int rc = cluster_device(device, dev);
    if (rc) return rc;
    DeviceGuard guard(dev);
    spiir_trigger_stream *ts = new (std::nothrow) spiir_trigger_stream();
    if (!ts) return fail(SPIIR_ENOMEM, "out of host memory");
    ts->device = dev;
    ts->thr = threshold;
    ts->W = window;
    ts->B = max_block;
    const int64_t cap = 2 * (int64_t)window + max_block;   // the window never holds more
    ts->ws_bytes = cluster_workspace_bytes(cap);
    hipError_t e = hipSuccess;
    for (int c = 0; c < 2 && e == hipSuccess; ++c) {
        e = dalloc(&ts->wm[c], (size_t)cap);
        if (e == hipSuccess) e = dalloc(&ts->wj[c], (size_t)cap);
    }
    if (e == hipSuccess) e = hipMalloc(&ts->ws, std::max<size_t>(256, ts->ws_bytes));
    if (e != hipSuccess) {
        ts_free(ts);
        delete ts;
        return fail(SPIIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    *out = ts;
    return SPIIR_OK;
}

int spiir_trigger_stream_destroy(spiir_trigger_stream *ts) {
    if (!ts) return SPIIR_OK;
    {
        DeviceGuard guard(ts->device);
        (void)hipDeviceSynchronize();
        ts_free(ts);
    }
    delete ts;
    return SPIIR_OK;
}

int spiir_trigger_stream_reset(spiir_trigger_stream *ts, void *stream) {
    if (!ts) return fail(SPIIR_EINVAL, "trigger stream is null");
    (void)stream;   // no device state to clear: the window is rebuilt from the next push
    ts->cur = 0;
    ts->base = ts->len = ts->total = ts->final_end = 0;
    return SPIIR_OK;
}

static int ts_check_out(int64_t *idx, int32_t *tpl, float *val, int64_t cap, int64_t *count) {
    if (!count) return fail(SPIIR_EINVAL, "count_dev is null");
    if (cap < 0) return fail(SPIIR_EINVAL, "capacity must be >= 0");
    if (cap > 0 && (!idx || !tpl || !val)) return fail(SPIIR_EINVAL, "null output array with capacity %lld",
                                                     (long long)cap);
    return SPIIR_OK;
}

int spiir_trigger_stream_push(spiir_trigger_stream *ts, const float *max_dev, const int32_t *argmax_dev, int64_t n,
                              int64_t *index_dev, int32_t *template_dev, float *snr_dev, int64_t capacity,
                              int64_t *count_dev, void *stream) {
    if (!ts) return fail(SPIIR_EINVAL, "trigger stream is null");
    int rc = ts_check_out(index_dev, template_dev, snr_dev, capacity, count_dev);
    if (rc) return rc;
    if (n < 0 || n > ts->B) return fail(SPIIR_EINVAL, "n must be in [0, max_block = %lld] (got %lld)",
                                        (long long)ts->B, (long long)n);
    if (n > 0 && (!max_dev || !argmax_dev)) return fail(SPIIR_EINVAL, "null max / argmax block");
    DeviceGuard guard(ts->device);
    hipStream_t st = as_stream(stream);
    const int c = ts->cur;
    if (n > 0) {
        HIPCHK(hipMemcpyAsync(ts->wm[c] + ts->len, max_dev, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(ts->wj[c] + ts->len, argmax_dev, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice,
                              st));
    }
    ts->len += n;
    ts->total += n;
    const int64_t new_end = std::max(ts->final_end, ts->total - ts->W);
    return ts_step(ts, new_end, index_dev, template_dev, snr_dev, capacity, count_dev, st);
}

int spiir_trigger_stream_flush(spiir_trigger_stream *ts, int64_t *index_dev, int32_t *template_dev, float *snr_dev,
                               int64_t capacity, int64_t *count_dev, void *stream) {
    if (!ts) return fail(SPIIR_EINVAL, "trigger stream is null");
    int rc = ts_check_out(index_dev, template_dev, snr_dev, capacity, count_dev);
    if (rc) return rc;
    DeviceGuard guard(ts->device);
    return ts_step(ts, ts->total, index_dev, template_dev, snr_dev, capacity, count_dev, as_stream(stream));
}

int spiir_cluster_workspace_size(int64_t n, size_t *nbytes) {
    if (!nbytes) return fail(SPIIR_EINVAL, "null argument");
    if (n < 0 || n > kMaxClusterN) return fail(SPIIR_EINVAL, "n must be in [0, 2^40] (got %lld)", (long long)n);
    *nbytes = cluster_workspace_bytes(n);
    return SPIIR_OK;
}

int spiir_cluster_triggers(const float *max_dev, const int32_t *argmax_dev, int64_t n, float threshold,
                           int32_t window, void *workspace_dev, size_t workspace_bytes, int64_t *index_dev,
                           int32_t *template_dev, float *snr_dev, int64_t capacity, int64_t *count_dev,
                           int32_t device, void *stream) {
    if (!count_dev) return fail(SPIIR_EINVAL, "count_dev is null");
    if (n < 0 || n > kMaxClusterN) return fail(SPIIR_EINVAL, "n must be in [0, 2^40] (got %lld)", (long long)n);
    if (window < 0) return fail(SPIIR_EINVAL, "window must be >= 0 (got %d)", window);
    if (capacity < 0) return fail(SPIIR_EINVAL, "capacity must be >= 0");
    if (capacity > 0 && (!index_dev || !template_dev || !snr_dev))
        return fail(SPIIR_EINVAL, "null output array with capacity %lld", (long long)capacity);
    if (n > 0) {
        if (!max_dev || !argmax_dev) return fail(SPIIR_EINVAL, "null max / argmax series");
        if (!workspace_dev) return fail(SPIIR_EINVAL, "null workspace");
        const size_t need = cluster_workspace_bytes(n);
        if (workspace_bytes < need)
            return fail(SPIIR_EINVAL, "workspace of %zu bytes is below the %zu bytes needed for n = %lld",
                        workspace_bytes, need, (long long)n);
    }
    int dev = 0;
    const int rc = cluster_device(device, dev);
    if (rc) return rc;
    DeviceGuard guard(dev);
    HIPCHK(launch_cluster(max_dev, argmax_dev, n, threshold, window, workspace_dev, capacity, index_dev,
                          template_dev, snr_dev, count_dev, static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

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
    // interpolation launches one workgroup per (template, 1,024 outputs)
    if (((B + 1023) / 1024) * (int64_t)T > INT32_MAX)
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
    mr->bank.assign(R + 1, nullptr);
    mr->zrow.assign(R + 1, nullptr);
    mr->xbuf.assign(R + 1, nullptr);
    mr->z.assign(R + 1, nullptr);
    mr->w.assign(R + 1, nullptr);
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
    for (int r = 0; r <= R; ++r) {
        const int64_t *off = filter_offsets[r];
        std::vector<int32_t> row(T, -1);
        std::vector<int64_t> offc(1, 0);
        for (int j = 0; j < T; ++j)
            if (off[j + 1] > off[j]) {
                row[j] = (int32_t)(offc.size() - 1);
                offc.push_back(off[j + 1]);
            }
        hipError_t e = dalloc(&mr->zrow[r], (size_t)T);
        if (e != hipSuccess) return alloc_fail(e);
        e = hipMemcpy(mr->zrow[r], row.data(), T * sizeof(int32_t), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "row map upload");
        if (off[T] == 0) continue;
        spiir_bank_opts orr = o;
        orr.device = dev;
        orr.max_block = (int32_t)std::max<int64_t>(8, B >> r);
        // a level whose filters leave most of the device idle is a short serial
        // recursion per call: let the automatic time split cut it into up to 32
        // segments, with 64-sample chunks so that segments can be that short
        const bool small = o.time_split == 0 && off[T] <= 128 * (int64_t)df.n_cu;
        if (small) orr.chunk_len = 64;
        spiir_bank *bk = nullptr;
        rc = orr.autotune ? spiir_bank_create(&bk, (int32_t)(offc.size() - 1), offc.data(), a[r], b[r], d[r], &orr)
                          : create_bank(&bk, (int32_t)(offc.size() - 1), offc.data(), a[r], b[r], d[r], orr,
                                        small ? 32 : 8);
        if (rc) {
            g_err = "level " + std::to_string(r) + ": " + g_err;
            return bail(rc);
        }
        mr->bank[r] = bk;
        e = dalloc(&mr->z[r], (size_t)(offc.size() - 1) * (size_t)(B >> r));
        if (e != hipSuccess) return alloc_fail(e);
    }
    for (int r = 1; r <= top; ++r) {
        hipError_t e = dalloc(&mr->xbuf[r], (size_t)(B >> r));
        for (int c = 0; c < 2 && e == hipSuccess; ++c) {
            e = dalloc(&mr->dh[c][r], (size_t)std::max(1, mr->lh - 1));
            if (e == hipSuccess) e = dalloc(&mr->wh[c][r], (size_t)T * std::max(1, mr->hh));
        }
        if (e == hipSuccess && r < top) e = dalloc(&mr->w[r], (size_t)T * (size_t)(B >> r));
        if (e != hipSuccess) return alloc_fail(e);
    }
    {
        hipError_t e = dalloc(&mr->w0, (size_t)T * (size_t)B);
        if (e == hipSuccess) e = dalloc(&mr->keys, (size_t)mr_key_chunks(T) * (size_t)B);
        if (e == hipSuccess) e = dalloc(&mr->h, (size_t)mr->lh);
        if (e == hipSuccess) e = dalloc(&mr->g, (size_t)mr->lg);
        if (e != hipSuccess) return alloc_fail(e);
    }
    mr->lstream.assign(R + 1, nullptr);
    mr->ldone.assign(R + 1, nullptr);
    {
        hipError_t e = hipEventCreateWithFlags(&mr->fork, hipEventDisableTiming);
        for (int r = 0; r <= R && e == hipSuccess; ++r)
            if (mr->bank[r]) {
                e = hipStreamCreateWithFlags(&mr->lstream[r], hipStreamNonBlocking);
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
            bk->hist_cur = 0;
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

int spiir_whitener_create(spiir_whitener **out, int32_t frame_len, int32_t max_block, int32_t device) {
    if (!out) return fail(SPIIR_EINVAL, "out is null");
    *out = nullptr;
    int logn = 0;
    while ((1 << logn) < frame_len) ++logn;
    if (frame_len < 16 || frame_len > 8192 || (1 << logn) != frame_len)
        return fail(SPIIR_EINVAL, "frame_len must be a power of two in [16, 8192] (got %d)", frame_len);
    if (max_block < 0) return fail(SPIIR_EINVAL, "max_block must be >= 0");
    const int H = frame_len / 2;
    int64_t B = max_block ? max_block : 65536;
    B = std::max<int64_t>(H, B / H * H);
    int dev = device;
    if (dev < 0) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) return fail(SPIIR_ENODEV, "no HIP device available");
        HIPCHK(hipGetDevice(&dev));
    }
    DeviceFacts df;
    int rc = device_facts(dev, df);
    if (rc) return rc;
    DeviceGuard guard(dev);
    spiir_whitener *wh = new (std::nothrow) spiir_whitener();
    if (!wh) return fail(SPIIR_ENOMEM, "out of host memory");
    wh->device = dev;
    wh->N = frame_len;
    wh->logN = logn;
    wh->H = H;
    wh->B = B;
    auto bail = [&](int code) {
        (void)hipDeviceSynchronize();
        wh_free(wh);
        delete wh;
        return code;
    };
    hipError_t e = dalloc(&wh->wtab, (size_t)frame_len);
    if (e == hipSuccess) e = dalloc(&wh->tw, (size_t)H);
    if (e == hipSuccess) e = dalloc(&wh->S, (size_t)H + 1);
    if (e == hipSuccess) e = dalloc(&wh->inv, (size_t)H + 1);
    for (int c = 0; c < 2 && e == hipSuccess; ++c) {
        e = dalloc(&wh->hist[c], (size_t)H);
        if (e == hipSuccess) e = dalloc(&wh->pend[c], (size_t)H);
    }
    if (e == hipSuccess) e = dalloc(&wh->y, (size_t)(B / H) * (size_t)frame_len);
    if (e != hipSuccess) return bail(fail(SPIIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e)));
    std::vector<float> w(frame_len);
    std::vector<float2> tw(H);
    double ws = 0.0;
    for (int t = 0; t < frame_len; ++t) {
        const double s1 = std::sin(M_PI * t / frame_len);
        w[t] = (float)(s1 * s1);
        ws += (s1 * s1) * (s1 * s1);
    }
    for (int k = 0; k < H; ++k) {
        const double ang = -2.0 * M_PI * k / frame_len;
        tw[k] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    wh->wsum2 = ws;
    e = hipMemcpy(wh->wtab, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(wh->tw, tw.data(), tw.size() * sizeof(float2), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(fail(SPIIR_EHIP, "window upload: %s", hipGetErrorString(e)));
    for (int c = 0; c < 2; ++c) {
        if (launch_fill_zero(wh->hist[c], (size_t)H * sizeof(float), nullptr) != hipSuccess ||
            launch_fill_zero(wh->pend[c], (size_t)H * sizeof(float), nullptr) != hipSuccess)
            return bail(fail(SPIIR_EHIP, "history clear failed"));
    }
    e = hipDeviceSynchronize();
    if (e != hipSuccess) return bail(fail(SPIIR_EHIP, "whitener set-up: %s", hipGetErrorString(e)));
    *out = wh;
    return SPIIR_OK;
}

int spiir_whitener_destroy(spiir_whitener *wh) {
    if (!wh) return SPIIR_OK;
    {
        DeviceGuard guard(wh->device);
        (void)hipDeviceSynchronize();
        wh_free(wh);
    }
    delete wh;
    return SPIIR_OK;
}

int spiir_whitener_estimate_psd(spiir_whitener *wh, const float *train, int64_t n, void *stream) {
    if (!wh) return fail(SPIIR_EINVAL, "whitener is null");
    if (!train) return fail(SPIIR_EINVAL, "null device pointer");
    if (n < wh->N) return fail(SPIIR_EINVAL, "training stretch of %lld samples is shorter than a frame (%d)",
                               (long long)n, wh->N);
    DeviceGuard guard(wh->device);
    hipStream_t st = as_stream(stream);
    const int64_t K = (n - wh->N) / wh->H + 1;
    if (K > INT32_MAX) return fail(SPIIR_EINVAL, "training stretch of %lld frames is too long", (long long)K);
    if (K > wh->pw_frames) {
        HIPCHK(hipStreamSynchronize(st));
        dfree(wh->pw);
        wh->pw_frames = 0;
        hipError_t e = dalloc(&wh->pw, (size_t)K * (size_t)(wh->H + 1));
        if (e != hipSuccess) return fail(SPIIR_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
        wh->pw_frames = K;
    }
    HIPCHK(launch_wh_frames(true, nullptr, 0, train, wh->wtab, wh->tw, wh->N, wh->logN, nullptr, nullptr, wh->pw, K,
                            st));
    HIPCHK(launch_wh_psd_reduce(wh->pw, K, wh->H, wh->wsum2, wh->S, wh->inv, st));
    wh->has_psd = true;
    return SPIIR_OK;
}

int spiir_whitener_set_psd(spiir_whitener *wh, const double *psd) {
    if (!wh || !psd) return fail(SPIIR_EINVAL, "null argument");
    for (int f = 0; f <= wh->H; ++f)
        if (!std::isfinite(psd[f]) || psd[f] < 0.0) return fail(SPIIR_EINVAL, "psd[%d] is negative or not finite", f);
    DeviceGuard guard(wh->device);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(wh->S, psd, (size_t)(wh->H + 1) * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(launch_wh_inv(wh->S, wh->H, wh->inv, nullptr));
    HIPCHK(hipDeviceSynchronize());
    wh->has_psd = true;
    return SPIIR_OK;
}

int spiir_whitener_get_psd(spiir_whitener *wh, double *psd) {
    if (!wh || !psd) return fail(SPIIR_EINVAL, "null argument");
    if (!wh->has_psd) return fail(SPIIR_ESTATE, "no PSD set or estimated");
    DeviceGuard guard(wh->device);
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(psd, wh->S, (size_t)(wh->H + 1) * sizeof(double), hipMemcpyDeviceToHost));
    return SPIIR_OK;
}

int spiir_whitener_reset(spiir_whitener *wh, void *stream) {
    if (!wh) return fail(SPIIR_EINVAL, "whitener is null");
    DeviceGuard guard(wh->device);
    hipStream_t st = as_stream(stream);
    for (int c = 0; c < 2; ++c) {
        HIPCHK(launch_fill_zero(wh->hist[c], (size_t)wh->H * sizeof(float), st));
        HIPCHK(launch_fill_zero(wh->pend[c], (size_t)wh->H * sizeof(float), st));
    }
    wh->cur = 0;
    return SPIIR_OK;
}

int spiir_whitener_process(spiir_whitener *wh, const float *x, int64_t n, float *out, void *stream) {
    if (!wh) return fail(SPIIR_EINVAL, "whitener is null");
    if (n < 0) return fail(SPIIR_EINVAL, "n must be >= 0");
    if (n % wh->H) return fail(SPIIR_EINVAL, "n (%lld) must be a multiple of half the frame (%d)", (long long)n, wh->H);
    if (!wh->has_psd) return fail(SPIIR_ESTATE, "no PSD set or estimated");
    if (n == 0) return SPIIR_OK;
    if (!x || !out) return fail(SPIIR_EINVAL, "null device pointer");
    DeviceGuard guard(wh->device);
    hipStream_t st = as_stream(stream);
    for (int64_t P = 0; P < n; P += wh->B) {
        const int64_t np = std::min<int64_t>(wh->B, n - P);
        const int64_t nf = np / wh->H;
        const int c = wh->cur;
        HIPCHK(launch_wh_frames(false, wh->hist[c], wh->H, x + P, wh->wtab, wh->tw, wh->N, wh->logN, wh->inv, wh->y,
                                nullptr, nf, st));
        HIPCHK(launch_wh_ola(wh->y, nf, wh->N, wh->pend[c], wh->pend[c ^ 1], x + P, np, wh->hist[c ^ 1], out + P, st));
        wh->cur ^= 1;
    }
    return SPIIR_OK;
}

const char *spiir_version(void) { return "spiir-mi355x 0.1.0 (gfx950)"; }

}  // extern "C"
