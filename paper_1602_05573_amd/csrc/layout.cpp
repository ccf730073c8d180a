// Host-side plan of a filter bank (declared in layout.h). No HIP calls: the
// library links it, and the tests build it with g++ under AddressSanitizer
// and UBSan.
#include "layout.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <tuple>

namespace spiir {
namespace layout {

namespace {

int bad(std::string &err, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int bad(std::string &err, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return SPIIR_EINVAL;
}

// Places the filters ks of one template (or part) into its rows r0 .. r0+nr-1 of
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
// gather in few passes. Padding lanes read the address of their column's first
// lane (a broadcast).
void deal_template(const std::vector<int32_t> &ks, const int32_t *d, int g, int wpg, int fl, int r0, int nr,
                   Layout &lay) {
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
    for (int32_t k : ks) bycls[d[k] & 31].push_back(k);
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

}  // namespace

void cpow(double re, double im, long e, double &out_re, double &out_im) {
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
    out_re = rr;
    out_im = ri;
}

int rows_of(int64_t k, int fl) { return (int)((k + kRowLanes * fl - 1) / (kRowLanes * fl)); }

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

int choose_fl(int T, const int64_t *off, int n_cu) {
    for (int fl = 4; fl >= 1; --fl) {
        const Plan p = plan_rows(T, off, fl);
        if (p.max_nr > 4 * kMaxWaves) return std::min(4, fl + 1);
        if ((p.total_rows + 3) / 4 >= (int64_t)7 * n_cu) return fl;
    }
    return 1;
}

size_t fwd_lds_bytes(int wpg, int dmax, int nb, bool x_in_lds, int tt) {
    const size_t win = x_in_lds ? (size_t)((dmax + nb + tt + 3) & ~3) * 4 : 0;
    return win + (size_t)wpg * tt * 64 * 8 + ((size_t)2 * tt * (4 * wpg + 1) + 16) * 8 + (size_t)2 * tt * 8;
}

// The strain window (max_delay + nb samples) in LDS when it fits, and 16-step
// tiles when they fit beside it. The forward kernel closes a chunk (FP64
// carry correction, tape entry) only at a tile end, so the tile length must
// divide L: chunk lengths that are not a multiple of 16 take 8-step tiles.
Geometry plan_geometry(int wpg, int dmax, int L, int max_block, size_t lds_cap) {
    Geometry best;
    bool have = false;
    for (int tt : {16, 8}) {
        if (L % tt) continue;
        Geometry g;
        g.tt = tt;
        const int64_t fixed = (int64_t)fwd_lds_bytes(wpg, 0, 0, false, tt);
        int64_t nb = ((int64_t)lds_cap - fixed - 4 * (int64_t)(dmax + tt) - 64) / (4 * L) * L;
        nb = std::min<int64_t>(nb, max_block);
        g.xlds = nb >= L;
        g.nb = g.xlds ? (int)nb : max_block;
        g.lds = fwd_lds_bytes(wpg, dmax, g.nb, g.xlds, tt);
        if (!have) {
            best = g;
            have = true;
            if (!g.xlds || g.nb >= std::min(max_block, 2048)) return g;
        } else if (g.xlds && (!best.xlds || g.nb > best.nb)) {
            return g;
        }
    }
    return best;
}

int check_bank_args(int32_t T, const int64_t *off, const double *a, const double *b, const int32_t *d,
                    const spiir_bank_opts &o, int &dmax_out, std::string &err) {
    if (T < 1) return bad(err, "n_templates must be >= 1 (got %d)", T);
    if (!off || !a || !b || !d) return bad(err, "null coefficient / offset / delay array");
    if (off[0] != 0) return bad(err, "filter_offsets[0] must be 0");
    for (int j = 0; j < T; ++j)
        if (off[j + 1] <= off[j]) return bad(err, "template %d has no filters (offsets must strictly increase)", j);
    const int64_t F = off[T];
    if (F > (int64_t)INT32_MAX) return bad(err, "too many filters (%lld)", (long long)F);
    int dm = 0;
    for (int64_t k = 0; k < F; ++k) {
        const double ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
        if (!std::isfinite(ar) || !std::isfinite(ai) || !std::isfinite(br) || !std::isfinite(bi))
            return bad(err, "filter %lld has a non-finite coefficient", (long long)k);
        if (std::hypot(ar, ai) >= 1.0)
            return bad(err, "filter %lld is not stable: |a| = %.17g >= 1", (long long)k, std::hypot(ar, ai));
        if (d[k] < 0) return bad(err, "filter %lld has a negative delay", (long long)k);
        dm = std::max(dm, d[k]);
    }
    if (o.max_delay < 0) return bad(err, "max_delay must be >= 0");
    if (o.max_delay > 0 && dm > o.max_delay) return bad(err, "a delay (%d) exceeds max_delay (%d)", dm, o.max_delay);
    const int dmax = o.max_delay > 0 ? o.max_delay : dm;
    if (dmax > (1 << 26)) return bad(err, "max_delay %d too large", dmax);
    if (o.chunk_len != 0 && (o.chunk_len < 8 || o.chunk_len > 4096 || o.chunk_len % 8))
        return bad(err, "chunk_len must be a multiple of 8 in [8, 4096] (got %d)", o.chunk_len);
    if (o.filters_per_lane < 0 || o.filters_per_lane > 4)
        return bad(err, "filters_per_lane must be 0..4 (got %d)", o.filters_per_lane);
    if (o.precision < 0 || o.precision > 2) return bad(err, "precision must be 0, 1 or 2");
    if (o.max_block < 0) return bad(err, "max_block must be >= 0");
    if (o.waves_per_group < 0 || o.waves_per_group > kMaxWaves)
        return bad(err, "waves_per_group must be 0..%d", kMaxWaves);
    if (o.time_split < 0 || o.time_split > 32) return bad(err, "time_split must be 0..32");
    if (o.delay_band < 0) return bad(err, "delay_band must be 0 (no bands) or a band width >= 1");
    dmax_out = dmax;
    return SPIIR_OK;
}

int build_layout(int T, const int64_t *off, const int32_t *d, int fl, int wpg, int band, Layout &lay,
                 std::string &err) {
    (void)err;
    const int R = 4 * wpg;
    const int64_t row_cap = (int64_t)kRowLanes * fl;   // filters per row
    // packing items: a whole template, or one part of a split template; with
    // delay bands every item holds filters of one band only
    struct Item {
        int tpl, part, nr, band;
        std::vector<int32_t> ks;
    };
    std::vector<Item> items;
    std::vector<int> first_part((size_t)T, -1);
    lay.n_parts = 0;
    lay.part_tpl.clear();
    lay.split_tpl.clear();
    lay.split_off.assign(1, 0);
    lay.band = band;
    for (int j = 0; j < T; ++j) {
        // the template's filters by band (one piece without bands), in filter order
        std::vector<std::vector<int32_t>> pieces;
        std::vector<int> piece_band;
        if (band <= 0) {
            pieces.emplace_back();
            piece_band.push_back(0);
            for (int64_t k = off[j]; k < off[j + 1]; ++k) pieces.back().push_back((int32_t)k);
        } else {
            std::vector<std::pair<int, int32_t>> bk;
            for (int64_t k = off[j]; k < off[j + 1]; ++k) bk.emplace_back(d[k] / band, (int32_t)k);
            std::stable_sort(bk.begin(), bk.end(),
                             [](const std::pair<int, int32_t> &x, const std::pair<int, int32_t> &y) {
                                 return x.first < y.first;
                             });
            for (size_t i = 0; i < bk.size(); ++i) {
                if (i == 0 || bk[i].first != bk[i - 1].first) {
                    pieces.emplace_back();
                    piece_band.push_back(bk[i].first);
                }
                pieces.back().push_back(bk[i].second);
            }
        }
        // pieces longer than a workgroup are cut into balanced row counts
        std::vector<Item> mine;
        for (size_t q = 0; q < pieces.size(); ++q) {
            const std::vector<int32_t> &pk = pieces[q];
            const int nr = rows_of((int64_t)pk.size(), fl);
            const int np = (nr + R - 1) / R;
            size_t at = 0;
            int done = 0;
            for (int c = 0; c < np; ++c) {
                const int rq = (nr - done + (np - c) - 1) / (np - c);
                const size_t to = std::min(pk.size(), at + (size_t)(rq * row_cap));
                Item it;
                it.tpl = j;
                it.part = -1;
                it.band = piece_band[q];
                it.ks.assign(pk.begin() + (long)at, pk.begin() + (long)to);
                it.nr = rows_of((int64_t)it.ks.size(), fl);
                mine.push_back(std::move(it));
                done += rq;
                at = to;
            }
        }
        if (mine.size() > 1) {
            lay.split_tpl.push_back(j);
            first_part[(size_t)j] = lay.n_parts;
            for (Item &it : mine) {
                it.part = lay.n_parts++;
                lay.part_tpl.push_back(j);
            }
            lay.split_off.push_back(lay.n_parts);
        }
        for (Item &it : mine) items.push_back(std::move(it));
    }
    // first-fit decreasing per band: a workgroup holds filters of one band
    std::vector<int> order(items.size());
    for (size_t i = 0; i < items.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return items[x].band != items[y].band ? items[x].band < items[y].band : items[x].nr > items[y].nr;
    });
    std::vector<int> room, gband;           // free rows and band per group
    std::vector<std::vector<int>> members;  // items per group
    size_t band_first = 0;                  // first group of the current band
    for (size_t oi = 0; oi < order.size(); ++oi) {
        const int i = order[oi];
        if (oi > 0 && items[i].band != items[order[oi - 1]].band) band_first = room.size();
        size_t g = band_first;
        for (; g < room.size(); ++g)
            if (room[g] >= items[i].nr) break;
        if (g == room.size()) {
            room.push_back(R);
            gband.push_back(items[i].band);
            members.emplace_back();
        }
        room[g] -= items[i].nr;
        members[g].push_back(i);
    }
    lay.fl = fl;
    lay.wpg = wpg;
    lay.groups = (int)members.size();
    lay.nslots = (int64_t)lay.groups * wpg * fl * 64;
    lay.rows.assign((size_t)lay.groups * R, RowInfo{-1, 0, 0, -1});
    lay.slot_filter.assign((size_t)lay.nslots, -1);
    lay.pad_src.assign((size_t)lay.nslots, -1);
    lay.tpl_group.assign(T, -1);
    lay.group_lo.assign((size_t)lay.groups, 0);
    for (int g = 0; g < lay.groups; ++g) {
        lay.group_lo[(size_t)g] = band > 0 ? gband[(size_t)g] * band : 0;
        std::vector<int> &mem = members[g];
        std::sort(mem.begin(), mem.end());   // items are in template order, parts in part order
        int r0 = 0;
        for (int i : mem) {
            const Item &it = items[i];
            if (it.part < 0 || it.part == first_part[(size_t)it.tpl]) lay.tpl_group[it.tpl] = g;
            for (int r = 0; r < it.nr; ++r)
                lay.rows[(size_t)g * R + r0 + r] = RowInfo{it.tpl, r0, it.nr, it.part};
            deal_template(it.ks, d, g, wpg, fl, r0, it.nr, lay);
            r0 += it.nr;
        }
    }
    return SPIIR_OK;
}

void slot_arrays(const Layout &lay, const double *a, const double *b, const int32_t *d, int dmax, int L,
                 SlotHost &o) {
    const size_t S = (size_t)lay.nslots;
    o.a32.assign(S, F2{0.f, 0.f});
    o.b32.assign(S, F2{0.f, 0.f});
    o.xoff.assign(S, 0);
    o.flags.assign(S, 0);
    o.aL.assign(S, D2{0.0, 0.0});
    o.dL.assign(S, D2{0.0, 0.0});
    o.a64.assign(S, D2{0.0, 0.0});
    for (size_t s = 0; s < S; ++s) {
        const int32_t k = lay.slot_filter[s];
        if (k < 0) {
            const int64_t src = lay.pad_src[s];
            if (src >= 0) o.xoff[s] = dmax - d[lay.slot_filter[(size_t)src]];
            continue;
        }
        const double ar = a[2 * (size_t)k], ai = a[2 * (size_t)k + 1];
        const float far = (float)ar, fai = (float)ai;
        o.a32[s] = F2{far, fai};
        o.b32[s] = F2{(float)b[2 * (size_t)k], (float)b[2 * (size_t)k + 1]};
        o.xoff[s] = dmax - d[k];
        double pr, pi, qr, qi;
        cpow(ar, ai, L, pr, pi);
        cpow((double)far, (double)fai, L, qr, qi);
        o.aL[s] = D2{pr, pi};
        o.dL[s] = D2{pr - qr, pi - qi};
        o.a64[s] = D2{ar, ai};
        o.flags[s] = std::hypot(ar, ai) > 1.0 - 1e-5 ? 1 : 0;
    }
}

}  // namespace layout
}  // namespace spiir
