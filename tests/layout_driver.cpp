// CPU check of the bank plan (layout.cpp): random banks through the argument
// checks, the slot layout, the per-slot coefficient arrays and the LDS
// geometry, with every structural invariant the kernels rely on asserted.
// Built by tests/test_layout_sanitized.py with g++ under AddressSanitizer and
// UBSan; exits non-zero on the first violated invariant.
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "layout.h"

using namespace spiir;
using namespace spiir::layout;

namespace {

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
    uint64_t next() {
        s ^= s << 13;
        s ^= s >> 7;
        s ^= s << 17;
        return s;
    }
    int uni(int lo, int hi) { return lo + (int)(next() % (uint64_t)(hi - lo + 1)); }
    double u01() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

int g_fail = 0;

#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            g_fail = 1;                                   \
            return;                                       \
        }                                                 \
    } while (0)

struct TestBank {
    int T = 0;
    std::vector<int64_t> off;
    std::vector<double> a, b;
    std::vector<int32_t> d;
    int dmax = 0;
};

TestBank random_bank(Rng &r, int T, int klo, int khi, int dmax) {
    TestBank tb;
    tb.T = T;
    tb.off.assign(1, 0);
    for (int j = 0; j < T; ++j) {
        int k = r.uni(klo, khi);
        tb.off.push_back(tb.off.back() + k);
    }
    const int64_t F = tb.off.back();
    tb.dmax = dmax;
    for (int64_t k = 0; k < F; ++k) {
        const double rad = 0.5 + 0.49999 * r.u01(), w = 3.14159 * r.u01();
        tb.a.push_back(rad * std::cos(w));
        tb.a.push_back(rad * std::sin(w));
        tb.b.push_back(r.u01() - 0.5);
        tb.b.push_back(r.u01() - 0.5);
        tb.d.push_back(r.uni(0, dmax));
    }
    return tb;
}

void check_layout(const TestBank &tb, int fl, int wpg, int L, int band) {
    Layout lay;
    std::string err;
    const int T = tb.T;
    const int rc = build_layout(T, tb.off.data(), tb.d.data(), fl, wpg, band, lay, err);
    CHECK(rc == SPIIR_OK, "build_layout failed: %s", err.c_str());
    const int R = 4 * wpg;
    // split templates: exactly those with more rows than a workgroup, parts consecutive
    std::vector<int> nparts(T, 0);
    CHECK(lay.split_off.size() == lay.split_tpl.size() + 1 && lay.split_off[0] == 0 &&
              lay.split_off.back() == lay.n_parts && (int)lay.part_tpl.size() == lay.n_parts,
          "part tables");
    for (size_t i = 0; i < lay.split_tpl.size(); ++i) {
        const int j = lay.split_tpl[i];
        CHECK(j >= 0 && j < T && (i == 0 || lay.split_tpl[i - 1] < j), "split template list");
        CHECK(lay.split_off[i + 1] - lay.split_off[i] >= 2, "a split template with fewer than two parts");
        for (int q = lay.split_off[i]; q < lay.split_off[i + 1]; ++q) CHECK(lay.part_tpl[q] == j, "part owner");
        nparts[j] = lay.split_off[i + 1] - lay.split_off[i];
    }
    for (int j = 0; j < T; ++j) {
        bool one_band = true;
        for (int64_t k = tb.off[j]; band > 0 && k < tb.off[j + 1]; ++k)
            one_band = one_band && tb.d[k] / band == tb.d[tb.off[j]] / band;
        CHECK((rows_of(tb.off[j + 1] - tb.off[j], fl) > R || !one_band) == (nparts[j] > 0),
              "template %d split wrongly", j);
    }
    CHECK(lay.band == band && lay.group_lo.size() == (size_t)lay.groups, "band tables");
    CHECK(lay.groups >= 1 && lay.nslots == (int64_t)lay.groups * wpg * fl * 64, "slot count");
    CHECK(lay.rows.size() == (size_t)lay.groups * R && lay.slot_filter.size() == (size_t)lay.nslots &&
              lay.pad_src.size() == (size_t)lay.nslots && lay.tpl_group.size() == (size_t)T,
          "array sizes");
    const int64_t F = tb.off.back();
    std::vector<int32_t> owner(F);
    for (int j = 0; j < T; ++j)
        for (int64_t k = tb.off[j]; k < tb.off[j + 1]; ++k) owner[k] = j;
    // rows: each whole template (each part) is one contiguous run of rows in one group; the
    // rows of a split template's parts add up to its row count
    std::vector<int> part_rows(lay.n_parts, 0), part_group(lay.n_parts, -1);
    for (int g = 0; g < lay.groups; ++g) {
        for (int row = 0; row < R; ++row) {
            const RowInfo ri = lay.rows[(size_t)g * R + row];
            if (ri.tpl < 0) continue;
            CHECK(ri.tpl < T, "row template out of range");
            CHECK(ri.r0 <= row && row < ri.r0 + ri.nr && ri.r0 + ri.nr <= R, "row range of template %d", ri.tpl);
            for (int q = ri.r0; q < ri.r0 + ri.nr; ++q)
                CHECK(lay.rows[(size_t)g * R + q].tpl == ri.tpl && lay.rows[(size_t)g * R + q].part == ri.part,
                      "template %d rows not contiguous", ri.tpl);
            if (ri.part < 0) {
                CHECK(nparts[ri.tpl] == 0, "whole rows of a split template");
                CHECK(lay.tpl_group[ri.tpl] == g, "template %d in group %d but rows in %d", ri.tpl,
                      lay.tpl_group[ri.tpl], g);
                CHECK(ri.nr == rows_of(tb.off[ri.tpl + 1] - tb.off[ri.tpl], fl), "row count of template %d", ri.tpl);
            } else {
                CHECK(ri.part < lay.n_parts && lay.part_tpl[ri.part] == ri.tpl, "part of another template");
                CHECK(part_group[ri.part] < 0 || part_group[ri.part] == g, "a part in two groups");
                part_group[ri.part] = g;
                if (row == ri.r0) part_rows[ri.part] += ri.nr;
            }
        }
    }
    for (size_t i = 0; i < lay.split_tpl.size(); ++i) {
        const int j = lay.split_tpl[i];
        int rows = 0;
        for (int q = lay.split_off[i]; q < lay.split_off[i + 1]; ++q) {
            CHECK(part_group[q] >= 0 && part_rows[q] >= 1 && part_rows[q] <= R, "part %d unplaced", q);
            rows += part_rows[q];
        }
        CHECK(rows <= rows_of(tb.off[j + 1] - tb.off[j], fl) + nparts[j], "rows of split template %d", j);
        CHECK(lay.tpl_group[j] == part_group[lay.split_off[i]], "group of a split template's first part");
    }
    for (int j = 0; j < T; ++j) CHECK(lay.tpl_group[j] >= 0 && lay.tpl_group[j] < lay.groups, "template unplaced");
    // every filter in exactly one slot, of a row serving its template
    std::vector<int> seen(F, 0);
    for (int64_t s = 0; s < lay.nslots; ++s) {
        const int lane = (int)(s % 64);
        const int64_t colw = s / 64;       // (g * wpg + wave) * fl + f
        const int64_t gw = colw / fl;
        const int g = (int)(gw / wpg), wave = (int)(gw % wpg);
        const int row = wave * 4 + lane / kRowLanes;
        const RowInfo ri = lay.rows[(size_t)g * R + row];
        const int32_t k = lay.slot_filter[(size_t)s];
        if (k >= 0) {
            CHECK(k < F, "slot filter out of range");
            ++seen[k];
            CHECK(band == 0 ? lay.group_lo[(size_t)g] == 0
                            : tb.d[k] >= lay.group_lo[(size_t)g] && tb.d[k] < lay.group_lo[(size_t)g] + band,
                  "filter %d (delay %d) outside its group's band [%d, +%d)", k, tb.d[k], lay.group_lo[(size_t)g], band);
            CHECK(ri.tpl == owner[k], "filter %d of template %d sits in a row of template %d", k, owner[k], ri.tpl);
            CHECK(lay.pad_src[(size_t)s] == -1, "real slot with a padding source");
        } else {
            const int64_t src = lay.pad_src[(size_t)s];
            if (src >= 0) {
                CHECK(src < lay.nslots && lay.slot_filter[(size_t)src] >= 0, "padding source is not a filter");
                CHECK(owner[lay.slot_filter[(size_t)src]] == ri.tpl, "padding source of another template");
                CHECK((src / 64) % fl == colw % fl && src / 64 / fl == gw, "padding source in another slot column");
            }
        }
    }
    for (int64_t k = 0; k < F; ++k) CHECK(seen[k] == 1, "filter %lld placed %d times", (long long)k, seen[k]);
    // per-slot arrays
    SlotHost h;
    slot_arrays(lay, tb.a.data(), tb.b.data(), tb.d.data(), tb.dmax, L, h);
    for (int64_t s = 0; s < lay.nslots; ++s) {
        const int32_t k = lay.slot_filter[(size_t)s];
        CHECK(h.xoff[(size_t)s] >= 0 && h.xoff[(size_t)s] <= tb.dmax, "window offset out of range");
        if (k < 0) {
            CHECK(h.a32[(size_t)s].x == 0.f && h.b32[(size_t)s].x == 0.f && h.b32[(size_t)s].y == 0.f,
                  "padding slot with coefficients");
            continue;
        }
        CHECK(h.a32[(size_t)s].x == (float)tb.a[2 * k] && h.a32[(size_t)s].y == (float)tb.a[2 * k + 1], "fl32(a)");
        CHECK(h.b32[(size_t)s].x == (float)tb.b[2 * k] && h.b32[(size_t)s].y == (float)tb.b[2 * k + 1], "fl32(b)");
        CHECK(h.xoff[(size_t)s] == tb.dmax - tb.d[k], "window offset");
        const std::complex<double> a(tb.a[2 * k], tb.a[2 * k + 1]);
        const std::complex<double> p = std::pow(a, L);
        const std::complex<double> got(h.aL[(size_t)s].x, h.aL[(size_t)s].y);
        CHECK(std::abs(got - p) <= 1e-12 * std::max(1e-300, std::abs(p)) + 1e-300, "a^L");
        const std::complex<double> a32((float)tb.a[2 * k], (float)tb.a[2 * k + 1]);
        const std::complex<double> dl(h.dL[(size_t)s].x, h.dL[(size_t)s].y);
        CHECK(std::abs(dl - (p - std::pow(a32, L))) <= 1e-10 * std::abs(p) + 1e-300, "a^L - fl32(a)^L");
        CHECK(h.flags[(size_t)s] == (std::abs(a) > 1.0 - 1e-5 ? 1 : 0), "carry flag");
    }
}

void check_geometry(Rng &r) {
    const size_t cap = 160 * 1024;
    for (int it = 0; it < 4000; ++it) {
        const int wpg = r.uni(1, kMaxWaves);
        const int dmax = r.next() % 4 == 0 ? r.uni(0, 70000) : r.uni(0, 20000);
        const int L = 8 * r.uni(1, 512);
        const int mb0 = r.uni(1, 8) * 4096;
        const int max_block = std::max(L, mb0 / L * L);
        const Geometry g = plan_geometry(wpg, dmax, L, max_block, cap);
        CHECK(g.tt == 16 || g.tt == 8, "tile length %d", g.tt);
        CHECK(L % g.tt == 0, "tile length %d does not divide L %d", g.tt, L);
        CHECK(g.lds == fwd_lds_bytes(wpg, dmax, g.nb, g.xlds, g.tt), "lds bytes");
        if (g.xlds) {
            CHECK(g.nb >= L && g.nb % L == 0 && g.nb <= max_block, "sub-block %d (L %d, max %d)", g.nb, L, max_block);
            CHECK(g.lds <= cap, "LDS %zu over the cap", g.lds);
        } else {
            CHECK(g.nb == max_block, "global window sub-block");
            CHECK(fwd_lds_bytes(wpg, 0, 0, false, g.tt) <= cap, "tiles alone over the LDS cap");
        }
    }
}

void check_args() {
    const int64_t off[3] = {0, 2, 3};
    double a[6] = {0.5, 0.1, 0.9, 0.0, -0.3, 0.2}, b[6] = {1, 0, 0, 1, 1, 1};
    int32_t d[3] = {0, 5, 7};
    spiir_bank_opts o;
    o.chunk_len = 256;
    o.filters_per_lane = 0;
    o.max_delay = 0;
    o.precision = 0;
    o.device = -1;
    o.max_block = 0;
    o.waves_per_group = 0;
    o.autotune = 0;
    o.time_split = 0;
    o.delay_band = 0;
    std::string err;
    int dm = -1;
    CHECK(check_bank_args(2, off, a, b, d, o, dm, err) == SPIIR_OK && dm == 7, "valid bank rejected: %s", err.c_str());
    struct Case {
        const char *what;
        void (*mut)(int64_t *, double *, double *, int32_t *, spiir_bank_opts &);
    };
    const Case cases[] = {
        {"unstable a", [](int64_t *, double *aa, double *, int32_t *, spiir_bank_opts &) { aa[2] = 1.0; }},
        {"nan b", [](int64_t *, double *, double *bb, int32_t *, spiir_bank_opts &) { bb[3] = std::nan(""); }},
        {"negative d", [](int64_t *, double *, double *, int32_t *dd, spiir_bank_opts &) { dd[1] = -1; }},
        {"empty template", [](int64_t *oo, double *, double *, int32_t *, spiir_bank_opts &) { oo[1] = 0; }},
        {"offset 0", [](int64_t *oo, double *, double *, int32_t *, spiir_bank_opts &) { oo[0] = 1; }},
        {"chunk 12", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.chunk_len = 12; }},
        {"chunk 8192", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.chunk_len = 8192; }},
        {"fl 5", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.filters_per_lane = 5; }},
        {"precision 3", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.precision = 3; }},
        {"max_delay", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.max_delay = 6; }},
        {"wpg 9", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.waves_per_group = 9; }},
        {"split 33", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.time_split = 33; }},
        {"band -1", [](int64_t *, double *, double *, int32_t *, spiir_bank_opts &oo) { oo.delay_band = -1; }},
    };
    for (const Case &c : cases) {
        int64_t o2[3] = {off[0], off[1], off[2]};
        double a2[6], b2[6];
        for (int i = 0; i < 6; ++i) {
            a2[i] = a[i];
            b2[i] = b[i];
        }
        int32_t d2[3] = {d[0], d[1], d[2]};
        spiir_bank_opts oo = o;
        c.mut(o2, a2, b2, d2, oo);
        err.clear();
        CHECK(check_bank_args(2, o2, a2, b2, d2, oo, dm, err) == SPIIR_EINVAL && !err.empty(), "%s accepted", c.what);
    }
}

}  // namespace

int main(int argc, char **argv) {
    const int seeds = argc > 1 ? std::atoi(argv[1]) : 40;
    check_args();
    Rng r(1602);
    check_geometry(r);
    int banks = 0, layouts = 0;
    for (int sd = 0; sd < seeds && !g_fail; ++sd) {
        Rng rb(1000 + sd);
        TestBank tb;
        switch (sd % 6) {
            case 0: tb = random_bank(rb, rb.uni(1, 40), 1, 600, 2047); break;
            case 1: tb = random_bank(rb, rb.uni(1, 12), 100, 800, 16384); break;
            case 2: tb = random_bank(rb, 3, 2048, 2048, 100); break;     // one full workgroup at fl = 4
            case 5: tb = random_bank(rb, rb.uni(2, 6), 1, 9000, 3000); break;  // templates split into parts
            case 3: tb = random_bank(rb, rb.uni(1, 64), 1, 40, 31); break;    // many tiny templates
            default: tb = random_bank(rb, rb.uni(2, 20), 16, 16 * rb.uni(1, 8), 4096); break;  // exact rows
        }
        ++banks;
        for (int fl = 1; fl <= 4 && !g_fail; ++fl)
            for (int wpg = 1; wpg <= kMaxWaves && !g_fail; wpg += (sd % 2 ? 3 : 1)) {
                const int L = 8 * rb.uni(1, 64);
                check_layout(tb, fl, wpg, L, 0);
                const int band = tb.dmax > 0 ? rb.uni(1, tb.dmax + 1) : 1;   // delay bands of random width
                check_layout(tb, fl, wpg, L, band);
                layouts += 2;
            }
    }
    if (g_fail) return 1;
    std::printf("layout ok: %d banks, %d layouts\n", banks, layouts);
    return 0;
}
