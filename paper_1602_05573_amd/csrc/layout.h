// Host-side plan of a filter bank on the device: argument checks, the
// filter-to-slot layout, the LDS geometry of the forward kernel and the FP64
// per-slot coefficients. Plain C++ with no HIP dependency, so that the tests
// can build it with g++ under AddressSanitizer and UBSan and drive it with
// random banks; the library compiles the same source.
#ifndef SPIIR_LAYOUT_H
#define SPIIR_LAYOUT_H

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "spiir.h"

namespace spiir {

constexpr int kMaxWaves = 8;    // 64-lane waves per workgroup (512 threads)
constexpr int kRowLanes = 16;   // lanes per row; a row serves exactly one template

// Per 16-lane row of a workgroup: the template it serves (-1: none), the
// first row of that template (or of its part) inside the workgroup, its number
// of rows there, and the part index when the template is split over several
// workgroups (-1: the whole template is in this workgroup).
struct RowInfo {
    int32_t tpl, r0, nr, part;
};

namespace layout {

// Filter-to-slot layout of one bank: a workgroup of wpg waves holds 4 wpg
// rows of 16 lanes, every lane fl filter slots; slot index
// ((g * wpg + wave) * fl + f) * 64 + lane.
struct Layout {
    int fl = 1, wpg = 1, groups = 0;
    int64_t nslots = 0;
    std::vector<RowInfo> rows;            // [groups * wpg * 4]
    std::vector<int32_t> slot_filter;     // [nslots], -1 = padding
    std::vector<int64_t> pad_src;         // [nslots], padding: slot whose window offset it reuses (-1: none)
    std::vector<int32_t> tpl_group;       // [T] (a split template: the group of its first part)
    // Templates with more rows than a workgroup has are split into parts of at
    // most 4 wpg rows, each packed like a template; parts of one template have
    // consecutive indices.
    int n_parts = 0;
    std::vector<int32_t> part_tpl;        // [n_parts] template of each part
    std::vector<int32_t> split_tpl;       // [n_split] split templates, increasing
    std::vector<int32_t> split_off;       // [n_split + 1] parts of split_tpl[i]: split_off[i] .. split_off[i+1]-1
    // Delay bands (band > 0): every workgroup holds filters with delays in
    // [group_lo[g], group_lo[g] + band) only, so that its strain window is band
    // + block samples long; a template with filters in several bands is split
    // into parts by band.
    int band = 0;
    std::vector<int32_t> group_lo;        // [groups] lowest delay of the group's band (0 without bands)
};

struct Plan {
    int64_t total_rows = 0;
    int max_nr = 0;
};

// LDS plan of the forward kernel for one workgroup size.
struct Geometry {
    int tt = 16;         // steps per tile; always divides the chunk length
    int nb = 0;          // samples per LDS window fill (a multiple of the chunk length)
    bool xlds = true;    // the strain window sits in LDS
    size_t lds = 0;      // LDS bytes per workgroup
};

// Two floats / two doubles laid out as the device's float2 / double2.
struct F2 {
    float x, y;
};
struct D2 {
    double x, y;
};

// Per-slot arrays as uploaded to the device (padding slots: zero
// coefficients, the window offset of their column's first filter).
struct SlotHost {
    std::vector<F2> a32, b32;     // fl32(a), fl32(b)
    std::vector<int32_t> xoff;    // max_delay - d
    std::vector<int32_t> flags;   // bit 0: |a| > 1 - 1e-5
    std::vector<D2> aL, dL, a64;  // a^L, a^L - fl32(a)^L, a (FP64)
};

// Rows of 16 lanes x fl filters that k filters need.
int rows_of(int64_t k, int fl);
Plan plan_rows(int T, const int64_t *off, int fl);
// Waves per workgroup that spread the rows over n_cu compute units, at least
// enough for the largest template, at most kMaxWaves.
int auto_wpg(int64_t total_rows, int max_nr, int n_cu);
// Filters per lane: the largest count that still gives about seven waves per
// compute unit; 1 for small banks.
int choose_fl(int T, const int64_t *off, int n_cu);
// LDS bytes of a forward workgroup: strain window (when in LDS), one tile of
// lane partial sums per wave, double-buffered row sums and the key slots.
size_t fwd_lds_bytes(int wpg, int dmax, int nb, bool x_in_lds, int tt);
Geometry plan_geometry(int wpg, int dmax, int L, int max_block, size_t lds_cap);

// Validates the arguments of spiir_bank_create; returns SPIIR_OK and the
// effective max_delay, or SPIIR_EINVAL with a message in err.
int check_bank_args(int32_t T, const int64_t *off, const double *a, const double *b, const int32_t *d,
                    const spiir_bank_opts &o, int &dmax_out, std::string &err);
// First-fit decreasing packing of templates into workgroups of 4 wpg rows (a
// template with more rows than that is first split into parts of balanced row
// counts, each packed as one item; with band > 0 a template is first cut by
// delay band d / band and workgroups hold one band each), then the
// delay-aware dealing of every template's (or part's) filters over its slot
// columns. Returns SPIIR_OK.
int build_layout(int T, const int64_t *off, const int32_t *d, int fl, int wpg, int band, Layout &lay,
                 std::string &err);
// FP64 powers and FP32 roundings of every slot's coefficients (a, b complex128
// interleaved [F], caller order).
void slot_arrays(const Layout &lay, const double *a, const double *b, const int32_t *d, int dmax, int L,
                 SlotHost &out);
// (re + i im)^e by binary powering in FP64.
void cpow(double re, double im, long e, double &out_re, double &out_im);

}  // namespace layout
}  // namespace spiir

#endif  // SPIIR_LAYOUT_H
