// Internal declarations shared by the kernels and the host side of libspiir.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "layout.h"

namespace spiir {

constexpr int kSub = 16;        // adjoint: steps of strain and G loaded together
constexpr float kFlagRadius = 1.0f - 1e-5f;

enum Mode { kModeSnr = 0, kModeKeys = 1, kModeZ = 2 };
enum Prec { kPrecHybrid = 0, kPrecFp32 = 1, kPrecFp64 = 2 };

// Per filter slot (lane-major inside each wave and slot column).
struct SlotArrays {
    const float2 *a32;    // fl32(a)
    const float2 *b32;    // fl32(b)
    const int32_t *xoff;  // max_delay - d: offset of x[m - d] inside the window
    const double2 *aL;    // a^L in FP64
    const double2 *dL;    // a^L - fl32(a)^L in FP64
    const double2 *a64;   // a in FP64 (powers for ragged chunks)
    const int32_t *flags; // bit 0: |a| > 1 - 1e-5 (FP64 carry in hybrid mode)
};

// The next call's strain history: the last dmax samples of old_h[0..dmax) ++ x[0..n).
struct HistCopy {
    const float *old_h;
    float *new_h;   // a different buffer than old_h
    const float *x;
    int64_t n;
    int dmax;
};

struct FwdArgs {
    SlotArrays s;
    float4 *state;        // (hi.re, hi.im, lo.re, lo.im) per slot; null: cold start, not stored
    const float *x;       // samples; launch sample t is x[xbase + t]
    const float *hist;    // max_delay samples before x[0] (null: zeros); hist[dmax + m], m < 0
    const float *xwin;    // global-window mode: xwin[dmax + m] = sample m (m >= -dmax)
    int64_t xbase;
    int64_t n;            // samples in this launch
    int32_t dmax, L, nb, prec, wpg, only_tpl;
    int32_t gbase;        // group of blockIdx.x == 0
    int32_t band_w;       // LDS window: delays of a group lie in [lo, lo + band_w]; max_delay without bands
    const int32_t *group_lo;  // [groups] lowest delay of each group's band (null: no bands, lo = 0)
    const RowInfo *rows;  // [groups * wpg * 4]
    int64_t obase;        // output column of launch sample 0
    int64_t ld;           // row length of snr / z / keys
    float *snr;           // kModeSnr: snr[tpl * ld + obase + t]
    uint64_t *keys;       // kModeKeys: keys[group * ld + t]
    float2 *z;            // kModeZ: z[tpl * ld + obase + t]
    float2 *zpart;        // rows of split templates' parts: zpart[part * ld_part + t] (piece-local t)
    int64_t ld_part;
    int64_t nslots;
    // time split of one launch into nseg segments of seg_len samples
    int32_t groups;       // workgroups of the bank (item = segment * groups + group)
    int32_t n_templates;
    int64_t seg_len;
    float4 *seg_end;      // [nseg][nslots] state at each segment end (local from zero for segments > 0)
    float4 *seg_start;    // [nseg][nslots] true state at each segment start (segments > 0)
    float2 *zl;           // [nseg - 1][T][seg_len] local z of segments > 0
    HistCopy hist_next;   // time split: history copy done by the chain launch (dmax 0: none)
    // seg_end / seg_start hold slots [seg_slot0, seg_slot0 + seg_stride) of every segment
    // (entry [seg][slot - seg_slot0]); the whole bank: 0 and nslots
    int64_t seg_slot0, seg_stride;
};

struct BwdArgs {
    SlotArrays s;
    const RowInfo *rows;
    const int32_t *slot_filter;  // slot -> caller filter index (-1 padding)
    const int32_t *filter_slot;  // caller filter index -> slot
    const int4 *bwaves;          // [n_bwaves] (template, first filter, end filter, 0): the backward's waves
    int32_t n_bwaves, pad0;
    const float *xwin;           // xwin[dmax + m] = x[m] for m in [-dmax, n)
    const float2 *gz;            // [T][n]
    float4 *pair_loc;            // scratch [nseg][nslots]: segment-local (lambda, nu) at the segment start
    float4 *pair_in;             // scratch [nseg][nslots]: true (lambda, nu) entering each segment from the right
    double2 *gpart;              // scratch [nseg][2][nslots]: per-segment sum nu x, sum lambda x
    float2 *grad_a, *grad_b;     // [F] caller order
    int64_t n, nslots;
    int32_t dmax, L, prec, wpg;
    int32_t nseg, seg_chunks;    // time segments of seg_chunks chunks each (the last may be shorter)
};

// Time-split streaming z calls of several banks (each on its own strain) in
// one launch per pass: pass workgroups [first[b], first[b + 1]) belong to
// bank b (segment pass: groups x nseg; chain: chain_blocks plus the history
// copy's blocks; carry pass: groups x (nseg - 1)).
constexpr int kMultiMax = 8;
struct MultiFwd {
    FwdArgs a[kMultiMax];
    int32_t seg_first[kMultiMax + 1];
    int32_t chain_first[kMultiMax + 1];
    int32_t carry_first[kMultiMax + 1];
    int32_t nseg[kMultiMax];
    int32_t chain_blocks[kMultiMax];
    int32_t count;
};

// One stream of a batch, as the persistent kernel sees it.
struct BatchStream {
    FwdArgs args;       // bank part filled at creation; x = whole stream, xbase/n per step
    int64_t len;
    int32_t groups;
    int32_t pad;
    float *max_out;
    int32_t *arg_out;
};

// Launch helpers (kernels.hip). All enqueue on `stream` and return the launch error.
// Optional kernel timestamps: when set, `start` takes the start time of the
// first forward kernel of a launch and `stop` the end time of the last one
// (recorded by the dispatch itself, so no packet is added between kernels).
struct KernelEvents {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};

hipError_t launch_forward(const FwdArgs &a, int mode, int fl, int tt, bool x_in_lds, int groups,
                          size_t lds, hipStream_t stream, KernelEvents ev = KernelEvents());
// Time-split launch (modes kModeSnr / kModeKeys / kModeZ): local pass over every
// segment, FP64 carry chain, carry-only pass with the local z added.
hipError_t launch_forward_split(const FwdArgs &a, int mode, int fl, int tt, bool x_in_lds, int nseg,
                                size_t lds, size_t lds_carry, const int32_t *slot_filter,
                                hipStream_t stream, KernelEvents ev = KernelEvents());
// The three passes of a MultiFwd (z mode, strain windows in LDS); every bank
// shares fl, tt and the workgroup size wpg * 64.
hipError_t launch_forward_split_multi(const MultiFwd &m, int fl, int tt, int wpg, size_t lds, size_t lds_carry,
                                      hipStream_t stream);
int forward_occupancy(int fl, int tt, int wpg, size_t lds);
// Adjoint over nseg time segments: segment-local (lambda, nu) scan, FP64 chain,
// per-segment backward, FP64 reduction of the per-segment gradients.
hipError_t launch_backward(const BwdArgs &a, hipStream_t stream);
// Per-sample max over the groups' keys; with hc, the same launch also writes
// the history copy (one launch fewer per streaming call).
hipError_t launch_finalize_keys(const uint64_t *keys, int groups, int64_t ld, int64_t n,
                                float *mx, int32_t *am, hipStream_t stream, const HistCopy *hc = nullptr);
// Sums the parts of split templates and writes the mode's output for them
// (key_row: the per-sample maximum key over the split templates).
hipError_t launch_combine_parts(const float2 *zpart, int64_t ld_part, const int32_t *split_tpl,
                                const int32_t *split_off, int n_split, int64_t n, int mode, float *snr, float2 *z,
                                int64_t ld, int64_t obase, uint64_t *key_row, hipStream_t stream);
// Slot arrays of a bank from caller-order complex128 a, b on the device.
hipError_t launch_set_coeffs(const double *a, const double *b, const int32_t *slot_filter, int64_t nslots, int L,
                             float2 *a32, float2 *b32, double2 *aL, double2 *dL, double2 *a64, int32_t *flags,
                             hipStream_t stream);
hipError_t launch_rows_argmax(const float *snr, int T, int64_t ld, int64_t n, float *mx,
                              int32_t *am, hipStream_t stream);
hipError_t launch_hist_update(const float *old_h, float *new_h, const float *x, int64_t n,
                              int dmax, hipStream_t stream);
hipError_t launch_window_fill(float *xwin, const float *hist, const float *x, int64_t n,
                              int dmax, hipStream_t stream);
int batch_occupancy(int fl, int tt, int wpg, size_t lds);
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t stream);
hipError_t launch_batch(const BatchStream *streams, const int2 *items, int nitems,
                        int *counter, const int64_t *pos, int block_len, int fl, int tt, int grid,
                        int wpg, size_t lds, hipStream_t stream);
// Time-split batch step: local pass over (stream, group << 4 | segment) items,
// per-stream FP64 carry chain, carry-only pass over the items of segments >= 1.
hipError_t launch_batch_split(const BatchStream *streams, const int2 *seg_items, int n_seg_items,
                              const int2 *carry_items, int n_carry_items, const int64_t *pos, int block_len,
                              int nstreams, int64_t max_slots, int fl, int tt, int wpg, size_t lds,
                              size_t lds_carry, hipStream_t stream);
hipError_t launch_batch_finalize(const BatchStream *streams, int nstreams, const uint64_t *keys,
                                 int64_t key_stride, const int64_t *pos, int block_len,
                                 int max_groups, hipStream_t stream);
hipError_t launch_batch_advance(int64_t *pos, const BatchStream *streams, int nstreams,
                                int *counter, int block_len, hipStream_t stream);
hipError_t launch_noise_fill(float *x, int64_t n, uint32_t seed, hipStream_t stream);
int forward_max_threads();

// Multi-rate bank: decimation by two with history (one launch per level, or
// every level in one launch when the levels fit in LDS), then the
// interpolation of every level back to the full rate in one launch, fused
// with the full-rate z or with the per-sample keys over chunks of template
// rows for finalize_keys.
constexpr int kMaxLevels = 8;
struct MrPyramid {
    const float *hist[kMaxLevels];   // [r >= 1]: the previous lh - 1 samples of level r - 1
    float *hist_new[kMaxLevels];     // [r >= 1]: the next call's (a different buffer)
    float *dst[kMaxLevels];          // [r >= 1]: level r's samples, n >> r
};
struct MrChain {
    const float2 *z[kMaxLevels];       // level sums [rows][ld_z] (null: the level has no filters)
    int64_t ld_z[kMaxLevels];
    const int32_t *zrow[kMaxLevels];   // template j -> row of z[r] (-1: none)
    const float2 *whist[kMaxLevels];   // [r >= 1]: the previous hh samples of W_r, [T][hh]
    float2 *whist_new[kMaxLevels];     // [r >= 1]: the next call's (a different buffer)
};
hipError_t launch_mr_decimate(const float *src, int64_t n_src, const float *hist, float *hist_new,
                              const float *h, int lh, float *dst, hipStream_t stream);
size_t mr_pyramid_lds(int64_t B, int top, int lh);
hipError_t launch_mr_pyramid(const float *x, int64_t n, int top, const MrPyramid &pm, const float *h, int lh,
                             int64_t B, hipStream_t stream);
size_t mr_chain_lds(int top, int lg);
// keys != null: keys[chunk][p] = max over the chunk's rows of (|z|^2 bits << 32 | ~j);
// else the full-rate z to out[j * ld_out + p].
hipError_t launch_mr_chain(const MrChain &c, int top, int hh, const float *g, int lg, int64_t n_out, int T,
                           uint64_t *keys, int64_t ld_keys, float2 *out, int64_t ld_out, hipStream_t stream);
int mr_key_chunks(int T);
hipError_t launch_mr_copy_out(float *mx, const float *mxo, int32_t *am, const int32_t *amo, int64_t n,
                              hipStream_t stream);

// Whitening front end: frame FFTs (PSD or whitening mode), PSD average,
// 1/sqrt(S) from a given PSD, overlap-add with history and pending half-frame.
hipError_t launch_wh_frames(bool psd, const float *hist, int64_t hlen, const float *x, const float *wtab,
                            const float2 *tw, int n, int logn, const float *inv, float *y, float *pw,
                            int64_t frames, hipStream_t stream);
hipError_t launch_wh_psd_reduce(const float *pw, int64_t frames, int H, double wsum2, double *S, float *inv,
                                hipStream_t stream);
hipError_t launch_wh_inv(const double *S, int H, float *inv, hipStream_t stream);
hipError_t launch_wh_ola(const float *y, int64_t nf, int n, const float *pend, float *pend_new, const float *x,
                         int64_t nx, float *hist_new, float *out, hipStream_t stream);

// Trigger clustering over a max/argmax series (block maxima, window test,
// ordered compaction); the workspace holds the block maxima, masks and counts.
size_t cluster_workspace_bytes(int64_t n);
// Candidates are limited to samples [c_lo, c_hi) (c_hi < 0: up to n; the rest
// are window neighbours only) and written indices are offset by index_base.
hipError_t launch_cluster(const float *max, const int32_t *argmax, int64_t n, float threshold,
                          int64_t window, void *workspace, int64_t capacity, int64_t *index,
                          int32_t *tmpl, float *snr, int64_t *count, hipStream_t stream,
                          int64_t c_lo = 0, int64_t c_hi = -1, int64_t index_base = 0);
// Trigger stream window: dm/dj = sm/sj[0..keep) ++ bm/bj[0..n) (no overlap).
hipError_t launch_ts_compose(const float *sm, const int32_t *sj, int64_t keep, const float *bm, const int32_t *bj,
                             int64_t n, float *dm, int32_t *dj, hipStream_t stream);

}  // namespace spiir
