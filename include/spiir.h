/*
 * spiir.h - C ABI of the MI355X (gfx950) summed parallel IIR (SPIIR) library.
 *
 * The operation (Sect. "GPU accelerated SPIIR method", subsections "SPIIR
 * method" and "Optimized GPU implementation of SPIIR"): a template's SNR is
 * approximated by the summed output of a parallel bank of single-pole IIR
 * filters run over the (whitened) detector stream; each filter's output is
 * fed back as its next input, and the template's SNR needs the outputs of all
 * its filters. In this library, for template j with filters k and samples m:
 *
 *   y_k[m]   = a_k * y_k[m-1] + b_k * x[m - d_k]          (complex a_k, b_k; real x)
 *   z_j[m]   = sum_k y_k[m]
 *   snr_j[m] = Re(z_j[m])^2 + Im(z_j[m])^2
 *   max[m]   = max_j snr_j[m],  argmax[m] = smallest j attaining it
 *
 * The recursion runs in FP32 complex arithmetic; every chunk_len samples each
 * filter's carried state is corrected in FP64 (see spiir_precision).
 *
 * Conventions for every function below:
 *  - Return value: SPIIR_OK (0) or a negative spiir_status. The message of the
 *    last failure on the calling thread is returned by spiir_last_error().
 *  - Pointers named *_dev are device pointers (hipMalloc / torch CUDA tensors)
 *    owned by the caller; the library never frees them. Pointers without the
 *    suffix are host pointers, read during the call only.
 *  - stream is a hipStream_t passed as void* (NULL = the null stream). Device
 *    work is enqueued asynchronously on it; argument errors are reported
 *    before anything is enqueued; device faults surface at the caller's next
 *    synchronisation.
 *  - A bank is not thread safe: use it from one host thread and one stream at
 *    a time. Banks keep streaming state (filter states and the last max_delay
 *    samples), so consecutive calls continue one stream.
 *  - Complex arrays are interleaved (re, im): complex128 on the host, complex64
 *    on the device.
 */
#ifndef SPIIR_H
#define SPIIR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spiir_bank spiir_bank;
typedef struct spiir_tape spiir_tape;
typedef struct spiir_batch spiir_batch;
typedef struct spiir_multirate spiir_multirate;
typedef struct spiir_whitener spiir_whitener;
typedef struct spiir_trigger_stream spiir_trigger_stream;

typedef enum {
    SPIIR_OK = 0,
    SPIIR_EINVAL = -1,  /* bad argument: null pointer, size, |a| >= 1, d out of range, ... */
    SPIIR_ENOMEM = -2,  /* host or device allocation failed */
    SPIIR_EHIP = -3,    /* a HIP runtime call failed; spiir_last_error() has its message */
    SPIIR_ESTATE = -4,  /* object used in the wrong state (stale tape, foreign bank, ...) */
    SPIIR_ENODEV = -5   /* no usable gfx950 device */
} spiir_status;

/* Precision plan of the recursion (the bulk loop is FP32 in every mode). */
typedef enum {
    /* FP64 chunk-carry powers a^L, and FP64 cross-chunk carry propagation for
     * filters with |a| > 1 - 1e-5; other filters get an FP32 correction by
     * (a^L - fl32(a)^L) times the chunk's starting state. Default. */
    SPIIR_PREC_HYBRID = 0,
    /* plain FP32 recursion with fl32(a), fl32(b); no correction */
    SPIIR_PREC_FP32 = 1,
    /* FP64 carry propagation for every filter */
    SPIIR_PREC_FP64_CARRY = 2
} spiir_precision;

typedef struct {
    int32_t chunk_len;        /* L: samples between carry corrections; multiple of 8 in
                                 [8, 4096]; 0 = 256 */
    int32_t filters_per_lane; /* filters held in registers by each lane: 1..4;
                                 0 = chosen from the bank size */
    int32_t max_delay;        /* upper bound on every d_k (size of the kept history);
                                 0 = max_k d_k */
    int32_t precision;        /* spiir_precision */
    int32_t device;           /* HIP device ordinal; -1 = the current device */
    int32_t max_block;        /* most samples handled by one kernel launch (longer calls
                                 are split); 0 = 16384 */
    int32_t waves_per_group;  /* 64-lane waves per workgroup, 1..8; 0 = automatic */
    int32_t autotune;         /* 1: time the candidate (chunk_len, filters_per_lane)
                                 pairs on this bank and keep the fastest */
    int32_t time_split;       /* segments each launch (spiir_filter_block,
                                 spiir_trigger_max, spiir_forward_z) is cut into when the
                                 bank alone cannot fill the device: every segment is
                                 filtered from rest in parallel, then the true
                                 segment-start states follow from a carry chain in FP64
                                 (with fl32(a) in SPIIR_PREC_FP32 mode) and their free
                                 response is added. spiir_backward likewise cuts the
                                 reverse scan into segments (automatic count up to 16
                                 for 0, the given count for 2..32). 0 = automatic, 1 = off,
                                 2..32 = forced. Not used by the per-template comparator.
                                 With filters_per_lane, waves_per_group and time_split all
                                 0, a bank of more than 128 filters per compute unit that
                                 the automatic lane count cannot spread over 7 waves per
                                 CU, with max_block >= 8192 and the strain window in LDS,
                                 takes 4 filters per lane, 8-wave workgroups and up to 16
                                 segments. */
    int32_t delay_band;       /* 0 = no delay bands (default: the strain window is staged in
                                 LDS when it fits, else read from global memory); w >= 1 =
                                 delay bands of width w: every workgroup holds filters with
                                 delays in one band [k*w, (k+1)*w) and stages only that
                                 band's window (w - 1 + sub-block samples, the sub-block at
                                 most w rounded up to chunk_len) in LDS; a template with
                                 filters in several bands is split into parts. EINVAL if a
                                 band's window does not fit LDS */
} spiir_bank_opts;

/* Layout facts of a created bank (for tests, tuning reports and benchmarks). */
typedef struct {
    int32_t n_templates;
    int64_t n_filters;
    int32_t max_delay;
    int32_t chunk_len;
    int32_t filters_per_lane;
    int32_t waves_per_group;
    int32_t n_groups;         /* workgroups per forward launch */
    int64_t n_slots;          /* filter slots incl. padding (n_groups * waves * 64 * F) */
    int32_t lds_bytes;        /* LDS per workgroup of the forward kernel */
    int32_t x_in_lds;         /* 1: the delayed strain window is staged in LDS */
    int32_t sub_block;        /* samples per LDS window fill */
    int32_t precision;
    int32_t device;
    int32_t n_cu;             /* compute units of the device */
    int32_t time_split;       /* segments per streaming launch (1 = no split) */
    int32_t n_parts;          /* parts of the templates split over workgroups (0: none) */
    int32_t delay_band;       /* delay band width (0: no bands) */
} spiir_bank_info;

/* Fills *opts with the defaults listed above. */
void spiir_bank_opts_default(spiir_bank_opts *opts);

/*
 * Builds a bank on the device (the per-template parameter arrays of subsection
 * "Optimized GPU implementation of SPIIR": aligned, contiguous, loaded with
 * coalesced accesses).
 *   n_templates     T >= 1
 *   filter_offsets  int64 [T+1]: filters of template j are offsets[j] .. offsets[j+1]-1;
 *                   offsets[0] = 0, strictly increasing (every template has >= 1 filter)
 *   a, b            complex128 [F] (interleaved), F = offsets[T]; |a_k| < 1 required
 *   d               int32 [F], 0 <= d_k <= max_delay
 *   opts            NULL = defaults
 * Filters are reordered into device slots internally; every per-filter output
 * (gradients, state) is reported in the caller's order. A template with more
 * filters than one workgroup holds (4 x waves_per_group rows of 16 lanes x
 * filters_per_lane; 2,048 at 8 waves and 4 filters per lane) is split into
 * parts in separate workgroups; each part's partial sum is written to a bank
 * buffer and a combine launch adds the parts, in part order, before the SNR,
 * z or key of that template. Banks with split templates are not accepted by
 * spiir_trigger_max_per_template and spiir_batch_create. The bank starts cold
 * (zero states, zero history). *out receives the bank, or NULL on failure.
 */
int spiir_bank_create(spiir_bank **out, int32_t n_templates, const int64_t *filter_offsets,
                      const double *a, const double *b, const int32_t *d,
                      const spiir_bank_opts *opts);

/* Frees the bank and its device buffers (synchronises its device). NULL is ignored. */
int spiir_bank_destroy(spiir_bank *bank);

/* Returns the layout facts of the bank. */
int spiir_bank_get_info(const spiir_bank *bank, spiir_bank_info *info);

/* Cold start: zero filter states and history, enqueued on stream. */
int spiir_bank_reset(spiir_bank *bank, void *stream);

/*
 * Replaces every a_k and b_k (same F, same d, same layout); the streaming
 * state is kept. Host arrays complex128 [F] in the caller's filter order,
 * |a_k| < 1. Synchronous with respect to the device (copies complete on
 * return).
 */
int spiir_bank_set_coeffs(spiir_bank *bank, const double *a, const double *b);

/*
 * The same replacement from device arrays, enqueued on stream (no host copy,
 * no synchronisation): the gradient step of a coefficient fit can stay on the
 * device between spiir_backward and the next spiir_forward_z (the fit is this
 * library's extension; see spiir_forward_z).
 *   a_dev, b_dev  complex128 [F] (interleaved), caller's filter order, device
 * The slot values are formed by a kernel exactly as the host call forms them
 * (fl32 roundings, a^chunk_len and its FP32 drift in FP64, the FP64-carry
 * flag). The values are not checked: the caller keeps every |a_k| < 1 and
 * every value finite (the host call rejects others with EINVAL). Work already
 * enqueued on other streams that uses this bank must complete first (a bank
 * is used from one stream at a time). Tapes made before the call become stale
 * (spiir_backward returns SPIIR_ESTATE for them). EINVAL for null pointers.
 */
int spiir_bank_set_coeffs_dev(spiir_bank *bank, const double *a_dev, const double *b_dev, void *stream);

/* Size in bytes of a state checkpoint of this bank. */
int spiir_bank_state_size(const spiir_bank *bank, size_t *nbytes);

/*
 * Checkpoint / resume of the streaming state (filter states and history).
 * host_buf must hold spiir_bank_state_size() bytes. Both calls synchronise the
 * device. Resuming from a checkpoint continues the stream bit for bit.
 */
int spiir_bank_get_state(const spiir_bank *bank, void *host_buf, size_t nbytes);
int spiir_bank_set_state(spiir_bank *bank, const void *host_buf, size_t nbytes);

/*
 * Filters the next n samples of the stream and writes every template's SNR.
 * Defined by Sect. "GPU accelerated SPIIR method": subsection "SPIIR method"
 * (a template's SNR approximated by a parallel bank of single-pole IIR
 * filters) and subsection "Optimized GPU implementation of SPIIR" (the SNR of
 * a template at a time point needs its parameter array and the data window,
 * and sums the outputs of all its filters). The paper prints no formula; the
 * recursion with an input delay and the SNR as the raw |z|^2 (no
 * normalisation, no square root) are this library's readings, stated at the
 * top of this file.
 *   x_dev    float32 [n], the next n samples
 *   snr_dev  float32, row-major [T][ld_snr], ld_snr >= n; row j receives snr_j
 * n = 0 is a no-op. One launch covers all templates. EINVAL for a null bank or
 * pointer, n < 0 or ld_snr < n.
 */
int spiir_filter_block(spiir_bank *bank, const float *x_dev, int64_t n,
                       float *snr_dev, int64_t ld_snr, void *stream);

/*
 * Filters the next n samples of the stream and writes every template's
 * complex sum z_j (the quantity whose squared modulus is the SNR; the summed
 * filter outputs of subsection "Optimized GPU implementation of SPIIR").
 *   z_dev  complex64, row-major [T][ld_z] (interleaved), ld_z >= n
 * n = 0 is a no-op. Continues the same stream as spiir_filter_block. EINVAL as
 * for spiir_filter_block.
 */
int spiir_filter_block_z(spiir_bank *bank, const float *x_dev, int64_t n, float *z_dev,
                         int64_t ld_z, void *stream);

/*
 * Filters the next n samples and writes only the per-sample maximum of the
 * SNR over templates and its smallest attaining template index; the [T][n]
 * SNR is never stored (fused epilogue). The paper has no trigger step: its
 * subsection "SPIIR method" states the purpose (identifying the presence of a
 * signal in noisy data with zero latency); the per-sample maximum over the
 * bank, ties to the lowest template index, is this library's reading of it.
 *   x_dev       float32 [n]
 *   max_dev     float32 [n]
 *   argmax_dev  int32 [n]
 * n = 0 is a no-op; EINVAL for a null bank or pointer or n < 0.
 */
int spiir_trigger_max(spiir_bank *bank, const float *x_dev, int64_t n,
                      float *max_dev, int32_t *argmax_dev, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * call as spiir_trigger_max, with the same arguments, results and stream
 * semantics (it continues the same stream; the two may be mixed call by
 * call), but its working memory (per-workgroup partial keys, the time split's
 * segment states and local sums, the strain window when it is not staged in
 * LDS) lives in a fixed 32 MiB array per device that the library holds until
 * the process ends. It calls no hipMalloc/hipFree. Needed bytes:
 *   groups * min(n, max_block) * 8
 *   + (time split) 2 * segments * slots * 16 + (segments - 1) * T * segment_len * 8
 *   + (window not in LDS) (n + max_delay + 16) * 4,
 * each rounded up to 256; the 1,024-template bank at 4,096 samples per call
 * needs 7.9 MB. When the bank's time segments do not fit, the call cuts its
 * launches into as many segments as do (results then agree with
 * spiir_trigger_max to FP32 rounding instead of bitwise). EINVAL (nothing
 * launched) when a call needs more than 32 MiB even without segments;
 * otherwise as spiir_trigger_max. Every call on one device shares that
 * device's array, which keeps the last call's contents: calls that overlap in
 * time on one device (several streams or host threads) race and must not be
 * issued; calls on one stream are ordered and safe.
 */
int spiir_trigger_max_noalloc(spiir_bank *bank, const float *x_dev, int64_t n,
                              float *max_dev, int32_t *argmax_dev, void *stream);

/*
 * Reference design for comparison: the same outputs as spiir_trigger_max
 * (within the same error against the FP64 oracle; not bitwise), but computed
 * template by template (the template-to-block mapping of subsection
 * "Optimized GPU implementation of SPIIR"), each template's launches writing
 * its SNR row to snr_scratch_dev (float32 [T][n], caller-owned), followed by
 * a separate max/argmax pass over the stored rows. Each template's launches
 * fill the device on their own: every piece of at most max_block samples is
 * cut into segments of chunk_len samples, one workgroup each, whose carries
 * are chained in FP64 (three launches per template and piece; one launch
 * when the piece is a single chunk); their strain is read from a window of
 * the call's samples in global memory. The segment scratch (two states per
 * slot of one workgroup and segment, one complex sum per template-sample)
 * and the window are allocated on first use. Continues the same stream as spiir_trigger_max.
 * n = 0 is a no-op; EINVAL for a null bank or pointer, n < 0, or a bank with
 * templates split over workgroups.
 */
int spiir_trigger_max_per_template(spiir_bank *bank, const float *x_dev, int64_t n,
                                   float *max_dev, int32_t *argmax_dev,
                                   float *snr_scratch_dev, void *stream);

/*
 * One-shot forward from a cold start over x[0..n), independent of the
 * bank's streaming state (which is left untouched). The forward half of the
 * coefficient fit: the paper reports that a SPIIR bank reaches more than 99%
 * overlap with the matched filter (subsection "SPIIR method") but gives no
 * procedure; fitting (a_k, b_k) by gradient descent on an overlap loss is this
 * library's extension, and this call records what its adjoint needs. Writes z_j[m] as complex64
 * into z_dev [T][n] (interleaved). If tape_out is not NULL, *tape_out receives
 * a tape for spiir_backward: a device copy of the call's strain (with
 * max_delay leading zeros) and the coefficient version it ran with; no filter
 * output or state is stored (the adjoint does not need y, see
 * spiir_backward). x_dev may be reused once the call's work has completed.
 */
int spiir_forward_z(spiir_bank *bank, const float *x_dev, int64_t n, float *z_dev,
                    spiir_tape **tape_out, void *stream);

/*
 * Reverse-time adjoint of spiir_forward_z for a real loss L of z (the
 * gradient half of the coefficient fit described at spiir_forward_z; not in
 * the paper, derived here from the recursion by the chain rule).
 *   grad_z_dev  complex64 [T][n]: dL/dRe(z) + i dL/dIm(z)
 *   grad_a_dev, grad_b_dev  complex64 [F], caller's filter order, same convention
 * lambda_k[m] = G_j[m] + conj(a_k) lambda_k[m+1] runs backwards from
 * lambda_k[n] = 0; grad_b_k = sum_m lambda_k[m] x[m-d_k] and
 * grad_a_k = sum_m lambda_k[m] conj(y_k[m-1]). The library forms the second
 * sum without y: from a cold start it equals conj(b_k) sum_m nu_k[m] x[m-d_k]
 * with nu_k[m] = lambda_k[m+1] + conj(a_k) nu_k[m+1] (nu_k[n-1] = 0), a second
 * reverse recursion run beside lambda. The pair is carried in FP32 with an
 * FP32 correction for fl32(a_k) every chunk_len samples; time segments (see
 * spiir_bank_opts.time_split) are composed in FP64. Per-chunk sums are FP32
 * and are accumulated across chunks in FP64. Returns SPIIR_ESTATE if the tape
 * belongs to another bank or the coefficients changed since it was made;
 * EINVAL for null pointers.
 */
int spiir_backward(spiir_bank *bank, const spiir_tape *tape, const float *grad_z_dev,
                   float *grad_a_dev, float *grad_b_dev, void *stream);

/* Frees a tape (after the work that uses it has completed). NULL is ignored. */
int spiir_tape_destroy(spiir_tape *tape);

/*
 * Batched streams: n_streams banks, each filtering its own stream, advanced
 * together one block per step by one persistent kernel launch recorded in a
 * HIP graph (created on stream). All banks must share filters_per_lane.
 * Subsection "Optimized GPU implementation of SPIIR" maps templates of uneven
 * size onto the thread hierarchy and sizes blocks for full occupancy; here the
 * uneven unit is a (stream, workgroup) item taken from a device work list, so
 * banks of uneven size and streams of uneven length share one launch.
 *   banks       [n_streams] banks (not used elsewhere while the batch lives)
 *   x_dev       [n_streams] float32 streams, whole, resident on the device
 *   lengths     [n_streams] samples of each stream (>= 1)
 *   max_dev     [n_streams] float32 [length] per-sample maxima (outputs)
 *   argmax_dev  [n_streams] int32 [length] argmax template indices (outputs)
 *   block_len   samples per step and stream, multiple of 8 (e.g. 4096)
 * The stream positions live on the device, so each replay of the same graph
 * advances every live stream by one block; ended streams are skipped and the
 * last block of a stream may be partial. Banks start cold. EINVAL for banks
 * that differ in layout, keep their strain window outside LDS, or hold
 * templates split over workgroups.
 */
int spiir_batch_create(spiir_batch **out, int32_t n_streams, spiir_bank *const *banks,
                       const float *const *x_dev, const int64_t *lengths,
                       float *const *max_dev, int32_t *const *argmax_dev,
                       int32_t block_len, void *stream);

/* One graph replay on stream: one block of every live stream.
 *
 * A batch holds two graphs. The plain one runs each (stream, workgroup) item
 * over the whole block. The time-split one cuts each live stream's block into
 * segments of whole chunks (as spiir_bank_opts.time_split does for one bank:
 * segment-local pass, FP64 carry chain, carry-only pass), which multiplies the
 * parallelism of the streams still running. By default a replay uses the
 * time-split graph when the live streams' workgroups fill at most half of the
 * device's resident workgroup slots (e.g. the tail of uneven streams); the
 * results agree with the plain graph to FP32 rounding. */
int spiir_batch_step(spiir_batch *batch, void *stream);

/* Graph choice of later replays: mode 0 = automatic (above), 1 = always the
 * plain graph (bitwise equal to per-bank streaming with time_split = 1),
 * 2 = always the time-split graph. EINVAL for another mode, or for mode 2 when
 * no stream's block holds two chunks (then no time-split graph exists). */
int spiir_batch_set_time_split(spiir_batch *batch, int32_t mode);

/* Number of steps until every stream has ended (host-side count). */
int spiir_batch_steps_total(const spiir_batch *batch, int64_t *steps);

/* Rewinds every stream to its start and resets the banks (cold start). */
int spiir_batch_reset(spiir_batch *batch, void *stream);

int spiir_batch_destroy(spiir_batch *batch);

/*
 * Autotuner: times the candidate chunk lengths {64, 128, 256, 512} and filters
 * per lane {1, 2, 3, 4} on the given bank definitions (the same arguments as
 * spiir_bank_create, for n_banks banks at once, run as a batch over
 * block_len-sample blocks of synthetic input) and writes the fastest pair.
 * Results are cached per device and bank signature for the process.
 *   n_banks           >= 1
 *   n_templates       [n_banks]
 *   filter_offsets    [n_banks] pointers to int64 [T+1]
 *   a, b, d           [n_banks] pointers, as in spiir_bank_create
 *   max_delay         as spiir_bank_opts.max_delay (0 = max d)
 *   table             optional float [16] receiving ns per block-step for
 *                     (L index * 4 + F-1), L index over {64,128,256,512}; NULL allowed
 */
int spiir_autotune(int32_t n_banks, const int32_t *n_templates,
                   const int64_t *const *filter_offsets, const double *const *a,
                   const double *const *b, const int32_t *const *d, int32_t max_delay,
                   int32_t block_len, int32_t device, int32_t *chunk_len_out,
                   int32_t *filters_per_lane_out, float *table);

/* Kernel timing of a bank's forward launches (measurement aid; results do not
 * depend on it).
 *
 * spiir_bank_time_kernels(bank, 1) makes every later forward launch of the bank
 * (spiir_filter_block, spiir_trigger_max, spiir_forward_z; one launch per piece
 * of at most max_block samples) record the start time of its first forward
 * kernel and the end time of its last forward kernel with HIP events attached
 * to the kernel dispatches themselves; the max/argmax finalisation and history
 * copy are not included. 0 switches it off and frees the events. Enabling
 * clears the running totals.
 *
 * spiir_bank_kernel_time waits for the recorded launches to finish, returns the
 * summed kernel time in milliseconds and the number of launches since the last
 * read, and clears both. The events live in a ring of 256 pairs: a launch that
 * would reuse a pair first waits on the host for the launch 256 calls earlier.
 * Returns SPIIR_ESTATE if timing is off.
 */
int spiir_bank_time_kernels(spiir_bank *bank, int32_t enable);
int spiir_bank_kernel_time(spiir_bank *bank, double *total_ms, int64_t *launches);

/*
 * Multi-rate bank. The paper notes that the slow frequency evolution of an
 * inspiral lets the data and the templates run at a reduced sampling rate
 * (Sect. "Multimessenger astronomy"). This library's reading: the filters
 * of every template are split over levels r = 0..R; level r runs at 1/2^r of
 * the input rate, on the stream decimated r times by two, and its template
 * sums are interpolated back one halving at a time and added:
 *
 *   x_0 = x,  x_r[q] = sum_i h[i] x_{r-1}[2q + 1 - i]             (decimation)
 *   z_r[j] = sum over template j's level-r filters of y_k, run on x_r
 *   w_R = z_R,  w_r[p] = z_r[p] + sum_q g[p - 2q] w_{r+1}[q]     (interpolation)
 *   z = w_0,  snr_j = |z_j|^2,  max / argmax over templates as spiir_trigger_max
 *
 * h and g are causal FIR filters given by the caller (a lowpass for each;
 * g with each polyphase half summing to 1 keeps a constant's level).
 * Samples before the stream start are 0. All arithmetic is FP32 apart from
 * the banks' FP64 chunk carries.
 *
 *   n_levels         R + 1, 1..8
 *   n_templates      T >= 1, the same templates at every level
 *   filter_offsets   [n_levels] pointers to int64 [T+1], non-decreasing (a
 *                    template may have no filters at a level; at least one
 *                    level must hold a filter)
 *   a, b, d          [n_levels] pointers as in spiir_bank_create, coefficients
 *                    and delays in that level's samples (NULL for a level
 *                    without filters)
 *   decim_taps       float64 [n_decim_taps], 1..64 taps (h)
 *   interp_taps      float64 [n_interp_taps], 1..64 taps (g)
 *   opts             applied to every level's bank; max_block counts full-rate
 *                    samples (rounded down to a multiple of 2^R; level r gets
 *                    max_block / 2^r). With time_split = 0, a level of at most
 *                    128 filters per compute unit (a short serial recursion
 *                    per call) takes up to 32 time segments instead of 8.
 *                    Two or more such levels run as one group of launches
 *                    when their banks agree in layout (with waves_per_group
 *                    = 0 they are built with the group's largest workgroup
 *                    size, at least 4 waves), and one bank call each while
 *                    kernel timing is on; a single such level uses 64-sample
 *                    chunks instead of chunk_len.
 * Calls take n a multiple of 2^R and continue one stream. Device memory held:
 * the level banks, the decimated streams, the level sums and ceil(T / 16) x
 * max_block uint64 keys. The interpolation runs in one launch per piece, each
 * workgroup forming the interpolated sums its full-rate samples need in LDS,
 * so neither those sums nor the full-rate z are stored (z is only written to
 * the caller's buffer by spiir_multirate_filter_block_z). The decimation of
 * every level also runs in one launch when max_block / 2 + max_block / 4
 * samples fit in 64 KB of LDS, else one launch per level.
 */
int spiir_multirate_create(spiir_multirate **out, int32_t n_levels, int32_t n_templates,
                           const int64_t *const *filter_offsets, const double *const *a,
                           const double *const *b, const int32_t *const *d,
                           const double *decim_taps, int32_t n_decim_taps,
                           const double *interp_taps, int32_t n_interp_taps,
                           const spiir_bank_opts *opts);
int spiir_multirate_destroy(spiir_multirate *mr);

/* Cold start: every level's bank and every resampling history. */
int spiir_multirate_reset(spiir_multirate *mr, void *stream);

/* The next n samples (n a multiple of 2^R): full-rate z into z_dev, complex64
 * row-major [T][ld_z], ld_z >= n. */
int spiir_multirate_filter_block_z(spiir_multirate *mr, const float *x_dev, int64_t n,
                                   float *z_dev, int64_t ld_z, void *stream);

/* The next n samples: per-sample max over templates of |z_j|^2 and the
 * smallest attaining template (float32 max_dev [n], int32 argmax_dev [n]). */
int spiir_multirate_trigger_max(spiir_multirate *mr, const float *x_dev, int64_t n,
                                float *max_dev, int32_t *argmax_dev, void *stream);

/* Graph replay of trigger calls (on by default): once a piece has run
 * eagerly, every spiir_multirate_trigger_max piece of exactly max_block
 * samples replays a HIP graph of the whole piece (decimation, level banks,
 * interpolation, max / argmax), captured on first use for each history
 * parity; the block is copied into an internal buffer and the results out
 * of one. Results are identical to the eager path. Other piece lengths,
 * spiir_multirate_filter_block_z and runs with kernel timing enabled on a
 * level bank take the eager path. 0 switches the graphs off. */
int spiir_multirate_set_graph(spiir_multirate *mr, int32_t enable);

/* The bank that runs level `level` (NULL when the level holds no filters),
 * owned by the multi-rate bank: for spiir_bank_get_info and kernel timing
 * only; filtering through it directly would desynchronise the levels. Its
 * templates are the templates with filters at that level, in order. */
int spiir_multirate_level_bank(spiir_multirate *mr, int32_t level, spiir_bank **bank);

/*
 * Whitening front end. The bank filters whitened strain; the paper's SPIIR
 * section starts from noisy detector data ("SPIIR method"), so this is the
 * step before the bank. This library's reading, with frames of N samples at
 * hop H = N/2 and the periodic Hann window w[t] = sin^2(pi t / N) (which sums
 * to 1 over overlapping frames):
 *
 *   PSD        S[f] = mean over the frames k of a training stretch of
 *                     |sum_t w[t] s[kH + t] exp(-2 pi i f t / N)|^2 / sum_t w[t]^2,
 *                     f = 0..N/2 (white noise of variance v gives S = v)
 *   whitening  with xp = H zeros followed by the stream x, frame j covers
 *              xp[jH, jH + N); its windowed DFT is divided by sqrt(S[min(f, N-f)])
 *              (bins with S = 0 are zeroed) and the inverse DFT is added into
 *              the output at jH. The output is the whitened stream delayed by H
 *              samples; with S = 1 it is x delayed by H exactly.
 *
 * Transforms run in FP32 on the device (radix-2 FFT per frame in LDS); the
 * PSD average is accumulated in FP64.
 *
 *   frame_len   N, a power of two in [16, 8192]
 *   max_block   most samples per internal piece (0 = 65536; rounded to a
 *               multiple of H); longer calls are split
 *   device      HIP device ordinal; -1 = current
 */
int spiir_whitener_create(spiir_whitener **out, int32_t frame_len, int32_t max_block, int32_t device);
int spiir_whitener_destroy(spiir_whitener *wh);

/* PSD from train_dev float32 [n] (n >= N: (n - N) / H + 1 frames), enqueued on
 * stream. Grows its frame buffer on demand (allocation: not for use under
 * graph capture). */
int spiir_whitener_estimate_psd(spiir_whitener *wh, const float *train_dev, int64_t n, void *stream);

/* Host PSD float64 [N/2 + 1], finite and >= 0; synchronous. */
int spiir_whitener_set_psd(spiir_whitener *wh, const double *psd);
int spiir_whitener_get_psd(spiir_whitener *wh, double *psd);

/* Whitens the next n samples (n a multiple of N/2) into out_dev float32 [n]
 * (out_dev must not overlap x_dev); the stream continues across calls.
 * SPIIR_ESTATE until a PSD has been set or estimated. */
int spiir_whitener_process(spiir_whitener *wh, const float *x_dev, int64_t n, float *out_dev,
                           void *stream);

/* Cold start: zero history and pending output (the PSD is kept). */
int spiir_whitener_reset(spiir_whitener *wh, void *stream);

/*
 * Trigger clustering over a per-sample max / argmax series such as the output
 * of spiir_trigger_max: thresholding the detection statistic and keeping one
 * peak (sample, template, SNR) per cluster. The paper uses the SNR output to
 * decide whether a signal is present (Sect. "GPU accelerated SPIIR method",
 * subsection "SPIIR method") and names low-latency trigger generation as the
 * purpose (Sect. "Multimessenger astronomy"); it gives no clustering rule, so
 * this library reads it as a peak finder over a window of W samples:
 *
 *   m is a trigger  <=>  max[m] >= threshold,
 *                        max[i] <  max[m] for every i in [m - W, m),
 *                        max[i] <= max[m] for every i in (m, m + W],
 *
 * with the windows clipped to [0, n). Among equal values the earliest sample
 * wins, so triggers are more than W samples apart. Comparisons are float32;
 * -0 equals +0, a NaN never triggers and suppresses every sample within W of
 * it. Triggers are written in increasing sample order.
 *
 * The rule depends on the series only within W of each sample, so a stream can
 * be clustered piecewise: a call on samples [s, e) of a longer series gives the
 * whole series' answer for every m with s + W <= m < e - W (overlap calls by 2W).
 *
 *   max_dev, argmax_dev  float32 [n], int32 [n]; device memory (may be NULL when
 *                        n = 0). Any alignment of 4 bytes.
 *   threshold            SNR threshold (a NaN threshold selects nothing)
 *   window               W >= 0; W = 0 keeps every sample at or above threshold
 *   workspace_dev        device scratch of spiir_cluster_workspace_size(n) bytes or
 *                        more, owned by the caller; contents need no clearing and
 *                        are overwritten. NULL allowed when n = 0.
 *   index_dev            int64 [capacity]: trigger sample indices, ascending
 *   template_dev         int32 [capacity]: argmax[index]
 *   snr_dev              float32 [capacity]: max[index]
 *                        (all three may be NULL when capacity = 0)
 *   count_dev            int64 [1], device memory: the total number of triggers,
 *                        also when it exceeds capacity (then only the first
 *                        capacity triggers are written)
 *   device               HIP device ordinal of every buffer and of stream; -1 = current
 * Everything is enqueued on stream (no host synchronisation, no allocation);
 * calls sharing a workspace must be ordered on one stream. Errors: EINVAL for
 * null pointers, n outside [0, 2^40], W < 0, capacity < 0 or a short workspace;
 * ENODEV for a missing or non-gfx950 device.
 */
int spiir_cluster_workspace_size(int64_t n, size_t *nbytes);
int spiir_cluster_triggers(const float *max_dev, const int32_t *argmax_dev, int64_t n,
                           float threshold, int32_t window, void *workspace_dev,
                           size_t workspace_bytes, int64_t *index_dev, int32_t *template_dev,
                           float *snr_dev, int64_t capacity, int64_t *count_dev, int32_t device,
                           void *stream);

/*
 * Streaming trigger clustering (the rule of spiir_cluster_triggers) for a
 * max / argmax series that arrives block by block, as spiir_trigger_max
 * produces it. A sample's triggers are final once the W samples after it have
 * arrived, so each push emits, in increasing order and with absolute sample
 * indices, the triggers among the samples that became final with it: the
 * latency is W samples. Across all pushes and the final flush the output is
 * exactly spiir_cluster_triggers on the whole series.
 *
 *   create   threshold and window W >= 0 as in spiir_cluster_triggers;
 *            max_block = most samples per push (1 .. 2^32). Device memory:
 *            two windows of 2W + max_block samples and a clustering workspace.
 *   push     max_dev float32 [n], argmax_dev int32 [n], 0 <= n <= max_block;
 *            writes up to capacity triggers (index_dev int64, template_dev
 *            int32, snr_dev float32; NULL allowed with capacity 0) and their
 *            count (also when above capacity) to count_dev int64 [1].
 *   flush    end of the stream: emits the triggers of the last W samples (their
 *            windows clipped at the end). Push after flush only after reset.
 *   reset    starts a new stream at sample 0.
 * Everything is enqueued on stream; the object keeps host-side positions, so
 * its calls must be made from one thread in stream order.
 */
int spiir_trigger_stream_create(spiir_trigger_stream **out, float threshold, int32_t window,
                                int64_t max_block, int32_t device);
int spiir_trigger_stream_push(spiir_trigger_stream *ts, const float *max_dev,
                              const int32_t *argmax_dev, int64_t n, int64_t *index_dev,
                              int32_t *template_dev, float *snr_dev, int64_t capacity,
                              int64_t *count_dev, void *stream);
int spiir_trigger_stream_flush(spiir_trigger_stream *ts, int64_t *index_dev, int32_t *template_dev,
                               float *snr_dev, int64_t capacity, int64_t *count_dev, void *stream);
int spiir_trigger_stream_reset(spiir_trigger_stream *ts, void *stream);
int spiir_trigger_stream_destroy(spiir_trigger_stream *ts);

/* Message of the last failure on the calling thread ("" if none). */
const char *spiir_last_error(void);

/* Library version string. */
const char *spiir_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPIIR_H */
