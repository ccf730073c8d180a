// Host side of trigger clustering (spiir_cluster_*, spiir_trigger_stream_*).
// Declared in include/spiir.h.
#include "host_common.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

using namespace spiir;
using namespace spiir::host;

namespace {

constexpr int64_t kMaxClusterN = (int64_t)1 << 40;

}  // namespace

// Streaming trigger clustering: a window of the series, [base, base + len),
// holds the samples whose triggers are not final yet plus W samples before
// them; each push appends a block, clusters the window with candidates
// limited to the newly final samples [final_end, total - W) and keeps the
// last W samples before the new final_end. The window sits at offset off of
// buffer cur: a step only moves off past the dropped samples, and the next
// push with data writes the kept samples and the new block into the other
// buffer in one launch (ping-pong buffers).
struct spiir_trigger_stream {
    int device = 0;
    float thr = 0.0f;
    int64_t W = 0, B = 0;
    float *wm[2] = {nullptr, nullptr};
    int32_t *wj[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t off = 0;   // window start inside wm[cur] / wj[cur]
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
    HIPCHK(launch_cluster(ts->wm[c] + ts->off, ts->wj[c] + ts->off, ts->len, ts->thr, ts->W, ts->ws, cap, idx, tpl,
                          val, count, st, ts->final_end - ts->base, new_end - ts->base, ts->base));
    ts->final_end = new_end;
    const int64_t keep_from = std::max(ts->base, ts->final_end - ts->W) - ts->base;
    ts->off += keep_from;
    ts->base += keep_from;
    ts->len -= keep_from;
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
    int rc = resolve_device(device, dev);
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
    ts->off = ts->base = ts->len = ts->total = ts->final_end = 0;
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
    if (n > 0 && ts->off > 0) {   // kept samples and the block into the other buffer
        HIPCHK(launch_ts_compose(ts->wm[c] + ts->off, ts->wj[c] + ts->off, ts->len, max_dev, argmax_dev, n,
                                 ts->wm[c ^ 1], ts->wj[c ^ 1], st));
        ts->cur = c ^ 1;
        ts->off = 0;
    } else if (n > 0) {           // the window starts the buffer: append the block
        HIPCHK(launch_ts_compose(nullptr, nullptr, 0, max_dev, argmax_dev, n, ts->wm[c] + ts->len,
                                 ts->wj[c] + ts->len, st));
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
    const int rc = resolve_device(device, dev);
    if (rc) return rc;
    DeviceGuard guard(dev);
    HIPCHK(launch_cluster(max_dev, argmax_dev, n, threshold, window, workspace_dev, capacity, index_dev,
                          template_dev, snr_dev, count_dev, static_cast<hipStream_t>(stream)));
    return SPIIR_OK;
}

}  // extern "C"
