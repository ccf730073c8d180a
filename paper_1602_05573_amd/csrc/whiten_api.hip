// Host side of the whitening front end (spiir_whitener_*). Declared in
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

}  // extern "C"
