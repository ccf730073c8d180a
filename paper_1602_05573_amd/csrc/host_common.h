// Host-side helpers shared by the library's C-ABI sources (api.hip,
// multirate_api.hip, whiten_api.hip, cluster_api.hip): error reporting,
// device selection, allocation, and the few bank operations the extension
// objects need. Internal; not installed.
#ifndef SPIIR_HOST_COMMON_H
#define SPIIR_HOST_COMMON_H

#include "spiir.h"
#include "spiir_internal.h"

#include <cstdarg>
#include <string>

namespace spiir {
namespace host {

// Records the message of a failure for spiir_last_error and returns code.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
extern thread_local std::string g_err;

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

struct DeviceFacts {
    int n_cu = 0;
    size_t lds_cap = 0;
};

// Device count, ordinal and gfx950 checks; fills the facts.
int device_facts(int dev, DeviceFacts &f);
// -1 = the current device; the gfx950 check is cached per ordinal.
int resolve_device(int32_t device, int &dev);

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

// Bank operations used by the multi-rate bank (the bank stays opaque here).
int bank_stream_z(spiir_bank *bk, const float *x, int64_t n, float *z, int64_t ld, hipStream_t st);
int bank_create_capped(spiir_bank **out, int32_t T, const int64_t *off, const double *a, const double *b,
                       const int32_t *d, const spiir_bank_opts &o, int seg_cap);
int bank_hist_cur(const spiir_bank *bk);
void bank_set_hist_cur(spiir_bank *bk, int v);
bool bank_timing_on(const spiir_bank *bk);
int bank_wpg(const spiir_bank *bk);
// Whether banks bks[0..nb) can take streaming z calls of n[b] samples through
// banks_stream_z_multi: each call one time-split piece (at most max_block
// samples, two segments or more) with the strain window in LDS, no split
// templates, no kernel timing, one device, and the same filters per lane,
// tile length and workgroup size.
bool banks_multi_ok(spiir_bank *const *bks, int nb, const int64_t *n);
// Streaming z calls of several banks, bank b on x[b][0..n[b]) into z[b] (row
// stride ld[b]), as one launch per time-split pass for all of them; the same
// results and state as one bank_stream_z call per bank.
int banks_stream_z_multi(spiir_bank *const *bks, int nb, const float *const *x, const int64_t *n, float *const *z,
                         const int64_t *ld, hipStream_t st);

}  // namespace host
}  // namespace spiir

#define HIPCHK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(SPIIR_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#endif  // SPIIR_HOST_COMMON_H
