/*
 * FP64 CPU oracle for the summed parallel IIR (SPIIR) filter bank.
 *
 * TEST INFRASTRUCTURE ONLY. Called by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark. It shares no code, header or constant
 * with the HIP library it checks, and the library never calls it.
 *
 * What is computed (Sect. "GPU accelerated SPIIR method", subsection
 * "SPIIR method": a template's SNR is approximated by the summed output of a
 * parallel bank of single-pole IIR filters; subsection "Optimized GPU
 * implementation of SPIIR": each filter's output feeds its next iteration and
 * a template's SNR needs the outputs of all its filters). With the readings
 * recorded in the design notes, for template j with filters k in
 * [off[j], off[j+1]) and samples m = 0 .. n-1:
 *
 *   y_k[m]   = a_k * y_k[m-1] + b_k * x[m - d_k],  y_k[-1] = 0, x[<0] = 0
 *   z_j[m]   = sum_k y_k[m]
 *   snr_j[m] = Re(z_j[m])^2 + Im(z_j[m])^2
 *   M[m]     = max_j snr_j[m],  J[m] = smallest j attaining M[m]
 *
 * Everything is double precision, written out in real arithmetic, built
 * without fast-math and without floating-point contraction. Complex arrays are
 * interleaved (re, im).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* One filter over the whole input, accumulated into z (length 2n). */
static void run_filter(double ar, double ai, double br, double bi, int64_t d,
                       const double *x, int64_t n, double *z)
{
    double yr = 0.0, yi = 0.0;
    for (int64_t m = 0; m < n; ++m) {
        double xin = (m - d >= 0) ? x[m - d] : 0.0;
        double nr = ar * yr - ai * yi + br * xin;
        double ni = ar * yi + ai * yr + bi * xin;
        yr = nr;
        yi = ni;
        z[2 * m] += yr;
        z[2 * m + 1] += yi;
    }
}

/* z of one template (filters k0..k1-1). Filters are split over nthreads
 * contiguous ranges; the per-thread partial sums are added in thread order,
 * so the result depends only on nthreads. */
static int template_z(const double *a, const double *b, const int32_t *d,
                      int64_t k0, int64_t k1, const double *x, int64_t n,
                      double *z, int nthreads)
{
    memset(z, 0, sizeof(double) * 2 * (size_t)n);
    int64_t nk = k1 - k0;
    if (nk <= 0 || n <= 0) return 0;
    if (nthreads <= 1 || nk < 2) {
        for (int64_t k = k0; k < k1; ++k)
            run_filter(a[2 * k], a[2 * k + 1], b[2 * k], b[2 * k + 1], d[k], x, n, z);
        return 0;
    }
    if (nthreads > nk) nthreads = (int)nk;
    double *part = (double *)calloc((size_t)nthreads * 2 * (size_t)n, sizeof(double));
    if (!part) return -2;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
        int64_t lo = k0 + nk * t / nthreads, hi = k0 + nk * (t + 1) / nthreads;
        double *zt = part + (size_t)t * 2 * (size_t)n;
        for (int64_t k = lo; k < hi; ++k)
            run_filter(a[2 * k], a[2 * k + 1], b[2 * k], b[2 * k + 1], d[k], x, n, zt);
    }
    for (int t = 0; t < nthreads; ++t) {
        const double *zt = part + (size_t)t * 2 * (size_t)n;
        for (int64_t i = 0; i < 2 * n; ++i) z[i] += zt[i];
    }
    free(part);
    return 0;
}

/* z_j for the listed templates, each over samples 0..n-1 from a cold start.
 * z_out is [ntpl][2n]. Templates run in parallel when there are several;
 * a single template is split over its filters instead. */
int oracle_z(const int64_t *off, const double *a, const double *b, const int32_t *d,
             const int32_t *tpl, int32_t ntpl, const double *x, int64_t n,
             double *z_out, int32_t nthreads)
{
    if (!off || !a || !b || !d || !tpl || !x || !z_out || n < 0 || ntpl < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    int rc = 0;
    if (ntpl * 2 <= nthreads) {
        /* few templates: one at a time, each split over its filters */
        for (int32_t i = 0; i < ntpl; ++i) {
            int r = template_z(a, b, d, off[tpl[i]], off[tpl[i] + 1], x, n,
                               z_out + (size_t)i * 2 * (size_t)n, nthreads);
            if (r) rc = r;
        }
        return rc;
    }
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int32_t i = 0; i < ntpl; ++i) {
        int r = template_z(a, b, d, off[tpl[i]], off[tpl[i] + 1], x, n,
                           z_out + (size_t)i * 2 * (size_t)n, 1);
        if (r) rc = r;
    }
    return rc;
}

/* snr_j[m] = |z_j[m]|^2 for the listed templates: snr_out is [ntpl][n]. */
int oracle_snr(const int64_t *off, const double *a, const double *b, const int32_t *d,
               const int32_t *tpl, int32_t ntpl, const double *x, int64_t n,
               double *snr_out, int32_t nthreads)
{
    if (!snr_out || n < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    int rc = 0;
    /* few templates: one at a time, each split over its filters */
    int outer = (ntpl * 2 <= nthreads) ? 1 : nthreads;
    int inner = (outer == 1) ? nthreads : 1;
#pragma omp parallel for num_threads(outer) schedule(dynamic, 1)
    for (int32_t i = 0; i < ntpl; ++i) {
        double *z = (double *)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
        if (!z) { rc = -2; continue; }
        int r = template_z(a, b, d, off[tpl[i]], off[tpl[i] + 1], x, n, z, inner);
        if (r) rc = r;
        double *s = snr_out + (size_t)i * (size_t)n;
        for (int64_t m = 0; m < n; ++m) s[m] = z[2 * m] * z[2 * m] + z[2 * m + 1] * z[2 * m + 1];
        free(z);
    }
    return rc;
}

/* Per-sample maximum of snr over all T templates and the smallest template
 * index attaining it. Templates are split into contiguous ranges, one per
 * thread; within a range a strictly larger value replaces the running
 * maximum, and ranges are merged in increasing order with the same rule, so
 * ties always resolve to the smallest index. peak_out (NULL allowed) receives
 * every template's largest snr over the n samples, the scale of the
 * admissible-set rule for argmax ties. */
int oracle_trigger(const int64_t *off, const double *a, const double *b, const int32_t *d,
                   int32_t T, const double *x, int64_t n,
                   double *max_out, int32_t *arg_out, double *peak_out, int32_t nthreads)
{
    if (!off || !a || !b || !d || !x || !max_out || !arg_out || T < 1 || n < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > T) nthreads = T;
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *pm = (double *)malloc(sizeof(double) * nn * (size_t)nthreads);
    int32_t *pj = (int32_t *)malloc(sizeof(int32_t) * nn * (size_t)nthreads);
    if (!pm || !pj) { free(pm); free(pj); return -2; }
    int rc = 0;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
    for (int t = 0; t < nthreads; ++t) {
        int32_t j0 = (int32_t)((int64_t)T * t / nthreads);
        int32_t j1 = (int32_t)((int64_t)T * (t + 1) / nthreads);
        double *m_t = pm + (size_t)t * nn;
        int32_t *j_t = pj + (size_t)t * nn;
        double *z = (double *)malloc(sizeof(double) * 2 * nn);
        if (!z) { rc = -2; continue; }
        for (int64_t m = 0; m < n; ++m) { m_t[m] = -1.0; j_t[m] = -1; }
        for (int32_t j = j0; j < j1; ++j) {
            template_z(a, b, d, off[j], off[j + 1], x, n, z, 1);
            double pk = 0.0;
            for (int64_t m = 0; m < n; ++m) {
                double s = z[2 * m] * z[2 * m] + z[2 * m + 1] * z[2 * m + 1];
                if (s > m_t[m]) { m_t[m] = s; j_t[m] = j; }
                if (s > pk) pk = s;
            }
            if (peak_out) peak_out[j] = pk;
        }
        free(z);
    }
    for (int64_t m = 0; m < n; ++m) { max_out[m] = -1.0; arg_out[m] = -1; }
    for (int t = 0; t < nthreads; ++t) {
        const double *m_t = pm + (size_t)t * nn;
        const int32_t *j_t = pj + (size_t)t * nn;
        for (int64_t m = 0; m < n; ++m)
            if (j_t[m] >= 0 && m_t[m] > max_out[m]) { max_out[m] = m_t[m]; arg_out[m] = j_t[m]; }
    }
    free(pm);
    free(pj);
    return rc;
}

/*
 * Reverse-time adjoint of the filter bank for a real loss of z.
 *
 * G is [T][2n]: the loss gradient with respect to z in the convention
 * G = dL/dRe(z) + i dL/dIm(z). For filter k of template j, with
 *   lambda_k[m] = G_j[m] + conj(a_k) * lambda_k[m+1],  lambda_k[n] = 0,
 * the gradients in the same convention are
 *   grad_b_k = sum_m lambda_k[m] * x[m - d_k]
 *   grad_a_k = sum_m lambda_k[m] * conj(y_k[m-1]).
 * The forward outputs y_k are recomputed per filter and kept whole.
 * Filters run in parallel; each gradient is a plain sequential sum.
 */
int oracle_backward(const int64_t *off, const double *a, const double *b, const int32_t *d,
                    int32_t T, const double *x, int64_t n, const double *G,
                    double *grad_a, double *grad_b, int32_t nthreads)
{
    if (!off || !a || !b || !d || !x || !G || !grad_a || !grad_b || T < 1 || n < 0) return -1;
    if (nthreads < 1) nthreads = 1;
    int64_t F = off[T];
    int32_t *owner = (int32_t *)malloc(sizeof(int32_t) * (size_t)(F > 0 ? F : 1));
    if (!owner) return -2;
    for (int32_t j = 0; j < T; ++j)
        for (int64_t k = off[j]; k < off[j + 1]; ++k) owner[k] = j;
    int rc = 0;
#pragma omp parallel num_threads(nthreads)
    {
        double *y = (double *)malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
        if (!y) rc = -2;
#pragma omp for schedule(dynamic, 16)
        for (int64_t k = 0; k < F; ++k) {
            if (!y) continue;
            double ar = a[2 * k], ai = a[2 * k + 1], br = b[2 * k], bi = b[2 * k + 1];
            int64_t dk = d[k];
            const double *Gj = G + (size_t)owner[k] * 2 * (size_t)n;
            double yr = 0.0, yi = 0.0;
            for (int64_t m = 0; m < n; ++m) {
                double xin = (m - dk >= 0) ? x[m - dk] : 0.0;
                double nr = ar * yr - ai * yi + br * xin;
                double ni = ar * yi + ai * yr + bi * xin;
                yr = nr; yi = ni;
                y[2 * m] = yr; y[2 * m + 1] = yi;
            }
            double lr = 0.0, li = 0.0;      /* lambda_k[m+1] */
            double gar = 0.0, gai = 0.0, gbr = 0.0, gbi = 0.0;
            for (int64_t m = n - 1; m >= 0; --m) {
                /* lambda[m] = G[m] + conj(a) * lambda[m+1] */
                double nr = Gj[2 * m] + (ar * lr + ai * li);
                double ni = Gj[2 * m + 1] + (ar * li - ai * lr);
                lr = nr; li = ni;
                double xin = (m - dk >= 0) ? x[m - dk] : 0.0;
                gbr += lr * xin;
                gbi += li * xin;
                if (m >= 1) {
                    /* lambda * conj(y[m-1]) */
                    double pr = y[2 * (m - 1)], pi = y[2 * (m - 1) + 1];
                    gar += lr * pr + li * pi;
                    gai += li * pr - lr * pi;
                }
            }
            grad_a[2 * k] = gar; grad_a[2 * k + 1] = gai;
            grad_b[2 * k] = gbr; grad_b[2 * k + 1] = gbi;
        }
        free(y);
    }
    free(owner);
    return rc;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

/*
 * Trigger clustering, the step after the per-sample max (Sect. "GPU
 * accelerated SPIIR method", subsection "SPIIR method": the search identifies
 * the presence of a signal in noisy data; Sect. "Multimessenger astronomy",
 * subsection on the event timescale: low-latency searches must generate
 * triggers quickly). The paper states no clustering rule; the reading used
 * here keeps the loudest sample of every window: sample m is a trigger when
 *
 *   M[m] >= threshold,
 *   M[i] <  M[m] for every i in [m - W, m)      (inside [0, n)),
 *   M[i] <= M[m] for every i in (m, m + W]      (inside [0, n)),
 *
 * so equal values go to the earliest sample and triggers are more than W
 * apart. M is the float32 fused maximum; comparisons are made on those float32
 * values. Triggers are listed in increasing m with J[m] and M[m]; at most cap
 * are written, the return value is their total number.
 */
int64_t oracle_clusters(const float *M, const int32_t *J, int64_t n, float threshold, int32_t W,
                        int64_t *idx, int32_t *tpl, float *val, int64_t cap) {
    int64_t cnt = 0;
    for (int64_t m = 0; m < n; ++m) {
        const float v = M[m];
        if (!(v >= threshold)) continue;
        int keep = 1;
        const int64_t lo = m - W < 0 ? 0 : m - W;
        for (int64_t i = lo; i < m && keep; ++i)
            if (!(M[i] < v)) keep = 0;
        const int64_t hi = m + W >= n ? n - 1 : m + W;
        for (int64_t i = m + 1; i <= hi && keep; ++i)
            if (!(M[i] <= v)) keep = 0;
        if (!keep) continue;
        if (cnt < cap) {
            idx[cnt] = m;
            tpl[cnt] = J[m];
            val[cnt] = v;
        }
        ++cnt;
    }
    return cnt;
}
