"""Shared helpers of the parity tests: error metrics and the argmax rule."""
import numpy as np

SNR_TOL = 1e-4      # peak-normalised SNR error gate for the FP32 paths
ARG_EPS = 1e-4      # half-width of the admissible set for argmax ties


def snr_err(gpu, ref):
    """max_j max_n |gpu - ref| / max_n ref, per template, and its maximum."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    peak = np.maximum(ref.max(axis=-1), 1e-300)
    per = np.abs(gpu - ref).max(axis=-1) / peak
    return float(np.max(per)), per


def check_argmax(gpu_max, gpu_arg, snr_ref, eps=ARG_EPS):
    """Checks the fused max/argmax against the oracle SNR matrix [T, n].

    Oracle argmax J = lowest index attaining the max. Admissible set
    A[n] = {j : ref_j[n] >= ref_J[n] - eps (P_j + P_J)} with P_j the peak of
    template j. The GPU index must equal J where |A| = 1 and lie in A
    otherwise; the GPU max must be within eps P of the oracle max.
    Returns the number of documented ties (|A| > 1).
    """
    ref = np.asarray(snr_ref, np.float64)
    T, n = ref.shape
    P = ref.max(axis=1)
    J = np.argmax(ref, axis=0)           # numpy argmax returns the first (lowest) index
    refJ = ref[J, np.arange(n)]
    thresh = refJ[None, :] - eps * (P[:, None] + P[J][None, :])
    adm = ref >= thresh
    nadm = adm.sum(axis=0)
    ga = np.asarray(gpu_arg).astype(np.int64)
    assert ga.min() >= 0 and ga.max() < T, "argmax out of range"
    unique = nadm == 1
    bad_unique = np.nonzero(unique & (ga != J))[0]
    assert bad_unique.size == 0, "argmax differs at unique samples %s" % bad_unique[:10]
    ok = adm[ga, np.arange(n)]
    assert ok.all(), "argmax outside the admissible set at %s" % np.nonzero(~ok)[0][:10]
    gm = np.asarray(gpu_max, np.float64)
    merr = np.abs(gm - refJ) / np.maximum(P[ga], 1e-300)
    assert merr.max() <= eps, "fused max error %.3g" % merr.max()
    return int((~unique).sum())
