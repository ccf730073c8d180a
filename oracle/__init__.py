"""FP64 CPU oracle for the SPIIR filter bank: TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package. It shares no code with the HIP library (the C source is
``spiir_oracle.c``, built with gcc into ``liboracle.so`` next to it).

Functions (all double precision; see the C source for the definitions):
  z(bank, x, templates)          complex128 [len(templates), n]
  snr(bank, x, templates)        float64    [len(templates), n]
  trigger(bank, x, peaks)        (float64 max [n], int32 argmax [n][, float64 peak [T]])
  backward(bank, x, G)           (grad_a, grad_b) complex128 [F]
  overlap_loss(z, g)             per-template loss and its gradient G
  clusters(M, J, threshold, W)   (index int64, template int32, value float32) of the triggers
  multirate_z(levels, h, g, x)   complex128 [T, n]: multi-rate bank, full-rate template sums
  multirate_trigger(levels, h, g, x)  (float64 max [n], int32 argmax [n]) of |multirate_z|^2
  welch_psd(s, N)                float64 [N/2+1]: averaged windowed periodogram
  whiten(x, S, N)                float64 [n]: frame-wise division by sqrt(S), overlap-added

Parity status: every function here is pinned by tests in
``tests/test_oracle_pins.py`` against closed forms, a library IIR routine,
brute-force convolution, superposition, finite differences and an
independent autograd implementation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spiir_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, OpenMP, no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_z.argtypes = [P, P, P, P, P, i32, P, i64, P, i32]
        lib.oracle_snr.argtypes = [P, P, P, P, P, i32, P, i64, P, i32]
        lib.oracle_trigger.argtypes = [P, P, P, P, i32, P, i64, P, P, P, i32]
        lib.oracle_backward.argtypes = [P, P, P, P, i32, P, i64, P, P, P, i32]
        for f in (lib.oracle_z, lib.oracle_snr, lib.oracle_trigger, lib.oracle_backward):
            f.restype = ctypes.c_int
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_clusters.argtypes = [P, P, i64, ctypes.c_float, i32, P, P, P, i64]
        lib.oracle_clusters.restype = i64
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _p(arr):
    return arr.ctypes.data_as(ctypes.c_void_p)


def _bank_arrays(bank):
    off = np.ascontiguousarray(bank.offsets, dtype=np.int64)
    a = np.ascontiguousarray(np.asarray(bank.a, dtype=np.complex128))
    b = np.ascontiguousarray(np.asarray(bank.b, dtype=np.complex128))
    d = np.ascontiguousarray(bank.d, dtype=np.int32)
    return off, a, b, d


def _threads(nthreads):
    return max_threads() if nthreads is None else int(nthreads)


def z(bank, x, templates=None, nthreads=None) -> np.ndarray:
    """Summed filter output z_j[m] (complex128 [len(templates), n]) from a cold start."""
    lib = _load()
    off, a, b, d = _bank_arrays(bank)
    T = len(off) - 1
    tpl = np.arange(T, dtype=np.int32) if templates is None else np.asarray(templates, np.int32)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((len(tpl), len(xd)), np.complex128)
    rc = lib.oracle_z(_p(off), _p(a), _p(b), _p(d), _p(tpl), len(tpl), _p(xd), len(xd),
                      _p(out), _threads(nthreads))
    if rc:
        raise RuntimeError("oracle_z failed (%d)" % rc)
    return out


def snr(bank, x, templates=None, nthreads=None) -> np.ndarray:
    """SNR_j[m] = |z_j[m]|^2 (float64 [len(templates), n])."""
    lib = _load()
    off, a, b, d = _bank_arrays(bank)
    T = len(off) - 1
    tpl = np.arange(T, dtype=np.int32) if templates is None else np.asarray(templates, np.int32)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros((len(tpl), len(xd)), np.float64)
    rc = lib.oracle_snr(_p(off), _p(a), _p(b), _p(d), _p(tpl), len(tpl), _p(xd), len(xd),
                        _p(out), _threads(nthreads))
    if rc:
        raise RuntimeError("oracle_snr failed (%d)" % rc)
    return out


def trigger(bank, x, nthreads=None, peaks=False):
    """Per-sample max over templates of SNR and the smallest index attaining
    it; with peaks=True also every template's largest SNR over the stream
    (float64 [T])."""
    lib = _load()
    off, a, b, d = _bank_arrays(bank)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    mx = np.zeros(len(xd), np.float64)
    am = np.zeros(len(xd), np.int32)
    pk = np.zeros(len(off) - 1, np.float64)
    rc = lib.oracle_trigger(_p(off), _p(a), _p(b), _p(d), len(off) - 1, _p(xd), len(xd),
                            _p(mx), _p(am), _p(pk) if peaks else None, _threads(nthreads))
    if rc:
        raise RuntimeError("oracle_trigger failed (%d)" % rc)
    return (mx, am, pk) if peaks else (mx, am)


def clusters(M, J, threshold, window):
    """Triggers of a fused max/argmax series: the loudest sample of every
    +-window neighbourhood at or above the threshold (earliest on ties)."""
    lib = _load()
    M = np.ascontiguousarray(M, np.float32)
    J = np.ascontiguousarray(J, np.int32)
    n = len(M)
    cap = n // (int(window) + 1) + 1   # triggers are more than `window` apart
    idx = np.zeros(cap, np.int64)
    tpl = np.zeros(cap, np.int32)
    val = np.zeros(cap, np.float32)
    cnt = lib.oracle_clusters(_p(M), _p(J), n, ctypes.c_float(threshold), int(window), _p(idx), _p(tpl),
                              _p(val), cap)
    if cnt > cap:
        raise RuntimeError("oracle_clusters: %d triggers exceed the bound %d" % (cnt, cap))
    return idx[:cnt], tpl[:cnt], val[:cnt]


def backward(bank, x, G, nthreads=None):
    """Gradients (grad_a, grad_b), complex128 [F], of a real loss whose gradient
    with respect to z is G (complex128 [T, n], convention dL/dRe + i dL/dIm)."""
    lib = _load()
    off, a, b, d = _bank_arrays(bank)
    T = len(off) - 1
    xd = np.ascontiguousarray(x, dtype=np.float64)
    Gc = np.ascontiguousarray(G, dtype=np.complex128)
    if Gc.shape != (T, len(xd)):
        raise ValueError("G must be [T, n]")
    ga = np.zeros(len(a), np.complex128)
    gb = np.zeros(len(a), np.complex128)
    rc = lib.oracle_backward(_p(off), _p(a), _p(b), _p(d), T, _p(xd), len(xd), _p(Gc),
                             _p(ga), _p(gb), _threads(nthreads))
    if rc:
        raise RuntimeError("oracle_backward failed (%d)" % rc)
    return ga, gb


def overlap_loss(zs: np.ndarray, gs: np.ndarray):
    """Template-overlap loss L_j = 1 - |<z_j, g_j>| / (|z_j| |g_j|), with
    <u, v> = sum_m u[m] conj(v[m]), and G_j = dL_j/dRe(z_j) + i dL_j/dIm(z_j):

      G = -(1/(Z Gn)) [ (c/|c|) g - (|c|/Z^2) z ],  c = <z, g>, Z = |z|, Gn = |g|.

    Inputs complex128 [T, n]; returns (loss [T] float64, G [T, n] complex128).
    """
    zs = np.asarray(zs, np.complex128)
    gs = np.asarray(gs, np.complex128)
    c = np.sum(zs * np.conj(gs), axis=1)
    Z = np.sqrt(np.sum(np.abs(zs) ** 2, axis=1))
    Gn = np.sqrt(np.sum(np.abs(gs) ** 2, axis=1))
    ac = np.abs(c)
    loss = 1.0 - ac / (Z * Gn)
    phase = np.where(ac > 0, c / np.where(ac > 0, ac, 1.0), 0.0)
    G = -(1.0 / (Z * Gn))[:, None] * (phase[:, None] * gs - (ac / Z ** 2)[:, None] * zs)
    return loss, G


def decimate(x, h):
    """One halving of the sample rate: x_r[q] = sum_i h[i] x[2q + 1 - i]
    (causal FIR h, x[m < 0] = 0), len(x) // 2 outputs."""
    x = np.asarray(x)
    full = np.convolve(x, np.asarray(h, np.float64))
    return full[1:len(x):2].copy()


def upsample(w, g, n_out):
    """One doubling of the sample rate: U(w)[p] = sum_q g[p - 2q] w[q] over
    0 <= p - 2q < len(g), i.e. w zero-stuffed to the doubled rate and passed
    through the causal FIR g, first n_out outputs."""
    w = np.asarray(w)
    s = np.zeros(n_out, w.dtype)
    s[0::2] = w[:(n_out + 1) // 2]
    return np.convolve(s, np.asarray(g, np.float64))[:n_out]


def multirate_z(levels, h, g, x, nthreads=None) -> np.ndarray:
    """Full-rate template sums of a multi-rate bank (the paper's remark that the
    sampling rate of data and templates can be lowered where the signal
    evolves slowly, Sect. "Multimessenger astronomy"; the steps are this
    library's reading of it). levels[r] is a bank whose filters run at
    1 / 2^r of the input rate, every level with the same templates (a
    template may have no filters at a level); coefficients and delays are in
    that level's samples.

      x_0 = x,  x_r = decimate(x_{r-1}, h)                  (r = 1..R)
      z_r[j] = sum over the level-r filters of template j of y_k, run on x_r
      w_R = z_R,  w_r = z_r + upsample(w_{r+1}, g)           (r = R-1..0)
      result = w_0

    Cold start; len(x) must be a multiple of 2^R. FP64."""
    R = len(levels) - 1
    x = np.asarray(x, np.float64)
    n = len(x)
    if n % (1 << R):
        raise ValueError("len(x) must be a multiple of 2^%d" % R)
    T = levels[0].n_templates
    xs = [x]
    for r in range(1, R + 1):
        xs.append(decimate(xs[-1], h))
    w = None
    for r in range(R, -1, -1):
        lv = levels[r]
        if lv.n_templates != T:
            raise ValueError("every level needs the same templates")
        nr = len(xs[r])
        zr = z(lv, xs[r], nthreads=nthreads) if lv.n_filters > 0 else np.zeros((T, nr), np.complex128)
        if w is not None:
            for j in range(T):
                zr[j] += upsample(w[j], g, nr)
        w = zr
    return w


def multirate_trigger(levels, h, g, x, nthreads=None):
    """Per-sample max over templates of |multirate_z|^2 and the smallest index
    attaining it."""
    zz = multirate_z(levels, h, g, x, nthreads=nthreads)
    s = zz.real ** 2 + zz.imag ** 2
    return s.max(axis=0), np.argmax(s, axis=0).astype(np.int32)


def hann(N):
    """Periodic Hann window w[t] = sin^2(pi t / N); w[t] + w[t + N/2] = 1."""
    t = np.arange(N)
    return np.sin(np.pi * t / N) ** 2


def welch_psd(s, N):
    """Noise power spectral density of a training stretch, the whitening
    filter's input (the path filters whitened strain; the paper's SPIIR
    section takes noisy detector data as its input, "SPIIR method"). Frames
    of N samples at hop N/2 (as many as fit), periodic Hann window w:
    S[f] = mean over frames of |sum_t w[t] s[kH + t] e^{-2 pi i f t / N}|^2
    divided by sum_t w[t]^2, for f = 0..N/2 (white noise of variance v gives
    S = v)."""
    s = np.asarray(s, np.float64)
    H = N // 2
    K = (len(s) - N) // H + 1
    if K < 1:
        raise ValueError("need at least N samples")
    w = hann(N)
    acc = np.zeros(N)
    for k in range(K):
        X = np.fft.fft(w * s[k * H:k * H + N])
        acc += X.real ** 2 + X.imag ** 2
    return acc[:H + 1] / K / np.sum(w * w)


def whiten(x, S, N):
    """Whitened stream, delayed by H = N/2 samples: with xp = H zeros followed
    by x, frame j covers xp[jH, jH + N); its windowed DFT is divided by
    sqrt(S[f]) (f and N - f share S[f]; bins with S <= 0 are zeroed), the
    inverse DFT is overlap-added at jH; frames j = 0 .. len(x)/H - 1, first
    len(x) outputs. With S = 1 the output is x delayed by H exactly (the
    window sums to 1 over overlapping frames)."""
    x = np.asarray(x, np.float64)
    S = np.asarray(S, np.float64)
    H = N // 2
    n = len(x)
    if n % H:
        raise ValueError("len(x) must be a multiple of N/2")
    xp = np.concatenate([np.zeros(H), x])
    inv = np.where(S > 0, 1.0 / np.sqrt(np.where(S > 0, S, 1.0)), 0.0)
    f = np.arange(N)
    inv_full = inv[np.minimum(f, N - f)]
    w = hann(N)
    out = np.zeros(n + N)
    for j in range(n // H):
        X = np.fft.fft(w * xp[j * H:j * H + N])
        out[j * H:j * H + N] += np.fft.ifft(X * inv_full).real
    return out[:n]
