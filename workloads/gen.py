"""Seeded generators for the five synthetic SPIIR workloads.

The paper's SPIIR experiment (Sect. "GPU accelerated SPIIR method",
subsection "Experimental results") ran on real pipeline data and real
template banks that are not public. These generators stand in for them with
banks of first-order complex IIR filters of the shapes the workloads name.

Seeds: ``numpy.random.default_rng([1602, family, role, idx])`` with role 0 =
strain, 1 = bank, 2 = chirp parameters, and idx = stream / template index.
The float32 strain array is canonical; bank coefficients are canonical in
complex128 (the library rounds them itself).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

SEED_ROOT = 1602
ROLE_STRAIN, ROLE_BANK, ROLE_CHIRP = 0, 1, 2

FS = 4096.0                 # sample rate of the chirp workloads (Hz)
T_SUN = 4.925491025543576e-06  # G * M_sun / c^3 in seconds


def _rng(family: int, role: int, idx: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_ROOT, family, role, idx])


@dataclass
class Bank:
    """A bank of templates, each a list of first-order complex IIR filters.

    offsets: int64 [T+1], filters of template j are offsets[j]:offsets[j+1]
    a, b:    complex128 [F] pole and gain of every filter
    d:       int32 [F] input delay in samples
    dmax:    int, the delay bound the bank is built for (>= max d)
    """

    offsets: np.ndarray
    a: np.ndarray
    b: np.ndarray
    d: np.ndarray
    dmax: int

    @property
    def n_templates(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_filters(self) -> int:
        return int(self.offsets[-1])

    def counts(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subset(self, templates) -> "Bank":
        """A bank made of the listed templates, in the given order."""
        templates = [int(j) for j in templates]
        parts = [slice(int(self.offsets[j]), int(self.offsets[j + 1])) for j in templates]
        cnt = np.array([s.stop - s.start for s in parts], dtype=np.int64)
        off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        cat = lambda v: np.concatenate([v[s] for s in parts])  # noqa: E731
        return Bank(off, cat(self.a), cat(self.b), cat(self.d).astype(np.int32), self.dmax)


def strain(n: int, family: int, idx: int = 0) -> np.ndarray:
    """Whitened strain stand-in: seeded white Gaussian noise, sigma = 1, float32."""
    return _rng(family, ROLE_STRAIN, idx).standard_normal(int(n)).astype(np.float32)


def random_bank(family: int, idx: int, n_templates: int, k_lo: int, k_hi: int,
                r_lo: float, r_hi: float, dmax: int,
                w_lo: float = 0.001 * math.pi, w_hi: float = 0.5 * math.pi) -> Bank:
    """Random bank: K_j ~ U{k_lo..k_hi}; per filter r ~ U[r_lo, r_hi],
    omega ~ U[w_lo, w_hi], a = r e^{i omega}; b circular complex normal
    (Re, Im iid N(0, 1/2)) scaled by 1/sqrt(K_j); d ~ U{0..dmax}.

    Draw order: all K_j first, then per template r, omega, Re b, Im b, d.
    """
    rng = _rng(family, ROLE_BANK, idx)
    k = rng.integers(k_lo, k_hi + 1, size=n_templates).astype(np.int64)
    off = np.concatenate([[0], np.cumsum(k)]).astype(np.int64)
    nf = int(off[-1])
    a = np.empty(nf, np.complex128)
    b = np.empty(nf, np.complex128)
    d = np.empty(nf, np.int32)
    s = math.sqrt(0.5)
    for j in range(n_templates):
        kj = int(k[j])
        sl = slice(int(off[j]), int(off[j + 1]))
        r = rng.uniform(r_lo, r_hi, kj)
        w = rng.uniform(w_lo, w_hi, kj)
        br = rng.standard_normal(kj) * s
        bi = rng.standard_normal(kj) * s
        dd = rng.integers(0, dmax + 1, size=kj)
        a[sl] = r * np.exp(1j * w)
        b[sl] = (br + 1j * bi) / math.sqrt(kj)
        d[sl] = dd
    return Bank(off, a, b, d, int(dmax))


# ---------------------------------------------------------------------------
# The five workloads. Each returns (bank(s), strain(s)) at full size unless a
# smaller n is asked for (tests use prefixes or reduced template counts).
# ---------------------------------------------------------------------------

def bank_4x128(n: int = 16384):
    """4 templates x 128 filters, r ~ U[0.99, 0.9999], d ~ U{0..2047}, 16,384 samples."""
    bank = random_bank(0, 0, 4, 128, 128, 0.99, 0.9999, 2047)
    return bank, strain(n, 0)


def bank_1024(n: int = 4194304, n_templates: int = 1024):
    """1,024 templates, K_j ~ U{100..800}, r ~ U[0.99, 1-1e-5], d ~ U{0..16384},
    4,194,304 samples at 4,096 Hz, processed in 4,096-sample blocks."""
    bank = random_bank(1, 0, n_templates, 100, 800, 0.99, 1.0 - 1e-5, 16384)
    return bank, strain(n, 1)


def batch_stream_lengths(n_streams: int = 8) -> np.ndarray:
    """Stream lengths round(2^u), u ~ U[18, 22]."""
    u = _rng(2, ROLE_STRAIN, 1000).uniform(18.0, 22.0, n_streams)
    return np.round(2.0 ** u).astype(np.int64)


def batch_streams(n_streams: int = 8, n_templates: int = 256, length_scale: float = 1.0):
    """8 streams of uneven length, each with its own 256-template bank of
    U{200..600} filters (coefficients as the 1,024-template bank, d <= 16,384)."""
    lengths = batch_stream_lengths(n_streams)
    if length_scale != 1.0:
        lengths = np.maximum(1, np.round(lengths * length_scale)).astype(np.int64)
    banks = [random_bank(2, s, n_templates, 200, 600, 0.99, 1.0 - 1e-5, 16384)
             for s in range(n_streams)]
    xs = [strain(int(lengths[s]), 2, s) for s in range(n_streams)]
    return banks, xs


def precision_bank(n: int = 16777216, n_templates: int = 64):
    """64 templates x 1,000 filters with poles between 1-1e-4 and 1-1e-6 in
    radius (the interval is stated as [1-1e-6, 1-1e-4]; read as its sorted
    form), d ~ U{0..2047}, 16,777,216 samples."""
    bank = random_bank(4, 0, n_templates, 1000, 1000, 1.0 - 1e-4, 1.0 - 1e-6, 2047)
    return bank, strain(n, 4)


# ---------------------------------------------------------------------------
# Chirp targets for the adjoint fit (256 templates x 400 filters).
# ---------------------------------------------------------------------------

def _chirp_tau_of_f(f, mc):
    """Time to coalescence at GW frequency f (leading-order quadrupole)."""
    return (5.0 / 256.0) * (math.pi * f) ** (-8.0 / 3.0) * (mc * T_SUN) ** (-5.0 / 3.0)


def chirp_target(mc: float, n: int = 65536, fs: float = FS,
                 f_lo: float = 30.0, f_hi: float = 1000.0) -> np.ndarray:
    """Time-reversed analytic Newtonian chirp g[n] = conj(h_c[N-1-n]).

    h_c(t) = f(t)^{2/3} exp(i phi(t)), tau = t_c - t,
    f(tau) = (1/pi) (5/(256 tau))^{3/8} (Mc T_sun)^{-5/8},
    phi(tau) = -2 (tau / (5 Mc T_sun))^{5/8}; zero outside [f_lo, f_hi].
    t_c is placed so that f = f_hi at the last sample. Real part of h_c is the
    A f^{2/3} cos(phi) waveform with A = 1 (the overlap loss is scale free).
    """
    tau_last = _chirp_tau_of_f(f_hi, mc)
    # g[m] corresponds to original index N-1-m, i.e. tau = tau_last + m/fs
    tau = tau_last + np.arange(n, dtype=np.float64) / fs
    f = (1.0 / math.pi) * (5.0 / (256.0 * tau)) ** (3.0 / 8.0) * (mc * T_SUN) ** (-5.0 / 8.0)
    phi = -2.0 * (tau / (5.0 * mc * T_SUN)) ** (5.0 / 8.0)
    h = f ** (2.0 / 3.0) * np.exp(1j * phi)
    h[(f < f_lo) | (f > f_hi * (1 + 1e-12))] = 0.0
    return np.conj(h)


def chirp_fit_masses(n_templates: int = 256) -> np.ndarray:
    return _rng(3, ROLE_CHIRP, 0).uniform(1.0, 30.0, n_templates)


def chirp_init_bank(g: np.ndarray, k: int, fs: float = FS):
    """Heuristic starting bank for fitting one target g with k filters.

    The support of g is cut into k equal segments; filter i starts at its
    segment (d = segment start), rotates at the local phase increment of g,
    decays over about one segment and takes the target sample as its gain.
    Returns (a, b, d) as complex128, complex128, int32.
    """
    nz = np.nonzero(np.abs(g) > 0)[0]
    n0, n1 = (int(nz[0]), int(nz[-1]) + 1) if nz.size else (0, len(g))
    edges = np.linspace(n0, n1, k + 1)
    starts = np.floor(edges[:-1]).astype(np.int64)
    seg = np.maximum(1.0, np.diff(edges))
    ph = np.unwrap(np.angle(g))
    nxt = np.minimum(starts + 1, len(g) - 1)
    w = ph[nxt] - ph[starts]
    w = np.where(np.abs(g[nxt]) > 0, w, 2 * math.pi * 30.0 / fs)
    r = np.minimum(np.exp(-1.0 / seg), 1.0 - 1e-6)
    a = r * np.exp(1j * w)
    b = np.where(np.abs(g[starts]) > 0, g[starts], 1e-6)
    return a.astype(np.complex128), b.astype(np.complex128), starts.astype(np.int32)


def chirp_fit(n: int = 65536, n_templates: int = 256, k: int = 400):
    """256 templates x 400 filters fitted to time-reversed Newtonian chirps with
    chirp masses ~ U[1, 30] M_sun, 30-1,000 Hz, 65,536 samples at 4,096 Hz.
    Input x is a unit impulse, so the bank output is its impulse response.

    Returns (initial bank, x, targets g [T, n] complex128, chirp masses)."""
    mcs = chirp_fit_masses(n_templates)
    gs = np.empty((n_templates, n), np.complex128)
    a = np.empty(n_templates * k, np.complex128)
    b = np.empty_like(a)
    d = np.empty(n_templates * k, np.int32)
    for j, mc in enumerate(mcs):
        g = chirp_target(float(mc), n)
        gs[j] = g
        aj, bj, dj = chirp_init_bank(g, k)
        a[j * k:(j + 1) * k] = aj
        b[j * k:(j + 1) * k] = bj
        d[j * k:(j + 1) * k] = dj
    off = np.arange(n_templates + 1, dtype=np.int64) * k
    x = np.zeros(n, np.float32)
    x[0] = 1.0
    return Bank(off, a, b, d, int(n - 1)), x, gs, mcs


# ---------------------------------------------------------------------------
# Inputs of the trigger clustering step: a fused max/argmax series.
# ---------------------------------------------------------------------------

def trigger_series(n: int, idx: int = 0, n_templates: int = 1024, peaks: int = 64,
                   plateau: int = 8):
    """A float32 max series shaped like the fused output over noise (chi-square
    background) with `peaks` injected bumps, some of them flat-topped plateaus of
    exactly equal values, and an int32 template index per sample (family 5)."""
    rng = _rng(5, ROLE_STRAIN, idx)
    M = rng.chisquare(2.0, n).astype(np.float64)
    J = rng.integers(0, n_templates, n).astype(np.int32)
    if n > 0:
        at = rng.integers(0, n, peaks)
        amp = rng.uniform(10.0, 100.0, peaks)
        width = rng.integers(1, 200, peaks)
        for c, h, w in zip(at, amp, width):
            lo, hi = max(0, c - 3 * w), min(n, c + 3 * w + 1)
            t = np.arange(lo, hi)
            M[lo:hi] = np.maximum(M[lo:hi], h * np.exp(-0.5 * ((t - c) / w) ** 2))
        for c in rng.integers(0, n, max(1, peaks // 4)):   # flat tops: runs of equal values
            lo, hi = max(0, c), min(n, c + plateau)
            M[lo:hi] = M[lo:hi].max() + 1.0
    return M.astype(np.float32), J



# ---------------------------------------------------------------------------
# Multi-rate bank (family 6): filters placed on halved sample rates.
# ---------------------------------------------------------------------------

def resample_taps(n_taps: int = 24):
    """FIR taps for halving (h) and doubling (g) the sample rate: a
    Hann-windowed sinc with its cutoff at a quarter of the higher rate. h sums
    to 1; each polyphase half of g (even and odd taps) sums to 1, so a constant
    passes through decimation and interpolation unchanged. float64."""
    i = np.arange(n_taps)
    m = i - (n_taps - 1) / 2.0
    win = 0.5 - 0.5 * np.cos(2.0 * np.pi * (i + 1) / (n_taps + 1))
    base = 0.5 * np.sinc(0.5 * m) * win
    h = base / base.sum()
    g = np.empty(n_taps)
    g[0::2] = base[0::2] / base[0::2].sum()
    g[1::2] = base[1::2] / base[1::2].sum()
    return h, g


def multirate_bank(n_templates: int = 1024, k_lo: int = 100, k_hi: int = 800, levels: int = 5,
                   f_lo: float = 20.0, f_hi: float = 1024.0, r_lo: float = 0.98, r_hi: float = 0.999,
                   dmax: int = 2047, idx: int = 0):
    """Chirp-like bank for a multi-rate filter bank (family 6). Template j has
    K_j ~ U{k_lo..k_hi} filters whose frequencies follow p(f) ~ f^(-11/3) on
    [f_lo, f_hi] Hz (the time an inspiral chirp spends per frequency band, so
    most filters are slow). A filter of frequency f goes to the lowest rate
    FS / 2^r (r < levels) at which f stays below a quarter of the rate, and is
    drawn at that rate: omega = 2 pi f 2^r / FS, |a| ~ U[r_lo, r_hi], b
    circular complex normal / sqrt(K_j), d ~ U{0..dmax >> r}.

    Draw order: all K_j, then per template u (frequency), |a|, Re b, Im b, v
    (delay). Returns the list of per-level Banks (same templates at every
    level; a template may have no filters at a level)."""
    rng = _rng(6, ROLE_BANK, idx)
    K = rng.integers(k_lo, k_hi + 1, n_templates)
    e = -8.0 / 3.0
    lo, hi = f_lo ** e, f_hi ** e
    per = [[[] for _ in range(n_templates)] for _ in range(levels)]
    for j in range(n_templates):
        k = int(K[j])
        u = rng.random(k)
        r = rng.uniform(r_lo, r_hi, k)
        br = rng.standard_normal(k) * math.sqrt(0.5 / k)
        bi = rng.standard_normal(k) * math.sqrt(0.5 / k)
        v = rng.random(k)
        f = (lo - u * (lo - hi)) ** (1.0 / e)
        for q in range(k):
            lev = 0
            while lev + 1 < levels and f[q] < FS / 2.0 ** (lev + 3):
                lev += 1
            om = 2.0 * math.pi * f[q] * 2.0 ** lev / FS
            dm = dmax >> lev
            per[lev][j].append((r[q] * np.exp(1j * om), br[q] + 1j * bi[q], int(v[q] * (dm + 1))))
    banks = []
    for lev in range(levels):
        cnt = np.array([len(per[lev][j]) for j in range(n_templates)], np.int64)
        off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        flat = [t for j in range(n_templates) for t in per[lev][j]]
        a = np.array([t[0] for t in flat], np.complex128)
        b = np.array([t[1] for t in flat], np.complex128)
        d = np.array([t[2] for t in flat], np.int32)
        banks.append(Bank(off, a, b, d, dmax >> lev))
    return banks



# ---------------------------------------------------------------------------
# Coloured noise for the whitening front end (family 7).
# ---------------------------------------------------------------------------

COLOUR_B = (1.0,)
COLOUR_A = (1.0, -1.8, 0.85)   # a resonant low-pass: power rises ~100x towards low frequencies


def coloured_noise(n: int, idx: int = 0, floor: float = 0.1) -> np.ndarray:
    """Raw-strain stand-in: white Gaussian noise through the resonant low-pass
    1 / (1 - 1.8 z^-1 + 0.85 z^-2) plus a white floor of standard deviation
    `floor`, float32 (family 7)."""
    import scipy.signal
    rng = _rng(7, ROLE_STRAIN, idx)
    w = rng.standard_normal(int(n))
    v = rng.standard_normal(int(n))
    return (scipy.signal.lfilter(COLOUR_B, COLOUR_A, w) + floor * v).astype(np.float32)
