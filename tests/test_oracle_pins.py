"""Pins of the FP64 oracle against results fixed by mathematics, not by itself.

Each test targets a plausible mistake in the oracle (a dropped term, a wrong
sign, an off-by-one delay, a transposed conjugate, a wrong tie rule):
  * closed-form impulse response b a^(m-d) of a delayed single-pole filter
  * scipy.signal.lfilter with complex coefficients (a library IIR routine)
  * exact finite convolution written out by brute force on tiny inputs
  * FFT convolution with the full (untruncated) kernel on longer inputs
  * superposition / linearity / time shift / permutation of filters
  * closed-form energy of the impulse response of a whole template
  * the tie rule of the per-sample argmax (duplicated template)
  * adjoint: closed-form derivatives at an impulse, central finite
    differences in FP64, and an independent torch autograd implementation
"""
import math

import numpy as np
import pytest
import scipy.signal

import oracle
from workloads import Bank, random_bank, strain

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def one_filter_bank(a, b, d, dmax=None):
    return Bank(np.array([0, 1], np.int64), np.array([a], np.complex128),
                np.array([b], np.complex128), np.array([d], np.int32),
                int(d if dmax is None else dmax))


def small_bank(seed=0, T=3, klo=2, khi=6, dmax=9, rlo=0.5, rhi=0.97):
    return random_bank(90 + seed, 0, T, klo, khi, rlo, rhi, dmax)


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# --------------------------------------------------------------------------
# single filter
# --------------------------------------------------------------------------

@pytest.mark.parametrize("d", [0, 1, 17])
def test_impulse_response_closed_form(d):
    a = 0.995 * np.exp(1j * 0.3)
    b = 0.7 - 0.4j
    n = 400
    x = np.zeros(n)
    x[0] = 1.0
    z = oracle.z(one_filter_bank(a, b, d), x)[0]
    m = np.arange(n)
    expect = np.where(m >= d, b * a ** np.maximum(m - d, 0), 0.0)
    assert np.all(z[:d] == 0)
    assert rel(z, expect) < 1e-13


def test_matches_lfilter_complex():
    rng = np.random.default_rng(5)
    n = 3000
    x = rng.standard_normal(n)
    for a, b, d in [(0.99 * np.exp(0.1j), 1 + 2j, 0),
                    (0.9999 * np.exp(-1.2j), -0.3 + 0.05j, 5),
                    (0.5 * np.exp(2.9j), 0.2j, 123)]:
        z = oracle.z(one_filter_bank(a, b, d), x)[0]
        xs = np.concatenate([np.zeros(d), x])[:n]
        ref = scipy.signal.lfilter([b], [1.0, -a], xs)
        assert rel(z, ref) < 1e-11, (a, b, d)


def test_bruteforce_finite_convolution():
    # y[m] = b * sum_{i=0}^{m-d} a^i x[m-d-i]: exact for a finite input
    rng = np.random.default_rng(11)
    bank = small_bank(1, T=2, klo=3, khi=4, dmax=7)
    n = 37
    x = rng.standard_normal(n)
    got = oracle.z(bank, x)
    for j in range(bank.n_templates):
        for m in range(n):
            acc = 0j
            for k in range(int(bank.offsets[j]), int(bank.offsets[j + 1])):
                a, b, d = complex(bank.a[k]), complex(bank.b[k]), int(bank.d[k])
                for i in range(0, m - d + 1):
                    acc += b * a ** i * x[m - d - i]
            assert abs(got[j, m] - acc) <= 1e-12 * (1 + abs(acc))


def test_fft_convolution_long():
    rng = np.random.default_rng(12)
    bank = small_bank(2, T=2, klo=5, khi=8, dmax=300, rlo=0.99, rhi=0.9999)
    n = 6000
    x = rng.standard_normal(n)
    got = oracle.z(bank, x)
    i = np.arange(n)
    for j in range(bank.n_templates):
        h = np.zeros(n, np.complex128)
        for k in range(int(bank.offsets[j]), int(bank.offsets[j + 1])):
            d = int(bank.d[k])
            h[d:] += bank.b[k] * bank.a[k] ** i[: n - d]
        ref = scipy.signal.fftconvolve(x, h)[:n]
        assert rel(got[j], ref) < 1e-9


# --------------------------------------------------------------------------
# template sum: superposition, linearity, shift, permutation, energy
# --------------------------------------------------------------------------

def test_linearity_in_x():
    rng = np.random.default_rng(3)
    bank = small_bank(3, T=3)
    n = 500
    x1, x2 = rng.standard_normal(n), rng.standard_normal(n)
    al, be = 1.7, -0.45
    lhs = oracle.z(bank, al * x1 + be * x2)
    rhs = al * oracle.z(bank, x1) + be * oracle.z(bank, x2)
    assert rel(lhs, rhs) < 1e-12


def test_bank_is_sum_of_single_filters():
    rng = np.random.default_rng(4)
    bank = small_bank(4, T=2, klo=4, khi=7)
    n = 700
    x = rng.standard_normal(n)
    z = oracle.z(bank, x)
    for j in range(bank.n_templates):
        acc = np.zeros(n, np.complex128)
        for k in range(int(bank.offsets[j]), int(bank.offsets[j + 1])):
            acc += oracle.z(one_filter_bank(bank.a[k], bank.b[k], bank.d[k]), x)[0]
        assert rel(z[j], acc) < 1e-13


def test_filter_permutation_and_threads():
    rng = np.random.default_rng(6)
    bank = small_bank(5, T=1, klo=40, khi=40, dmax=50)
    x = rng.standard_normal(1000)
    perm = rng.permutation(bank.n_filters)
    pb = Bank(bank.offsets, bank.a[perm], bank.b[perm], bank.d[perm], bank.dmax)
    z1 = oracle.z(bank, x, nthreads=1)
    z2 = oracle.z(pb, x, nthreads=1)
    z3 = oracle.z(bank, x, nthreads=4)
    assert rel(z1, z2) < 1e-13
    assert rel(z1, z3) < 1e-13


def test_time_shift():
    rng = np.random.default_rng(7)
    bank = small_bank(6, T=2)
    n, s = 400, 23
    x = rng.standard_normal(n)
    xs = np.concatenate([np.zeros(s), x[: n - s]])
    z = oracle.z(bank, x)
    zs = oracle.z(bank, xs)
    assert np.all(zs[:, :s] == 0)
    assert rel(zs[:, s:], z[:, : n - s]) < 1e-13


def test_impulse_energy_closed_form():
    # |z|^2 summed over m < N for x = delta:
    #   sum_{k,l} b_k conj(b_l) a_k^(M-d_k) conj(a_l)^(M-d_l) (1 - (a_k conj a_l)^(N-M)) / (1 - a_k conj a_l)
    # with M = max(d_k, d_l)
    bank = small_bank(7, T=2, klo=5, khi=9, dmax=40, rlo=0.9, rhi=0.99)
    N = 900
    x = np.zeros(N)
    x[0] = 1.0
    z = oracle.z(bank, x)
    for j in range(bank.n_templates):
        ks = range(int(bank.offsets[j]), int(bank.offsets[j + 1]))
        e = 0j
        for k in ks:
            for l in ks:
                ak, al = bank.a[k], bank.a[l]
                M = max(int(bank.d[k]), int(bank.d[l]))
                q = ak * np.conj(al)
                e += (bank.b[k] * np.conj(bank.b[l]) * ak ** (M - bank.d[k])
                      * np.conj(al) ** (M - bank.d[l]) * (1 - q ** (N - M)) / (1 - q))
        direct = np.sum(np.abs(z[j]) ** 2)
        assert abs(e.imag) < 1e-10 * abs(e.real)
        assert abs(direct - e.real) < 1e-11 * e.real


def test_snr_is_abs_squared():
    rng = np.random.default_rng(8)
    bank = small_bank(8, T=3)
    x = rng.standard_normal(300)
    z = oracle.z(bank, x)
    s = oracle.snr(bank, x)
    assert np.array_equal(s, z.real ** 2 + z.imag ** 2)


# --------------------------------------------------------------------------
# max / argmax over templates
# --------------------------------------------------------------------------

def test_trigger_tie_rule_lowest_index():
    rng = np.random.default_rng(9)
    base = small_bank(9, T=3, klo=3, khi=5)
    # template order: 0, 1, 2, then duplicates of 1 and 0 at indices 3, 4
    bank = base.subset([0, 1, 2, 1, 0])
    x = rng.standard_normal(400)
    s = oracle.snr(bank, x)
    first = np.argmax(s == s.max(axis=0)[None, :], axis=0)
    for nt in (1, 2, 3, 5):
        mx, am = oracle.trigger(bank, x, nthreads=nt)
        assert np.array_equal(mx, s.max(axis=0))
        assert np.all(am <= 2)          # duplicates never win
        assert np.array_equal(am, first)


def test_trigger_peaks_and_merge_of_template_subsets():
    """Per-template peaks equal the maxima of the SNR rows; the trigger of a
    bank equals the merge (max, lowest index among equal values) of the
    triggers of a partition of its templates, which is how the full-size GPU
    parity tests split the oracle's work. Duplicated templates put exact ties
    across the parts."""
    rng = np.random.default_rng(12)
    base = small_bank(12, T=5, klo=2, khi=6)
    bank = base.subset([0, 1, 2, 3, 4, 1, 0, 3])
    x = rng.standard_normal(500)
    s = oracle.snr(bank, x)
    mx, am, pk = oracle.trigger(bank, x, nthreads=3, peaks=True)
    assert np.array_equal(pk, s.max(axis=1))
    for parts in ([[0, 1, 2], [3, 4, 5, 6, 7]], [[0, 1], [2, 3], [4, 5], [6, 7]]):
        M = np.full(len(x), -1.0)
        J = np.full(len(x), -1, np.int64)
        for p in parts:
            m, j = oracle.trigger(bank.subset(p), x, nthreads=2)
            j = np.asarray(p)[j]
            take = (m > M) | ((m == M) & (j < J))
            M = np.where(take, m, M)
            J = np.where(take, j, J)
        assert np.array_equal(M, mx) and np.array_equal(J, am)


def test_trigger_threads_agree():
    rng = np.random.default_rng(10)
    bank = small_bank(10, T=7, klo=2, khi=5)
    x = rng.standard_normal(333)
    m1, j1 = oracle.trigger(bank, x, nthreads=1)
    m4, j4 = oracle.trigger(bank, x, nthreads=4)
    assert np.array_equal(m1, m4) and np.array_equal(j1, j4)


# --------------------------------------------------------------------------
# adjoint
# --------------------------------------------------------------------------

def test_backward_impulse_closed_form():
    # x = delta: dz[m]/db_k = a_k^(m-d_k), dz[m]/da_k = b_k (m-d_k) a_k^(m-d_k-1);
    # grad = sum_m G[m] conj(dz[m]/dp) in the dL/dRe + i dL/dIm convention.
    rng = np.random.default_rng(13)
    bank = small_bank(11, T=2, klo=3, khi=5, dmax=20, rlo=0.9, rhi=0.99)
    n = 300
    x = np.zeros(n)
    x[0] = 1.0
    G = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    ga, gb = oracle.backward(bank, x, G)
    m = np.arange(n)
    for j in range(2):
        for k in range(int(bank.offsets[j]), int(bank.offsets[j + 1])):
            a, b, d = bank.a[k], bank.b[k], int(bank.d[k])
            on = m >= d
            e = np.maximum(m - d, 0)
            dzb = np.where(on, a ** e, 0)
            dza = np.where(m >= d + 1, b * e * a ** np.maximum(e - 1, 0), 0)
            assert abs(gb[k] - np.sum(G[j] * np.conj(dzb))) < 1e-10 * np.sum(np.abs(G[j]))
            assert abs(ga[k] - np.sum(G[j] * np.conj(dza))) < 1e-9 * np.sum(np.abs(G[j] * dza))


def _loss_of(bank, x, g):
    z = oracle.z(bank, x)
    loss, G = oracle.overlap_loss(z, g)
    return float(np.sum(loss)), G


def test_backward_matches_central_differences():
    rng = np.random.default_rng(14)
    bank = small_bank(12, T=2, klo=3, khi=4, dmax=15, rlo=0.9, rhi=0.99)
    n = 200
    x = rng.standard_normal(n)
    g = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    L0, G = _loss_of(bank, x, g)
    ga, gb = oracle.backward(bank, x, G)
    h = 1e-6
    for k in range(bank.n_filters):
        for which, grad in (("a", ga), ("b", gb)):
            fd = 0j
            for unit, part in ((1.0, 1.0), (1j, 1j)):
                vals = []
                for s in (+1, -1):
                    a2, b2 = bank.a.copy(), bank.b.copy()
                    (a2 if which == "a" else b2)[k] += s * h * unit
                    vals.append(_loss_of(Bank(bank.offsets, a2, b2, bank.d, bank.dmax), x, g)[0])
                fd += part * (vals[0] - vals[1]) / (2 * h)
            assert abs(grad[k] - fd) <= 1e-6 * max(1e-3, abs(fd)), (which, k, grad[k], fd)


def test_backward_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(15)
    bank = small_bank(13, T=2, klo=2, khi=3, dmax=6, rlo=0.8, rhi=0.98)
    n = 60
    x = rng.standard_normal(n)
    g = rng.standard_normal((2, n)) + 1j * rng.standard_normal((2, n))
    a = torch.tensor(bank.a, dtype=torch.complex128, requires_grad=True)
    b = torch.tensor(bank.b, dtype=torch.complex128, requires_grad=True)
    xt = torch.tensor(x, dtype=torch.float64)
    gt = torch.tensor(g)
    total = 0
    for j in range(2):
        zj = [torch.zeros((), dtype=torch.complex128) for _ in range(n)]
        for k in range(int(bank.offsets[j]), int(bank.offsets[j + 1])):
            y = torch.zeros((), dtype=torch.complex128)
            d = int(bank.d[k])
            for m in range(n):
                xin = xt[m - d] if m >= d else torch.zeros((), dtype=torch.float64)
                y = a[k] * y + b[k] * xin
                zj[m] = zj[m] + y
        zv = torch.stack(zj)
        c = torch.sum(zv * torch.conj(gt[j]))
        total = total + 1 - torch.abs(c) / (torch.linalg.norm(zv) * torch.linalg.norm(gt[j]))
    total.backward()
    L0, G = _loss_of(bank, x, g)
    assert abs(float(total) - L0) < 1e-12
    ga, gb = oracle.backward(bank, x, G)
    assert rel(ga, a.grad.numpy()) < 1e-10
    assert rel(gb, b.grad.numpy()) < 1e-10


def test_overlap_loss_gradient_fd():
    rng = np.random.default_rng(16)
    z = rng.standard_normal((2, 50)) + 1j * rng.standard_normal((2, 50))
    g = rng.standard_normal((2, 50)) + 1j * rng.standard_normal((2, 50))
    loss, G = oracle.overlap_loss(z, g)
    # scale invariance of the overlap
    l2, _ = oracle.overlap_loss(3.7 * np.exp(0.4j) * z, g)
    assert np.allclose(loss, l2, atol=1e-14)
    assert np.all((loss >= -1e-15) & (loss <= 1 + 1e-15))
    h = 1e-6
    for j in range(2):
        for m in (0, 7, 49):
            fd = 0j
            for unit in (1.0, 1j):
                zp, zm = z.copy(), z.copy()
                zp[j, m] += h * unit
                zm[j, m] -= h * unit
                fd += unit * (oracle.overlap_loss(zp, g)[0][j] - oracle.overlap_loss(zm, g)[0][j]) / (2 * h)
            assert abs(G[j, m] - fd) < 1e-7


def test_identical_target_has_zero_loss():
    rng = np.random.default_rng(17)
    z = rng.standard_normal((1, 64)) + 1j * rng.standard_normal((1, 64))
    loss, G = oracle.overlap_loss(z, 2.5j * z)
    assert abs(loss[0]) < 1e-14
    assert np.max(np.abs(G)) < 1e-12


# --------------------------------------------------------------------------
# generators
# --------------------------------------------------------------------------

def test_generators_are_deterministic_and_in_range():
    b1 = random_bank(1, 0, 20, 100, 800, 0.99, 1 - 1e-5, 16384)
    b2 = random_bank(1, 0, 20, 100, 800, 0.99, 1 - 1e-5, 16384)
    assert np.array_equal(b1.a, b2.a) and np.array_equal(b1.d, b2.d)
    r = np.abs(b1.a)
    w = np.angle(b1.a)
    assert r.min() >= 0.99 and r.max() <= 1 - 1e-5 + 1e-15
    assert w.min() >= 0.001 * math.pi - 1e-12 and w.max() <= 0.5 * math.pi + 1e-12
    assert b1.d.min() >= 0 and b1.d.max() <= 16384
    k = b1.counts()
    assert k.min() >= 100 and k.max() <= 800
    x1, x2 = strain(1000, 1), strain(1000, 1)
    assert x1.dtype == np.float32 and np.array_equal(x1, x2)
    assert not np.array_equal(strain(1000, 1), strain(1000, 0))


# --- trigger clustering ----------------------------------------------------

def _clusters_brute(M, J, threshold, W):
    """Independent restatement: keep m when it is at or above the threshold and
    no sample within W before it reaches its value, none within W after exceeds it."""
    n = len(M)
    out = []
    for m in range(n):
        v = float(M[m])
        if v < threshold:
            continue
        left = [float(u) for u in M[max(0, m - W):m]]
        right = [float(u) for u in M[m + 1:min(n, m + W + 1)]]
        if (not left or max(left) < v) and (not right or max(right) <= v):
            out.append(m)
    return np.array(out, np.int64)


@pytest.mark.parametrize("W,threshold", [(1, 0.0), (3, 2.0), (7, 5.0), (50, 0.0)])
def test_clusters_brute_force_with_ties(W, threshold):
    rng = np.random.default_rng(40 + W)
    M = rng.integers(0, 9, 3000).astype(np.float32)   # many exact ties
    J = rng.integers(0, 100, 3000).astype(np.int32)
    idx, tpl, val = oracle.clusters(M, J, threshold, W)
    ref = _clusters_brute(M, J, threshold, W)
    assert np.array_equal(idx, ref)
    assert np.array_equal(tpl, J[ref]) and np.array_equal(val, M[ref])
    assert np.all(np.diff(idx) > W)   # triggers are more than W apart


def test_clusters_match_maximum_filter_for_distinct_values():
    import scipy.ndimage
    from workloads import trigger_series
    M, J = trigger_series(200000, 1)
    # distinct values with the same ordering (ranks, exact in float32), where the
    # tie rule plays no part
    rank = np.empty(len(M), np.int64)
    rank[np.argsort(M, kind="stable")] = np.arange(len(M))
    M = rank.astype(np.float32)
    assert len(np.unique(M)) == len(M)
    for W in (5, 200, 4096):
        mf = scipy.ndimage.maximum_filter(M, size=2 * W + 1, mode="constant", cval=-np.inf)
        thr = float(np.quantile(M, 0.999))
        ref = np.nonzero((M >= thr) & (M == mf))[0]
        idx, _, _ = oracle.clusters(M, J, thr, W)
        assert np.array_equal(idx, ref), W


def test_clusters_closed_form_cases():
    J = np.arange(40, dtype=np.int32)
    # one triangular bump: its apex
    M = np.array([0, 1, 2, 3, 4, 3, 2, 1, 0] + [0] * 31, np.float32)
    assert oracle.clusters(M, J, 0.5, 10)[0].tolist() == [4]
    # a flat top: its first sample
    M = np.zeros(40, np.float32)
    M[10:15] = 7.0
    assert oracle.clusters(M, J, 1.0, 3)[0].tolist() == [10]
    # a value exactly at the threshold counts
    assert oracle.clusters(M, J, 7.0, 3)[0].tolist() == [10]
    # two bumps further apart than W: both; within W: the larger one
    M = np.zeros(40, np.float32)
    M[5], M[20] = 3.0, 4.0
    assert oracle.clusters(M, J, 1.0, 14)[0].tolist() == [5, 20]
    assert oracle.clusters(M, J, 1.0, 15)[0].tolist() == [20]
    # windows are clipped at both ends of the series
    M = np.zeros(40, np.float32)
    M[0], M[39] = 2.0, 2.0
    assert oracle.clusters(M, J, 1.0, 5)[0].tolist() == [0, 39]
    # nothing at or above the threshold; an empty series
    assert len(oracle.clusters(M, J, 3.0, 5)[0]) == 0
    assert len(oracle.clusters(np.zeros(0, np.float32), np.zeros(0, np.int32), 0.0, 5)[0]) == 0


# --- multi-rate bank ---------------------------------------------------------

def _mr_levels(T, per_level, R, seed=0, r_max=0.95):
    """Random small multi-rate bank: per_level[r] = filters per template at level r."""
    from workloads import Bank
    rng = np.random.default_rng(900 + seed)
    out = []
    for r in range(R + 1):
        k = per_level[r]
        off = np.arange(T + 1, dtype=np.int64) * k
        F = T * k
        a = rng.uniform(0.3, r_max, F) * np.exp(1j * rng.uniform(0, np.pi / 2, F))
        b = rng.standard_normal(F) + 1j * rng.standard_normal(F)
        d = rng.integers(0, 5, F).astype(np.int32)
        out.append(Bank(off, a, b, d, 8))
    return out


def test_multirate_resampling_matches_library_routines():
    """A single pass-through filter (a = 0, b = 1, d = 0) at level R: the result
    is x decimated R times and interpolated R times, built here from
    scipy.signal.lfilter and scipy.signal.upfirdn."""
    import scipy.signal
    from workloads import Bank
    rng = np.random.default_rng(5)
    h, g = rng.standard_normal(13), rng.standard_normal(10)   # asymmetric: index direction matters
    x = rng.standard_normal(512)
    for R in (1, 2, 3):
        levels = [Bank(np.zeros(2, np.int64), np.zeros(0, complex), np.zeros(0, complex),
                       np.zeros(0, np.int32), 0) for _ in range(R)]
        levels.append(Bank(np.array([0, 1], np.int64), np.array([0j]), np.array([1 + 0j]),
                           np.array([0], np.int32), 0))
        v = x.copy()
        for _ in range(R):
            v = scipy.signal.lfilter(h, [1.0], v)[1::2]
        for r in range(R, 0, -1):
            v = scipy.signal.upfirdn(g, v, up=2)[:len(x) >> (r - 1)]
        got = oracle.multirate_z(levels, h, g, x)
        assert got.shape == (1, len(x))
        assert np.max(np.abs(got[0] - v)) < 1e-12, R


def test_multirate_constant_input_steady_state():
    """x = 1: decimation keeps the constant (h sums to 1), each filter settles at
    b / (1 - a) in its own level's samples, interpolation keeps a constant
    (each polyphase half of g sums to 1), so z_j settles at the sum of
    b / (1 - a) over all of the template's filters at every level."""
    from workloads import resample_taps
    h, g = resample_taps(24)
    R = 3
    levels = _mr_levels(3, [2, 3, 1, 4], R, seed=1, r_max=0.8)
    got = oracle.multirate_z(levels, h, g, np.ones(4096))
    for j in range(3):
        want = sum(np.sum(lv.b[lv.offsets[j]:lv.offsets[j + 1]] / (1 - lv.a[lv.offsets[j]:lv.offsets[j + 1]]))
                   for lv in levels)
        assert abs(got[j, -1] - want) < 1e-9 * abs(want)


def _mr_brute(levels, h, g, x):
    R = len(levels) - 1
    xs = [list(map(float, x))]
    for r in range(1, R + 1):
        p = xs[-1]
        xs.append([sum(h[i] * p[2 * q + 1 - i] for i in range(len(h)) if 0 <= 2 * q + 1 - i < len(p))
                   for q in range(len(p) // 2)])
    T = levels[0].n_templates
    w = None
    for r in range(R, -1, -1):
        lv, xr = levels[r], xs[r]
        zr = [[0j] * len(xr) for _ in range(T)]
        for j in range(T):
            for k in range(int(lv.offsets[j]), int(lv.offsets[j + 1])):
                y = 0j
                for m in range(len(xr)):
                    y = lv.a[k] * y + lv.b[k] * (xr[m - lv.d[k]] if m - lv.d[k] >= 0 else 0.0)
                    zr[j][m] += y
            if w is not None:
                for p in range(len(xr)):
                    zr[j][p] += sum(g[p - 2 * q] * w[j][q] for q in range(len(w[j])) if 0 <= p - 2 * q < len(g))
        w = zr
    return np.array(w)


def test_multirate_brute_force_tiny():
    rng = np.random.default_rng(8)
    h, g = rng.standard_normal(7), rng.standard_normal(6)   # asymmetric taps
    levels = _mr_levels(2, [1, 2, 1], 2, seed=2)
    levels[1].offsets = np.array([0, 0, 2], np.int64)      # template 0 has no level-1 filter
    levels[1].a, levels[1].b, levels[1].d = levels[1].a[:2], levels[1].b[:2], levels[1].d[:2]
    x = np.random.default_rng(6).standard_normal(48)
    got = oracle.multirate_z(levels, h, g, x)
    ref = _mr_brute(levels, h, g, x)
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_multirate_shift_and_linearity():
    from workloads import resample_taps
    h, g = resample_taps(12)
    R = 2
    levels = _mr_levels(2, [2, 1, 3], R, seed=3)
    rng = np.random.default_rng(7)
    x, y = rng.standard_normal(256), rng.standard_normal(256)
    zx, zy = oracle.multirate_z(levels, h, g, x), oracle.multirate_z(levels, h, g, y)
    assert np.allclose(oracle.multirate_z(levels, h, g, 2.0 * x - 0.5 * y), 2.0 * zx - 0.5 * zy, atol=1e-10)
    s = 3 << R   # shifts by whole multiples of 2^R keep the decimation phase
    xs = np.concatenate([np.zeros(s), x])[:len(x)]
    assert np.allclose(oracle.multirate_z(levels, h, g, xs)[:, s:], zx[:, :len(x) - s], atol=1e-10)


def test_multirate_single_level_is_the_bank():
    from workloads import random_bank, resample_taps, strain
    h, g = resample_taps(8)
    bank = random_bank(0, 3, 3, 10, 20, 0.9, 0.99, 16)
    x = strain(300, 0, 3)
    assert np.array_equal(oracle.multirate_z([bank], h, g, x), oracle.z(bank, x))
    mx, am = oracle.multirate_trigger([bank], h, g, x)
    m2, a2 = oracle.trigger(bank, x)
    assert np.allclose(mx, m2, rtol=1e-12) and np.array_equal(am, a2)


# --- whitening front end -----------------------------------------------------

def test_welch_psd_matches_scipy():
    """scipy.signal.welch with the same frames and window, density scaling at
    fs = 1, one-sided: its bins 1..N/2-1 are doubled, DC and Nyquist are not."""
    import scipy.signal
    from workloads import coloured_noise
    x = coloured_noise(40000, 1).astype(np.float64)
    for N in (64, 512, 2048):
        S = oracle.welch_psd(x, N)
        f, P = scipy.signal.welch(x, fs=1.0, window="hann", nperseg=N, noverlap=N // 2, detrend=False,
                                  return_onesided=True, scaling="density", average="mean")
        want = P.copy()
        want[1:N // 2] /= 2.0
        assert np.allclose(S, want, rtol=1e-10, atol=0), N


def test_whiten_unit_psd_is_a_delay():
    """S = 1: the Hann frames sum to 1 at 50% overlap, so the output is x
    delayed by N/2 exactly; S = c scales it by 1/sqrt(c)."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal(4096)
    for N in (16, 256, 1024):
        H = N // 2
        y = oracle.whiten(x, np.ones(H + 1), N)
        assert np.max(np.abs(y[H:] - x[:-H])) < 1e-12 and np.max(np.abs(y[:H])) < 1e-12
        y4 = oracle.whiten(x, np.full(H + 1, 4.0), N)
        assert np.max(np.abs(y4[H:] - x[:-H] / 2.0)) < 1e-12


def _whiten_brute(x, S, N):
    H = N // 2
    xp = [0.0] * H + list(map(float, x))
    n = len(x)
    out = [0.0] * (n + N)
    w = [np.sin(np.pi * t / N) ** 2 for t in range(N)]
    inv = [0.0 if S[min(f, N - f)] <= 0 else 1.0 / np.sqrt(S[min(f, N - f)]) for f in range(N)]
    for j in range(n // H):
        X = [sum(w[t] * xp[j * H + t] * np.exp(-2j * np.pi * f * t / N) for t in range(N)) for f in range(N)]
        for t in range(N):
            out[j * H + t] += (sum(X[f] * inv[f] * np.exp(2j * np.pi * f * t / N) for f in range(N)) / N).real
    return np.array(out[:n])


def test_whiten_brute_force_tiny():
    rng = np.random.default_rng(12)
    N = 8
    S = rng.uniform(0.2, 3.0, N // 2 + 1)
    S[2] = 0.0                       # a zeroed bin
    x = rng.standard_normal(40)
    assert np.max(np.abs(oracle.whiten(x, S, N) - _whiten_brute(x, S, N))) < 1e-12


def test_whiten_flattens_coloured_noise():
    """Coloured noise whose PSD spans four decades comes out with a flat PSD
    of unit level (statistical: 50 frames per estimate)."""
    from workloads import coloured_noise
    N = 512
    x = coloured_noise(1 << 16, 2)
    S = oracle.welch_psd(x, N)
    assert S.max() / S.min() > 1e3
    y = oracle.whiten(x, S, N)
    S2 = oracle.welch_psd(y[N:], N)
    assert abs(S2.mean() - 1.0) < 0.02 and S2.min() > 0.75 and S2.max() < 1.3


def test_whiten_zero_bin_removes_a_tone():
    """A tone exactly on bin f0 disappears when S[f0] = 0 (after the first frame)."""
    N = 256
    f0 = 20
    t = np.arange(8192)
    x = np.cos(2 * np.pi * f0 * t / N)
    S = np.ones(N // 2 + 1)
    S[f0] = 0.0
    y = oracle.whiten(x, S, N)
    assert np.max(np.abs(y[N:])) < 1e-9
    assert np.max(np.abs(oracle.whiten(x, np.ones(N // 2 + 1), N)[N:])) > 0.99
