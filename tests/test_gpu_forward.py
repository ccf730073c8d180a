"""GPU parity of the forward path (filter recursion, template sum, SNR, fused
max/argmax, streaming state) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from helpers import SNR_TOL, check_argmax, snr_err
from workloads import Bank, bank_4x128, random_bank, strain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1602_05573_amd import load
    load()


def mk(bank, **kw):
    from paper_1602_05573_amd import SpiirBank
    return SpiirBank.from_bank(bank, **kw)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def banner(msg):
    print("[case] " + msg, flush=True)


# ---------------------------------------------------------------------------
# 4 templates x 128 filters, 16,384 samples
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def c0():
    bank, x = bank_4x128()
    ref = oracle.snr(bank, x)
    return bank, x, ref


@pytest.mark.parametrize("fl", [0, 1, 2, 4])
def test_bank4x128_snr_parity(c0, fl):
    bank, x, ref = c0
    banner("bank_4x128 snr fl=%d" % fl)
    with mk(bank, filters_per_lane=fl) as bk:
        snr = bk.filter_block(dev(x)).cpu().numpy()
    err, _ = snr_err(snr, ref)
    print("bank_4x128 fl=%d err=%.3g" % (fl, err))
    assert err <= SNR_TOL


def test_bank4x128_trigger_parity(c0):
    bank, x, ref = c0
    banner("bank_4x128 trigger")
    with mk(bank) as bk:
        mx, am = bk.trigger_max(dev(x))
        mx, am = mx.cpu().numpy(), am.cpu().numpy()
    ties = check_argmax(mx, am, ref)
    print("bank_4x128 documented ties: %d of %d" % (ties, len(x)))


def test_fused_equals_max_of_plain_rows(c0):
    bank, x, _ = c0
    banner("fused vs plain rows")
    xd = dev(x)
    with mk(bank) as b1, mk(bank) as b2:
        snr = b1.filter_block(xd)
        mx, am = b2.trigger_max(xd)
        torch.cuda.synchronize()
    s = snr.cpu().numpy()
    m = s.max(axis=0)
    first = np.argmax(s == m[None, :], axis=0)
    assert np.array_equal(mx.cpu().numpy(), m)
    assert np.array_equal(am.cpu().numpy(), first)


@pytest.mark.parametrize("L,cuts", [(256, (0, 16384)), (16, (0, 5000, 16384)), (64, (0, 3001, 9000, 16384))])
def test_per_template_launches_parity(c0, L, cuts):
    """The per-template comparator (each template's launches split into
    chunk-length segments over that template's workgroup only; here all four
    templates share one workgroup) over several calls of one stream, pieces
    of 4,096 samples and ragged tails: every template's SNR row of every call
    within the gate, and the max/argmax by the argmax rule."""
    bank, x, ref = c0
    banner("per-template L=%d cuts %s" % (L, cuts))
    xd = dev(x)
    n = len(x)
    mx = torch.empty(n, dtype=torch.float32, device="cuda")
    am = torch.empty(n, dtype=torch.int32, device="cuda")
    with mk(bank, chunk_len=L, max_block=4096, filters_per_lane=1, waves_per_group=8) as bk:
        assert bk.info["n_groups"] == 1
        for c0_, c1_ in zip(cuts[:-1], cuts[1:]):
            rows = torch.empty((bank.n_templates, c1_ - c0_), dtype=torch.float32, device="cuda")
            bk.trigger_max_per_template(xd[c0_:c1_], out=(mx[c0_:c1_], am[c0_:c1_]), snr_scratch=rows)
            err, _ = snr_err(rows.cpu().numpy(), ref[:, c0_:c1_])
            assert err <= SNR_TOL, "samples %d..%d: SNR error %.3g" % (c0_, c1_, err)
        torch.cuda.synchronize()
    check_argmax(mx.cpu().numpy(), am.cpu().numpy(), ref)


def test_per_template_launches_many_groups(mid):
    """Several workgroups of several templates each: the per-template launches
    leave every other template's state alone (two calls of one stream)."""
    bank, x, ref = mid
    banner("per-template, many groups")
    xd = dev(x)
    n = len(x)
    mx = torch.empty(n, dtype=torch.float32, device="cuda")
    am = torch.empty(n, dtype=torch.int32, device="cuda")
    h = n // 2 + 37
    with mk(bank, chunk_len=64, max_block=4096, filters_per_lane=2, waves_per_group=8) as bk:
        assert bk.info["n_groups"] >= 2
        bk.trigger_max_per_template(xd[:h], out=(mx[:h], am[:h]))
        bk.trigger_max_per_template(xd[h:], out=(mx[h:], am[h:]))
        torch.cuda.synchronize()
    check_argmax(mx.cpu().numpy(), am.cpu().numpy(), ref)


def test_determinism(c0):
    bank, x, _ = c0
    banner("determinism")
    xd = dev(x)
    with mk(bank) as bk:
        s1 = bk.filter_block(xd).clone()
        bk.reset()
        s2 = bk.filter_block(xd).clone()
        bk.reset()
        m1, a1 = bk.trigger_max(xd)
        m1, a1 = m1.clone(), a1.clone()
        bk.reset()
        m2, a2 = bk.trigger_max(xd)
    assert torch.equal(s1, s2)
    assert torch.equal(m1, m2) and torch.equal(a1, a2)


@pytest.mark.parametrize("tsplit", [1, 0])
def test_block_split_invariance(c0, tsplit):
    """Without a time split, cutting the stream at multiples of L is bitwise
    invisible; with it (the segments follow the call length) within the gate."""
    bank, x, ref = c0
    banner("block split time_split=%d" % tsplit)
    xd = dev(x)
    with mk(bank, chunk_len=256, time_split=tsplit) as bk:
        whole = bk.filter_block(xd).clone()
        bk.reset()
        parts = []
        for a, b in [(0, 4096), (4096, 4608), (4608, 8192), (8192, 16384)]:   # multiples of L
            parts.append(bk.filter_block(xd[a:b].contiguous()).clone())
        split = torch.cat(parts, dim=1)
        bk.reset()
        rag = []
        for a, b in [(0, 1000), (1000, 1003), (1003, 9000), (9000, 16384)]:    # arbitrary cuts
            rag.append(bk.filter_block(xd[a:b].contiguous()).clone())
        ragged = torch.cat(rag, dim=1)
    if tsplit == 1:
        assert torch.equal(whole, split)
    for s in (whole, split, ragged):
        err, _ = snr_err(s.cpu().numpy(), ref)
        assert err <= SNR_TOL


def test_state_checkpoint_resume(c0):
    bank, x, _ = c0
    banner("checkpoint")
    xd = dev(x)
    with mk(bank) as b1, mk(bank) as b2:
        b1.filter_block(xd[:6000].contiguous())
        blob = b1.get_state()
        rest1 = b1.filter_block(xd[6000:].contiguous()).clone()
        b2.set_state(blob)
        rest2 = b2.filter_block(xd[6000:].contiguous()).clone()
    assert torch.equal(rest1, rest2)


def test_exact_ties_resolve_to_lowest_index():
    """Duplicated templates that occupy the same lane positions (every template
    here fills exactly one wave: 4 rows of 16 filters) produce bitwise equal SNR,
    and the fused argmax then returns the smallest index."""
    banner("ties")
    base = random_bank(50, 0, 3, 60, 64, 0.99, 0.9999, 300)
    bank = base.subset([0, 1, 2, 1, 0, 2])       # 3..5 duplicate 1, 0, 2
    x = strain(3000, 50)
    with mk(bank, filters_per_lane=1) as bk:
        snr = bk.filter_block(dev(x)).cpu().numpy()
        bk.reset()
        mx, am = bk.trigger_max(dev(x))
        am = am.cpu().numpy()
    assert np.array_equal(snr[0], snr[4]) and np.array_equal(snr[1], snr[3]) and np.array_equal(snr[2], snr[5])
    assert am.max() <= 2
    ref = oracle.snr(bank, x)
    check_argmax(mx.cpu().numpy(), am, ref)


def test_near_ties_stay_admissible():
    """Duplicates at different lane positions sum their filters in a different
    order; their SNRs agree to rounding and the argmax stays in the admissible set."""
    banner("near ties")
    base = random_bank(50, 1, 3, 40, 90, 0.99, 0.9999, 300)
    bank = base.subset([0, 1, 2, 1, 0, 2])
    x = strain(3000, 50)
    with mk(bank) as bk:
        mx, am = bk.trigger_max(dev(x))
    ref = oracle.snr(bank, x)
    ties = check_argmax(mx.cpu().numpy(), am.cpu().numpy(), ref)
    assert ties > 0


# ---------------------------------------------------------------------------
# layouts, precisions, ragged sizes, edge cases
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def mid():
    # 12 templates, 1..700 filters, several waves per template, ragged length
    bank = random_bank(51, 0, 12, 1, 700, 0.99, 1 - 1e-5, 1500)
    x = strain(5003, 51)
    return bank, x, oracle.snr(bank, x)


def test_segment_layout_for_banks_that_cannot_fill_the_device():
    """A bank of more than 128 filters per compute unit that cannot fill the
    device even at 4 filters per lane gets, when the layout is left to the
    library, 4 filters per lane, 8-wave workgroups and 16 time segments;
    SNR rows and the fused max/argmax against the oracle over two calls."""
    bank = random_bank(61, 0, 40, 900, 1000, 0.99, 1 - 1e-5, 2047)
    n, h = 20000, 12288
    x = strain(n, 61)
    banner("segment layout: %d templates, %d filters" % (bank.n_templates, bank.n_filters))
    ref = oracle.snr(bank, x, nthreads=oracle.max_threads())
    xd = dev(x)
    with mk(bank) as bk:
        info = bk.info
        assert info["filters_per_lane"] == 4 and info["waves_per_group"] == 8
        assert info["time_split"] == 16
        s = torch.cat([bk.filter_block(xd[:h]), bk.filter_block(xd[h:])], dim=1).cpu().numpy()
        bk.reset()
        mx = torch.empty(n, dtype=torch.float32, device="cuda")
        am = torch.empty(n, dtype=torch.int32, device="cuda")
        bk.trigger_max(xd[:h], out=(mx[:h], am[:h]))
        bk.trigger_max(xd[h:], out=(mx[h:], am[h:]))
        torch.cuda.synchronize()
    err, _ = snr_err(s, ref)
    assert err <= SNR_TOL
    check_argmax(mx.cpu().numpy(), am.cpu().numpy(), ref)


@pytest.mark.parametrize("fl,L,wpg,prec", [
    (2, 64, 0, 0), (2, 256, 0, 0), (3, 128, 8, 0), (4, 512, 0, 0),
    (2, 8, 0, 0), (2, 256, 8, 2), (3, 256, 6, 2), (4, 64, 3, 0)])
def test_layouts_and_precisions(mid, fl, L, wpg, prec):
    bank, x, ref = mid
    banner("layout fl=%d L=%d wpg=%d prec=%d" % (fl, L, wpg, prec))
    with mk(bank, filters_per_lane=fl, chunk_len=L, waves_per_group=wpg, precision=prec) as bk:
        snr = bk.filter_block(dev(x)).cpu().numpy()
        info = bk.info
    err, _ = snr_err(snr, ref)
    print("layout", info, "err=%.3g" % err)
    assert err <= SNR_TOL


@pytest.mark.parametrize("L", [24, 40, 8])
def test_chunk_len_not_multiple_of_16(L):
    """Chunk lengths that are a multiple of 8 but not of 16 take 8-step tiles,
    so every chunk end still falls on a tile end and gets its FP64 carry
    correction. Poles within 2e-5 of the unit circle over 16,384-sample
    launches: the corrected recursion must beat the plain FP32 one (the
    precision mode without corrections) by a wide margin, as it does at L = 48,
    and stay within the gate."""
    banner("chunk_len %d" % L)
    bank = random_bank(55, 0, 6, 50, 300, 1 - 2e-5, 1 - 1e-6, 1000)
    x = strain(32768, 55)
    ref = oracle.snr(bank, x)
    err = {}
    for prec, chunk in ((0, L), (1, L), (0, 48)):
        with mk(bank, chunk_len=chunk, max_block=16384, precision=prec, time_split=1) as bk:
            assert bk.info["sub_block"] % chunk == 0
            s = torch.cat([bk.filter_block(dev(x[:16384])).clone(), bk.filter_block(dev(x[16384:]))], dim=1)
        err[(prec, chunk)], _ = snr_err(s.cpu().numpy(), ref)
    print("chunk_len %d: hybrid %.3g, all-FP32 %.3g, hybrid at L=48 %.3g"
          % (L, err[(0, L)], err[(1, L)], err[(0, 48)]))
    assert err[(0, L)] <= SNR_TOL
    assert err[(0, L)] <= 0.1 * err[(1, L)]


def test_template_too_large_for_one_workgroup(mid):
    """At one filter per lane a workgroup holds 512 filters: the larger
    templates of the bank are split into parts (time split on and off)."""
    bank, x, ref = mid
    assert bank.counts().max() > 512
    for ts in (1, 0):
        banner("templates over 512 filters at fl=1, time_split=%d" % ts)
        with mk(bank, filters_per_lane=1, time_split=ts) as bk:
            assert bk.info["n_parts"] >= 2
            snr = bk.filter_block(dev(x)).cpu().numpy()
        err, _ = snr_err(snr, ref)
        assert err <= SNR_TOL, "time_split %d: %.3g" % (ts, err)


def test_all_fp32_mode_runs(mid):
    bank, x, ref = mid
    banner("all fp32")
    with mk(bank, precision=1) as bk:
        snr = bk.filter_block(dev(x)).cpu().numpy()
    err, _ = snr_err(snr, ref)
    print("all-fp32 err=%.3g" % err)
    assert np.isfinite(snr).all() and err < 0.05
    # the time split keeps the mode's arithmetic (rounded coefficient, no correction)
    out = {}
    for ts in (1, 6):
        with mk(bank, precision=1, time_split=ts) as bk:
            out[ts] = bk.filter_block(dev(x)).cpu().numpy()
    d, _ = snr_err(out[6], out[1])
    print("all-fp32 split vs unsplit %.3g" % d)
    assert d <= 1e-4


def test_multi_piece_calls(mid):
    bank, x, ref = mid
    banner("pieces")
    with mk(bank, max_block=1024, chunk_len=128) as bk:       # one call, five launches
        snr = bk.filter_block(dev(x)).cpu().numpy()
    err, _ = snr_err(snr, ref)
    assert err <= SNR_TOL


def test_small_lds_sub_blocks(mid):
    bank, x, ref = mid
    banner("sub-blocks")
    # a long stream with windows refilled several times per launch
    with mk(bank, chunk_len=64, max_block=16384) as bk:
        assert bk.info["x_in_lds"] == 1
        mx, am = bk.trigger_max(dev(x))
        mx, am = mx.cpu().numpy(), am.cpu().numpy()
    check_argmax(mx, am, ref)


@pytest.mark.parametrize("band", [0, 4096, 16384])
def test_strain_window_in_global_memory(band):
    """240 KB of history does not fit LDS: without delay bands the window stays
    in global memory; with bands each workgroup stages its band's window in
    LDS (templates spanning bands are split into parts)."""
    banner("long delay window, delay_band=%d" % band)
    bank = random_bank(52, 0, 5, 20, 200, 0.99, 0.9999, 60000)
    x = strain(7000, 52)
    ref = oracle.snr(bank, x)
    with mk(bank, delay_band=band) as bk:
        info = bk.info
        assert info["x_in_lds"] == (0 if band == 0 else 1)
        assert info["delay_band"] == band
        snr = bk.filter_block(dev(x[:3000])).clone()
        snr2 = bk.filter_block(dev(x[3000:]))
        s = torch.cat([snr, snr2], dim=1).cpu().numpy()
    err, _ = snr_err(s, ref)
    assert err <= SNR_TOL


def test_single_filter_templates_and_zero_delay():
    banner("tiny templates")
    off = np.array([0, 1, 2, 66, 67], np.int64)
    rng = np.random.default_rng(3)
    F = 67
    a = 0.995 * np.exp(1j * rng.uniform(0.01, 1.5, F))
    b = (rng.standard_normal(F) + 1j * rng.standard_normal(F)) / 8
    d = rng.integers(0, 40, F).astype(np.int32)
    d[0] = 0
    bank = Bank(off, a, b, d, 40)
    x = strain(777, 53)
    ref = oracle.snr(bank, x)
    with mk(bank) as bk:
        s = bk.filter_block(dev(x)).cpu().numpy()
        mx, am = bk.trigger_max(dev(np.zeros(0, np.float32)))
    assert mx.numel() == 0
    err, _ = snr_err(s, ref)
    assert err <= SNR_TOL


@pytest.mark.parametrize("nseg,max_block,L", [(2, 4096, 256), (4, 2048, 128), (8, 16384, 64), (3, 5000, 8),
                                             (16, 8192, 64), (32, 16384, 64), (32, 4096, 256), (4, 4096, 24)])
def test_time_split_parity(mid, nseg, max_block, L):
    """Launches cut into segments filtered in parallel, joined by the FP64 carry
    chain: SNR rows and the fused max against the oracle, over several calls."""
    bank, x, ref = mid
    banner("time split nseg=%d max_block=%d L=%d" % (nseg, max_block, L))
    with mk(bank, time_split=nseg, max_block=max_block, chunk_len=L) as bk:
        assert bk.info["time_split"] == min(nseg, max(1, (max_block // L * L) // L))
        s1 = bk.filter_block(dev(x[:3001])).clone()
        s2 = bk.filter_block(dev(x[3001:]))
        snr = torch.cat([s1, s2], dim=1).cpu().numpy()
        bk.reset()
        mx, am = bk.trigger_max(dev(x))
    err, _ = snr_err(snr, ref)
    assert err <= SNR_TOL, err
    check_argmax(mx.cpu().numpy(), am.cpu().numpy(), ref)


def test_time_split_checkpoint_and_stream_continuity(mid):
    bank, x, ref = mid
    banner("time split checkpoint")
    xd = dev(x)
    with mk(bank, time_split=4, max_block=1024, chunk_len=64) as b1, mk(bank, time_split=4, max_block=1024,
                                                                          chunk_len=64) as b2:
        a = b1.filter_block(xd[:2500].contiguous()).clone()
        blob = b1.get_state()
        r1 = b1.filter_block(xd[2500:].contiguous()).clone()
        b2.set_state(blob)
        r2 = b2.filter_block(xd[2500:].contiguous()).clone()
    assert torch.equal(r1, r2)
    err, _ = snr_err(torch.cat([a, r1], dim=1).cpu().numpy(), ref)
    assert err <= SNR_TOL


def test_impulse_response_on_gpu():
    banner("impulse")
    bank = random_bank(54, 0, 3, 100, 300, 0.99, 0.9999, 200)
    n = 4000
    x = np.zeros(n, np.float32)
    x[0] = 1.0
    ref = oracle.snr(bank, x)
    with mk(bank) as bk:
        s = bk.filter_block(dev(x)).cpu().numpy()
    err, _ = snr_err(s, ref)
    assert err <= SNR_TOL


def test_kernel_timing_api(c0):
    """spiir_bank_time_kernels / spiir_bank_kernel_time: one timed launch per
    block call, positive durations, totals cleared on read, ESTATE when off."""
    from paper_1602_05573_amd import SpiirError
    bank, x, _ = c0
    banner("kernel timing")
    with mk(bank) as bk:
        with pytest.raises(SpiirError, match="timing is off"):
            bk.kernel_time()
        xd = dev(x)
        bk.time_kernels(True)
        for i in range(0, len(x), 4096):
            bk.trigger_max(xd[i:i + 4096])
        ms, n = bk.kernel_time()
        assert n == (len(x) + 4095) // 4096 and ms > 0
        assert bk.kernel_time() == (0.0, 0)
        # more launches than the event ring holds: the oldest pairs are collected on reuse
        for _ in range(300):
            bk.trigger_max(xd[:256])
        ms, n = bk.kernel_time()
        assert n == 300 and ms > 0
        bk.time_kernels(False)
        with pytest.raises(SpiirError, match="timing is off"):
            bk.kernel_time()


@pytest.mark.parametrize("tsplit", [1, 0])
def test_irregular_call_sizes(mid, tsplit):
    """The stream fed in calls of 1, 2, 3, 7, 15, 16, 17, 100, 1000 samples and
    the rest (partial tiles, partial chunks, calls shorter than a segment):
    SNR and fused outputs against the oracle."""
    bank, x, ref = mid
    banner("irregular calls time_split=%d" % tsplit)
    cuts = np.cumsum([0, 1, 1, 2, 3, 7, 15, 16, 17, 100, 1000])
    cuts = np.append(cuts, len(x))
    with mk(bank, time_split=tsplit) as bk:
        parts = [bk.filter_block(dev(x[c0:c1])).cpu().numpy() for c0, c1 in zip(cuts[:-1], cuts[1:])]
    snr = np.concatenate(parts, axis=1)
    err, _ = snr_err(snr, ref)
    print("irregular calls err=%.3g" % err)
    assert err <= SNR_TOL
    with mk(bank, time_split=tsplit) as bk:
        outs = [bk.trigger_max(dev(x[c0:c1])) for c0, c1 in zip(cuts[:-1], cuts[1:])]
    mx = torch.cat([o[0] for o in outs]).cpu().numpy()
    am = torch.cat([o[1] for o in outs]).cpu().numpy()
    check_argmax(mx, am, ref)


def test_degenerate_coefficients_and_largest_template():
    """a = 0 (a pure delayed tap), b = 0 (a silent filter), d = max_delay, and a
    template that fills a whole workgroup (8 waves x 4 rows x 16 lanes x 4
    filters = 2,048 filters) beside a one-filter template."""
    banner("degenerate coefficients, largest template")
    rng = np.random.default_rng(11)
    K0, dmax = 2048, 1200
    off = np.array([0, K0, K0 + 1, K0 + 4], np.int64)
    F = int(off[-1])
    a = 0.999 * np.exp(1j * rng.uniform(0.01, 1.5, F))
    b = (rng.standard_normal(F) + 1j * rng.standard_normal(F)) / 40
    d = rng.integers(0, dmax + 1, F).astype(np.int32)
    a[5] = 0.0            # y = b x[n - d]
    b[6] = 0.0            # contributes nothing
    d[7] = dmax
    a[K0] = 0.0           # one-filter template that is a pure tap at the longest delay
    d[K0] = dmax
    a[K0 + 1:] = 0.5 - 0.25j
    bank = Bank(off, a, b, d, dmax)
    x = strain(6007, 57)
    ref = oracle.snr(bank, x)
    for tsplit in (1, 0):
        with mk(bank, filters_per_lane=4, time_split=tsplit) as bk:
            assert bk.info["waves_per_group"] == 8
            s = bk.filter_block(dev(x)).cpu().numpy()
            bk.reset()
            mx, am = bk.trigger_max(dev(x))
        err, _ = snr_err(s, ref)
        print("degenerate time_split=%d err=%.3g" % (tsplit, err))
        assert err <= SNR_TOL
        check_argmax(mx.cpu().numpy(), am.cpu().numpy(), ref)
    # the one-tap template is exactly |b|^2 x[n - dmax]^2 (x = 0 before the stream)
    tap = np.zeros(len(x))
    tap[dmax:] = np.abs(b[K0]) ** 2 * x[:-dmax].astype(np.float64) ** 2
    assert np.allclose(ref[1], tap, rtol=1e-12, atol=1e-300)



# ---------------------------------------------------------------------------
# Templates longer than one workgroup: split into parts, summed by a combine
# launch before the SNR / z / keys
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def big():
    # templates of 5,000 and 2,500 filters (3 and 2 parts at 8 waves x 4 filters
    # per lane) among small ones
    b0 = random_bank(81, 0, 6, 20, 400, 0.99, 1 - 1e-5, 3000)
    b1 = random_bank(81, 1, 1, 5000, 5000, 0.99, 1 - 1e-5, 3000)
    b2 = random_bank(81, 2, 1, 2500, 2500, 0.99, 0.9999, 3000)
    parts = [b0.subset([0, 1]), b1, b0.subset([2, 3, 4]), b2, b0.subset([5])]
    off = [0]
    for p in parts:
        off += list(off[-1] + p.offsets[1:])
    bank = Bank(np.array(off, np.int64), np.concatenate([p.a for p in parts]),
                np.concatenate([p.b for p in parts]), np.concatenate([p.d for p in parts]).astype(np.int32), 3000)
    x = strain(9000, 81)
    return bank, x, oracle.snr(bank, x)


@pytest.mark.parametrize("tsplit", [1, 4])
def test_split_templates_snr_and_trigger(big, tsplit):
    bank, x, ref = big
    banner("split templates time_split=%d" % tsplit)
    xd = dev(x)
    with mk(bank, filters_per_lane=4, waves_per_group=8, chunk_len=128, max_block=4096,
            time_split=tsplit) as bk:
        info = bk.info
        assert info["n_parts"] == 5, info
        s1 = bk.filter_block(xd[:5000]).clone()
        s2 = bk.filter_block(xd[5000:])
        snr = torch.cat([s1, s2], dim=1).cpu().numpy()
        bk.reset()
        mx, am = bk.trigger_max(xd)
        mx, am = mx.cpu().numpy(), am.cpu().numpy()
    err, _ = snr_err(snr, ref)
    print("split templates: SNR error %.3g" % err)
    assert err <= SNR_TOL
    check_argmax(mx, am, ref)


def test_split_templates_forward_z_and_adjoint(big):
    bank, x, _ = big
    banner("split templates forward_z + backward")
    n = 3000
    xs = x[:n]
    zr = oracle.z(bank, xs)
    rng = np.random.default_rng(8101)
    G = (rng.standard_normal(zr.shape) + 1j * rng.standard_normal(zr.shape)) / 50
    ga_ref, gb_ref = oracle.backward(bank, xs, G)
    with mk(bank, filters_per_lane=4, waves_per_group=8, chunk_len=128, max_block=2048) as bk:
        assert bk.info["n_parts"] == 5
        z, tape = bk.forward_z(dev(xs), want_tape=True)
        ga, gb = bk.backward(tape, torch.from_numpy(G.astype(np.complex64)).cuda())
        tape.close()
        z, ga, gb = z.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()
    peak = np.abs(zr).max(axis=1)
    zerr = float(np.max(np.abs(z - zr).max(axis=1) / peak))
    print("split templates: z error %.3g" % zerr)
    assert zerr <= SNR_TOL
    for g, gref, what in ((ga, ga_ref, "grad_a"), (gb, gb_ref, "grad_b")):
        for j in range(bank.n_templates):
            sl = slice(int(bank.offsets[j]), int(bank.offsets[j + 1]))
            e = np.linalg.norm(g[sl] - gref[sl]) / np.linalg.norm(gref[sl])
            assert e <= 1e-3, "%s template %d: %.3g" % (what, j, e)


def test_split_templates_refused_by_comparator_and_batch(big):
    from paper_1602_05573_amd import SpiirBatch, SpiirError
    bank, x, _ = big
    banner("split templates refused")
    xd = dev(x[:4096])
    with mk(bank, filters_per_lane=4, waves_per_group=8) as bk:
        with pytest.raises(SpiirError, match="one workgroup"):
            bk.trigger_max_per_template(xd)
        with pytest.raises(SpiirError, match="split"):
            SpiirBatch([bk], [xd], block_len=4096)


@pytest.mark.parametrize("band,tsplit,L", [(512, 1, 256), (700, 4, 128), (64, 0, 64)])
def test_forced_delay_bands(mid, band, tsplit, L):
    """Delay bands forced on a bank whose window fits LDS anyway: every
    template is split by band; SNR over two calls, the fused trigger, and
    z / gradients of the adjoint against the oracle."""
    bank, x, ref = mid
    banner("forced delay bands %d, time_split %d, L %d" % (band, tsplit, L))
    xd = dev(x)
    with mk(bank, delay_band=band, time_split=tsplit, chunk_len=L, max_block=4096) as bk:
        info = bk.info
        assert info["delay_band"] == band and info["x_in_lds"] == 1 and info["n_parts"] > 0
        s1 = bk.filter_block(xd[:2500]).clone()
        s2 = bk.filter_block(xd[2500:])
        snr = torch.cat([s1, s2], dim=1).cpu().numpy()
        bk.reset()
        mx, am = bk.trigger_max(xd)
        mx, am = mx.cpu().numpy(), am.cpu().numpy()
        n = 2000
        zr = oracle.z(bank, x[:n])
        rng = np.random.default_rng(9101)
        G = (rng.standard_normal(zr.shape) + 1j * rng.standard_normal(zr.shape)) / 40
        ga_ref, gb_ref = oracle.backward(bank, x[:n], G)
        z, tape = bk.forward_z(dev(x[:n]), want_tape=True)
        ga, gb = bk.backward(tape, torch.from_numpy(G.astype(np.complex64)).cuda())
        tape.close()
        z, ga, gb = z.cpu().numpy(), ga.cpu().numpy(), gb.cpu().numpy()
    err, _ = snr_err(snr, ref)
    print("delay bands %d: SNR error %.3g, %d parts" % (band, err, info["n_parts"]))
    assert err <= SNR_TOL
    check_argmax(mx, am, ref)
    peak = np.abs(zr).max(axis=1)
    assert float(np.max(np.abs(z - zr).max(axis=1) / peak)) <= SNR_TOL
    for g, gref in ((ga, ga_ref), (gb, gb_ref)):
        for j in range(bank.n_templates):
            sl = slice(int(bank.offsets[j]), int(bank.offsets[j + 1]))
            assert np.linalg.norm(g[sl] - gref[sl]) <= 1e-3 * np.linalg.norm(gref[sl])
