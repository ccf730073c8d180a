"""Multi-rate bank on the GPU (spiir_multirate_*) against the oracle's
multi-rate definition: decimation, per-level filtering, interpolation and
summation, then |z|^2 and the per-sample max / argmax."""
import numpy as np
import pytest

import oracle
from helpers import SNR_TOL, check_argmax, snr_err
from workloads import Bank, multirate_bank, resample_taps, strain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def banner(msg):
    print("[case] " + msg, flush=True)


def rand_levels(T, per, seed, r_lo=0.9, r_hi=0.999, dmax=40):
    """per[r] = most filters per template at level r (0 = none); counts drawn
    in 0..per[r], so some templates have no filters at a level."""
    rng = np.random.default_rng(300 + seed)
    out = []
    for k in per:
        cnt = rng.integers(0, k + 1, T) if k else np.zeros(T, np.int64)
        off = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
        F = int(off[-1])
        a = rng.uniform(r_lo, r_hi, F) * np.exp(1j * rng.uniform(0.001 * np.pi, 0.5 * np.pi, F))
        b = (rng.standard_normal(F) + 1j * rng.standard_normal(F)) / 4
        d = rng.integers(0, dmax + 1, F).astype(np.int32)
        out.append(Bank(off, a, b, d, dmax))
    return out


def z_err(got, ref):
    """max over templates of max |dz| / max |z_ref| (templates with z = 0 must be 0)."""
    worst = 0.0
    for j in range(ref.shape[0]):
        p = np.max(np.abs(ref[j]))
        e = np.max(np.abs(got[j] - ref[j]))
        worst = max(worst, e / p if p > 0 else e)
    return worst


CONFIGS = [
    # (templates, max filters per template per level, decimation taps, interpolation taps, n, max_block)
    (6, [8, 12, 20], 24, 24, 8192, 0),
    (5, [0, 10, 0, 30], 16, 20, 6144, 2048),      # empty levels, pieces of 2,048
    (4, [30], 8, 8, 3000, 0),                     # one level: an ordinary bank
    (7, [4, 0, 0, 0, 25], 24, 24, 4096, 1024),    # 5 levels, only the top and the bottom hold filters
    (3, [0, 0, 16], 7, 9, 4000, 0),               # odd tap counts, only the top level
    (4, [6, 10, 14], 24, 24, 36864, 32768),       # a piece above the one-launch decimation size, then a short one
    (5, [4, 8, 12], 64, 64, 6144, 2048),          # longest taps: the largest interpolation windows
]


@pytest.mark.parametrize("cfg", range(len(CONFIGS)))
def test_multirate_z_parity(cfg):
    from paper_1602_05573_amd import SpiirMultiRate
    T, per, lh, lg, n, mb = CONFIGS[cfg]
    levels = rand_levels(T, per, cfg)
    if lh == lg == 24:
        h, g = resample_taps(24)
    else:
        rng = np.random.default_rng(cfg)
        h, g = rng.standard_normal(lh) / lh, rng.standard_normal(lg) / lg
    x = strain(n, 6, cfg)
    banner("multirate z cfg %d: T=%d per=%s taps=%d/%d n=%d max_block=%d" % (cfg, T, per, lh, lg, n, mb))
    ref = oracle.multirate_z(levels, h, g, x)
    with SpiirMultiRate(levels, h, g, max_block=mb) as mr:
        z = mr.filter_block_z(torch.from_numpy(x).cuda()).cpu().numpy()
    e = z_err(z, ref)
    print("cfg %d: z error %.3g" % (cfg, e))
    assert e <= SNR_TOL


@pytest.mark.parametrize("cfg", [0, 1, 3, 6])
def test_multirate_trigger_parity(cfg):
    from paper_1602_05573_amd import SpiirMultiRate
    T, per, lh, lg, n, mb = CONFIGS[cfg]
    levels = rand_levels(T, per, cfg)
    h, g = resample_taps(24)
    x = strain(n, 6, 10 + cfg)
    banner("multirate trigger cfg %d" % cfg)
    zz = oracle.multirate_z(levels, h, g, x)
    ref = zz.real ** 2 + zz.imag ** 2
    with SpiirMultiRate(levels, h, g, max_block=mb) as mr:
        mx, am = mr.trigger_max(torch.from_numpy(x).cuda())
        mx, am = mx.cpu().numpy(), am.cpu().numpy()
    err, _ = snr_err(mx[None, :], ref.max(axis=0)[None, :])
    assert err <= SNR_TOL
    ties = check_argmax(mx, am, ref)
    print("cfg %d: max error %.3g, %d documented ties" % (cfg, err, ties))


def test_multirate_streaming_and_reset():
    """Irregular call lengths (multiples of 2^R) continue one stream; reset
    restores the cold start."""
    from paper_1602_05573_amd import SpiirMultiRate
    T, per = 5, [6, 10, 14, 20]
    levels = rand_levels(T, per, 21)
    h, g = resample_taps(20)
    n = 8192
    x = strain(n, 6, 21)
    banner("multirate streaming")
    ref = oracle.multirate_z(levels, h, g, x)
    xd = torch.from_numpy(x).cuda()
    cuts = [0, 8, 1024, 1032, 4096, 4104, 8192]
    with SpiirMultiRate(levels, h, g, max_block=2048) as mr:
        parts = [mr.filter_block_z(xd[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
        z = torch.cat(parts, dim=1).cpu().numpy()
        assert z_err(z, ref) <= SNR_TOL
        mr.reset()
        z2 = mr.filter_block_z(xd).cpu().numpy()
        assert z_err(z2, ref) <= SNR_TOL
        # fused max over the same stream after another reset
        mr.reset()
        mx, am = mr.trigger_max(xd)
        # the fused max is taken over the same full-rate z
        s = np.abs(z2.astype(np.complex128)) ** 2
        assert np.max(np.abs(mx.cpu().numpy() - s.max(axis=0))) <= 1e-6 * s.max()
        check_argmax(mx.cpu().numpy(), am.cpu().numpy(), s)


def test_multirate_graph_replay_equals_eager():
    """Trigger pieces replayed from the captured graphs equal the eager path
    bitwise, across mixed call lengths (graph pieces, shorter eager pieces),
    a reset, timing switched on and off, and many replays of both parities."""
    from paper_1602_05573_amd import SpiirMultiRate
    T, per = 9, [5, 8, 0, 24]
    levels = rand_levels(T, per, 40)
    h, g = resample_taps(24)
    B = 1024
    n = 40 * B
    x = strain(n, 6, 40)
    banner("multirate graph replay")
    xd = torch.from_numpy(x).cuda()
    cuts = [0, B, 2 * B, 2 * B + 256, 3 * B + 256, 7 * B + 256, 7 * B + 512, 20 * B, n]

    def run(graph, timing_at=None):
        mx = torch.empty(n, dtype=torch.float32, device="cuda")
        am = torch.empty(n, dtype=torch.int32, device="cuda")
        with SpiirMultiRate(levels, h, g, max_block=B) as mr:
            mr.set_graph(graph)
            for k, (a, b) in enumerate(zip(cuts[:-1], cuts[1:])):
                if timing_at is not None and k == timing_at:
                    mr.time_kernels(True)
                if timing_at is not None and k == timing_at + 2:
                    mr.kernel_time()
                    mr.time_kernels(False)
                mr.trigger_max(xd[a:b], out=(mx[a:b], am[a:b]))
            torch.cuda.synchronize()
            first = (mx.clone(), am.clone())
            mr.reset()
            mr.trigger_max(xd, out=(mx, am))
            torch.cuda.synchronize()
        return first, (mx, am)

    (e1, e2) = run(False)
    (g1, g2) = run(True, timing_at=4)
    assert torch.equal(e1[0], g1[0]) and torch.equal(e1[1], g1[1])
    assert torch.equal(e2[0], g2[0]) and torch.equal(e2[1], g2[1])
    zz = oracle.multirate_z(levels, h, g, x)
    s = zz.real ** 2 + zz.imag ** 2
    assert np.max(np.abs(g2[0].cpu().numpy() - s.max(axis=0))) <= SNR_TOL * s.max()


def test_multirate_grouped_small_levels_equal_per_level_calls():
    """Small levels (few filters per compute unit) run as one group of
    time-split launches; with kernel timing on, every level is its own bank
    call. Both give the same full-rate z and max / argmax bitwise over
    several calls, and the grouped banks share one workgroup size."""
    from paper_1602_05573_amd import SpiirMultiRate
    T, per = 12, [6, 10, 0, 16, 30]
    levels = rand_levels(T, per, 41)
    h, g = resample_taps(24)
    B = 2048
    n = 5 * B
    x = strain(n, 6, 41)
    banner("multirate grouped small levels")
    xd = torch.from_numpy(x).cuda()

    def run(timing):
        z = torch.empty((T, n), dtype=torch.complex64, device="cuda")
        mx = torch.empty(n, dtype=torch.float32, device="cuda")
        am = torch.empty(n, dtype=torch.int32, device="cuda")
        with SpiirMultiRate(levels, h, g, max_block=B) as mr:
            wpg = {mr.level_info(r)["waves_per_group"] for r in (0, 1, 3, 4)}
            mr.set_graph(False)
            mr.time_kernels(timing)
            for k in range(0, n, B):
                z[:, k:k + B] = mr.filter_block_z(xd[k:k + B])
            mr.reset()
            for k in range(0, n, B):
                mr.trigger_max(xd[k:k + B], out=(mx[k:k + B], am[k:k + B]))
            torch.cuda.synchronize()
            if timing:
                mr.kernel_time()
        return wpg, z.cpu(), mx.cpu(), am.cpu()

    wg, zg, mg, ag = run(False)
    wt, zt, mt, at = run(True)
    assert len(wg) == 1 and wg == wt
    assert torch.equal(zg, zt)
    assert torch.equal(mg, mt) and torch.equal(ag, at)
    zz = oracle.multirate_z(levels, h, g, x)
    assert z_err(zg.numpy(), zz) <= SNR_TOL


def test_multirate_graph_after_odd_reset():
    """Reset after an odd number of pieces, then graph replays mixed with eager
    pieces: equal to the same calls with graphs off (the graphs bake in which
    history buffer of each level bank is current)."""
    from paper_1602_05573_amd import SpiirMultiRate
    levels = rand_levels(6, [4, 6, 12], 41)
    h, g = resample_taps(16)
    B = 1024
    x = strain(40 * B, 6, 41)
    xd = torch.from_numpy(x).cuda()
    banner("multirate graph after odd reset")
    plan = [(0, 3 * B), "reset", (3 * B, 5 * B), (5 * B, 5 * B + 256), (5 * B + 256, 9 * B + 256), "reset",
            (0, B), (B, B + 512), (B + 512, 12 * B + 512)]

    def run(graph):
        outs = []
        with SpiirMultiRate(levels, h, g, max_block=B) as mr:
            mr.set_graph(graph)
            for step in plan:
                if step == "reset":
                    mr.reset()
                    continue
                a, b = step
                mx, am = mr.trigger_max(xd[a:b])
                outs.append((mx.clone(), am.clone()))
            torch.cuda.synchronize()
        return outs

    eager, graph = run(False), run(True)
    for (em, ea), (gm, ga) in zip(eager, graph):
        assert torch.equal(em, gm) and torch.equal(ea, ga)


def test_multirate_level_banks():
    """Each level runs a bank of exactly the templates that have filters there;
    a level without filters has no bank."""
    from paper_1602_05573_amd import SpiirMultiRate
    levels = rand_levels(8, [3, 0, 9, 5], 42)
    h, g = resample_taps(8)
    with SpiirMultiRate(levels, h, g, max_block=2048) as mr:
        for r, lv in enumerate(levels):
            info = mr.level_info(r)
            present = int(np.count_nonzero(np.diff(lv.offsets)))
            if lv.n_filters == 0:
                assert info is None and mr.level_bank_handle(r) is None
            else:
                assert info["n_templates"] == present and info["n_filters"] == lv.n_filters


def test_multirate_rejects_bad_arguments():
    from paper_1602_05573_amd import SpiirError, SpiirMultiRate
    levels = rand_levels(3, [4, 4], 30)
    h, g = resample_taps(8)
    with pytest.raises(SpiirError, match="taps"):
        SpiirMultiRate(levels, np.zeros(0), g)
    with pytest.raises(SpiirError, match="no level"):
        SpiirMultiRate(rand_levels(3, [0, 0], 31), h, g)
    bad = rand_levels(3, [4, 4], 32)
    bad[1].offsets = bad[1].offsets[::-1].copy()
    with pytest.raises(SpiirError):
        SpiirMultiRate(bad, h, g)
    with SpiirMultiRate(levels, h, g) as mr:
        with pytest.raises(SpiirError, match="multiple"):
            mr.filter_block_z(torch.zeros(101, device="cuda"))


def test_multirate_chirp_bank_sampled_full_size():
    """The bench workload: 1,024 chirp-like templates over 5 levels, 4,194,304
    samples in 4,096-sample blocks; sampled templates against the oracle over
    the whole stream, and the fused max against the sampled SNRs."""
    from paper_1602_05573_amd import SpiirMultiRate
    levels = multirate_bank()
    h, g = resample_taps(24)
    N, B = 1 << 22, 4096
    x = strain(N, 6)
    pick = [0, 411, 1023]
    banner("multirate chirp bank full size")
    xd = torch.from_numpy(x).cuda()
    with SpiirMultiRate(levels, h, g, max_block=B) as mr:
        mx = torch.empty(N, dtype=torch.float32, device="cuda")
        am = torch.empty(N, dtype=torch.int32, device="cuda")
        for i in range(N // B):
            sl = slice(i * B, (i + 1) * B)
            mr.trigger_max(xd[sl], out=(mx[sl], am[sl]))
        mr.reset()
        zs = torch.empty((len(pick), N), dtype=torch.complex64, device="cuda")
        zb = torch.empty((levels[0].n_templates, B), dtype=torch.complex64, device="cuda")
        sel = torch.tensor(pick, device="cuda")
        for i in range(N // B):
            mr.filter_block_z(xd[i * B:(i + 1) * B], z=zb)
            zs[:, i * B:(i + 1) * B] = zb.index_select(0, sel)
        torch.cuda.synchronize()
    sub = [lv.subset(pick) for lv in levels]
    ref = oracle.multirate_z(sub, h, g, x)
    got = zs.cpu().numpy()
    e = z_err(got, ref)
    print("chirp bank sampled-template z error %.3g" % e)
    assert e <= SNR_TOL
    m, a = mx.cpu().numpy(), am.cpu().numpy()
    s = np.abs(ref) ** 2
    P = s.max(axis=1)
    for r, j in enumerate(pick):
        assert np.all(m >= s[r] - SNR_TOL * P[r])
        at = np.nonzero(a == j)[0]
        if at.size:
            assert np.max(np.abs(m[at] - s[r, at])) <= SNR_TOL * P[r]


def test_single_bank_streaming_z():
    """spiir_filter_block_z on an ordinary bank: streaming z equals the
    oracle's z, and |z|^2 equals filter_block's SNR bitwise."""
    from paper_1602_05573_amd import SpiirBank
    from workloads import bank_4x128
    bank, x = bank_4x128()
    banner("single bank streaming z")
    ref = oracle.z(bank, x)
    xd = torch.from_numpy(x).cuda()
    with SpiirBank.from_bank(bank) as bk:
        z = torch.cat([bk.filter_block_z(xd[:5000]), bk.filter_block_z(xd[5000:])], dim=1)
        bk.reset()
        snr = torch.cat([bk.filter_block(xd[:5000]), bk.filter_block(xd[5000:])], dim=1)
    zc = z.cpu().numpy()
    assert z_err(zc, ref) <= SNR_TOL
    zz = z.real.float() ** 2 + z.imag.float() ** 2
    assert float((zz - snr).abs().max()) <= 1e-6 * float(snr.max())
