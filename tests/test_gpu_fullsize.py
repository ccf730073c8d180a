"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times. The oracle computes what it can one by one
(sampled templates over the whole stream, every template over a prefix); the
rest is checked through properties that hold at any size (the fused max is
the max of the per-template rows, the batch equals per-bank streaming)."""
import numpy as np
import pytest

import oracle
from helpers import SNR_TOL, check_argmax, snr_err
from workloads import bank_1024, batch_streams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

B = 4096
PICK1 = [0, 517, 1023]            # sampled templates of the 1,024-template bank
SAMPLE_BLOCKS = (0, 1, 300, 1023)  # blocks where fused and plain outputs are compared whole


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def banner(msg):
    print("[case] " + msg, flush=True)


def test_bank1024_full_size():
    """1,024 templates x U{100..800} filters over 4,194,304 samples in
    4,096-sample blocks (the bench.py configuration)."""
    from paper_1602_05573_amd import SpiirBank
    banner("bank_1024 full size")
    bank, x = bank_1024()
    N, T = len(x), bank.n_templates
    xd = torch.from_numpy(x).cuda()
    with SpiirBank.from_bank(bank, chunk_len=256, max_block=B) as bk:
        mx = torch.empty(N, dtype=torch.float32, device="cuda")
        am = torch.empty(N, dtype=torch.int32, device="cuda")
        for i in range(N // B):
            sl = slice(i * B, (i + 1) * B)
            bk.trigger_max(xd[sl], out=(mx[sl], am[sl]))
        bk.reset()
        rows = torch.empty((len(PICK1), N), dtype=torch.float32, device="cuda")
        snr = torch.empty((T, B), dtype=torch.float32, device="cuda")
        pick = torch.tensor(PICK1, device="cuda")
        ar = torch.arange(B, device="cuda")
        for i in range(N // B):
            sl = slice(i * B, (i + 1) * B)
            s = bk.filter_block(xd[sl], snr=snr)
            rows[:, sl] = s.index_select(0, pick)
            if i in SAMPLE_BLOCKS:
                # fused epilogue = max over the plain rows, lowest index among equal values
                m = s.max(dim=0).values
                assert torch.equal(m, mx[sl]), "block %d: fused max differs from the rows" % i
                first = torch.argmax((s == m[None, :]).to(torch.int8), dim=0).to(torch.int32)
                assert torch.equal(first, am[sl]), "block %d: argmax is not the lowest maximal row" % i
        torch.cuda.synchronize()
    banner("bank_1024 oracle on templates %s" % PICK1)
    ref = oracle.snr(bank.subset(PICK1), x)
    got = rows.cpu().numpy()
    err, per = snr_err(got, ref)
    print("bank_1024 sampled-template SNR error %.3g (per template %s)" % (err, per))
    assert err <= SNR_TOL
    # wherever the fused argmax is a sampled template, the fused max is its oracle SNR
    m, a = mx.cpu().numpy(), am.cpu().numpy()
    P = ref.max(axis=1)
    for r, j in enumerate(PICK1):
        at = np.nonzero(a == j)[0]
        if at.size:
            assert np.max(np.abs(m[at] - ref[r, at])) <= SNR_TOL * P[r]
        # and the max over all templates is never below a sampled template's SNR
        assert np.all(m >= ref[r] - SNR_TOL * P[r])
    # trigger clustering of the fused output, as bench.py runs it
    from paper_1602_05573_amd import cluster_triggers
    thr, W = float(np.quantile(m, 0.9999)), 4096
    banner("bank_1024 clustering threshold %.6g window %d" % (thr, W))
    gi, gt, gv, total = cluster_triggers(mx, am, thr, W)
    ri, rt, rv = oracle.clusters(m, a, thr, W)
    rtotal = len(ri)
    assert total == rtotal and total > 0
    assert np.array_equal(gi.cpu().numpy(), ri) and np.array_equal(gt.cpu().numpy(), rt)
    assert np.array_equal(gv.cpu().numpy(), rv)


def test_batch_streams_full_size():
    """8 uneven streams (2^18..2^22 samples), 256-template banks of U{200..600}
    filters, autotuned L and filters per lane, automatic graph choice (the
    bench.py configuration)."""
    from paper_1602_05573_amd import SpiirBank, SpiirBatch, autotune, batch_banks
    banner("batch_streams full size")
    banks, xs = batch_streams()
    L, F, _ = autotune(banks, block_len=B)
    bks = batch_banks(banks, L, F)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    bt = SpiirBatch(bks, xd, block_len=B)
    for _ in range(bt.steps_total()):
        bt.step()
    torch.cuda.synchronize()
    npre = 8192
    for s, (b, x) in enumerate(zip(banks, xs)):
        # whole stream: per-bank streaming (no time split) on the same layout
        with SpiirBank.from_bank(b, chunk_len=L, filters_per_lane=F, time_split=1,
                                 waves_per_group=bks[s].info["waves_per_group"]) as rb:
            m, a = rb.trigger_max(xd[s])
        P = m.max().item()
        d = (bt.max[s] - m).abs().max().item()
        assert d <= SNR_TOL * P, "stream %d: batch vs streaming %.3g of the peak" % (s, d / P)
        # prefix: every template against the oracle
        ref = oracle.snr(b, x[:npre])
        check_argmax(bt.max[s][:npre].cpu().numpy(), bt.argmax[s][:npre].cpu().numpy(), ref)
        print("stream %d (%d samples): batch vs streaming %.3g of the peak" % (s, len(x), d / P))
    bt.close()
    for bk in bks:
        bk.close()
