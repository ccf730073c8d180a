"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times.

The 1,024-template bank (1,024 templates x U{100..800} filters, 4,194,304
samples in 4,096-sample blocks) is compared with the FP64 oracle in full:
every template's SNR row over the whole stream, element by element, and the
fused max/argmax over every sample with the admissible-set rule for ties.
The oracle's work is split into eight parts of 128 templates (each part is
one test, so progress shows); the per-sample maximum over templates is the
merge of the parts' maxima (max, lowest index among equal values), which the
oracle pins check against the oracle's own trigger.
"""
import time

import numpy as np
import pytest

import oracle
from helpers import ARG_EPS, SNR_TOL, check_argmax
from workloads import bank_1024, batch_streams

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

B = 4096
PARTS = 8                 # oracle parts of the 1,024-template bank
PREFIX_BLOCKS = 16        # blocks whose documented ties are counted exactly
_parts = {}               # part -> (M, J, P, ref at the GPU argmax, row errors), filled in order


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def banner(msg):
    print("[case] " + msg, flush=True)


@pytest.fixture(scope="module")
def c1():
    """The bench.py run of the bank (chunk_len 256, 4,096-sample blocks,
    library-chosen layout and time split): the fused max/argmax of every
    block, then, after a reset, every template's SNR row of every block (kept
    on the device, 17 GB). On every block the fused output must equal the max
    of the rows and the lowest row attaining it."""
    from paper_1602_05573_amd import SpiirBank
    banner("bank_1024 full size: GPU passes")
    bank, x = bank_1024()
    N, T = len(x), bank.n_templates
    xd = torch.from_numpy(x).cuda()
    with SpiirBank.from_bank(bank, chunk_len=256, filters_per_lane=0, time_split=0, waves_per_group=0,
                             max_block=B) as bk:
        info = bk.info
        mx = torch.empty(N, dtype=torch.float32, device="cuda")
        am = torch.empty(N, dtype=torch.int32, device="cuda")
        for i in range(N // B):
            sl = slice(i * B, (i + 1) * B)
            bk.trigger_max(xd[sl], out=(mx[sl], am[sl]))
        bk.reset()
        rows = torch.empty((T, N), dtype=torch.float32, device="cuda")
        bad_max, bad_arg = [], []
        for i in range(N // B):
            sl = slice(i * B, (i + 1) * B)
            s = bk.filter_block(xd[sl], snr=rows[:, sl])
            m = s.max(dim=0).values
            first = torch.argmax((s == m[None, :]).to(torch.int8), dim=0).to(torch.int32)
            if not torch.equal(m, mx[sl]):
                bad_max.append(i)
            if not torch.equal(first, am[sl]):
                bad_arg.append(i)
        torch.cuda.synchronize()
    print("bank_1024 layout %s" % info, flush=True)
    return {"bank": bank, "x": x, "rows": rows, "mx": mx.cpu().numpy(), "am": am.cpu().numpy(),
            "bad_max": bad_max, "bad_arg": bad_arg}


def test_bank1024_fused_is_max_of_rows(c1):
    """Fused epilogue = max over the per-template SNR rows, lowest index among
    equal values, bitwise, on all 1,024 blocks."""
    assert not c1["bad_max"], "fused max differs from the rows in blocks %s" % c1["bad_max"][:10]
    assert not c1["bad_arg"], "argmax is not the lowest maximal row in blocks %s" % c1["bad_arg"][:10]


def _part(c1, p):
    """Oracle SNR of templates [128 p, 128 (p + 1)) over the whole stream
    against the GPU rows, element by element; the part's per-sample max,
    lowest attaining index, per-template peaks, and the oracle SNR of the
    GPU's argmax template wherever that template is in the part."""
    if p in _parts:
        return _parts[p]
    bank, x = c1["bank"], c1["x"]
    T = bank.n_templates
    j0, j1 = T * p // PARTS, T * (p + 1) // PARTS
    t0 = time.time()
    ref = oracle.snr(bank, x, templates=np.arange(j0, j1))
    t_or = time.time() - t0
    got = c1["rows"][j0:j1].cpu().numpy()
    P = ref.max(axis=1)
    err = np.array([np.max(np.abs(got[r].astype(np.float64) - ref[r])) / P[r] for r in range(j1 - j0)])
    J = np.argmax(ref, axis=0)               # first (lowest) index attaining the part's max
    M = ref[J, np.arange(ref.shape[1])]
    g = c1["am"].astype(np.int64)
    at = np.nonzero((g >= j0) & (g < j1))[0]
    ref_g = ref[g[at] - j0, at]
    _parts[p] = (M, J + j0, P, at, ref_g, err)
    print("part %d (templates %d..%d): oracle %.1f s, max SNR error %.3g of the peak"
          % (p, j0, j1 - 1, t_or, err.max()), flush=True)
    del ref, got
    return _parts[p]


@pytest.mark.parametrize("p", range(PARTS))
def test_bank1024_every_template_full_stream(c1, p):
    banner("bank_1024 oracle part %d of %d" % (p, PARTS))
    err = _part(c1, p)[5]
    assert err.max() <= SNR_TOL, "template %d: SNR error %.3g" % (int(np.argmax(err)) + 1024 * p // PARTS,
                                                                 err.max())


def test_bank1024_fused_argmax_full_stream(c1):
    """The fused max/argmax of all 4,194,304 samples against the oracle: the
    GPU's template must be the oracle's (lowest maximal) one, or lie in the
    admissible set A[n] = {j : ref_j >= ref_J - eps (P_j + P_J)} (a documented
    tie); the fused max within eps of the GPU template's peak."""
    banner("bank_1024 fused argmax over the whole stream")
    N = len(c1["x"])
    M = np.full(N, -1.0)
    J = np.full(N, -1, np.int64)
    P = []
    ref_g = np.full(N, np.nan)
    for p in range(PARTS):
        m, j, pk, at, rg, _ = _part(c1, p)
        take = (m > M) | ((m == M) & (j < J))     # merge: max, lowest index among equal values
        M = np.where(take, m, M)
        J = np.where(take, j, J)
        P.append(pk)
        ref_g[at] = rg
    P = np.concatenate(P)
    g = c1["am"].astype(np.int64)
    gm = c1["mx"].astype(np.float64)
    assert not np.isnan(ref_g).any()
    diff = np.nonzero(g != J)[0]
    adm = ref_g[diff] >= M[diff] - ARG_EPS * (P[g[diff]] + P[J[diff]])
    merr = np.abs(gm - M) / P[g]
    print("bank_1024 full stream: %d of %d samples take another template than the oracle, all inside "
          "the admissible set: %s; max fused-max error %.3g of the template peak"
          % (diff.size, N, bool(adm.all()), merr.max()), flush=True)
    assert adm.all(), "argmax outside the admissible set at samples %s" % diff[~adm][:10]
    assert merr.max() <= ARG_EPS, "fused max error %.3g" % merr.max()


def test_bank1024_prefix_ties_counted(c1):
    """On the first 16 blocks every template's oracle row is at hand: the
    helper's exact rule (unique samples must match, the rest stay admissible)
    and the number of documented ties (samples with more than one admissible
    template)."""
    banner("bank_1024 prefix ties")
    n = PREFIX_BLOCKS * B
    ref = oracle.snr(c1["bank"], c1["x"][:n])
    ties = check_argmax(c1["mx"][:n], c1["am"][:n], ref)
    print("bank_1024 first %d samples: %d documented ties" % (n, ties), flush=True)


def test_bank1024_clustering_full_stream(c1):
    """Trigger clustering of the fused output, as bench.py runs it: identical to
    the oracle's clustering of the same series."""
    from paper_1602_05573_amd import cluster_triggers
    m, a = c1["mx"], c1["am"]
    thr, W = float(np.quantile(m, 0.9999)), 4096
    banner("bank_1024 clustering threshold %.6g window %d" % (thr, W))
    gi, gt, gv, total = cluster_triggers(torch.from_numpy(m).cuda(), torch.from_numpy(a).cuda(), thr, W)
    ri, rt, rv = oracle.clusters(m, a, thr, W)
    assert total == len(ri) and total > 0
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
