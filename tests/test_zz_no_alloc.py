"""The allocation-free trigger call (spiir_trigger_max_noalloc) against the
allocating one (spiir_trigger_max), through the C ABI: two banks built from
the same definition, one driven by each call, over two calls in a row (the
second shorter), must give identical max/argmax, which must also pass the
argmax rule against the FP64 oracle. Covered: a bank whose strain window sits
in LDS, a time-split bank (segment states and local sums in the scratch
array), a bank whose window stays in global memory (window in the scratch
array), a bank with a template split over workgroups, two banks sharing the
array call by call, a bank whose time segments must be cut to fit the array,
and the size limit."""
import numpy as np
import pytest

import oracle
from helpers import check_argmax
from workloads import random_bank, strain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SCRATCH_BYTES = 32 << 20


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    from paper_1602_05573_amd import load
    load()


def banner(msg):
    print("[case] " + msg, flush=True)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run_pair(bank, x, cuts, **opts):
    """Feeds x in pieces [cuts[i], cuts[i+1]) to two banks of the same
    definition, one per call; returns both (max, argmax) series and the
    first bank's info."""
    from paper_1602_05573_amd import SpiirBank
    n = len(x)
    xd = dev(x)
    outs = []
    with SpiirBank.from_bank(bank, **opts) as ba, SpiirBank.from_bank(bank, **opts) as bb:
        info = ba.info
        for bk, noalloc in ((ba, False), (bb, True)):
            mx = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
            am = torch.full((n,), -1, dtype=torch.int32, device="cuda")
            for c0, c1 in zip(cuts[:-1], cuts[1:]):
                out = (mx[c0:c1], am[c0:c1])
                if noalloc:
                    bk.trigger_max_noalloc(xd[c0:c1], out=out)
                else:
                    bk.trigger_max(xd[c0:c1], out=out)
            torch.cuda.synchronize()
            outs.append((mx.cpu().numpy(), am.cpu().numpy()))
    return outs, info


def check_same(bank, x, outs):
    (m0, a0), (m1, a1) = outs
    assert np.array_equal(m0, m1), "max differs at %s" % np.nonzero(m0 != m1)[0][:10]
    assert np.array_equal(a0, a1), "argmax differs at %s" % np.nonzero(a0 != a1)[0][:10]
    ties = check_argmax(m1, a1, oracle.snr(bank, x))
    print("identical to the allocating call; %d documented ties" % ties, flush=True)


@pytest.mark.parametrize("cuts", [(0, 6000, 7234), (0, 4096, 5120)])
def test_window_in_lds(cuts):
    banner("noalloc: window in LDS, cuts %s" % (cuts,))
    bank = random_bank(71, 0, 24, 60, 300, 0.99, 0.99999, 2047)
    x = strain(cuts[-1], 71)
    outs, info = run_pair(bank, x, list(cuts), chunk_len=64, max_block=4096, time_split=1)
    assert info["x_in_lds"] == 1 and info["time_split"] == 1
    check_same(bank, x, outs)


def test_time_split():
    banner("noalloc: time split")
    bank = random_bank(72, 0, 6, 100, 400, 0.99, 0.99999, 1500)
    x = strain(9000, 72)
    outs, info = run_pair(bank, x, [0, 5003, 9000], chunk_len=64, max_block=4096, time_split=4)
    assert info["time_split"] == 4
    check_same(bank, x, outs)


def test_window_in_global_memory():
    banner("noalloc: window in global memory")
    bank = random_bank(73, 0, 5, 20, 200, 0.99, 0.9999, 60000)   # 240 KB of history: not in LDS
    x = strain(7000, 73)
    outs, info = run_pair(bank, x, [0, 4500, 7000])
    assert info["x_in_lds"] == 0
    check_same(bank, x, outs)


def test_templates_split_over_workgroups():
    """A template of 5,000 filters (three parts) beside small ones: the key
    row of the split templates is carved from the array too."""
    banner("noalloc: split templates")
    b0 = random_bank(76, 0, 5, 20, 300, 0.99, 0.99999, 1000)
    b1 = random_bank(76, 1, 1, 5000, 5000, 0.99, 0.99999, 1000)
    from workloads import Bank
    off = np.concatenate([b0.offsets, b0.offsets[-1] + b1.offsets[1:]]).astype(np.int64)
    bank = Bank(off, np.concatenate([b0.a, b1.a]), np.concatenate([b0.b, b1.b]),
                np.concatenate([b0.d, b1.d]).astype(np.int32), 1000)
    x = strain(6000, 76)
    outs, info = run_pair(bank, x, [0, 4100, 6000], filters_per_lane=4, waves_per_group=8, max_block=4096)
    assert info["n_parts"] == 3
    check_same(bank, x, outs)


def test_two_banks_share_the_array():
    """Calls of two different banks alternate on the one array; each bank's
    series equals its allocating twin's."""
    from paper_1602_05573_amd import SpiirBank
    banner("noalloc: two banks alternate")
    b1 = random_bank(74, 0, 10, 50, 250, 0.99, 0.9999, 3000)
    b2 = random_bank(74, 1, 3, 300, 600, 0.99, 0.99999, 900)
    x = strain(8192, 74)
    xd = dev(x)
    cuts = [0, 5000, 8192]
    res = {}
    with SpiirBank.from_bank(b1, time_split=1) as p1, SpiirBank.from_bank(b2, time_split=3) as p2, \
            SpiirBank.from_bank(b1, time_split=1) as q1, SpiirBank.from_bank(b2, time_split=3) as q2:
        for name, bk, noalloc in (("p1", p1, True), ("p2", p2, True), ("q1", q1, False), ("q2", q2, False)):
            res[name] = (torch.empty(8192, dtype=torch.float32, device="cuda"),
                         torch.empty(8192, dtype=torch.int32, device="cuda"))
        for c0, c1 in zip(cuts[:-1], cuts[1:]):
            for name, bk, noalloc in (("p1", p1, True), ("p2", p2, True), ("q1", q1, False), ("q2", q2, False)):
                out = (res[name][0][c0:c1], res[name][1][c0:c1])
                if noalloc:
                    bk.trigger_max_noalloc(xd[c0:c1], out=out)
                else:
                    bk.trigger_max(xd[c0:c1], out=out)
        torch.cuda.synchronize()
        r = {k: (v[0].cpu().numpy(), v[1].cpu().numpy()) for k, v in res.items()}
    for bank, pn, qn in ((b1, "p1", "q1"), (b2, "p2", "q2")):
        check_same(bank, x, [r[qn], r[pn]])


def test_segments_cut_to_fit_the_array():
    """A bank whose own time split (16 segments of 65,536 slots) does not fit
    the array: the allocation-free call cuts its launches into fewer
    segments, so it agrees with the allocating call to FP32 rounding (not
    bitwise), and both pass the gate and the argmax rule against the oracle."""
    from helpers import SNR_TOL
    banner("noalloc: segments cut to fit")
    bank = random_bank(77, 0, 64, 1000, 1000, 0.99, 0.99999, 2047)
    x = strain(20000, 77)
    outs, info = run_pair(bank, x, [0, 12288, 20000])
    # the bank's segment states alone fill the array, beside the partial keys
    assert info["time_split"] == 16 and info["n_slots"] * 16 * 2 * 16 >= SCRATCH_BYTES
    (m0, a0), (m1, a1) = outs
    ref = oracle.snr(bank, x, nthreads=oracle.max_threads())
    peak = float(ref.max())
    assert np.max(np.abs(m0.astype(np.float64) - m1)) <= SNR_TOL * peak
    assert np.max(np.abs(m1.astype(np.float64) - ref.max(axis=0))) <= SNR_TOL * peak
    check_argmax(m0, a0, ref)
    check_argmax(m1, a1, ref)


def test_size_limit_is_an_error():
    """A call whose window would not fit the array is refused before any
    launch (x is a real buffer of that length all the same)."""
    from paper_1602_05573_amd import SpiirBank
    from paper_1602_05573_amd._lib import SPIIR_EINVAL, SpiirError
    banner("noalloc: size limit")
    bank = random_bank(75, 0, 2, 20, 40, 0.99, 0.999, 60000)
    n = SCRATCH_BYTES // 4          # the window alone needs (n + dmax + 16) * 4 bytes
    xd = torch.zeros(n, dtype=torch.float32, device="cuda")
    mx = torch.empty(n, dtype=torch.float32, device="cuda")
    am = torch.empty(n, dtype=torch.int32, device="cuda")
    with SpiirBank.from_bank(bank) as bk:
        assert bk.info["x_in_lds"] == 0
        with pytest.raises(SpiirError) as ei:
            bk.trigger_max_noalloc(xd, out=(mx, am))
        assert ei.value.code == SPIIR_EINVAL and "allocation-free" in str(ei.value)
        # the refused call left the stream untouched: a valid call still matches the oracle
        x = strain(3000, 75)
        m, a = bk.trigger_max_noalloc(dev(x), out=(mx[:3000], am[:3000]))
        torch.cuda.synchronize()
        check_argmax(m.cpu().numpy(), a.cpu().numpy(), oracle.snr(bank, x))
