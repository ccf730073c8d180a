"""Batched streams: one persistent launch per step, recorded in a HIP graph,
advancing several banks over uneven streams; checked against per-bank
streaming calls (bitwise) and against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from helpers import check_argmax
from workloads import random_bank, strain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def banner(msg):
    print("[case] " + msg, flush=True)


def make(n_streams=3, lengths=(10000, 25001, 4097), fl=2, L=256, wpg=4):
    from paper_1602_05573_amd import SpiirBank
    banks = [random_bank(70, s, 5 + s, 40, 400, 0.99, 1 - 1e-5, 3000) for s in range(n_streams)]
    xs = [strain(lengths[s], 70, s) for s in range(n_streams)]
    bks = [SpiirBank.from_bank(b, filters_per_lane=fl, chunk_len=L, waves_per_group=wpg) for b in banks]
    return banks, xs, bks


def test_batch_matches_streaming_and_oracle():
    from paper_1602_05573_amd import SpiirBank, SpiirBatch
    banner("batch vs streaming")
    banks, xs, bks = make()
    xd = [torch.from_numpy(x).cuda() for x in xs]
    bt = SpiirBatch(bks, xd, block_len=4096)
    bt.set_time_split(1)   # plain graph: bitwise equal to unsplit streaming
    steps = bt.steps_total()
    assert steps == (25001 + 4095) // 4096
    for _ in range(steps):
        bt.step()
    bt.step()   # every stream has ended: a no-op replay
    torch.cuda.synchronize()
    for s, (b, x) in enumerate(zip(banks, xs)):
        with SpiirBank.from_bank(b, filters_per_lane=2, chunk_len=256, waves_per_group=4, time_split=1) as ref_bk:
            m, a = ref_bk.trigger_max(xd[s])
        assert torch.equal(bt.max[s], m), "stream %d max differs" % s
        assert torch.equal(bt.argmax[s], a), "stream %d argmax differs" % s
    ref = oracle.snr(banks[1], xs[1])
    check_argmax(bt.max[1].cpu().numpy(), bt.argmax[1].cpu().numpy(), ref)
    # replays after a reset reproduce the run bit for bit
    first = [m.clone() for m in bt.max]
    bt.reset()
    for _ in range(steps):
        bt.step()
    torch.cuda.synchronize()
    for s in range(len(xs)):
        assert torch.equal(first[s], bt.max[s])
    bt.close()
    for bk in bks:
        bk.close()


@pytest.mark.parametrize("mode", [2, 0])
def test_batch_time_split_graph(mode):
    """Blocks cut into time segments inside the batch graph (always, or
    automatically for the tail where one stream is left) agree with the plain
    graph to rounding and pass the oracle's gate; ragged last blocks."""
    from paper_1602_05573_amd import SpiirBatch
    banner("batch time split mode %d" % mode)
    banks, xs, bks = make(lengths=(10000, 29001, 4097))
    xd = [torch.from_numpy(x).cuda() for x in xs]
    out = {}
    for m in (1, mode):
        bt = SpiirBatch(bks, xd, block_len=4096)
        bt.set_time_split(m)
        for _ in range(bt.steps_total()):
            bt.step()
        torch.cuda.synchronize()
        out[m] = ([t.clone() for t in bt.max], [t.clone() for t in bt.argmax])
        bt.close()
    for s, (b, x) in enumerate(zip(banks, xs)):
        ref = oracle.snr(b, x)
        P = ref.max()
        mx, am = out[mode][0][s].cpu().numpy(), out[mode][1][s].cpu().numpy()
        assert np.max(np.abs(mx - ref.max(axis=0))) <= 1e-4 * P, "stream %d" % s
        check_argmax(mx, am, ref)
        d = (out[mode][0][s] - out[1][0][s]).abs().max().item()
        assert d <= 1e-4 * P, "stream %d: split vs plain %.3g" % (s, d)
    for bk in bks:
        bk.close()


def test_batch_time_split_mode_errors():
    from paper_1602_05573_amd import SpiirBank, SpiirBatch, SpiirError
    banner("batch time split modes")
    b0 = random_bank(73, 0, 3, 40, 100, 0.99, 0.999, 100)
    x = torch.from_numpy(strain(5000, 73)).cuda()
    with SpiirBank.from_bank(b0, filters_per_lane=1, chunk_len=512) as k1:
        # 512-sample blocks hold one chunk: no time-split graph exists
        bt = SpiirBatch([k1], [x], block_len=512)
        with pytest.raises(SpiirError, match="no time-split"):
            bt.set_time_split(2)
        with pytest.raises(SpiirError, match="mode"):
            bt.set_time_split(3)
        bt.set_time_split(0)
        for _ in range(bt.steps_total()):
            bt.step()
        torch.cuda.synchronize()
        m, a = bt.max[0].clone(), bt.argmax[0].clone()
        bt.close()
    with SpiirBank.from_bank(b0, filters_per_lane=1, chunk_len=512, time_split=1) as ref:
        rm, ra = ref.trigger_max(x)
    assert torch.equal(m, rm) and torch.equal(a, ra)


def test_batch_rejects_mixed_layouts():
    from paper_1602_05573_amd import SpiirBank, SpiirBatch, SpiirError
    banner("batch mixed layouts")
    b0 = random_bank(71, 0, 3, 40, 100, 0.99, 0.999, 100)
    x = torch.from_numpy(strain(5000, 71)).cuda()
    with SpiirBank.from_bank(b0, filters_per_lane=1) as k1, SpiirBank.from_bank(b0, filters_per_lane=2) as k2:
        with pytest.raises(SpiirError, match="share"):
            SpiirBatch([k1, k2], [x, x], block_len=4096)
        with pytest.raises(SpiirError, match="twice"):
            SpiirBatch([k1, k1], [x, x], block_len=4096)


def test_autotune_picks_a_candidate():
    from paper_1602_05573_amd import autotune, SpiirBank
    banner("autotune")
    banks = [random_bank(72, s, 8, 100, 300, 0.99, 1 - 1e-5, 2000) for s in range(2)]
    L, F, table = autotune(banks, block_len=4096)
    assert L in (64, 128, 256, 512) and F in (1, 2, 3, 4)
    li = (64, 128, 256, 512).index(L)
    assert table[li, F - 1] > 0
    valid = table[table > 0]
    assert table[li, F - 1] == valid.min()
    # bank creation with autotune uses the tuner's choice
    with SpiirBank.from_bank(banks[0], autotune=1) as bk:
        assert bk.info["chunk_len"] in (64, 128, 256, 512)
