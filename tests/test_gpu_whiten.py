"""Whitening front end on the GPU (spiir_whitener_*) against the oracle's
Welch PSD and frame-wise whitening."""
import numpy as np
import pytest

import oracle
from workloads import coloured_noise

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# FP32 transforms: error relative to the largest value of the compared series
TOL = 1e-4


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def banner(msg):
    print("[case] " + msg, flush=True)


@pytest.mark.parametrize("N", [16, 256, 4096, 8192])
def test_psd_parity(N):
    from paper_1602_05573_amd import Whitener
    x = coloured_noise(40 * N + 123, 4)
    banner("psd N=%d" % N)
    ref = oracle.welch_psd(x, N)
    with Whitener(N) as wh:
        wh.estimate_psd(torch.from_numpy(x).cuda())
        got = wh.psd()
    rel = np.max(np.abs(got - ref) / ref)
    print("N=%d: PSD max relative error per bin %.3g (dynamic range %.3g)" % (N, rel, ref.max() / ref.min()))
    assert np.max(np.abs(got - ref)) <= TOL * ref.max()
    assert rel <= 1e-3


@pytest.mark.parametrize("N,max_block", [(64, 0), (1024, 2048), (4096, 0), (8192, 8192)])
def test_whiten_parity_streaming(N, max_block):
    """GPU PSD, then the stream whitened in calls of irregular lengths
    (multiples of N/2, some longer than max_block) against the oracle with
    the same PSD."""
    from paper_1602_05573_amd import Whitener
    H = N // 2
    n = 24 * N
    x = coloured_noise(n, 5)
    banner("whiten N=%d max_block=%d" % (N, max_block))
    xd = torch.from_numpy(x).cuda()
    cuts = [0, H, 3 * H, 10 * H, 11 * H, 40 * H, n]
    with Whitener(N, max_block=max_block) as wh:
        wh.estimate_psd(xd)
        S = wh.psd()
        parts = [wh.process(xd[a:b]) for a, b in zip(cuts[:-1], cuts[1:])]
        got = torch.cat(parts).cpu().numpy()
        wh.reset()
        again = wh.process(xd).cpu().numpy()
    ref = oracle.whiten(x, S, N)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("N=%d: whitened error %.3g of the peak" % (N, err))
    assert err <= TOL
    assert np.max(np.abs(again - ref)) <= TOL * np.max(np.abs(ref))


def test_unit_psd_is_a_delay():
    from paper_1602_05573_amd import Whitener
    N, H = 512, 256
    x = np.random.default_rng(3).standard_normal(64 * H).astype(np.float32)
    banner("unit psd")
    with Whitener(N) as wh:
        wh.set_psd(np.ones(H + 1))
        y = wh.process(torch.from_numpy(x).cuda()).cpu().numpy()
        assert np.array_equal(wh.psd(), np.ones(H + 1))
    assert np.max(np.abs(y[:H])) < 1e-6
    assert np.max(np.abs(y[H:] - x[:-H])) < 1e-5 * np.max(np.abs(x))


def test_whitened_noise_is_flat():
    """Coloured noise spanning four decades of power comes out flat at unit level."""
    from paper_1602_05573_amd import Whitener
    N = 1024
    x = coloured_noise(1 << 17, 6)
    banner("flatness")
    with Whitener(N) as wh:
        xd = torch.from_numpy(x).cuda()
        wh.estimate_psd(xd)
        y = wh.process(xd).cpu().numpy()
    S2 = oracle.welch_psd(y[N:], N)
    assert abs(S2.mean() - 1.0) < 0.02 and S2.min() > 0.75 and S2.max() < 1.3


def test_whitener_errors():
    from paper_1602_05573_amd import SpiirError, Whitener
    with pytest.raises(SpiirError, match="power of two"):
        Whitener(1000)
    with pytest.raises(SpiirError, match="power of two"):
        Whitener(16384)
    with Whitener(64) as wh:
        x = torch.zeros(64, device="cuda")
        with pytest.raises(SpiirError, match="no PSD"):
            wh.process(x)
        with pytest.raises(SpiirError, match="shorter"):
            wh.estimate_psd(torch.zeros(63, device="cuda"))
        bad = np.ones(33)
        bad[4] = -1.0
        with pytest.raises(SpiirError, match="negative"):
            wh.set_psd(bad)
        wh.set_psd(np.ones(33))
        with pytest.raises(SpiirError, match="multiple"):
            wh.process(torch.zeros(40, device="cuda"))


def test_whiten_full_size():
    """The bench configuration: 4,194,304 samples of coloured noise, 4,096-sample
    frames, PSD from the first 32 s, the whole stream whitened in 4,096-sample
    calls against the oracle."""
    from paper_1602_05573_amd import Whitener
    N, n = 4096, 1 << 22
    x = coloured_noise(n, 0)
    banner("whiten full size")
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    with Whitener(N) as wh:
        wh.estimate_psd(xd[:32 * 4096])
        S = wh.psd()
        for i in range(n // 4096):
            wh.process(xd[i * 4096:(i + 1) * 4096], out=out[i * 4096:(i + 1) * 4096])
        got = out.cpu().numpy()
    ref = oracle.whiten(x, S, N)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print("full size: whitened error %.3g of the peak" % err)
    assert err <= TOL
    Sref = oracle.welch_psd(x[:32 * 4096], N)
    assert np.max(np.abs(S - Sref)) <= TOL * Sref.max()
