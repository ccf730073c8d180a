"""The three stages composed as a streaming pipeline on the GPU: raw
(coloured) strain -> whitening -> fused bank trigger (max / argmax) ->
trigger clustering, block by block, against the oracle chain (whiten,
trigger, clusters) on the same input."""
import numpy as np
import pytest

import oracle
from helpers import SNR_TOL, check_argmax
from workloads import coloured_noise, random_bank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def test_pipeline_matches_oracle_chain():
    from paper_1602_05573_amd import SpiirBank, Whitener, cluster_triggers
    N, B, n = 1024, 2048, 32 * 2048
    x = coloured_noise(n, 9)
    bank = random_bank(7, 0, 24, 50, 120, 0.99, 0.9995, 300)
    print("[case] pipeline n=%d block=%d" % (n, B), flush=True)
    xd = torch.from_numpy(x).cuda()
    white = torch.empty_like(xd)
    mx = torch.empty(n, dtype=torch.float32, device="cuda")
    am = torch.empty(n, dtype=torch.int32, device="cuda")
    with Whitener(N) as wh, SpiirBank.from_bank(bank) as bk:
        wh.estimate_psd(xd[:16 * N])
        S = wh.psd()
        for i in range(n // B):
            sl = slice(i * B, (i + 1) * B)
            wh.process(xd[sl], out=white[sl])
            bk.trigger_max(white[sl], out=(mx[sl], am[sl]))
        thr = float(torch.quantile(mx[n // 2:], 0.999))
        ti, tt, tv, total = cluster_triggers(mx, am, thr, 1500)
        torch.cuda.synchronize()
    # oracle chain on the same raw input and the same PSD
    w_ref = oracle.whiten(x, S, N)
    w_gpu = white.cpu().numpy()
    assert np.max(np.abs(w_gpu - w_ref)) <= 1e-4 * np.max(np.abs(w_ref))
    # the bank on the GPU's whitened stream (whitening parity is checked above)
    ref = oracle.snr(bank, w_gpu)
    m, a = mx.cpu().numpy(), am.cpu().numpy()
    P = ref.max()
    assert np.max(np.abs(m - ref.max(axis=0))) <= SNR_TOL * P
    check_argmax(m, a, ref)
    ri, rt, rv = oracle.clusters(m, a, thr, 1500)
    assert total == len(ri) > 0
    assert np.array_equal(ti.cpu().numpy(), ri) and np.array_equal(tt.cpu().numpy(), rt)
    assert np.array_equal(tv.cpu().numpy(), rv)
