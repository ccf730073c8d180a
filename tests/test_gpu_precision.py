"""Precision plan of the recursion at full size (64 templates x 1,000 filters,
r ~ U[1-1e-6, 1-1e-4], 16,777,216 samples): FP32 recursion with FP64 chunk
carries against all-FP32 and against the FP64 oracle, on sampled templates."""
import numpy as np
import pytest

import oracle
from helpers import SNR_TOL, snr_err
from workloads import precision_bank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PICK = [5, 42]


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


@pytest.fixture(scope="module")
def c4():
    bank, x = precision_bank()
    print("[case] precision_bank oracle on templates %s" % PICK, flush=True)
    ref = oracle.snr(bank.subset(PICK), x)
    return bank, x, ref


def run(bank, x, precision):
    from paper_1602_05573_amd import SpiirBank
    with SpiirBank.from_bank(bank, precision=precision) as bk:
        xd = torch.from_numpy(x).cuda()
        out = torch.empty((len(PICK), len(x)), dtype=torch.float32)
        # stream the whole input in 1,048,576-sample calls; keep only the sampled rows
        snr = torch.empty((bank.n_templates, 1 << 20), dtype=torch.float32, device="cuda")
        for c0 in range(0, len(x), 1 << 20):
            c1 = min(len(x), c0 + (1 << 20))
            s = bk.filter_block(xd[c0:c1], snr=snr[:, : c1 - c0] if c1 - c0 == snr.shape[1] else None)
            out[:, c0:c1] = s[PICK].cpu()
    return out.numpy()


@pytest.mark.parametrize("precision,must_pass", [(0, True), (2, True), (1, False)])
def test_precision_bank_modes(c4, precision, must_pass):
    bank, x, ref = c4
    print("[case] precision_bank precision=%d" % precision, flush=True)
    got = run(bank, x, precision)
    err, per = snr_err(got, ref)
    print("precision %d: max relative SNR error %.3g (per template %s)" % (precision, err, per))
    if must_pass:
        assert err <= SNR_TOL
    else:
        assert np.isfinite(err)
