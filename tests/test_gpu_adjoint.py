"""GPU parity of the reverse-time adjoint (forward_z + tape + backward) and of
the autograd Function, against the FP64 oracle's gradients."""
import numpy as np
import pytest

import oracle
from workloads import Bank, chirp_target, chirp_fit, random_bank, strain

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# Gradient gate (FP32 adjoint against the FP64 oracle's gradient), per
# template: the error vector's norm relative to the oracle gradient's norm,
# and every entry of at least 1e-3 of the template's largest entry relative
# to itself, both at most GRAD_TOL.
GRAD_TOL = 1e-3


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def mk(bank, **kw):
    from paper_1602_05573_amd import SpiirBank
    return SpiirBank.from_bank(bank, **kw)


def banner(msg):
    print("[case] " + msg, flush=True)


def grad_close(g_gpu, g_ref, off, tol=GRAD_TOL, what="grad"):
    """Per-template norm error and large-entry error of g_gpu against g_ref,
    both asserted at tol; returns the worst norm error."""
    worst, worst_ent = 0.0, 0.0
    for j in range(len(off) - 1):
        sl = slice(int(off[j]), int(off[j + 1]))
        a, b = np.asarray(g_gpu[sl], np.complex128), g_ref[sl]
        nrm = np.linalg.norm(b)
        worst = max(worst, np.linalg.norm(a - b) / max(nrm, 1e-300))
        big = np.abs(b) >= 1e-3 * np.abs(b).max()
        worst_ent = max(worst_ent, float(np.max(np.abs(a[big] - b[big]) / np.abs(b[big]))))
    print("%s: worst per-template norm error %.3g, worst large-entry error %.3g" % (what, worst, worst_ent),
          flush=True)
    assert worst <= tol, "%s: norm error %.3g" % (what, worst)
    assert worst_ent <= tol, "%s: entry error %.3g" % (what, worst_ent)
    return worst


@pytest.mark.parametrize("tsplit,max_block", [(0, 0), (1, 0), (3, 4096), (8, 0)])
def test_forward_z_parity(tsplit, max_block):
    banner("forward_z time_split=%d max_block=%d" % (tsplit, max_block))
    bank = random_bank(60, 0, 6, 30, 500, 0.99, 1 - 1e-5, 800)
    x = strain(9001, 60)
    ref = oracle.z(bank, x)
    with mk(bank, chunk_len=128, time_split=tsplit, max_block=max_block) as bk:
        z = bk.forward_z(torch.from_numpy(x).cuda()).cpu().numpy()
        # forward_z leaves the streaming state alone: a streaming call still starts cold
        s = bk.filter_block(torch.from_numpy(x).cuda()).cpu().numpy()
    err = np.max(np.abs(z - ref).max(axis=1) / np.abs(ref).max(axis=1))
    assert err <= 1e-4, err
    sref = np.abs(ref) ** 2
    assert np.max(np.abs(s - sref).max(axis=1) / sref.max(axis=1)) <= 1e-4


@pytest.mark.parametrize("L,fl", [(64, 1), (256, 2), (512, 4), (24, 2), (40, 3)])
def test_backward_matches_oracle_random_upstream(L, fl):
    banner("backward L=%d fl=%d" % (L, fl))
    bank = random_bank(61, 0, 5, 20, 300, 0.99, 0.9999, 500)
    n = 5000
    x = strain(n, 61)
    rng = np.random.default_rng(7)
    G = (rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))) * 1e-2
    ga_ref, gb_ref = oracle.backward(bank, x, G)
    with mk(bank, chunk_len=L, filters_per_lane=fl) as bk:
        xd = torch.from_numpy(x).cuda()
        z, tape = bk.forward_z(xd, want_tape=True)
        ga, gb = bk.backward(tape, torch.from_numpy(G.astype(np.complex64)).cuda())
        ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
        tape.close()
    ea = grad_close(ga, ga_ref, bank.offsets, what="L=%d grad_a" % L)
    eb = grad_close(gb, gb_ref, bank.offsets, what="L=%d grad_b" % L)
    print("grad err a %.3g b %.3g" % (ea, eb))


@pytest.mark.parametrize("tsplit,prec", [(1, 0), (2, 0), (5, 0), (8, 2), (3, 1)])
def test_backward_time_segments(tsplit, prec):
    """The adjoint cut into time segments (segment-local lambda, FP64 chain,
    per-segment gradients) against the oracle and against the unsplit run;
    ragged last chunk and sub-chunk."""
    banner("backward time_split=%d precision=%d" % (tsplit, prec))
    bank = random_bank(62, 0, 7, 40, 200, 0.99, 1 - 1e-5, 900)
    n = 7777
    x = strain(n, 62)
    rng = np.random.default_rng(8)
    G = (rng.standard_normal((7, n)) + 1j * rng.standard_normal((7, n))) * 1e-2
    ga_ref, gb_ref = oracle.backward(bank, x, G)
    out = {}
    for ts in (1, tsplit):
        with mk(bank, chunk_len=128, filters_per_lane=2, time_split=ts, precision=prec) as bk:
            xd = torch.from_numpy(x).cuda()
            z, tape = bk.forward_z(xd, want_tape=True)
            ga, gb = bk.backward(tape, torch.from_numpy(G.astype(np.complex64)).cuda())
            out[ts] = (ga.cpu().numpy(), gb.cpu().numpy())
            tape.close()
    tol = GRAD_TOL if prec != 1 else 2e-2
    ga, gb = out[tsplit]
    ea = grad_close(ga, ga_ref, bank.offsets, tol, what="split %d prec %d grad_a" % (tsplit, prec))
    eb = grad_close(gb, gb_ref, bank.offsets, tol, what="split %d prec %d grad_b" % (tsplit, prec))
    # split and unsplit runs differ only by FP32 rounding order
    ga1, gb1 = out[1]
    da = np.linalg.norm(ga - ga1) / np.linalg.norm(ga1)
    db = np.linalg.norm(gb - gb1) / np.linalg.norm(gb1)
    print("grad err a %.3g b %.3g; split vs unsplit %.3g %.3g" % (ea, eb, da, db))
    assert da <= tol and db <= tol


def test_backward_of_overlap_loss_on_chirps():
    banner("overlap loss chirps")
    n = 16384
    masses = [1.5, 7.0, 22.0]
    k = 120
    a, b, d, gs = [], [], [], []
    from workloads import chirp_init_bank
    for mc in masses:
        g = chirp_target(mc, n)
        aj, bj, dj = chirp_init_bank(g, k)
        a.append(aj); b.append(bj); d.append(dj); gs.append(g)
    bank = Bank(np.arange(len(masses) + 1, dtype=np.int64) * k, np.concatenate(a), np.concatenate(b),
                np.concatenate(d).astype(np.int32), n - 1)
    gs = np.array(gs)
    x = np.zeros(n, np.float32)
    x[0] = 1.0
    zr = oracle.z(bank, x)
    loss_ref, G_ref = oracle.overlap_loss(zr, gs)
    ga_ref, gb_ref = oracle.backward(bank, x, G_ref)
    with mk(bank) as bk:
        xd = torch.from_numpy(x).cuda()
        z, tape = bk.forward_z(xd, want_tape=True)
        zc = z.cpu().numpy().astype(np.complex128)
        loss, G = oracle.overlap_loss(zc, gs)         # upstream gradient at the GPU's z
        ga, gb = bk.backward(tape, torch.from_numpy(G.astype(np.complex64)).cuda())
        ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
        tape.close()
    assert np.max(np.abs(loss - loss_ref)) < 1e-4
    grad_close(ga, ga_ref, bank.offsets, what="chirps grad_a")
    grad_close(gb, gb_ref, bank.offsets, what="chirps grad_b")


def test_spiirfn_autograd_and_fit_step():
    banner("SpiirFn")
    from paper_1602_05573_amd import SpiirFn
    n = 8192
    k = 64
    g = chirp_target(12.0, n)
    from workloads import chirp_init_bank
    a0, b0, d0 = chirp_init_bank(g, k)
    bank = Bank(np.array([0, k], np.int64), a0, b0, d0, n - 1)
    x = np.zeros(n, np.float32)
    x[0] = 1.0
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()

    def loss_fn(z):
        c = torch.sum(z[0] * torch.conj(gt))
        return 1 - torch.abs(c) / (torch.linalg.norm(z[0]) * torch.linalg.norm(gt))

    with mk(bank) as bk:
        a = torch.tensor(a0, dtype=torch.complex128, requires_grad=True)
        b = torch.tensor(b0, dtype=torch.complex128, requires_grad=True)
        xd = torch.from_numpy(x).cuda()
        z = SpiirFn.apply(a, b, bk, xd)
        loss = loss_fn(z)
        loss.backward()
        zr = oracle.z(bank, x)
        lref, Gref = oracle.overlap_loss(zr, g[None, :])
        ga_ref, gb_ref = oracle.backward(bank, x, Gref)
        assert abs(float(loss) - lref[0]) < 1e-4
        grad_close(a.grad.numpy(), ga_ref, bank.offsets, what="SpiirFn grad_a")
        grad_close(b.grad.numpy(), gb_ref, bank.offsets, what="SpiirFn grad_b")
        # a few optimiser steps reduce the loss (fit quality itself is not pinned)
        opt = torch.optim.Adam([a, b], lr=1e-4)
        first = float(loss)
        for _ in range(15):
            opt.zero_grad()
            l = loss_fn(SpiirFn.apply(a, b, bk, xd))
            l.backward()
            opt.step()
            with torch.no_grad():
                r = torch.abs(a)
                a.mul_(torch.where(r > 1 - 1e-6, (1 - 1e-6) / r, torch.ones_like(r)))
        last = float(loss_fn(SpiirFn.apply(a, b, bk, xd)))
        print("fit loss %.4f -> %.4f" % (first, last))
        assert last < first


def test_stale_tape_is_rejected():
    banner("stale tape")
    from paper_1602_05573_amd import SpiirError
    bank = random_bank(62, 0, 2, 10, 20, 0.9, 0.99, 10)
    with mk(bank) as bk:
        x = torch.from_numpy(strain(100, 62)).cuda()
        z, tape = bk.forward_z(x, want_tape=True)
        bk.set_coeffs(bank.a * 0.5, bank.b)
        with pytest.raises(SpiirError, match="changed"):
            bk.backward(tape, torch.zeros_like(z))
        tape.close()


def test_set_coeffs_from_device():
    """spiir_bank_set_coeffs_dev: new coefficients from device arrays give the
    oracle's z for those coefficients, agree with the host call to rounding,
    and make older tapes stale; padding slots and the FP64-carry flags are
    formed as the host forms them (a filter with |a| > 1 - 1e-5 included)."""
    banner("set coeffs from the device")
    from paper_1602_05573_amd import SpiirError
    bank = random_bank(63, 0, 5, 30, 300, 0.99, 1 - 1e-6, 1000)
    rng = np.random.default_rng(6301)
    F = bank.n_filters
    r = rng.uniform(0.99, 1 - 2e-6, F)
    r[3] = 1 - 3e-6                                   # FP64-carry filter
    a2 = r * np.exp(1j * rng.uniform(0.01, 1.5, F))
    b2 = bank.b * np.exp(1j * rng.uniform(0, 6.28, F))
    bank2 = Bank(bank.offsets, a2, b2, bank.d, bank.dmax)
    x = strain(6000, 63)
    xd = torch.from_numpy(x).cuda()
    with mk(bank, chunk_len=128) as hb, mk(bank, chunk_len=128) as db:
        z0, tape = db.forward_z(xd, want_tape=True)
        hb.set_coeffs(a2, b2)
        db.set_coeffs_dev(torch.from_numpy(a2).cuda(), torch.from_numpy(b2).cuda())
        with pytest.raises(SpiirError, match="changed"):
            db.backward(tape, torch.zeros_like(z0))
        tape.close()
        zh = hb.forward_z(xd).cpu().numpy()
        zd = db.forward_z(xd).cpu().numpy()
    ref = oracle.z(bank2, x)
    peak = np.abs(ref).max(axis=1)
    err_d = float(np.max(np.abs(zd - ref).max(axis=1) / peak))
    err_hd = float(np.max(np.abs(zd - zh).max(axis=1) / peak))
    print("device-set z error %.3g of the peak, device vs host %.3g" % (err_d, err_hd), flush=True)
    assert err_d <= 1e-4 and err_hd <= 1e-6


def test_spiirfn_on_device():
    """SpiirFn with a, b on the GPU: the coefficients go in by the device call
    and the gradients come back on the device, equal to the oracle's; a few
    device-resident Adam steps lower the loss."""
    banner("SpiirFn on the device")
    from paper_1602_05573_amd import SpiirFn
    bank = random_bank(64, 0, 3, 40, 120, 0.95, 0.999, 300)
    x = strain(3000, 64)
    rng = np.random.default_rng(6401)
    g = (rng.standard_normal((3, 3000)) + 1j * rng.standard_normal((3, 3000)))
    gt = torch.from_numpy(g.astype(np.complex64)).cuda()
    xd = torch.from_numpy(x).cuda()

    def loss_fn(z):
        c = torch.sum(z * torch.conj(gt), dim=1)
        return torch.sum(1 - torch.abs(c) / (torch.linalg.norm(z, dim=1) * torch.linalg.norm(gt, dim=1)))

    with mk(bank) as bk:
        a = torch.tensor(bank.a, dtype=torch.complex128, device="cuda", requires_grad=True)
        b = torch.tensor(bank.b, dtype=torch.complex128, device="cuda", requires_grad=True)
        loss = loss_fn(SpiirFn.apply(a, b, bk, xd))
        loss.backward()
        assert a.grad.is_cuda and b.grad.is_cuda
        zr = oracle.z(bank, x)
        lref, Gref = oracle.overlap_loss(zr, g)
        ga_ref, gb_ref = oracle.backward(bank, x, Gref)
        assert abs(float(loss.detach()) - float(np.sum(lref))) < 1e-4
        grad_close(a.grad.cpu().numpy(), ga_ref, bank.offsets, what="device SpiirFn grad_a")
        grad_close(b.grad.cpu().numpy(), gb_ref, bank.offsets, what="device SpiirFn grad_b")
        opt = torch.optim.Adam([a, b], lr=1e-4)
        first = float(loss.detach())
        for _ in range(10):
            opt.zero_grad()
            l = loss_fn(SpiirFn.apply(a, b, bk, xd))
            l.backward()
            opt.step()
            with torch.no_grad():
                r = torch.abs(a)
                a.mul_(torch.where(r > 1 - 1e-6, (1 - 1e-6) / r, torch.ones_like(r)))
        last = float(loss_fn(SpiirFn.apply(a, b, bk, xd)).detach())
        print("device fit loss %.4f -> %.4f" % (first, last), flush=True)
        assert last < first


def test_chirp_fit_full_size_every_template():
    """256 templates x 400 filters, 65,536 samples (the bench.py adjoint
    workload): GPU forward + adjoint over the whole bank, compared with the
    oracle for every template: z, the overlap loss, and both gradients."""
    banner("chirp_fit full size")
    bank, x, gs, _ = chirp_fit()
    T = bank.n_templates
    with mk(bank) as bk:
        xd = torch.from_numpy(x).cuda()
        z, tape = bk.forward_z(xd, want_tape=True)
        gt = torch.from_numpy(gs.astype(np.complex64)).cuda()
        zc = z.to(torch.complex128)
        gtc = gt.to(torch.complex128)
        c = torch.sum(zc * torch.conj(gtc), dim=1)
        Z = torch.linalg.norm(zc, dim=1)
        Gn = torch.linalg.norm(gtc, dim=1)
        ac = torch.abs(c)
        G = -(1 / (Z * Gn))[:, None] * ((c / ac)[:, None] * gtc - (ac / Z ** 2)[:, None] * zc)
        ga, gb = bk.backward(tape, G.to(torch.complex64).contiguous())
        ga, gb = ga.cpu().numpy(), gb.cpu().numpy()
        zs = z.cpu().numpy()
        tape.close()
    zr = oracle.z(bank, x)
    zerr = np.abs(zs.astype(np.complex128) - zr).max(axis=1) / np.abs(zr).max(axis=1)
    print("chirp_fit: z error %.3g of the peak (worst template %d)" % (zerr.max(), int(np.argmax(zerr))))
    assert zerr.max() <= 1e-4
    lref, Gref = oracle.overlap_loss(zr, gs)
    lgpu, _ = oracle.overlap_loss(zs.astype(np.complex128), gs)
    assert np.abs(lgpu - lref).max() <= 1e-4
    ga_ref, gb_ref = oracle.backward(bank, x, Gref)
    # the GPU gradient used the upstream gradient at its own z (FP32); the
    # oracle's at the exact z
    grad_close(ga, ga_ref, bank.offsets, what="chirp_fit grad_a")
    grad_close(gb, gb_ref, bank.offsets, what="chirp_fit grad_b")
