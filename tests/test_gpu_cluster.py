"""Trigger clustering on the GPU (spiir_cluster_triggers) against the oracle's
plain window scan: sample indices, templates, SNR values and the total count
must be identical (integer and selection work, float32 comparisons on both
sides)."""
import numpy as np
import pytest

import oracle
from workloads import trigger_series

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")


def banner(msg):
    print("[case] " + msg, flush=True)


def gpu_clusters(M, J, thr, W, capacity=None, offset=0):
    """Runs the library on device copies; offset > 0 places the series at a
    4-byte but not 16-byte aligned address."""
    from paper_1602_05573_amd import cluster_triggers
    n = len(M)
    md = torch.zeros(n + offset, dtype=torch.float32, device="cuda")
    jd = torch.zeros(n + offset, dtype=torch.int32, device="cuda")
    md[offset:] = torch.from_numpy(M)
    jd[offset:] = torch.from_numpy(J)
    i, t, v, total = cluster_triggers(md[offset:], jd[offset:], thr, W, capacity=capacity)
    torch.cuda.synchronize()
    return i.cpu().numpy(), t.cpu().numpy(), v.cpu().numpy(), total


def oracle_ref(M, J, thr, W):
    i, t, v = oracle.clusters(M, J, thr, W)
    return i, t, v, len(i)


def assert_same(got, ref, what):
    gi, gt, gv, total = got
    ri, rt, rv, rtotal = ref
    assert total == rtotal, "%s: %d triggers, oracle %d" % (what, total, rtotal)
    k = len(gi)
    assert np.array_equal(gi, ri[:k]), what
    assert np.array_equal(gt, rt[:k]), what
    assert np.array_equal(gv.view(np.uint32), rv[:k].view(np.uint32)), what


@pytest.mark.parametrize("n", [4097, 70001])
@pytest.mark.parametrize("W", [0, 1, 63, 64, 65, 4095, 4096, 50000, 2**31 - 1])
@pytest.mark.parametrize("q", [0.5, 0.999])
def test_cluster_parity(n, W, q):
    M, J = trigger_series(n, idx=n % 5, peaks=16, plateau=6)
    thr = float(np.quantile(M, q))
    banner("cluster n=%d W=%d q=%g" % (n, W, q))
    ref = oracle_ref(M, J, thr, W)
    got = gpu_clusters(M, J, thr, W, offset=1 if W % 2 else 0)
    assert_same(got, ref, "n=%d W=%d q=%g" % (n, W, q))
    assert ref[3] > 0


@pytest.mark.parametrize("W", [64, 4096, 65536])
def test_cluster_parity_long_series(W):
    """2^22 + 5 samples: thousands of 4,096-blocks and a ragged tail."""
    n = (1 << 22) + 5
    M, J = trigger_series(n, idx=3, peaks=256, plateau=8)
    thr = float(np.quantile(M, 0.9995))
    banner("cluster long n=%d W=%d" % (n, W))
    ref = oracle_ref(M, J, thr, W)
    got = gpu_clusters(M, J, thr, W)
    assert_same(got, ref, "long W=%d" % W)
    assert ref[3] > 10


def test_cluster_edge_cases():
    M, J = trigger_series(9000, idx=1, peaks=8)
    banner("cluster edge cases")
    # empty series
    e = np.zeros(0, np.float32)
    assert gpu_clusters(e, np.zeros(0, np.int32), 1.0, 4)[3] == 0
    # one sample, below and at the threshold
    one = np.array([3.0], np.float32)
    assert gpu_clusters(one, np.array([7], np.int32), 4.0, 2)[3] == 0
    i, t, v, total = gpu_clusters(one, np.array([7], np.int32), 3.0, 2)
    assert total == 1 and i.tolist() == [0] and t.tolist() == [7] and v.tolist() == [3.0]
    # nothing above the threshold
    assert gpu_clusters(M, J, float(M.max()) + 1.0, 64)[3] == 0
    # the window covers the whole series: only the first global maximum
    ref = oracle_ref(M, J, 0.0, len(M))
    got = gpu_clusters(M, J, 0.0, len(M))
    assert_same(got, ref, "W >= n")
    assert got[3] == 1 and got[0][0] == int(np.argmax(M))
    # capacity below the count: total reported, the first ones written
    ref = oracle_ref(M, J, float(np.quantile(M, 0.5)), 3)
    for cap in (0, 1, ref[3] // 2, ref[3], ref[3] + 5):
        got = gpu_clusters(M, J, float(np.quantile(M, 0.5)), 3, capacity=cap)
        assert len(got[0]) == min(cap, ref[3])
        assert_same(got, ref, "capacity %d" % cap)
    # a plateau of equal values: its first sample, for every window
    P = np.zeros(300, np.float32)
    P[100:140] = 9.0
    for W in (0, 1, 39, 40, 1000):
        ref = oracle_ref(P, np.arange(300, dtype=np.int32), 1.0, W)
        assert_same(gpu_clusters(P, np.arange(300, dtype=np.int32), 1.0, W), ref, "plateau W=%d" % W)


def test_cluster_special_values():
    """NaN suppresses its window and never triggers; -0 equals +0; inf peaks;
    NaN and infinite thresholds."""
    base = np.array([0.0, -0.0, 1.0, np.nan, 5.0, 5.0, 2.0, np.inf, np.inf, -np.inf, 3.0, 0.0], np.float32)
    M = np.tile(base, 700)
    J = np.arange(len(M), dtype=np.int32)
    banner("cluster special values")
    for W in (0, 1, 2, 3, 70, 5000):
        for thr in (-np.inf, 0.0, -0.0, 2.0, np.nan, np.inf):
            ref = oracle_ref(M, J, thr, W)
            assert_same(gpu_clusters(M, J, thr, W), ref, "W=%d thr=%r" % (W, thr))


def test_cluster_workspace_reuse():
    """One workspace for calls of decreasing size and different windows: no
    state leaks from one call into the next."""
    from paper_1602_05573_amd import TriggerClusterer
    banner("cluster workspace reuse")
    c = TriggerClusterer(200000, 5000)
    for n, W, q in ((200000, 64, 0.99), (70001, 4096, 0.5), (5000, 0, 0.9), (0, 8, 0.5), (150000, 1, 0.999)):
        M, J = trigger_series(n, idx=n % 3, peaks=32)
        thr = float(np.quantile(M, q)) if n else 0.0
        md, jd = torch.from_numpy(M).cuda(), torch.from_numpy(J).cuda()
        c.run(md, jd, thr, W)
        i, t, v, total = c.result()
        ref = oracle_ref(M, J, thr, W)
        assert_same((i.cpu().numpy(), t.cpu().numpy(), v.cpu().numpy(), total), ref, "n=%d W=%d" % (n, W))


def test_cluster_rejects_bad_tensors():
    from paper_1602_05573_amd import SpiirError, TriggerClusterer
    c = TriggerClusterer(100, 10)
    m = torch.zeros(200, device="cuda")
    j = torch.zeros(200, dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError):
        c.run(m, j, 1.0, 4)                      # longer than max_n
    with pytest.raises(ValueError):
        c.run(m[:50], j[:40], 1.0, 4)            # lengths differ
    with pytest.raises(SpiirError):
        c.run(m[:50], j[:50], 1.0, -3)           # negative window


def test_cluster_graph_replay():
    """The clustering call captured in a HIP graph: each replay, with eager
    work (new series copied into the captured buffers) in between, equals the
    oracle on the series the buffers hold at that replay."""
    from paper_1602_05573_amd import TriggerClusterer
    banner("cluster graph replay")
    n, W = 300000, 512
    series = [trigger_series(n, idx=k, peaks=48) for k in range(4)]
    thr = 30.0
    md = torch.empty(n, dtype=torch.float32, device="cuda")
    jd = torch.empty(n, dtype=torch.int32, device="cuda")
    md.copy_(torch.from_numpy(series[0][0]))
    jd.copy_(torch.from_numpy(series[0][1]))
    c = TriggerClusterer(n, n // (W + 1) + 1)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        c.run(md, jd, thr, W)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c.run(md, jd, thr, W)
    for rep in range(6):
        M, J = series[rep % 4]
        md.copy_(torch.from_numpy(M))
        jd.copy_(torch.from_numpy(J))
        g.replay()
        i, t, v, total = c.result()
        ref = oracle_ref(M, J, thr, W)
        assert ref[3] > 3
        assert_same((i.cpu().numpy(), t.cpu().numpy(), v.cpu().numpy(), total), ref, "replay %d" % rep)
        # eager call on another series between replays
        M2, J2 = series[(rep + 1) % 4]
        e = TriggerClusterer(n, 100)
        e.run(torch.from_numpy(M2).cuda(), torch.from_numpy(J2).cuda(), thr, W)
        assert e.result()[3] == oracle_ref(M2, J2, thr, W)[3]
    del g


def test_cluster_parity_scan_path():
    """A series of more than 8,192 4,096-blocks (2^25 + 12,365 samples): block
    offsets come from the separate one-workgroup scan instead of the write
    launch."""
    n = (1 << 25) + 3 * 4096 + 77
    M, J = trigger_series(n, idx=4, peaks=512, plateau=8)
    thr = float(np.quantile(M, 0.99995))
    banner("cluster scan path n=%d" % n)
    for W in (4096, 100000):
        ref = oracle_ref(M, J, thr, W)
        got = gpu_clusters(M, J, thr, W)
        assert_same(got, ref, "scan path W=%d" % W)
        assert ref[3] > 20


def test_cluster_piecewise_with_overlap():
    """The rule reaches W samples either side, so calls on [s, e) overlapping by
    2W give the whole series' triggers for every m with s + W <= m < e - W:
    stitching those ranges reproduces the whole-series result."""
    from paper_1602_05573_amd import cluster_triggers
    n, W, piece = 300000, 777, 40000
    M, J = trigger_series(n, idx=2, peaks=64, plateau=6)
    thr = float(np.quantile(M, 0.99))
    banner("cluster piecewise")
    whole = gpu_clusters(M, J, thr, W)
    md, jd = torch.from_numpy(M).cuda(), torch.from_numpy(J).cuda()
    got = []
    start = 0
    while start < n:
        s = max(0, start - W)
        e = min(n, start + piece + W)
        i, t, v, total = cluster_triggers(md[s:e], jd[s:e], thr, W)
        i = i.cpu().numpy() + s
        keep = (i >= start) & (i < min(n, start + piece))
        got.append(i[keep])
        start += piece
    stitched = np.concatenate(got)
    assert np.array_equal(stitched, whole[0])
    assert len(stitched) > 20


@pytest.mark.parametrize("W,block,q", [(0, 4096, 0.99), (1, 1000, 0.5), (777, 5000, 0.99), (5000, 2048, 0.999),
                                       (20000, 8192, 0.99)])
def test_trigger_stream_equals_whole_series(W, block, q):
    """Pushes of irregular lengths (at most max_block) and a flush give exactly
    the whole series' triggers; reset starts over."""
    from paper_1602_05573_amd import TriggerStream
    n = 120007
    M, J = trigger_series(n, idx=W % 4, peaks=48, plateau=6)
    thr = float(np.quantile(M, q))
    banner("trigger stream W=%d block=%d q=%g" % (W, block, q))
    ref = oracle_ref(M, J, thr, W)
    md, jd = torch.from_numpy(M).cuda(), torch.from_numpy(J).cuda()
    rng = np.random.default_rng(W)
    ts = TriggerStream(thr, W, block, capacity=n // (W + 1) + 2)
    for rep in range(2):
        got_i, got_t, got_v = [], [], []
        pos = 0
        while pos < n:
            k = int(min(n - pos, rng.integers(0, block + 1)))
            i, t, v, total = ts.push(md[pos:pos + k], jd[pos:pos + k])
            assert total == len(i)
            got_i.append(i.cpu().numpy()); got_t.append(t.cpu().numpy()); got_v.append(v.cpu().numpy())
            pos += k
        i, t, v, total = ts.flush()
        got_i.append(i.cpu().numpy()); got_t.append(t.cpu().numpy()); got_v.append(v.cpu().numpy())
        got = (np.concatenate(got_i), np.concatenate(got_t), np.concatenate(got_v))
        assert_same(got + (len(got[0]),), ref, "stream W=%d rep %d" % (W, rep))
        ts.reset()
    ts.close()
