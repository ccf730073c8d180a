"""Throughput of the SPIIR hot path on one MI355X.

Workload (default): 1,024 templates with K_j ~ U{100..800} first-order complex
IIR filters (r ~ U[0.99, 1-1e-5], d ~ U{0..16384}) over a 4,194,304-sample
float32 white-noise stream processed in 4,096-sample blocks. One step = a
cold start plus the whole stream through spiir_trigger_max, one call per
block (filter recursion, template sums, SNR, fused max/argmax). Inputs are
resident in HBM before timing.

Prints ONE JSON line with the throughput (complex filter-updates/s), the
roofline of the forward kernel (FP32 vector ALU), the plain one-launch-per-
template comparator on a sample of blocks, a parity check of the timed run
against the FP64 oracle on a prefix, and the oracle's own rate on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "complex IIR filter-updates/s + % FP32 vector peak; fused vs plain at 1e-4 err"
PEAK_FP32 = 157.3e12          # MI355X FP32 vector peak (packed FP32 issue), FLOP/s
PEAK_HBM = 8.0e12             # MI355X HBM3E bandwidth, bytes/s
# FP32 issue ceiling of the recursion loop without packed FP32 instructions:
# 256 CU x 2.4 GHz x 64 lanes x 12 FLOP per 8 VALU issues = 59.0 TFLOP/s
ISSUE_CEILING = 256 * 2.4e9 * 64 * 12 / 8
FLOP_UPDATE = 12              # a*y 6 + b*x 2 + add 2 + template accumulation 2
FLOP_SAMPLE = 4               # |z|^2 3 + compare 1, per template and sample
FLOP_ADJ = 30                 # adjoint per update, the scope table's figure: y 10, lambda 8, grad_b 4, grad_a 8
FLOP_ADJ_PAIR = 24            # as computed here (no y): lambda 8, nu 8, lambda x 4, nu x 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_traffic():
    """HBM bytes per forward launch and where the figure comes from: the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a device copy
    of known size) of this kernel source, not a measurement of this run; None
    when the kernel source changed since those counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            t = json.load(f)
        src = open(os.path.join(ROOT, "paper_1602_05573_amd", "csrc", "kernels.hip"), "rb").read()
        sha = hashlib.sha256(src).hexdigest()[:16]
        if sha != t["kernel_sha256_prefix"]:
            return None, ("null: kernels.hip (sha256 %s) changed since the committed counters (%s)"
                          % (sha, t["kernel_sha256_prefix"]))
        return (int(t["fetch_bytes"] + t["write_bytes"]),
                "committed rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel source (sha256 %s), %s"
                % (sha, t.get("source", "profiles/traffic.json")))
    except (OSError, KeyError, ValueError):
        return None, "null: no committed traffic counters"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--templates", type=int, default=1024)
    ap.add_argument("--samples", type=int, default=4194304)
    ap.add_argument("--block", type=int, default=4096)
    ap.add_argument("--chunk-len", type=int, default=256)
    ap.add_argument("--fl", type=int, default=0, help="filters per lane (0 = library choice)")
    ap.add_argument("--wpg", type=int, default=0)
    ap.add_argument("--time-split", type=int, default=0, help="time segments (0 = library choice, 1 = off)")
    ap.add_argument("--delay-band", type=int, default=0,
                    help="adjoint: delay band width (0 = none: the strain window stays in global memory)")
    ap.add_argument("--fit-steps", type=int, default=5, help="adjoint: optimiser steps of the chirp fit")
    ap.add_argument("--fit-lr", type=float, default=1e-4, help="adjoint: Adam learning rate of the fit")
    ap.add_argument("--plain-blocks", type=int, default=16)
    ap.add_argument("--check-blocks", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-cluster", action="store_true", help="bank: skip the trigger clustering leg")
    ap.add_argument("--cluster-window", type=int, default=4096,
                    help="bank: clustering window W in samples (4096 = 1 s at 4096 Hz)")
    ap.add_argument("--cluster-quantile", type=float, default=0.9999,
                    help="bank: clustering threshold as a quantile of the step's max series")
    ap.add_argument("--workload", choices=("bank", "batch", "adjoint", "precision", "multirate", "whiten",
                                           "pipeline"),
                    default="bank",
                    help="bank: the 1,024-template bank (default, the headline); "
                         "batch: 8 uneven streams with their own banks in one graph replay per block")
    ap.add_argument("--length-scale", type=float, default=1.0, help="batch: scale of the stream lengths")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 256 MiB device copy (reference for HBM traffic counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(templates would shard across GPUs with one max-key all-reduce per block)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read, 268435456 bytes written")
        del src, dst
    if args.workload == "batch":
        return run_batch(args, torch)
    if args.workload == "precision":
        return run_precision(args, torch)
    if args.workload == "adjoint":
        return run_adjoint(args, torch)
    if args.workload == "multirate":
        return run_multirate(args, torch)
    if args.workload == "whiten":
        return run_whiten(args, torch)
    if args.workload == "pipeline":
        return run_pipeline(args, torch)
    return run_bank(args, torch)


def argmax_outside_ties(oracle, bank, x, g_j, j_ref, nth, eps=1e-4):
    """Samples where the GPU argmax differs from the oracle's, and how many of
    them lie outside the admissible set ref_j >= ref_J - eps (P_j + P_J)
    (P = a template's peak over the sample): differences inside it are
    documented ties."""
    diff = np.nonzero(g_j != j_ref)[0]
    bad = 0
    if diff.size:
        pair = sorted(set(g_j[diff].tolist()) | set(j_ref[diff].tolist()))
        ref_pair = oracle.snr(bank.subset(pair), x, nthreads=nth)
        row = {j: k for k, j in enumerate(pair)}
        P = ref_pair.max(axis=1)
        for n_ in diff:
            a, b = row[int(g_j[n_])], row[int(j_ref[n_])]
            if ref_pair[a, n_] < ref_pair[b, n_] - eps * (P[a] + P[b]):
                bad += 1
    return int(diff.size), bad


def bench_plain(args, torch, bank, x, blocks, mx_fused, fused_value, info, m_ref, j_ref):
    """The one-launch-per-template comparator: every template's launches write
    its SNR row to HBM and a separate pass takes the max/argmax. Each
    template's launches fill the device (one workgroup per chunk-length
    segment of the block, chained in FP64); the chunk length sets the segment
    count, so the comparator is timed at chunk lengths 16, 64 and 256 (256, 64
    and 16 workgroups per template and block) and reported at its fastest,
    with its own error against the oracle on the timed blocks."""
    import oracle
    from paper_1602_05573_amd import SpiirBank
    T, F = bank.n_templates, bank.n_filters
    B = args.block
    nb = min(args.plain_blocks, len(blocks))
    n = nb * B
    pm = torch.empty(n, dtype=torch.float32, device="cuda")
    pa = torch.empty(n, dtype=torch.int32, device="cuda")
    scratch = torch.empty((T, B), dtype=torch.float32, device="cuda")
    sweep = {}
    best = None
    for L in (16, 64, 256):
        with SpiirBank.from_bank(bank, chunk_len=L, filters_per_lane=info["filters_per_lane"],
                                 waves_per_group=info["waves_per_group"], time_split=1,
                                 max_block=max(B, 4096)) as pb:
            pb.trigger_max_per_template(blocks[0], out=(pm[:B], pa[:B]), snr_scratch=scratch)  # warm-up
            pb.reset()
            torch.cuda.synchronize()
            tp = time.perf_counter()
            for i in range(nb):
                pb.trigger_max_per_template(blocks[i], out=(pm[i * B:(i + 1) * B], pa[i * B:(i + 1) * B]),
                                            snr_scratch=scratch)
            torch.cuda.synchronize()
            t = time.perf_counter() - tp
        rate = float(F) * n / t
        sweep[L] = {"value": rate, "ms_per_block": 1e3 * t / nb}
        log("plain chunk_len %d: %.3e updates/s, %.2f ms per block" % (L, rate, 1e3 * t / nb))
        if best is None or rate > best[1]:
            best = (L, rate, pm.clone(), pa.clone())
    L, rate, pm, pa = best
    g_m = pm.cpu().numpy().astype(np.float64)
    g_j = pa.cpu().numpy()
    f_m = mx_fused[:n].cpu().numpy().astype(np.float64)
    out = {"value": rate, "unit": "filter-updates/s",
           "pct_fp32_peak": 100.0 * FLOP_UPDATE * rate / PEAK_FP32,
           "chunk_len": L, "workgroups_per_template_launch": B // L,
           "launches_per_block": T * (3 if B // L >= 2 else 1) + 1,
           "sweep": sweep,
           "sample": "first %d blocks (%d samples), one template per launch group plus a max/argmax pass"
                     % (nb, n),
           "fused_speedup": fused_value / rate}
    if m_ref is not None and len(m_ref) >= n:
        peak = float(m_ref[:n].max())
        nth = oracle.max_threads()
        diff_n, bad = argmax_outside_ties(oracle, bank, x[:n], g_j, j_ref[:n], nth)
        rel = float(np.max(np.abs(g_m - m_ref[:n])) / peak)
        out["check"] = {"samples": n, "max_abs_err_over_peak": rel, "argmax_ties": diff_n,
                        "argmax_outside_ties": bad, "gate": 1e-4, "pass": rel <= 1e-4 and bad == 0,
                        "fused_max_abs_err_over_peak": float(np.max(np.abs(f_m - m_ref[:n])) / peak)}
    out["max_abs_diff_vs_fused_over_peak"] = float(np.max(np.abs(g_m - f_m)) / max(float(f_m.max()), 1e-30))
    log("plain: %.3e updates/s at chunk_len %d (fused %.1fx); check %s"
        % (rate, L, fused_value / rate, out.get("check")))
    return out


def run_bank(args, torch):
    from paper_1602_05573_amd import SpiirBank
    from workloads import bank_1024

    t0 = time.time()
    bank, x = bank_1024(n=args.samples, n_templates=args.templates)
    F = bank.n_filters
    T = bank.n_templates
    N = len(x)
    B = args.block
    nblk = (N + B - 1) // B
    log("workload: T=%d F=%d N=%d blocks=%d (gen %.1fs)" % (T, F, N, nblk, time.time() - t0))

    bk = SpiirBank.from_bank(bank, chunk_len=args.chunk_len, filters_per_lane=args.fl, time_split=args.time_split,
                             waves_per_group=args.wpg, max_block=max(B, 4096))
    info = bk.info
    log("bank:", info)
    xd = torch.from_numpy(x).cuda()
    blocks = [xd[i * B:min(N, (i + 1) * B)] for i in range(nblk)]
    mx = torch.empty(N, dtype=torch.float32, device="cuda")
    am = torch.empty(N, dtype=torch.int32, device="cuda")
    outs = [(mx[i * B:min(N, (i + 1) * B)], am[i * B:min(N, (i + 1) * B)]) for i in range(nblk)]
    stream = torch.cuda.current_stream()

    def step(events=None):
        bk.reset()
        for i in range(nblk):
            if events is not None:
                events[i][0].record(stream)
            bk.trigger_max(blocks[i], out=outs[i])
            if events is not None:
                events[i][1].record(stream)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nblk)] for _ in range(args.steps)]
    bk.time_kernels(True)   # start/stop timestamps of the forward kernel dispatches themselves
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    k_ms, k_launches = bk.kernel_time()
    bk.time_kernels(False)
    ms_step = 1e3 * t_total / args.steps
    updates = float(F) * N
    value = updates / (t_total / args.steps)
    # per-block call duration (forward kernel + its two small epilogue kernels)
    full = [i for i in range(nblk) if (i + 1) * B <= N]
    blk_ms = np.array([ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps) for i in full])
    blk_s = float(np.mean(blk_ms)) * 1e-3
    # forward kernel alone: every block is one launch of B samples when B divides N
    kern_s = k_ms * 1e-3 / k_launches if (k_launches and N % B == 0) else blk_s
    flops_launch = FLOP_UPDATE * float(F) * B + FLOP_SAMPLE * float(T) * B
    achieved = flops_launch / kern_s
    traffic, traffic_source = measured_traffic()
    log("step %.1f ms, %.3e updates/s, forward kernel %.1f us (%d launches), block call %.1f us "
        "(p50 %.1f, p99 %.1f)" % (ms_step, value, kern_s * 1e6, k_launches, blk_s * 1e6,
                                 np.percentile(blk_ms, 50) * 1e3, np.percentile(blk_ms, 99) * 1e3))

    result = {
        "metric": METRIC, "value": value, "unit": "filter-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded white noise and random banks; the paper's pipeline data are not public)",
        "config": {"workload": "template bank: %d templates x U{100..800} filters (F=%d), %d samples "
                               "at 4096 Hz in %d-sample blocks, fused max/argmax" % (T, F, N, B),
                   "global_batch": T, "seq_len": N, "parallelism": "single GPU",
                   "chunk_len": info["chunk_len"], "filters_per_lane": info["filters_per_lane"],
                   "waves_per_group": info["waves_per_group"], "workgroups": info["n_groups"]},
        "pct_fp32_peak": 100.0 * FLOP_UPDATE * value / PEAK_FP32,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": traffic,
                     "traffic_source": traffic_source,
                     "issue_ceiling": ISSUE_CEILING / 1e12, "frac_of_issue_ceiling": achieved / ISSUE_CEILING,
                     "kernel": "fwd_kernel<FL=%d, keys, LDS window>" % info["filters_per_lane"],
                     "launch_us": kern_s * 1e6, "launches_timed": k_launches,
                     "block_call_us": blk_s * 1e6, "flop_per_launch": flops_launch},
    }

    if not args.no_cluster:
        result["triggers"] = bench_clustering(args, torch, mx, am, stream)

    # parity of the timed configuration on a prefix (oracle over all templates)
    oracle_rate = None
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        nchk = min(N, args.check_blocks * B)
        nth = oracle.max_threads()
        t1 = time.perf_counter()
        m_ref, j_ref = oracle.trigger(bank, x[:nchk], nthreads=nth)
        t_or = time.perf_counter() - t1
        oracle_rate = float(F) * nchk / t_or
        g_m = mx[:nchk].cpu().numpy().astype(np.float64)
        g_j = am[:nchk].cpu().numpy()
        peak = float(m_ref.max())
        rel = float(np.max(np.abs(g_m - m_ref)) / peak)
        agree = float(np.mean(g_j == j_ref))
        diff_n, bad = argmax_outside_ties(oracle, bank, x[:nchk], g_j, j_ref, nth)
        result["check"] = {"samples": nchk, "max_abs_err_over_peak": rel, "argmax_agree": agree,
                           "argmax_ties": diff_n, "argmax_outside_ties": bad,
                           "gate": 1e-4, "pass": rel <= 1e-4 and bad == 0}
        log("check: max|dM|/peak %.3g argmax agree %.6f (%d documented ties, %d outside) (oracle %.1fs)"
            % (rel, agree, diff_n, bad, t_or))
        if not args.no_cpu_baseline:
            from workloads import bank_4x128
            small, xs_small = bank_4x128()
            t2 = time.perf_counter()
            oracle.trigger(small, xs_small, nthreads=1)
            rate1 = float(small.n_filters) * len(xs_small) / (time.perf_counter() - t2)
            result["cpu_baseline"] = {
                "value": oracle_rate, "unit": "filter-updates/s", "cores": nth, "kind": "oracle",
                "sample": "FP64 oracle trigger over the first %d samples of the same bank "
                          "(all %d templates, %.2e updates), %.1f s" % (nchk, T, float(F) * nchk, t_or),
                "one_thread_4x128_bank": rate1, "cpu_model": cpu_model(), "nproc": os.cpu_count()}

    if not args.no_plain and args.plain_blocks > 0:
        result["plain"] = bench_plain(args, torch, bank, x, blocks, mx, value, info,
                                      m_ref if oracle_rate is not None else None,
                                      j_ref if oracle_rate is not None else None)

    bk.close()
    print(json.dumps(result), flush=True)


def bench_clustering(args, torch, mx, am, stream, reps=50):
    """Trigger clustering of one step's fused max/argmax series (threshold = a
    high quantile of the series, window W), timed over back-to-back calls on
    the stream and over replays of the call captured in a graph; the oracle's
    scan of the same series is the CPU baseline and the check (identical
    triggers)."""
    from paper_1602_05573_amd import TriggerClusterer
    n = mx.numel()
    W = args.cluster_window
    m_host, a_host = mx.cpu().numpy(), am.cpu().numpy()
    thr = float(np.quantile(m_host, args.cluster_quantile))
    cl = TriggerClusterer(n, n // (W + 1) + 1)
    for _ in range(3):
        cl.run(mx, am, thr, W)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        cl.run(mx, am, thr, W)
    e1.record(stream)
    torch.cuda.synchronize()
    t_call = e0.elapsed_time(e1) * 1e-3 / reps
    # the same call captured in a HIP graph: replays are not bound by host submission
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        cl.run(mx, am, thr, W)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cl.run(mx, am, thr, W)
    graph.replay()
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        graph.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    t_graph = e0.elapsed_time(e1) * 1e-3 / reps
    del graph
    gi, gt, gv, total = cl.result()
    # algorithmic bytes: the max series read once, then argmax read and
    # (index, template, snr) written per trigger
    alg = 4.0 * n + 20.0 * total
    out = {"samples": n, "window": W, "threshold": thr, "threshold_quantile": args.cluster_quantile,
           "count": total, "us_per_call": t_call * 1e6, "us_per_graph_replay": t_graph * 1e6,
           "samples_per_s": n / t_call, "launches_per_call": 3,
           "roofline": {"bound": "hbm", "achieved": alg / t_call / 1e9, "peak": PEAK_HBM / 1e9,
                        "unit": "GB/s", "frac": alg / t_call / PEAK_HBM, "algorithmic_bytes": alg,
                        "note": "whole call (3 launches back to back); launch latency dominates at this size"}}
    log("clustering: %d triggers (W=%d, threshold %.4g), %.1f us per call, %.1f us per graph replay"
        % (total, W, thr, t_call * 1e6, t_graph * 1e6))
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        ri, rt, rv = oracle.clusters(m_host, a_host, thr, W)
        rtotal = len(ri)
        t_or = time.perf_counter() - t0
        same = (total == rtotal and np.array_equal(gi.cpu().numpy(), ri)
                and np.array_equal(gt.cpu().numpy(), rt) and np.array_equal(gv.cpu().numpy(), rv))
        out["cpu_baseline"] = {"value": n / t_or, "unit": "samples/s", "cores": 1, "kind": "oracle",
                               "sample": "oracle window scan of the same %d-sample series, %.3f s" % (n, t_or)}
        out["check"] = {"identical_to_oracle": bool(same), "oracle_count": int(rtotal)}
        log("clustering check: identical to the oracle: %s (oracle %.3f s)" % (same, t_or))
    return out


def run_batch(args, torch):
    """8 streams of round(2^U[18,22]) samples, each with its own 256-template
    bank of U{200..600} filters, advanced one 4,096-sample block per graph
    replay; chunk length and filters per lane from the autotuner."""
    from paper_1602_05573_amd import SpiirBatch, autotune, batch_banks
    from workloads import batch_streams

    t0 = time.time()
    banks, xs = batch_streams(length_scale=args.length_scale)
    lengths = [len(x) for x in xs]
    updates = float(sum(b.n_filters * len(x) for b, x in zip(banks, xs)))
    log("batch workload: %d streams, lengths %s, %.3e updates (gen %.1fs)"
        % (len(xs), lengths, updates, time.time() - t0))
    t1 = time.time()
    L, F, table = autotune(banks, block_len=args.block)
    log("autotune (%.1fs): chunk_len %d, filters/lane %d; ns per step:\n%s" % (time.time() - t1, L, F, table))
    bks = batch_banks(banks, L, F)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    bt = SpiirBatch(bks, xd, block_len=args.block)
    nsteps = bt.steps_total()
    stream = torch.cuda.current_stream()

    def one_pass(events=None):
        bt.reset()
        for i in range(nsteps):
            if events is not None:
                events[i][0].record(stream)
            bt.step()
            if events is not None:
                events[i][1].record(stream)

    for w in range(args.warmup):
        one_pass()
        torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(nsteps)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for k in range(args.steps):
        one_pass(ev[k])
    torch.cuda.synchronize()
    t_total = time.perf_counter() - ts
    lat = np.array([ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps) for i in range(nsteps)])
    value = updates * args.steps / t_total
    info = bks[0].info
    # algorithmic FLOP of the replays while all 8 streams are live
    live = min(lengths) // args.block
    flops_full = sum(FLOP_UPDATE * b.n_filters * args.block + FLOP_SAMPLE * b.n_templates * args.block
                     for b in banks)
    lat_full = np.array([ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps) for i in range(live)])
    achieved = flops_full / (float(np.mean(lat_full)) * 1e-3)
    res = {
        "metric": METRIC, "value": value, "unit": "filter-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded white noise and random banks)",
        "config": {"workload": "batched streams: 8 streams (%s samples), 256 templates x U{200..600} "
                               "filters each, %d-sample blocks, one persistent launch per block in a "
                               "HIP graph" % (",".join(map(str, lengths)), args.block),
                   "chunk_len": L, "filters_per_lane": F, "waves_per_group": info["waves_per_group"],
                   "graph_replays_per_step": nsteps},
        "pct_fp32_peak": 100.0 * FLOP_UPDATE * value / PEAK_FP32,
        "block_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "p50_all_streams_live": float(np.percentile(lat_full, 50)),
                             "p99_all_streams_live": float(np.percentile(lat_full, 99)),
                             "replays": int(len(lat))},
        "autotune_ns_per_step": {"chunk_len": [64, 128, 256, 512], "filters_per_lane": [1, 2, 3, 4],
                                 "table": table.tolist()},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": None,
                     "kernel": "batch_kernel (all streams live)"},
    }
    log("batch: %.3e updates/s, p50 %.3f ms p99 %.3f ms per block-step" % (value, res["block_latency_ms"]["p50"],
                                                                           res["block_latency_ms"]["p99"]))
    bt.close()
    for b in bks:
        b.close()
    print(json.dumps(res), flush=True)


def run_adjoint(args, torch):
    """256 templates x 400 filters fitted to time-reversed chirps over 65,536
    samples: forward_z with its tape (the strain window), the overlap loss and
    its gradient (torch, on the device), and the reverse-time adjoint
    (spiir_backward)."""
    from paper_1602_05573_amd import SpiirBank
    from workloads import chirp_fit

    bank, x, gs, _ = chirp_fit()
    F, T, N = bank.n_filters, bank.n_templates, len(x)
    bk = SpiirBank.from_bank(bank, filters_per_lane=args.fl, waves_per_group=args.wpg,
                             time_split=args.time_split, delay_band=args.delay_band)
    info = bk.info
    log("bank:", info)
    xd = torch.from_numpy(x).cuda()
    gt = torch.from_numpy(gs.astype(np.complex64)).cuda()
    stream = torch.cuda.current_stream()

    def upstream(z):
        c = torch.sum(z * torch.conj(gt), dim=1)
        Z = torch.linalg.norm(z, dim=1)
        Gn = torch.linalg.norm(gt, dim=1)
        ac = torch.abs(c)
        return (-(1 / (Z * Gn))[:, None] * ((c / ac)[:, None] * gt - (ac / Z ** 2)[:, None] * z)).contiguous()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        z, tape = bk.forward_z(xd, want_tape=True)
        if ev is not None:
            ev[1].record(stream)
        G = upstream(z)
        if ev is not None:
            ev[2].record(stream)
        ga, gb = bk.backward(tape, G)
        if ev is not None:
            ev[3].record(stream)
        torch.cuda.synchronize()
        tape.close()
        return ga

    for _ in range(args.warmup):
        step()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    ts = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    t_total = time.perf_counter() - ts
    fwd = np.mean([e[0].elapsed_time(e[1]) for e in evs])
    loss = np.mean([e[1].elapsed_time(e[2]) for e in evs])
    bwd = np.mean([e[2].elapsed_time(e[3]) for e in evs])
    updates = float(F) * N
    res = {
        "metric": METRIC, "value": updates / ((fwd + bwd) * 1e-3), "unit": "filter-updates/s (forward + adjoint)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * t_total / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (leading-order chirps, chirp masses U[1,30])",
        "config": {"workload": "adjoint fit: %d templates x 400 filters, %d samples, unit impulse input" % (T, N),
                   "chunk_len": info["chunk_len"], "filters_per_lane": info["filters_per_lane"],
                   "waves_per_group": info["waves_per_group"], "workgroups": info["n_groups"],
                   "time_split": info["time_split"], "delay_band": info["delay_band"],
                   "template_parts": info["n_parts"]},
        "forward_ms": fwd, "loss_ms": loss, "backward_ms": bwd,
        "forward_updates_per_s": updates / (fwd * 1e-3), "backward_updates_per_s": updates / (bwd * 1e-3),
        # backward call = (lambda, nu) scan + FP64 chain + per-segment backward + reduction
        # kernels, timed with events on the stream they run on; algorithmic work counted at the
        # scope table's 30 FLOP per update (frac_executed: the 24 FLOP this formulation computes)
        "roofline": {"bound": "alu", "achieved": FLOP_ADJ * updates / (bwd * 1e-3) / 1e12,
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": FLOP_ADJ * updates / (bwd * 1e-3) / PEAK_FP32, "traffic": None,
                     "frac_executed": FLOP_ADJ_PAIR * updates / (bwd * 1e-3) / PEAK_FP32,
                     "kernel": "spiir_backward (bwd_scan, bwd_chain, bwd_seg, bwd_reduce)",
                     "launch_us": bwd * 1e3, "flop_per_launch": FLOP_ADJ * updates},
        "roofline_forward": {"bound": "alu", "achieved": FLOP_UPDATE * updates / (fwd * 1e-3) / 1e12,
                             "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                             "frac": FLOP_UPDATE * updates / (fwd * 1e-3) / PEAK_FP32,
                             "kernel": "spiir_forward_z with tape", "launch_us": fwd * 1e3},
        "step_ms": fwd + loss + bwd,
    }
    log("adjoint: forward %.2f ms, loss %.2f ms, backward %.2f ms" % (fwd, loss, bwd))

    # a short fit through the autograd Function: loss before and after (fit quality is not a gate)
    from paper_1602_05573_amd import SpiirFn
    # coefficients, gradients and the optimiser state stay on the device
    a = torch.tensor(bank.a, dtype=torch.complex128, device="cuda", requires_grad=True)
    b = torch.tensor(bank.b, dtype=torch.complex128, device="cuda", requires_grad=True)
    Gn = torch.linalg.norm(gt, dim=1)

    def overlap_loss(z):
        c = torch.sum(z * torch.conj(gt), dim=1)
        return torch.mean(1 - torch.abs(c) / (torch.linalg.norm(z, dim=1) * Gn))

    opt = torch.optim.Adam([a, b], lr=args.fit_lr)
    losses = []
    tf = 0.0
    for it in range(args.fit_steps + 1):
        if it == 1:     # the first step carries the optimiser's and torch's first-use costs
            torch.cuda.synchronize()
            tf = time.perf_counter()
        opt.zero_grad()
        lval = overlap_loss(SpiirFn.apply(a, b, bk, xd))
        losses.append(lval.detach())   # read after the loop: no host sync inside a step
        if len(losses) > args.fit_steps:
            break
        lval.backward()
        opt.step()
        with torch.no_grad():   # keep every pole inside the unit circle
            r = torch.abs(a)
            a.mul_(torch.where(r > 1 - 1e-6, (1 - 1e-6) / r, torch.ones_like(r)))
    torch.cuda.synchronize()
    tf = time.perf_counter() - tf
    losses = [float(v) for v in losses]
    res["fit"] = {"steps": args.fit_steps, "optimizer": "Adam lr %g" % args.fit_lr,
                  "mean_loss_before": losses[0], "mean_loss_after": losses[-1],
                  "s_per_step": tf / max(1, args.fit_steps - 1) if args.fit_steps > 1 else None,
                  "timed_steps": max(0, args.fit_steps - 1),
                  "note": "coefficients, gradients and optimiser state on the device (spiir_bank_set_coeffs_dev)"}
    log("fit: mean overlap loss %.4f -> %.4f over %d steps (%.4f s per step after the first, coefficients set "
        "from the device)" % (losses[0], losses[-1], args.fit_steps, tf / max(1, args.fit_steps - 1)))
    bk.close()
    print(json.dumps(res), flush=True)


def run_multirate(args, torch):
    """Chirp-like bank on 5 rate levels (1,024 templates x U{100..800}
    filters placed at 4096/2^r Hz by frequency), 4,194,304 samples in
    4,096-sample blocks. value = full-rate-equivalent filter-updates/s (every
    filter counted at the input rate, the work a single-rate bank would do);
    the same filters run as one single-rate bank are timed beside it."""
    from paper_1602_05573_amd import SpiirBank, SpiirMultiRate
    from workloads import Bank, multirate_bank, resample_taps, strain

    t0 = time.time()
    levels = multirate_bank(n_templates=args.templates)
    h, g = resample_taps(24)
    N, B = args.samples, args.block
    x = strain(N, 6)
    F = [lv.n_filters for lv in levels]
    T = levels[0].n_templates
    nblk = N // B
    upd_eff = float(sum(F)) * N
    upd_act = float(sum(f * (N >> r) for r, f in enumerate(F)))
    log("multirate workload: T=%d filters per level %s (gen %.1fs)" % (T, F, time.time() - t0))
    mr = SpiirMultiRate(levels, h, g, max_block=B)
    infos = {r: mr.level_info(r) for r in range(len(levels))}
    xd = torch.from_numpy(x).cuda()
    mx = torch.empty(N, dtype=torch.float32, device="cuda")
    am = torch.empty(N, dtype=torch.int32, device="cuda")
    blocks = [(xd[i * B:(i + 1) * B], (mx[i * B:(i + 1) * B], am[i * B:(i + 1) * B])) for i in range(nblk)]

    def step():
        mr.reset()
        for xb, out in blocks:
            mr.trigger_max(xb, out=out)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    t_step = t_total / args.steps
    # the same step without graphs (every piece enqueued call by call)
    mr.set_graph(False)
    torch.cuda.synchronize()
    t0e = time.perf_counter()
    step()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0e
    # one more step with the level banks' forward kernels timed (eager path)
    mr.time_kernels(True)
    step()
    torch.cuda.synchronize()
    kt = mr.kernel_time()
    mr.time_kernels(False)
    mr.set_graph(True)
    value = upd_eff / t_step
    per_level = {}
    for r, (ms, nl) in kt.items():
        n_r = B >> r
        fl = FLOP_UPDATE * float(F[r]) * n_r + FLOP_SAMPLE * float(infos[r]["n_templates"]) * n_r
        us = ms * 1e3 / max(1, nl)
        per_level[r] = {"filters": F[r], "templates": infos[r]["n_templates"], "samples_per_launch": n_r,
                        "forward_us": us, "launches": nl, "tflops": fl / (us * 1e-6) / 1e12 if us > 0 else None}
    dom = max(per_level, key=lambda r: per_level[r]["forward_us"])
    d = per_level[dom]
    fl_dom = FLOP_UPDATE * float(F[dom]) * (B >> dom) + FLOP_SAMPLE * float(d["templates"]) * (B >> dom)
    achieved = fl_dom / (d["forward_us"] * 1e-6)
    fwd_sum_us = sum(v["forward_us"] for v in per_level.values())
    log("multirate: %.1f ms per step, %.3e effective / %.3e actual updates/s; per block %.1f us (graph replay; "
        "%.1f us enqueued call by call), forward kernels %.1f us (dominant level %d: %.1f us)"
        % (t_step * 1e3, value, upd_act / t_step, t_step / nblk * 1e6, t_eager / nblk * 1e6, fwd_sum_us, dom,
           d["forward_us"]))

    # the same filters as one single-rate bank (every filter at the input rate), timed on a prefix
    off = np.zeros(T + 1, np.int64)
    for lv in levels:
        off[1:] += np.diff(lv.offsets)
    off = np.cumsum(np.concatenate([[0], off[1:]]))
    aa = np.concatenate([lv.a[lv.offsets[j]:lv.offsets[j + 1]] for j in range(T) for lv in levels])
    bb = np.concatenate([lv.b[lv.offsets[j]:lv.offsets[j + 1]] for j in range(T) for lv in levels])
    dd = np.concatenate([lv.d[lv.offsets[j]:lv.offsets[j + 1]] for j in range(T) for lv in levels]).astype(np.int32)
    single = Bank(off.astype(np.int64), aa, bb, dd, int(dd.max()))
    nb_single = min(nblk, 64)
    with SpiirBank.from_bank(single, max_block=B) as sb:
        for i in range(4):
            sb.trigger_max(blocks[i][0])
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for i in range(nb_single):
            sb.trigger_max(blocks[i][0])
        torch.cuda.synchronize()
        t_single = (time.perf_counter() - ts) / nb_single
    single_rate = float(sum(F)) * B / t_single
    log("single-rate bank of the same filters: %.1f us per block, %.3e updates/s (multi-rate %.1fx faster)"
        % (t_single * 1e6, single_rate, value / single_rate))

    res = {
        "metric": METRIC, "value": value, "unit": "filter-updates/s (full-rate equivalent)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded white noise; chirp-like bank, filter frequencies ~ f^-11/3 on 20..1024 Hz)",
        "config": {"workload": "multi-rate bank: %d templates x U{100..800} filters on 5 rate levels "
                               "(4096..256 Hz), %d samples at 4096 Hz in %d-sample blocks, fused max/argmax"
                               % (T, N, B),
                   "filters_per_level": F, "global_batch": T, "seq_len": N, "parallelism": "single GPU"},
        "actual_updates_per_s": upd_act / t_step, "update_fraction": upd_act / upd_eff,
        "block_us": t_step / nblk * 1e6, "block_us_without_graph": t_eager / nblk * 1e6, "per_level": per_level,
        "single_rate_same_filters": {"updates_per_s": single_rate, "block_us": t_single * 1e6,
                                     "blocks_timed": nb_single, "multirate_speedup": value / single_rate},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": None,
                     "kernel": "level-%d forward kernel (%d filters, %d samples per launch)" % (dom, F[dom], B >> dom),
                     "launch_us": d["forward_us"], "flop_per_launch": fl_dom},
    }
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        nchk = min(N, 16 * B)
        t1 = time.perf_counter()
        m_ref, j_ref = oracle.multirate_trigger(levels, h, g, x[:nchk])
        t_or = time.perf_counter() - t1
        gm = mx[:nchk].cpu().numpy().astype(np.float64)
        gj = am[:nchk].cpu().numpy()
        peak = float(m_ref.max())
        rel = float(np.max(np.abs(gm - m_ref)) / peak)
        agree = float(np.mean(gj == j_ref))
        res["check"] = {"samples": nchk, "max_abs_err_over_peak": rel, "argmax_agree": agree, "gate": 1e-4,
                        "pass": rel <= 1e-4}
        log("multirate check: max|dM|/peak %.3g, argmax agree %.6f (oracle %.1fs)" % (rel, agree, t_or))
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = {"value": float(sum(F)) * nchk / t_or, "unit": "filter-updates/s (full-rate equivalent)",
                                   "cores": oracle.max_threads(), "kind": "oracle",
                                   "sample": "FP64 multi-rate oracle over the first %d samples, %.1f s" % (nchk, t_or)}
    mr.close()
    print(json.dumps(res), flush=True)


def run_whiten(args, torch, frame=4096, train_s=32):
    """Whitening front end on 4,194,304 samples of coloured noise (4,096 Hz):
    PSD from the first 32 s, then the stream whitened in 4,096-sample calls
    (streaming) and in 65,536-sample calls (throughput). value = samples/s of
    the streaming pass."""
    from paper_1602_05573_amd import Whitener
    from workloads import coloured_noise

    N, B = args.samples, args.block
    x = coloured_noise(N, 0)
    xd = torch.from_numpy(x).cuda()
    out = torch.empty_like(xd)
    stream = torch.cuda.current_stream()
    wh = Whitener(frame)
    ntrain = train_s * 4096
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wh.estimate_psd(xd[:ntrain])
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(10):
        wh.estimate_psd(xd[:ntrain])
    e1.record(stream)
    torch.cuda.synchronize()
    t_psd = e0.elapsed_time(e1) * 1e-3 / 10

    def one_pass(block):
        wh.reset()
        for i in range(N // block):
            wh.process(xd[i * block:(i + 1) * block], out=out[i * block:(i + 1) * block])

    res_pass = {}
    for label, block in (("streaming", B), ("throughput", 65536)):
        for _ in range(args.warmup):
            one_pass(block)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            one_pass(block)
        e1.record(stream)
        torch.cuda.synchronize()
        res_pass[label] = e0.elapsed_time(e1) * 1e-3 / args.steps
    t_step = res_pass["streaming"]
    value = N / t_step
    alg = 8.0 * N   # the raw stream read once, the whitened stream written once
    log("whiten: PSD of %d s in %.1f us; %.3e samples/s in %d-sample calls (%.1f ms per pass), %.3e in 65,536"
        % (train_s, t_psd * 1e6, value, B, t_step * 1e3, N / res_pass["throughput"]))
    res = {
        "metric": "whitened samples/s", "value": value, "unit": "samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic coloured noise (white noise through 1/(1 - 1.8 z^-1 + 0.85 z^-2) plus a white floor)",
        "config": {"workload": "whitening front end: %d samples at 4096 Hz, %d-sample frames (Hann, half overlap), "
                               "PSD from the first %d s, %d-sample calls" % (N, frame, train_s, B),
                   "parallelism": "single GPU"},
        "psd_us": t_psd * 1e6, "throughput_65536_calls": N / res_pass["throughput"],
        "roofline": {"bound": "hbm", "achieved": alg / t_step / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                     "frac": alg / t_step / PEAK_HBM, "traffic": None,
                     "note": "8 B per sample (read and write once); frame FFT + overlap-add launches per call",
                     "achieved_65536_calls": alg / res_pass["throughput"] / 1e9},
    }
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        S = wh.psd()
        t1 = time.perf_counter()
        ref = oracle.whiten(x, S, frame)
        t_or = time.perf_counter() - t1
        got = out.cpu().numpy()
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        res["check"] = {"samples": N, "max_abs_err_over_peak": err, "gate": 1e-4, "pass": err <= 1e-4}
        log("whiten check: %.3g of the peak (oracle %.1f s)" % (err, t_or))
        if not args.no_cpu_baseline:
            res["cpu_baseline"] = {"value": N / t_or, "unit": "samples/s", "cores": 1, "kind": "oracle",
                                   "sample": "numpy FP64 oracle whitening of the same %d samples, %.1f s" % (N, t_or)}
    wh.close()
    print(json.dumps(res), flush=True)


def run_pipeline(args, torch, frame=4096, window=4096):
    """Streaming pipeline on raw strain: coloured noise (4,194,304 samples at
    4,096 Hz) -> whitening (4,096-sample frames, PSD from the first 32 s) ->
    the 1,024-template bank's fused max/argmax -> streaming trigger clustering
    (W = 4,096: each block's final triggers, one second of latency). Per-block
    latency is whitening + filtering + clustering of one 4,096-sample block
    (HIP events on the stream). value = raw samples/s of the whole job."""
    from paper_1602_05573_amd import SpiirBank, TriggerStream, Whitener
    from workloads import bank_1024, coloured_noise

    bank, _ = bank_1024(n=args.samples, n_templates=args.templates)
    N, B = args.samples, args.block
    x = coloured_noise(N, 0)
    xd = torch.from_numpy(x).cuda()
    white = torch.empty_like(xd)
    mx = torch.empty(N, dtype=torch.float32, device="cuda")
    am = torch.empty(N, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    wh = Whitener(frame)
    wh.estimate_psd(xd[:32 * 4096])
    bk = SpiirBank.from_bank(bank, max_block=B)
    nblk = N // B
    cap = (B + window) // (window + 1) + 2
    t_idx = torch.empty((nblk + 1, cap), dtype=torch.int64, device="cuda")
    t_tpl = torch.empty((nblk + 1, cap), dtype=torch.int32, device="cuda")
    t_snr = torch.empty((nblk + 1, cap), dtype=torch.float32, device="cuda")
    t_cnt = torch.zeros(nblk + 1, dtype=torch.int64, device="cuda")
    ts = None

    def one_pass(events=None):
        wh.reset()
        bk.reset()
        ts.reset()
        for i in range(nblk):
            sl = slice(i * B, (i + 1) * B)
            if events is not None:
                events[i][0].record(stream)
            wh.process(xd[sl], out=white[sl])
            bk.trigger_max(white[sl], out=(mx[sl], am[sl]))
            ts.push_into(mx[sl], am[sl], t_idx[i], t_tpl[i], t_snr[i], t_cnt[i:i + 1])
            if events is not None:
                events[i][1].record(stream)
        ts.flush_into(t_idx[nblk], t_tpl[nblk], t_snr[nblk], t_cnt[nblk:nblk + 1])

    # threshold from a first pass of the filter output (a high quantile of the max series)
    wh.reset()
    bk.reset()
    for i in range(nblk):
        sl = slice(i * B, (i + 1) * B)
        wh.process(xd[sl], out=white[sl])
        bk.trigger_max(white[sl], out=(mx[sl], am[sl]))
    torch.cuda.synchronize()
    thr = float(torch.quantile(mx[N // 2:N // 2 + (1 << 20)], 0.9999))
    ts = TriggerStream(thr, window, B, capacity=cap)
    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nblk)]
          for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s_ in range(args.steps):
        one_pass(ev[s_])
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / args.steps
    lat = np.array([ev[s_][i][0].elapsed_time(ev[s_][i][1]) for s_ in range(args.steps) for i in range(nblk)])
    counts = t_cnt.cpu().numpy()
    total = int(counts.sum())
    value = N / t_step
    log("pipeline: %.1f ms per pass = %.3e raw samples/s (%.1fx real time at 4,096 Hz); block latency p50 %.1f us, "
        "p99 %.1f us; %d triggers (threshold %.4g, W = %d)"
        % (t_step * 1e3, value, value / 4096.0, np.percentile(lat, 50) * 1e3, np.percentile(lat, 99) * 1e3, total,
           thr, window))
    res = {
        "metric": "raw strain samples/s through whitening, filtering and clustering", "value": value,
        "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_step * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic coloured noise; random 1,024-template bank",
        "config": {"workload": "pipeline: %d samples of coloured noise -> whitening (%d-sample frames) -> "
                               "%d-template bank fused max/argmax in %d-sample blocks -> streaming clustering "
                               "(W = %d)" % (N, frame, bank.n_templates, B, window),
                   "parallelism": "single GPU"},
        "realtime_factor": value / 4096.0, "triggers": total, "threshold": thr,
        "block_latency_us": {"p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
                             "max": float(lat.max() * 1e3)},
        "filter_updates_per_s": float(bank.n_filters) * N / t_step,
    }
    if not args.no_check or not args.no_cpu_baseline:
        import oracle
        m_h, a_h = mx.cpu().numpy(), am.cpu().numpy()
        ri = oracle.clusters(m_h, a_h, thr, window)[0]
        got = np.concatenate([t_idx[i, :min(cap, int(counts[i]))].cpu().numpy() for i in range(nblk + 1)])
        res["check"] = {"streamed_triggers_equal_whole_series_oracle": bool(np.array_equal(got, ri)),
                        "oracle_triggers": int(len(ri))}
        log("pipeline check: streamed triggers equal the oracle's on the whole series: %s" % np.array_equal(got, ri))
    wh.close()
    bk.close()
    ts.close()
    print(json.dumps(res), flush=True)


def run_precision(args, torch):
    """64 templates x 1,000 filters with r ~ U[1-1e-4, 1-1e-6] over 16,777,216
    samples: throughput of the fused trigger per precision mode, and the max
    relative SNR error of two sampled templates against the FP64 oracle."""
    from paper_1602_05573_amd import SpiirBank
    from workloads import precision_bank
    import oracle

    pick = [5, 42]
    bank, x = precision_bank()
    F, T, N = bank.n_filters, bank.n_templates, len(x)
    xd = torch.from_numpy(x).cuda()
    C = 1 << 20   # samples per call
    t0 = time.perf_counter()
    ref = oracle.snr(bank.subset(pick), x, nthreads=oracle.max_threads())
    log("oracle on templates %s: %.1fs" % (pick, time.perf_counter() - t0))
    P = ref.max(axis=1)
    modes = {}
    for prec, name in ((0, "fp32 + fp64 carries for |a| > 1-1e-5"), (2, "fp32 + fp64 carries for all"),
                       (1, "all fp32")):
        with SpiirBank.from_bank(bank, precision=prec, filters_per_lane=args.fl, waves_per_group=args.wpg,
                                 time_split=args.time_split) as bk:
            if prec == 0:
                log("bank:", bk.info)
            mx = torch.empty(C, dtype=torch.float32, device="cuda")
            am = torch.empty(C, dtype=torch.int32, device="cuda")

            def one_pass():
                bk.reset()
                for c0 in range(0, N, C):
                    c1 = min(N, c0 + C)
                    bk.trigger_max(xd[c0:c1], out=(mx[: c1 - c0], am[: c1 - c0]))

            for _ in range(args.warmup):
                one_pass()
            torch.cuda.synchronize()
            ts = time.perf_counter()
            for _ in range(args.steps):
                one_pass()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - ts) / args.steps
            # error of the sampled templates (separate pass keeping their SNR rows)
            bk.reset()
            rows = np.empty((len(pick), N), np.float32)
            snr = torch.empty((T, C), dtype=torch.float32, device="cuda")
            for c0 in range(0, N, C):
                c1 = min(N, c0 + C)
                s = bk.filter_block(xd[c0:c1], snr=snr[:, : c1 - c0] if c1 - c0 == C else None)
                rows[:, c0:c1] = s[pick].cpu().numpy()
            err = float(np.max(np.max(np.abs(rows - ref), axis=1) / P))
            info = bk.info
            modes[prec] = {"mode": name, "filter_updates_per_s": F * N / dt, "ms_per_pass": dt * 1e3,
                           "max_rel_snr_err": err, "time_split": info["time_split"],
                           "filters_per_lane": info["filters_per_lane"],
                           "waves_per_group": info["waves_per_group"], "workgroups": info["n_groups"]}
            log("precision %d (%s): %.3e updates/s, %.1f ms per pass, max rel SNR err %.3g"
                % (prec, name, F * N / dt, dt * 1e3, err))
    res = {
        "metric": METRIC, "value": modes[0]["filter_updates_per_s"], "unit": "filter-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": modes[0]["ms_per_pass"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded white noise and random banks)",
        "config": {"workload": "precision stress: %d templates x 1000 filters, r in [1-1e-4, 1-1e-6], "
                               "%d samples in %d-sample calls, fused max/argmax" % (T, N, C)},
        "pct_fp32_peak": 100.0 * FLOP_UPDATE * modes[0]["filter_updates_per_s"] / PEAK_FP32,
        "precision_modes": modes,
        "error_sample": "templates %s over the whole stream against the FP64 oracle; error = "
                        "max |SNR - SNR_ref| / max SNR_ref per template" % pick,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
