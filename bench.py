"""Benchmark: exact top-k LCP retrieval on one MI355X.

Workload (default): N = 2,000,000 rows, L = 32 uint16 tokens, V = 4,096 from
the 16/16/16 hierarchy + Zipf(1.1) generator; a batch of Q = 8,192 queries
from the same generator, k = 10 for every query.  The index is built once
(timed separately); inputs are resident in HBM before the timed region.

A step is one call of the index path (lcp_topk) over the whole batch.  The
full scan (lcp_scan_topk) is timed on the same batch for comparison, and the
scan kernel's HBM bandwidth is measured separately at a bandwidth-bound tile.

Prints ONE JSON line.  Run `python bench.py --help` for options.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--queries", type=int, default=8192)
    ap.add_argument("--scan-steps", type=int, default=5)
    ap.add_argument("--scan-bw-queries", type=int, default=32,
                    help="batch size for the scan-bandwidth measurement (HBM-bound regime)")
    ap.add_argument("--streams", type=int, default=2,
                    help="streams the index-path steps are issued on, round-robin")
    ap.add_argument("--large-n", type=int, default=8_000_000,
                    help="rows of the larger-than-Infinity-Cache database (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target wall time of the CPU baseline sample")
    ap.add_argument("--serve-seconds", type=float, default=4.0,
                    help="duration of each fixed-rate serving run (0 disables)")
    ap.add_argument("--serve-rates", type=str, default="1000,10000,100000")
    ap.add_argument("--saturation-qps", type=float, default=1_000_000.0,
                    help="offered load of a one-second serving burst that the synchronous scan cannot keep up with (0: skip)")
    ap.add_argument("--no-uneven", dest="uneven", action="store_false",
                    help="skip the uneven-k batch comparison")
    ap.add_argument("--sensor-steps", type=int, default=5000,
                    help="steps of the sensor-fusion stream (0 disables)")
    ap.add_argument("--energy-seconds", type=float, default=2.0,
                    help="sustained run per energy reading (0 disables the energy section)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain 1-byte elementwise copy of this size (profiler counter calibration)")
    ap.add_argument("--calib-gather-mib", type=int, default=0,
                    help="also gather this many MiB of random 64-byte rows from a 1 GiB table "
                         "(profiler counter calibration for scattered reads)")
    ap.add_argument("--quiet", action="store_true")
    return ap.parse_args()


def log(args, *a):
    if not args.quiet:
        print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the index and the scan run on a single MI355X; "
                                   "--gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2602_04936_amd as P

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = synth.c3_hierarchy(Q=args.queries, k_fixed=args.k)
    log(args, f"[bench] generated N={w.N} L={w.L} V={w.V} Q={w.Q} in {time.time() - t0:.1f}s")
    db_dev = P.to_device_tokens(w.db, dev)
    q_dev = P.to_device_tokens(w.queries, dev)
    ks = w.k.astype(np.int32)
    torch.cuda.synchronize()

    tb = time.perf_counter()
    idx = P.Index(db_dev, w.V)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - tb) * 1e3
    del db_dev
    log(args, f"[bench] index built in {build_ms:.1f} ms")

    total = int(ks.sum())
    ids = torch.empty(total, dtype=torch.int32, device=dev)
    lcps = torch.empty(total, dtype=torch.int32, device=dev)

    # ---- index path: warmup, then K timed steps.  Batches are independent, so
    # consecutive steps go round-robin to --streams streams (each with its own
    # output buffers): one batch's slowest waves overlap the next batch's start.
    # The same steps on one stream are timed too.
    nstreams = max(1, args.streams)
    streams = [torch.cuda.Stream(device=dev) for _ in range(nstreams)]
    outs = [(ids, lcps)] + [(torch.empty_like(ids), torch.empty_like(lcps)) for _ in range(nstreams - 1)]

    def timed_steps(n_str):
        for _ in range(args.warmup):
            for j in range(n_str):
                idx.topk(q_dev, args.k, out=outs[j], stream=streams[j])
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(args.steps):
            idx.topk(q_dev, args.k, out=outs[i % n_str], stream=streams[i % n_str])
        torch.cuda.synchronize()
        return time.perf_counter() - t

    dt_single = timed_steps(1)
    dt = timed_steps(nstreams)
    same_outputs = all(torch.equal(o[0], ids) and torch.equal(o[1], lcps) for o in outs[1:])

    def event_blocks(n_str, blocks=5):
        """GPU time of `blocks` further blocks of --steps steps each, from an
        event on the first stream that the others wait on, to an event there
        recorded after it waits for the others' last steps."""
        times = []
        for _ in range(blocks):
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(streams[0])
            for j in range(1, n_str):
                streams[j].wait_event(a)
            for i in range(args.steps):
                idx.topk(q_dev, args.k, out=outs[i % n_str], stream=streams[i % n_str])
            for j in range(1, n_str):
                e = torch.cuda.Event()
                e.record(streams[j])
                streams[0].wait_event(e)
            b.record(streams[0])
            b.synchronize()
            times.append(a.elapsed_time(b) / args.steps)
        return times

    blocks_multi = event_blocks(nstreams)
    blocks_single = event_blocks(1)
    # kernel duration: K launches back to back on one stream, between two HIP
    # events on that stream (the kernel runs on the stream it is given), in a
    # pass of its own so that the events do not sit inside the timed region
    s0 = streams[0]
    idx.topk(q_dev, args.k, out=outs[0], stream=s0)
    torch.cuda.synchronize()
    ea, eb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ea.record(s0)
    for _ in range(args.steps):
        idx.topk(q_dev, args.k, out=outs[0], stream=s0)
    eb.record(s0)
    eb.synchronize()
    k_avg_ms = ea.elapsed_time(eb) / args.steps
    ms_per_step = dt * 1e3 / args.steps
    qps = w.Q * args.steps / dt
    kn = args.steps
    log(args, f"[bench] index path: {ms_per_step:.4f} ms/step, {qps / 1e6:.2f} M queries/s on {nstreams} streams "
              f"({dt_single * 1e3 / args.steps:.4f} ms/step on one), kernel {k_avg_ms * 1e3:.1f} us avg over {kn}")
    got_ids = ids.cpu().numpy()
    got_lcp = lcps.cpu().numpy()

    # ---- full scan on the same batch
    sids = torch.empty_like(ids)
    slcp = torch.empty_like(lcps)
    idx.scan_topk(q_dev, ks, out=(sids, slcp))
    torch.cuda.synchronize()
    idx.set_kernel_timing(True)
    idx.kernel_time(1)
    idx.kernel_time(2)
    t2 = time.perf_counter()
    for _ in range(args.scan_steps):
        idx.scan_topk(q_dev, ks, out=(sids, slcp))
    torch.cuda.synchronize()
    sdt = time.perf_counter() - t2
    s_ms, s_n = idx.kernel_time(1)
    m_ms, m_n = idx.kernel_time(2)
    idx.set_kernel_timing(False)
    scan_qps = w.Q * args.scan_steps / sdt
    paths_agree = bool(torch.equal(sids, ids) and torch.equal(slcp, lcps))
    log(args, f"[bench] full scan: {sdt * 1e3 / args.scan_steps:.3f} ms/batch, {scan_qps / 1e6:.3f} M queries/s, "
              f"paths agree: {paths_agree}")

    # ---- the bucket range scan on the same batch at B = 1, 16, 256 prefix buckets
    bucket_scan = prefix_bucket_sweep(P, idx, q_dev, args.k)
    log(args, f"[bench] bucket range scan: {bucket_scan}")

    # ---- scan bandwidth at a bandwidth-bound tile (few queries per pass)
    nbw = args.scan_bw_queries
    qbw = q_dev[:nbw]
    kbw = ks[:nbw]
    bw_ids = torch.empty(int(kbw.sum()), dtype=torch.int32, device=dev)
    bw_lcp = torch.empty_like(bw_ids)
    for _ in range(2):
        idx.scan_topk(qbw, kbw, out=(bw_ids, bw_lcp))
    torch.cuda.synchronize()
    idx.set_kernel_timing(True)
    idx.kernel_time(1)
    idx.kernel_time(2)
    reps = 20
    tcall = time.perf_counter()
    for _ in range(reps):
        idx.scan_topk(qbw, kbw, out=(bw_ids, bw_lcp))
    torch.cuda.synchronize()
    bw_call_us = (time.perf_counter() - tcall) / reps * 1e6
    bw_ms, bw_n = idx.kernel_time(1)
    idx.kernel_time(2)
    idx.set_kernel_timing(False)
    row_bytes = w.L * 2
    groups_bw = idx.scan_info(nbw, args.k)[0]
    # the pass streams the 8-byte prefix plane (key words 0-1 of every row);
    # whole rows are read only for rows that tie on those 8 bytes.  Each query
    # group streams the plane, but the groups' blocks take the same rows at
    # the same time on one XCD, so HBM sees one pass (the FETCH_SIZE counter
    # agrees): the bytes charged are one pass plus the query rows
    plane_bytes = 8
    bw_bytes = w.N * plane_bytes + nbw * row_bytes
    bw_gbs = bw_bytes / (bw_ms / bw_n * 1e-3) / 1e9

    # ---- the same Q=32 pass with the 256 MB Infinity Cache flushed before each
    # rep, so the plane comes from HBM: a 512 MiB read (clean lines), and a
    # 512 MiB write (the dirty lines are written back while the pass runs)
    flush = torch.ones(512 << 20, dtype=torch.uint8, device=dev)

    def cold_pass(ix, q, kk, out, write_flush):
        times = []
        for _ in range(10):
            if write_flush:
                flush.fill_(1)
            else:
                flush.sum()
            torch.cuda.synchronize()
            ix.set_kernel_timing(True)
            ix.kernel_time(1)
            ix.scan_topk(q, kk, out=out)
            c_ms, c_n = ix.kernel_time(1)
            ix.set_kernel_timing(False)
            times.append(c_ms / max(c_n, 1))
        return float(np.median(times)) * 1e3

    cold_us = cold_pass(idx, qbw, kbw, (bw_ids, bw_lcp), False)
    cold_w_us = cold_pass(idx, qbw, kbw, (bw_ids, bw_lcp), True)
    cold_gbs = bw_bytes / (cold_us * 1e-6) / 1e9

    def stream_reference(nbytes):
        """torch.sum over nbytes of int64, hot and after the read flush: what a
        plain streaming reduction reaches on the same data size."""
        x = torch.ones(nbytes // 8, dtype=torch.int64, device=dev)
        res = {}
        for name, pre in (("hot", None), ("cold", lambda: flush.sum())):
            ts = []
            for _ in range(10):
                if pre:
                    pre()
                torch.cuda.synchronize()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                torch.sum(x)
                b.record()
                b.synchronize()
                ts.append(a.elapsed_time(b) * 1e3)
            us = float(np.median(ts))
            res[name + "_us"] = round(us, 2)
            res[name + "_GBps"] = round(nbytes / (us * 1e-6) / 1e9, 1)
        del x
        return res

    # ---- a database larger than the Infinity Cache: c3's generator at N=8M
    large = None
    if args.large_n > 0:
        wl = synth.c3_like(args.large_n, w.Q, seed=1003, k_fixed=args.k)
        lidx = P.Index(P.to_device_tokens(wl.db, dev), wl.V)
        lq = P.to_device_tokens(wl.queries, dev)
        lo = [(torch.empty(wl.Q * args.k, dtype=torch.int32, device=dev),
               torch.empty(wl.Q * args.k, dtype=torch.int32, device=dev)) for _ in range(nstreams)]
        for j in range(nstreams):
            lidx.topk(lq, args.k, out=lo[j], stream=streams[j])
        torch.cuda.synchronize()
        lsteps = max(20, args.steps // 4)
        t = time.perf_counter()
        for i in range(lsteps):
            lidx.topk(lq, args.k, out=lo[i % nstreams], stream=streams[i % nstreams])
        torch.cuda.synchronize()
        l_qps = wl.Q * lsteps / (time.perf_counter() - t)
        lbw = (torch.empty(32 * args.k, dtype=torch.int32, device=dev), torch.empty(32 * args.k, dtype=torch.int32, device=dev))
        lidx.scan_topk(lq[:32], args.k, out=lbw)
        torch.cuda.synchronize()
        lidx.set_kernel_timing(True)
        lidx.kernel_time(1)
        for _ in range(10):
            lidx.scan_topk(lq[:32], args.k, out=lbw)
        lm, ln = lidx.kernel_time(1)
        lidx.set_kernel_timing(False)
        l_pass_us = lm / max(ln, 1) * 1e3
        l_cold_us = cold_pass(lidx, lq[:32], args.k, lbw, False)
        l_groups = lidx.scan_info(32, args.k)[0]
        l_bytes = wl.N * plane_bytes + 32 * row_bytes
        t = time.perf_counter()
        for _ in range(2):
            lidx.scan_topk(lq, args.k, out=lo[0])
        torch.cuda.synchronize()
        l_scan_qps = wl.Q * 2 / (time.perf_counter() - t)
        large = {"N": wl.N, "db_bytes": int(wl.N * row_bytes),
                 "index_qps": round(l_qps, 1), "index_ms_per_step": round(wl.Q / l_qps * 1e3, 5),
                 "scan_qps": round(l_scan_qps, 1),
                 "scan_pass_q32_us": round(l_pass_us, 2),
                 "scan_pass_q32_GBps": round(l_bytes / (l_pass_us * 1e-6) / 1e9, 1),
                 "scan_pass_q32_cold_us": round(l_cold_us, 2),
                 "scan_pass_q32_cold_GBps": round(l_bytes / (l_cold_us * 1e-6) / 1e9, 1),
                 "scan_pass_q32_cold_frac": round(l_bytes / (l_cold_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                 "scan_pass_q32_bytes": int(l_bytes),
                 "query_groups_q32": l_groups,
                 "streaming_reference_torch_sum": stream_reference(wl.N * plane_bytes)}
        lidx.close()
        del wl, lq, lo
        log(args, f"[bench] larger than the Infinity Cache: {large}")

    # ---- parity of the whole bench batch against the CPU oracle (outside every timed region)
    parity = None
    try:
        import oracle
        wi, wl, _ = oracle.c_topk(w.db, w.queries, ks)
        parity = {"queries_checked": int(w.Q), "bit_exact": bool((got_ids == wi).all() and (got_lcp == wl).all())}
    except Exception as e:  # the oracle is a test dependency; report, do not fail the bench
        parity = {"error": repr(e)}

    # ---- roofline of the index-path kernel.  Algorithmic bytes per query: the
    # query row, the ceil(log2(N+1)) rows a comparison search must probe, one A
    # byte per row of the cutoff group G_c plus its two boundaries, one perm id
    # per row above or tied at the cutoff (the range scan's items), 8 bytes per
    # output entry.  The per-query counts come from the kernel itself.
    probes = int(np.ceil(np.log2(w.N + 1)))
    _, st = idx.topk_stats(q_dev, args.k)
    torch.cuda.synchronize()
    shape = work_shape(st.cpu().numpy(), w.N, args.k, row_bytes, probes)
    bytes_per_query = shape.pop("algorithmic_bytes_per_query")
    idx_bytes = shape.pop("algorithmic_bytes_per_launch")
    idx_gbs = idx_bytes / (k_avg_ms * 1e-3) / 1e9
    scan_kernel_ms = s_ms / max(s_n, 1)
    groups = idx.scan_info(w.Q, args.k)[0]
    scan_bytes = w.N * plane_bytes + w.Q * row_bytes

    # ---- serving at fixed offered load (Poisson arrivals, batches of 1-256 queries)
    serving = None
    if args.serve_seconds > 0:
        from paper_2602_04936_amd import serve
        serving = {"index_continuous_batching": {}, "scan_synchronous": {}}
        ref = got_ids.reshape(w.Q, args.k), got_lcp.reshape(w.Q, args.k)
        for rate in [float(r) for r in args.serve_rates.split(",") if r]:
            t, b, kk = synth.serving_schedule(rate, args.serve_seconds, seed=1004, k_mode="fixed", k_fixed=args.k)
            reqs = serve.requests_from_schedule(w.queries, t, b, kk)
            rep = serve.run_served(idx, reqs)
            rep["results_match_batch_run"] = served_match(reqs, ref, w.Q)
            serving["index_continuous_batching"][str(int(rate))] = rep
            log(args, f"[bench] served index path @{int(rate)}/s: {rep}")
            reqs = serve.requests_from_schedule(w.queries, t, b, kk)
            rep = serve.run_synchronous(idx, reqs, scan=True, max_wall_s=2 * args.serve_seconds + 5)
            serving["scan_synchronous"][str(int(rate))] = rep
            log(args, f"[bench] synchronous full scan @{int(rate)}/s: {rep}")
            t, b, kk = synth.serving_schedule(rate, args.serve_seconds, seed=1004, k_mode="uniform")
            reqs = serve.requests_from_schedule(w.queries, t, b, kk)
            rep = serve.run_served(idx, reqs)
            rep.update(served_check(idx, reqs, w.db))
            serving.setdefault("index_continuous_batching_k_uniform_1_100", {})[str(int(rate))] = rep
            log(args, f"[bench] served index path, k uniform 1..100 @{int(rate)}/s: {rep}")

        # where the two paths part: a one-second burst at 1,000,000 queries/s
        # (about 87,000 requests), the synchronous scan cut off after 3 s
        if args.saturation_qps > 0:
            sat = {"offered_qps": args.saturation_qps, "seconds": 1.0}
            t, b, kk = synth.serving_schedule(args.saturation_qps, 1.0, seed=1004, k_mode="fixed", k_fixed=args.k)
            reqs = serve.requests_from_schedule(w.queries, t, b, kk)
            sat["index_continuous_batching"] = serve.run_served(idx, reqs)
            sat["index_continuous_batching"]["results_match_batch_run"] = served_match(reqs, ref, w.Q)
            reqs = serve.requests_from_schedule(w.queries, t, b, kk)
            sat["scan_synchronous"] = serve.run_synchronous(idx, reqs, scan=True, max_wall_s=3.0)
            serving["saturation"] = sat
            log(args, f"[bench] burst at {args.saturation_qps:.0f} queries/s: {sat}")

    # ---- uneven batch: the same 8,192 queries with k uniform on {1, 10, 100}:
    # one plain launch, per-k-bucket plain launches, and one persistent launch
    # replayed from a captured HIP graph with the autotuned grid
    uneven = None
    if args.uneven:
        from paper_2602_04936_amd import batching
        ku = synth.uneven_k(w.Q)
        buckets = batching.split_by_k(ku)
        bq = {kv: q_dev[torch.from_numpy(sel).to(dev)] for kv, sel in buckets.items()}
        bout = {kv: (torch.empty(len(sel) * kv, dtype=torch.int32, device=dev),
                     torch.empty(len(sel) * kv, dtype=torch.int32, device=dev)) for kv, sel in buckets.items()}
        uo = (torch.empty(int(ku.sum()), dtype=torch.int32, device=dev),
              torch.empty(int(ku.sum()), dtype=torch.int32, device=dev))
        tune = batching.tune_launch(idx, q_dev, ku, reps=5)
        best = tune["best"] if tune["best"].mode != "plain" else min(
            (sh for sh in tune["tried"] if sh.mode != "plain"), key=lambda sh: sh.ms)
        tune["best"] = best
        cl = batching.CapturedLaunch(idx, cap_queries=w.Q, k_max=100,
                                     blocks=best.blocks if best.mode == "persistent" else 0)

        def timed(fn, reps=20):
            fn()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t) * 1e3 / reps

        def device_ms(fn, stream, reps=20):
            # GPU time of `reps` back-to-back calls, from events on `stream`
            fn()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                fn()
            b.record(stream)
            b.synchronize()
            return a.elapsed_time(b) / reps

        one = timed(lambda: idx.topk(q_dev, ku, out=uo))
        per_bucket = timed(lambda: [idx.topk(bq[kv], kv, out=bout[kv]) for kv in buckets])
        cur = torch.cuda.current_stream()
        per_bucket_dev = device_ms(lambda: [idx.topk(bq[kv], kv, out=bout[kv]) for kv in buckets], cur)
        # the batch is produced straight into the captured query buffer, in
        # the tuned launch order (the answers keep the batch's own layout)
        order = batching.launch_order(ku, w.Q, best.order)
        cl.q.copy_(q_dev if order is None else q_dev[torch.from_numpy(order).to(dev)])
        torch.cuda.synchronize()
        captured = timed(lambda: cl.run(None, ku, n=w.Q, order=order))
        reps_c = 20
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps_c)]
        for e in evs:
            cl.run(None, ku, n=w.Q, events=e, order=order)
        torch.cuda.synchronize()
        captured_dev = float(np.median([a.elapsed_time(b) for a, b in evs]))
        ref = idx.topk(q_dev, ku, out=uo)
        gi, gl, _ = cl.run(None, ku, n=w.Q, order=order)
        torch.cuda.synchronize()
        same = bool(torch.equal(gi, ref.ids) and torch.equal(gl, ref.lcps))
        # the batch staged on the device ahead of time (as the per-bucket
        # launches have their queries and k ready): the replay alone
        cl.stage(ku, w.Q, order=order)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps_c)]
        for e in evs:
            cl.replay(events=e)
        torch.cuda.synchronize()
        staged_dev = float(np.median([a.elapsed_time(b) for a, b in evs]))
        # the same replay timed like the per-bucket launches: back-to-back on
        # one stream (the captured launch's own) between two events
        def replays(reps=20):
            cl.replay()
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(cl.stream):
                a.record(cl.stream)
                for _ in range(reps):
                    cl.graph.replay()
                b.record(cl.stream)
            b.synchronize()
            return a.elapsed_time(b) / reps
        staged_b2b = replays()
        staged_same = bool(torch.equal(cl.ids[:int(ku.sum())], ref.ids) and torch.equal(cl.lcps[:int(ku.sum())], ref.lcps))
        # every shape the autotuner tried, and the per-bucket launches, against the C oracle on all queries
        shapes_exact = None
        try:
            import oracle
            wi_u, wl_u, woff_u = oracle.c_topk(w.db, w.queries, ku)
            cnt = torch.tensor([w.Q], dtype=torch.int64, device=dev)
            shapes_exact = {}
            for sh in tune["tried"]:
                si = torch.full_like(uo[0], -9)
                sl = torch.full_like(uo[1], -9)
                batching.run_shape(idx, sh, batching.shape_inputs(q_dev, ku, sh.order), 100, si, sl, cnt)
                torch.cuda.synchronize()
                shapes_exact[f"{sh.mode}:{sh.blocks}:{sh.order}"] = bool((si.cpu().numpy() == wi_u).all() and
                                                                         (sl.cpu().numpy() == wl_u).all())
            bucket_ok = True
            for kv, sel in buckets.items():
                bi = bout[kv][0].cpu().numpy().reshape(-1, kv)
                bl = bout[kv][1].cpu().numpy().reshape(-1, kv)
                for j, qi in enumerate(sel):
                    a, b = woff_u[qi], woff_u[qi + 1]
                    bucket_ok &= bool((bi[j] == wi_u[a:b]).all() and (bl[j] == wl_u[a:b]).all())
            shapes_exact["per_k_bucket"] = bucket_ok
            shapes_exact["captured"] = bool((gi.cpu().numpy() == wi_u).all() and (gl.cpu().numpy() == wl_u).all())
        except Exception as e:  # the oracle is a test dependency; report, do not fail the bench
            shapes_exact = {"error": repr(e)}
        uneven = {"queries": w.Q, "k_choices": [1, 10, 100],
                  "one_plain_launch_ms": round(one, 4), "per_k_bucket_launches_ms": round(per_bucket, 4),
                  "per_k_bucket_launches_gpu_ms": round(per_bucket_dev, 4),
                  "captured_ms": round(captured, 4), "captured_gpu_ms": round(captured_dev, 4),
                  "captured_staged_replay_gpu_ms": round(staged_dev, 4),
                  "back_to_back_gpu_ms": {"per_k_bucket_launches": round(per_bucket_dev, 4),
                                          "captured_staged_replay": round(staged_b2b, 4)},
                  "captured_staged_replay_equals_plain": staged_same,
                  "oracle_exact_by_shape": shapes_exact,
                  "captured_shape": (tune["best"].mode, tune["best"].blocks, tune["best"].order),
                  "captured_qps": round(w.Q / (captured * 1e-3), 1),
                  "autotune": [(sh.mode, sh.blocks, sh.order, round(sh.ms, 4)) for sh in tune["tried"]],
                  "captured_equals_plain": same}
        log(args, f"[bench] uneven batch: {uneven}")

    # ---- energy per query from the socket energy accumulator: idle draw, the
    # index path, the full scan, and the bucket range scan at B = 1, 16, 256
    # prefix buckets (each query scans only its own bucket)
    energy = None
    if args.energy_seconds > 0:
        from paper_2602_04936_amd import energy as E
        meter, why = E.try_meter(dev)
        if meter is None:
            energy = {"unavailable": why}
        else:
            es = args.energy_seconds
            iw = meter.idle_watts(es)
            energy = {"idle_watts": round(iw, 1) if iw is not None else None}

            def run_index():  # the timed steps' configuration: round-robin over the streams
                for j in range(nstreams):
                    idx.topk(q_dev, args.k, out=outs[j], stream=streams[j])
                return w.Q * nstreams

            def run_scan(ix):
                def f():
                    ix.scan_topk(q_dev, ks, out=(sids, slcp))
                    return w.Q
                return f

            energy["index"] = meter.measure(run_index, es, sync_every=64)
            energy["full_scan"] = meter.measure(run_scan(idx), es, sync_every=1)
            energy["prefix_bucket_scan"] = prefix_bucket_sweep(P, idx, q_dev, args.k, meter, es, idle=iw)
            ji, js = energy["index"].get("j_per_query"), energy["full_scan"].get("j_per_query")
            energy["index_vs_full_scan_energy_ratio"] = round(js / ji, 1) if ji and js else None
            meter.close()
        log(args, f"[bench] energy: {energy}")

    # ---- sensor-fusion stream: N=1M history, 1,000 queries per step (k=5) at a
    # 4,000 Hz target, that step's 1,000 readings appended every 1,000 steps
    sensor = None
    if args.sensor_steps > 0:
        from paper_2602_04936_amd import serve
        st = synth.SensorStream(seed=1005)
        hist = np.concatenate(list(st.steps(1000)), axis=0)
        sidx = P.Index(hist, synth.SensorStream.V)
        # room for every append of both runs below, so that no append allocates
        sidx.reserve(sidx.N + 2 * (args.sensor_steps // 1000 + 1) * st.S)

        def append(index, batch):
            index.append(batch)
            return index

        rep = serve.run_step_stream(sidx, st.steps(args.sensor_steps), rate_hz=4000.0, k=5, append_every=1000,
                                    append=append)
        rep["final_rows"] = rep.pop("index").N
        rep["append_mode"] = "lcp_index_append (sorted merge into the second sorted copy, room reserved beforehand)"
        rep["append_ms_median"] = round(float(np.median(rep["append_ms"])), 3) if rep["append_ms"] else None
        # the same loop unpaced: every step is released when the previous one is done
        un = serve.run_step_stream(sidx, st.steps(args.sensor_steps), rate_hz=None, k=5, append_every=1000,
                                   append=append)
        un.pop("index")
        rep["unpaced"] = {key: un[key] for key in ("steps", "achieved_hz", "p50_step_ms", "p99_step_ms",
                                                   "max_step_ms", "appends", "append_ms")}
        sidx.close()
        sensor = rep
        log(args, f"[bench] sensor stream: {sensor}")

    # ---- CPU baseline: the oracle as it is, on a bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, ks, args)
        log(args, f"[bench] cpu baseline: {cpu}")

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib << 20
        a = torch.ones(n, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.bitwise_not(a, out=b)
        torch.cuda.synchronize()
        del a, b
    if args.calib_gather_mib > 0:
        # rows of 64 bytes (16 int32) from a 1 GiB table at random positions:
        # reads n * (64 + 8) bytes (rows and int64 positions), writes n * 64
        table = torch.ones((1 << 30) // 64, 16, dtype=torch.int32, device=dev)
        n = (args.calib_gather_mib << 20) // 64
        pos = torch.randint(0, table.shape[0], (n,), device=dev, generator=torch.Generator(device=dev).manual_seed(7))
        out_g = torch.empty((n, 16), dtype=torch.int32, device=dev)
        for _ in range(3):
            torch.index_select(table, 0, pos, out=out_g)
        torch.cuda.synchronize()
        del table, pos, out_g

    out = {
        "metric": "queries/s at N=2M,L=32,k=10 (index vs full scan); p50/p99 ms at fixed QPS",
        "value": round(qps, 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "inputs_sha256": {"db": synth.sha256_of(w.db), "queries": synth.sha256_of(w.queries),
                          "numpy": np.__version__},
        "config": {"workload": "c3 hierarchy: N=2,000,000 L=32 uint16 V=4096, Q=8192 per step, k=10",
                   "N": w.N, "L": w.L, "V": w.V, "queries_per_step": w.Q, "k": args.k,
                   "path": "index (lcp_topk)", "parallelism": "single GPU",
                   "streams": nstreams},
        "single_stream": {"ms_per_step": round(dt_single * 1e3 / args.steps, 5),
                          "value": round(w.Q * args.steps / dt_single, 1)},
        "event_timed_blocks": {
            "blocks": len(blocks_multi), "steps_per_block": args.steps,
            "ms_per_step": [round(x, 5) for x in blocks_multi],
            "median_value": round(w.Q / (float(np.median(blocks_multi)) * 1e-3), 1),
            "single_stream_ms_per_step": [round(x, 5) for x in blocks_single],
            "single_stream_median_value": round(w.Q / (float(np.median(blocks_single)) * 1e-3), 1)},
        "streams_outputs_identical": same_outputs,
        "roofline": {"kernel": "k_index_query", "bound": "hbm", "achieved": round(idx_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(idx_gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(w.Q, args.k), "traffic_unit": "bytes per launch",
                     "avg_kernel_us": round(k_avg_ms * 1e3, 2), "launches_timed": kn,
                     "algorithmic_bytes_per_query": round(bytes_per_query, 1),
                     "algorithmic_bytes_per_launch": int(idx_bytes),
                     "traffic_over_algorithmic": (round(measured_traffic(w.Q, args.k) / idx_bytes, 3)
                                                  if measured_traffic(w.Q, args.k) else None)},
        "work_shape": shape,
        "scan": {"qps": round(scan_qps, 1), "ms_per_batch": round(sdt * 1e3 / args.scan_steps, 4),
                 "index_speedup": round(qps / scan_qps, 2), "scan_kernel_ms": round(scan_kernel_ms, 4),
                 "merge_kernel_ms": round(m_ms / max(m_n, 1), 4), "query_groups": groups,
                 "hbm_GBps": round(scan_bytes / (scan_kernel_ms * 1e-3) / 1e9, 1),
                 "l2_stream_GBps": round((w.N * plane_bytes * groups + w.Q * row_bytes) / (scan_kernel_ms * 1e-3) / 1e9, 1),
                 "pair_lcp_per_s": round(w.Q * w.N / (scan_kernel_ms * 1e-3), 1),
                 "paths_bit_identical": paths_agree},
        "scan_roofline": {"kernel": "k_scan", "bound": "hbm", "queries": nbw, "query_groups": groups_bw,
                          "bytes_per_launch": int(bw_bytes),
                          "achieved": round(bw_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(bw_gbs / HBM_PEAK_GBS, 4),
                          "avg_kernel_us": round(bw_ms / bw_n * 1e3, 2),
                          "avg_call_us": round(bw_call_us, 2),
                          "cold_kernel_us": round(cold_us, 2), "cold_achieved": round(cold_gbs, 1),
                          "cold_after_write_flush_us": round(cold_w_us, 2),
                          "streaming_reference_torch_sum": stream_reference(w.N * plane_bytes)},
        "large_db": large,
        "bucket_scan": bucket_scan,
        "build_ms": round(build_ms, 2),
        "serving": serving,
        "uneven_batch": uneven,
        "sensor_stream": sensor,
        "energy": energy,
        "parity": parity,
        "cpu_baseline": cpu,
    }
    idx.close()
    print(json.dumps(out), flush=True)


INDEX_KERNEL_SOURCES = ("query_kernels.hip", "device.hpp", "launch.hpp")
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hbm_counters_c3_index_and_scan.md")


def measured_traffic(queries, k):
    """HBM bytes per index-path launch from the committed counter summary, or
    None when the kernel sources changed since the counters were taken (or the
    workload differs)."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    m = re.search(r"traffic k_index_query bytes_per_launch=(\d+) queries=(\d+) k=(\d+) \S+ sha256=([0-9a-f]+)", text)
    if not m or int(m.group(2)) != queries or int(m.group(3)) != k:
        return None
    h = hashlib.sha256()
    for f in INDEX_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2602_04936_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return int(m.group(1)) if h.hexdigest() == m.group(4) else None


TIE_PATHS = ("none", "id_walk", "wave_minima", "bisection", "pruned", "sorted_list")


def work_shape(st, N, k, row_bytes, probes):
    """Per-query work of the index path from lcp_topk_stats rows (c, n_gt,
    tied, tie path): histograms, and the algorithmic bytes per query,
        R + ceil(log2(N+1)) R + (|G_c| + 2) + 4 (n_gt + |tied|) + 8 k,
    with |G_c| = n_gt + |tied|.  At c = 0 the method walks ids instead of the
    tied range (at most k' + 64 probes, no A bytes beyond the inner group), so
    those queries are charged that walk."""
    c, ngt, tied, path = (st[:, i].astype(np.int64) for i in range(4))
    kp = min(k, N)
    walk = c == 0
    a_bytes = np.where(walk, ngt + 2, ngt + tied + 2)
    ids_read = np.where(walk, ngt + np.minimum(tied, kp - ngt + 64), ngt + tied)
    per_q = row_bytes + probes * row_bytes + a_bytes + 4 * ids_read + 8 * k
    edges = [0, 1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192, 16384, 1 << 31]
    return {
        "queries": int(st.shape[0]),
        "c_counts": {str(v): int(n) for v, n in enumerate(np.bincount(c)) if n},
        "n_gt_mean": round(float(ngt.mean()), 2),
        "tied_mean": round(float(tied.mean()), 2),
        "tied_percentiles": {p: int(np.percentile(tied, int(p))) for p in ("50", "90", "99")},
        "tied_max": int(tied.max()),
        "tied_histogram": {"edges": edges, "counts": np.histogram(tied, bins=edges)[0].tolist()},
        "G_c_mean": round(float((ngt + tied).mean()), 2),
        "tie_path_counts": {TIE_PATHS[i]: int(n) for i, n in enumerate(np.bincount(path, minlength=6)) if n},
        "algorithmic_bytes_per_query": float(per_q.mean()),
        "algorithmic_bytes_per_launch": int(per_q.sum()),
    }


def prefix_bucket_sweep(P, idx, q_dev, k, meter=None, seconds=0.0, idle=None):
    """The bucket range scan of section 6.2 (lcp_bucket_scan_topk) over the
    whole batch, one call per depth d = 0, 1, 2: each query scans only the
    sorted rows that share its first d tokens (c3's 16-ary hierarchy gives
    B = 1, 16, 256 buckets).  Per depth: the GPU time of one call (events),
    the mean rows scanned per query and the queries whose bucket is empty
    (from the call's bucket bounds), and with a meter J/query, the share above
    the idle draw and the query rate under the meter."""
    import torch
    Q = int(q_dev.shape[0])
    o = (torch.empty(Q * k, dtype=torch.int32, device=q_dev.device),
         torch.empty(Q * k, dtype=torch.int32, device=q_dev.device))
    out = {}
    for d in (0, 1, 2):
        _, b = idx.bucket_scan_topk(q_dev, k, d, out=o, bounds=True)  # the first call lays out the sorted prefixes
        torch.cuda.synchronize()
        rows = (b[:, 1] - b[:, 0]).to(torch.float64)
        buckets = int(torch.unique(b[rows > 0, 0]).numel())
        reps = 4 if d == 0 else 20
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            idx.bucket_scan_topk(q_dev, k, d, out=o)
        e1.record()
        torch.cuda.synchronize()
        gpu_ms = e0.elapsed_time(e1) / reps
        # bytes a row the scan streams: key words 0-1 (8) until the prefix covers a whole word, then one word (4)
        per_row = 8 if d * idx.token_bytes < 4 else 4
        streamed = float(rows.sum()) * per_row
        rec = {"depth": d, "buckets_with_queries": buckets, "queries": Q,
               "mean_rows_scanned": round(float(rows.mean()), 1), "empty_bucket_queries": int((rows == 0).sum()),
               "gpu_ms_per_batch": round(gpu_ms, 4), "gpu_qps": round(Q / (gpu_ms * 1e-3), 1),
               "plane_bytes_per_row": per_row, "streamed_GBps": round(streamed / (gpu_ms * 1e-3) / 1e9, 1)}
        if meter is not None:
            def run():
                idx.bucket_scan_topk(q_dev, k, d, out=o)
                return Q

            rep = meter.measure(run, seconds, sync_every=8)
            above = None
            if idle is not None and rep.get("watts") and rep.get("queries_per_s"):
                above = (rep["watts"] - idle) / rep["queries_per_s"]
            rec.update({"j_per_query": rep.get("j_per_query"), "j_per_query_above_idle": above,
                        "watts": rep.get("watts"), "queries_per_s": rep.get("queries_per_s")})
        out[str(16 ** d)] = rec
    return out


def served_check(idx, reqs, db, n_oracle=40):
    """Served answers (k uniform on [1, 100]) against the same requests answered
    in one eager batch, and a spread sample of requests against the C oracle."""
    import torch
    qs = np.concatenate([r.queries for r in reqs])
    ks = np.concatenate([np.full(r.b, r.k, np.int32) for r in reqs])
    res = idx.topk(qs, ks)
    torch.cuda.synchronize()
    bi, bl = res.ids.cpu().numpy(), res.lcps.cpu().numpy()
    got_i = np.concatenate([r.ids.reshape(-1) for r in reqs])
    got_l = np.concatenate([r.lcps.reshape(-1) for r in reqs])
    out = {"results_match_batch_run": bool((got_i == bi).all() and (got_l == bl).all())}
    try:
        import oracle
        pick = sorted(set(np.linspace(0, len(reqs) - 1, min(n_oracle, len(reqs))).astype(int).tolist()))
        sq = np.concatenate([reqs[i].queries for i in pick])
        sk = np.concatenate([np.full(reqs[i].b, reqs[i].k, np.int32) for i in pick])
        wi, wl, _ = oracle.c_topk(db, sq, sk)
        gi = np.concatenate([reqs[i].ids.reshape(-1) for i in pick])
        gl = np.concatenate([reqs[i].lcps.reshape(-1) for i in pick])
        out["oracle_checked_requests"] = len(pick)
        out["oracle_bit_exact"] = bool((gi == wi).all() and (gl == wl).all())
    except Exception as e:  # the oracle is a test dependency; report, do not fail the bench
        out["oracle_error"] = repr(e)
    return out


def served_match(reqs, ref, Q):
    """Every served answer equals the same query's answer in the batch run."""
    ref_ids, ref_lcp = ref
    pos = 0
    for r in sorted(reqs, key=lambda r: r.rid):
        if r.ids is None:
            return False
        sel = (pos + np.arange(r.b)) % Q
        pos = (pos + r.b) % Q
        if not ((r.ids == ref_ids[sel]).all() and (r.lcps == ref_lcp[sel]).all()):
            return False
    return True


def cpu_baseline(w, ks, args):
    import numpy as np

    import oracle
    os.environ.setdefault("OMP_PROC_BIND", "close")
    threads = int(oracle.native_lib().oracle_threads(0))
    # calibrate on a small slice, then run a sample sized to about --cpu-seconds;
    # the reported rate is the median of three runs of that sample
    probe = 64
    t = time.perf_counter()
    oracle.c_topk(w.db, w.queries[:probe], ks[:probe], native=True)
    per_q = (time.perf_counter() - t) / probe
    n = int(min(w.Q, max(probe, args.cpu_seconds / 3 / max(per_q, 1e-9))))
    sel = np.arange(n)
    runs = []
    for _ in range(3):
        t = time.perf_counter()
        oracle.c_topk(w.db, w.queries[sel], ks[sel], native=True)
        runs.append(time.perf_counter() - t)
    el = float(np.median(runs))
    return {"value": round(n / el, 2), "unit": "queries/s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": f"first {n} of the {w.Q} bench queries against all N={w.N} rows, k={args.k}, "
                      f"C brute force (oracle/cpu_topk.c built -O3 -march=native on this host, OpenMP over "
                      f"queries, OMP_PROC_BIND={os.environ.get('OMP_PROC_BIND')}), median of 3 runs "
                      f"({', '.join(f'{x:.2f}' for x in runs)} s)"}


def cpu_model():
    """Host processor as /proc/cpuinfo and the scheduler describe it."""
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" in line:
                    key, val = (x.strip() for x in line.split(":", 1))
                    if key in ("model name", "cpu family", "model", "stepping", "cpu MHz") and key not in info:
                        info[key] = val
                    if key == "flags" and "flags" not in info:
                        info["flags"] = " ".join(x for x in val.split() if x in ("avx2", "avx512f", "avx512bw"))
    except OSError:
        pass
    info["logical_cpus_visible"] = os.cpu_count()
    try:
        info["cpus_allowed"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    return info


if __name__ == "__main__":
    main()
