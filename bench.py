"""Benchmark: sliding-window streaming IVF on one MI355X.

Workload (default): the sliding-window plain FP32 configuration - a window of
1,000,000 vectors, d=128, integer values 0..255 stored as fp32, 1,024 lists
(k-means centroids), slabs of 64; each step inserts 10,000 new vectors,
searches 10,000 queries (nprobe 32, k 10) and evicts the oldest 10,000
(the paper's insert -> search -> delete loop).  All inputs are generated on
the host, copied to HBM before timing, and synthetic (the paper's datasets are
not available).

Prints one JSON line.  value = queries answered per second of window-step
time (every step also inserts and deletes 10,000 vectors); per-operation
device rates, step-latency percentiles, recall@10, the roofline of the scan
kernel and the CPU oracle's rate on a bounded sample are reported beside it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 VALU peak with packed FP32 off: 256 CUs x 4 SIMD x 16 lanes x 2 flop
# (fma) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def recorded_traffic():
    """DRAM bytes per scan launch from the committed counter summary, or None
    when the scan source changed since the counters were taken."""
    import hashlib
    prof = os.path.join(ROOT, "profiles", "k_scan_window_1M.md")
    src = os.path.join(ROOT, "paper_2601_11808_amd", "csrc", "search.hip")
    try:
        kv = dict(l.split(": ", 1) for l in open(prof).read().splitlines() if l.startswith(("traffic_", "search_hip")))
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != kv["search_hip_sha256"].strip():
            return None
        return int(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="window", choices=["window", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--recall-queries", type=int, default=1000)
    ap.add_argument("--no-sweep", action="store_true", help="skip the nprobe / recall sweep")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (scale for DRAM byte counters)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def exact_topk(xw, idw, q, k):
    """Exact squared-L2 top-k (float64) of q against the window, ties by id."""
    xd = xw.astype(np.float64)
    x2 = (xd * xd).sum(1)
    out = np.empty((q.shape[0], k), np.int64)
    for s in range(0, q.shape[0], 64):
        qq = q[s:s + 64].astype(np.float64)
        dd = x2[None, :] - 2.0 * (qq @ xd.T) + (qq * qq).sum(1)[:, None]
        part = np.argpartition(dd, k, axis=1)[:, :k + 8]
        for i in range(qq.shape[0]):
            c = part[i]
            o = np.lexsort((idw[c], dd[i, c]))[:k]
            out[s + i] = idw[c[o]]
    return out


def cpu_baseline(w, x, ids, q, batches, nprobe, k, n_sample_q):
    """The CPU oracle on a bounded sample of the same workload: one window
    step (insert 10k, search a query sample, delete 10k) on the full
    window; the search time is scaled to the full query batch."""
    import oracle
    ix = oracle.OracleIndex(w.dim, w.nlist, w.centroids, w.metric, w.slab, 1 << 26, ids.shape[0] + 4 * w.batch)
    t0 = time.time()
    assert ix.add(x, ids) == 0
    build_s = time.time() - t0
    xb, idb, old = batches
    t0 = time.time()
    assert ix.add(xb, idb) == 0
    t_add = time.time() - t0
    t0 = time.time()
    st, _, _ = ix.search(q[:n_sample_q], k, nprobe)
    t_search = time.time() - t0
    t0 = time.time()
    st, nr = ix.remove(old)
    t_rm = time.time() - t0
    step_s = t_add + t_search * (q.shape[0] / n_sample_q) + t_rm
    ix.close()
    return {
        "value": q.shape[0] / step_s, "unit": "queries/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": (f"one window step on the full {ids.shape[0]}-vector window: insert {xb.shape[0]} "
                   f"({t_add:.2f} s), search {n_sample_q} of {q.shape[0]} queries ({t_search:.2f} s, scaled "
                   f"x{q.shape[0] / n_sample_q:.0f}), delete {old.shape[0]} ({t_rm:.3f} s); "
                   f"untimed window build {build_s:.1f} s"),
        "insert_vec_per_s": xb.shape[0] / t_add, "delete_vec_per_s": old.shape[0] / max(t_rm, 1e-9),
    }


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: every GPU box here has a single MI355X, so --gpus must be 1 "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2601_11808_amd as sivf
    import workloads

    if not os.path.exists(sivf.LIB_PATH):
        raise SystemExit("libsivf.so is not built: run python -c 'import __graft_entry__ as g; g.build()'")
    dev = torch.device("cuda:0")
    t0 = time.time()
    w = workloads.window() if a.workload == "window" else workloads.tiny()
    x, ids = w.base()
    q = w.queries()
    B, nq, k, nprobe = w.batch, q.shape[0], w.k, w.nprobe
    T = a.warmup + a.steps
    log(f"[bench] workload {w.name}: N={w.n_base} d={w.dim} nlist={w.nlist} C={w.slab} B={B} nq={nq} "
        f"(generated in {time.time() - t0:.1f} s)")
    num_slabs = int(1.15 * (w.n_base + 2 * B) / w.slab) + w.nlist
    id_cap = w.n_base + B * (T + a.steps + 2)   # timed loop, then as many graph-mode steps
    chunk = 65536
    ix = sivf.Index(w.dim, w.nlist, w.centroids, metric=w.metric, slab_capacity=w.slab, num_slabs=num_slabs,
                    id_capacity=id_cap, max_batch=max(chunk, B), max_queries=nq, max_k=16,
                    max_nprobe=max(128, nprobe), device="cuda:0")
    log(f"[bench] workspace {ix.workspace_bytes / 2**30:.2f} GiB")
    # bulk load (device time of the whole load)
    xd = torch.from_numpy(x).to(dev)
    idd = torch.from_numpy(ids).to(dev)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for s in range(0, x.shape[0], chunk):
        ix.add(xd[s:s + chunk], idd[s:s + chunk])
    e1.record()
    assert ix.sync() == 0
    bulk_ms = e0.elapsed_time(e1)
    log(f"[bench] bulk load {x.shape[0]} vectors: {bulk_ms:.1f} ms ({x.shape[0] / bulk_ms * 1e3 / 1e6:.2f} M vec/s)")
    # stream batches, resident in HBM before timing
    bx, bi, bo = [], [], []
    for t in range(1, T + 1):
        xb, idb = w.stream_batch(t)
        bx.append(torch.from_numpy(xb).to(dev))
        bi.append(torch.from_numpy(idb).to(dev))
        bo.append(torch.from_numpy(w.oldest_ids(t)).to(dev))
    qd = torch.from_numpy(q).to(dev)
    dist = torch.empty((nq, k), dtype=torch.float32, device=dev)
    lab = torch.empty((nq, k), dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    for t in range(a.warmup):
        ix.step(bx[t], bi[t], qd, k, nprobe, bo[t], out=(dist, lab))
    assert ix.sync() == 0
    ix.profile_read()
    ix.profile(True)
    step_ms = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    for t in range(a.warmup, T):
        ts = time.perf_counter()
        ix.step(bx[t], bi[t], qd, k, nprobe, bo[t], out=(dist, lab))
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
    elapsed = time.perf_counter() - t_all
    prof = ix.profile_read()
    ix.profile(False)
    assert ix.sync() == 0
    # scan roofline: distance evaluations of one search = sum over (query,
    # probe) of the probed list's length; 3 flops per dimension (sub + fma)
    probes = ix.probe(qd, nprobe).cpu().numpy()
    d = ix.dump()   # window state at the end of the timed region
    evals = int(d["list_len"].astype(np.int64)[probes[probes >= 0]].sum())
    scan_ms = prof["scan"][0] / max(prof["scan"][1], 1)
    log(f"[bench] {a.steps} steps in {elapsed:.3f} s; device ms per class: "
        + ", ".join(f"{kk}={v[0] / max(v[1], 1):.3f}" for kk, v in prof.items()))

    # graph mode: the same step captured once and replayed on refilled buffers
    T2 = T + a.steps
    gx = torch.empty_like(bx[0])
    gi = torch.empty_like(bi[0])
    go = torch.empty_like(bo[0])
    nrem = torch.zeros(1, dtype=torch.int64, device=dev)
    g = ix.step_graph(gx, gi, qd, k, nprobe, go, dist, lab, nrem)
    gsteps = []
    for t in range(T, T2):
        xb, idb = w.stream_batch(t + 1)
        bxt, bit = torch.from_numpy(xb).to(dev), torch.from_numpy(idb).to(dev)
        bot = torch.from_numpy(w.oldest_ids(t + 1)).to(dev)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        gx.copy_(bxt)
        gi.copy_(bit)
        go.copy_(bot)
        g.launch()
        torch.cuda.synchronize()
        gsteps.append((time.perf_counter() - ts) * 1e3)
    g.close()
    assert ix.sync() == 0
    gsm = np.sort(np.array(gsteps))
    log(f"[bench] graph steps: p50 {np.percentile(gsm, 50):.3f} ms, p99 {np.percentile(gsm, 99):.3f} ms")

    # recall@10 and the nprobe sweep on the final window (base ids >= B*T2
    # plus batches 1..T2) against exact kNN (float64)
    nrq = min(a.recall_queries, nq)
    keep = ids >= B * T2
    xw = np.concatenate([x[keep]] + [w.stream_batch(t)[0] for t in range(1, T2 + 1)])
    idw = np.concatenate([ids[keep]] + [w.stream_batch(t)[1] for t in range(1, T2 + 1)])
    gt = exact_topk(xw, idw, q[:nrq], k)

    def recall_of(labels):
        return float(np.mean([len(set(gt[i]) & set(labels[i])) / k for i in range(nrq)]))

    sweep = []
    ix.profile(True)
    for npb in ([1, 2, 4, 8, 16, 32, 64] if not a.no_sweep else [nprobe]):
        ix.search(qd, k, npb, out=(dist, lab))
        ix.sync()
        ix.profile_read()
        for _ in range(3):
            ix.search(qd, k, npb, out=(dist, lab))
        pr = ix.profile_read()
        sms = pr["search"][0] / max(pr["search"][1], 1)
        sweep.append({"nprobe": npb, "recall_at_10": round(recall_of(lab.cpu().numpy()), 4),
                      "search_qps": round(nq / (sms * 1e-3), 1)})
    ix.profile(False)
    recall = [r for r in sweep if r["nprobe"] == nprobe][0]["recall_at_10"]
    ok95 = [r for r in sweep if r["recall_at_10"] >= 0.95]
    best95 = max(ok95, key=lambda r: r["search_qps"]) if ok95 else None
    log(f"[bench] recall@{k} at nprobe {nprobe}: {recall:.4f}; sweep {sweep}")

    copy_info = None
    if a.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        copy_info = {"bytes_read": nbytes, "bytes_written": nbytes}
        del src, dst

    flops = evals * 3.0 * w.dim
    achieved = flops / (scan_ms * 1e-3) / 1e12
    # per-operation device rates
    add_ms = prof["add"][0] / max(prof["add"][1], 1)
    rm_ms = prof["remove"][0] / max(prof["remove"][1], 1)
    se_ms = prof["search"][0] / max(prof["search"][1], 1)
    sm = np.sort(np.array(step_ms))
    res = {
        "metric": "insert/delete vectors/s; search QPS at recall@10>=0.95; p99 window-step ms",
        "value": round(nq * a.steps / elapsed, 1),
        "unit": "queries/s (window step: +10k insert, 10k-query search, -10k delete)",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(elapsed / a.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: sliding window N={w.n_base}, d={w.dim}, nlist={w.nlist}, slab={w.slab}, "
                               f"+{B}/-{B} per step, {nq} queries, nprobe={nprobe}, k={k}, L2",
                   "global_batch": nq, "parallelism": "single GPU"},
        "recall_at_10": recall,
        "qps_at_recall95": best95,
        "nprobe_sweep": sweep,
        "graph_p50_step_ms": round(float(np.percentile(gsm, 50)), 4),
        "graph_p99_step_ms": round(float(np.percentile(gsm, 99)), 4),
        "search_qps": round(nq / (se_ms * 1e-3), 1),
        "insert_vec_per_s": round(B / (add_ms * 1e-3), 1),
        "delete_vec_per_s": round(B / (rm_ms * 1e-3), 1),
        "bulk_insert_vec_per_s": round(x.shape[0] / (bulk_ms * 1e-3), 1),
        "p50_step_ms": round(float(np.percentile(sm, 50)), 4),
        "p99_step_ms": round(float(np.percentile(sm, 99)), 4),
        "max_step_ms": round(float(sm[-1]), 4),
        "device_ms": {kk: round(v[0] / max(v[1], 1), 4) for kk, v in prof.items()},
        "roofline": {"bound": "alu", "kernel": "k_scan", "achieved": round(achieved, 3),
                     "peak": round(ALU_PEAK_TFLOPS, 2), "unit": "TFLOP/s", "frac": round(achieved / ALU_PEAK_TFLOPS, 4),
                     "traffic": recorded_traffic() if a.workload == "window" else None,
                     "traffic_unit": "bytes per launch (DRAM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "evals_per_launch": evals, "flops_per_eval": 3 * w.dim,
                     "avg_launch_ms": round(scan_ms, 4)},
    }
    if not a.no_cpu_baseline:
        t0 = time.time()
        xb, idb = w.stream_batch(1)
        res["cpu_baseline"] = cpu_baseline(w, x, ids, q, (xb, idb, w.oldest_ids(1)), nprobe, k,
                                           n_sample_q=200 if a.workload == "window" else nq)
        log(f"[bench] cpu baseline in {time.time() - t0:.1f} s")
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
