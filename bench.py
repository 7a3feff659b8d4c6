#!/usr/bin/env python3
"""Benchmark of the synchronous parallel Louvain hot path on one MI355X.

One step = the whole method on one resident synthetic graph: ingest from
device buffers (validation of offsets and column range, weighted degrees),
vertex following, Jones-Plassmann coloring of the early phases, the
synchronous local-moving sweeps with community-degree updates and exact
modularity, threshold cycling, and graph rebuilding between phases.

Printed value: local-move GTEPS = CSR entries gathered by the sweeps of the
iterations of a step (look-ahead sweeps that only measure Q are left out) /
wall time of the step (so coloring, rebuilding and ingest count against it);
ms_per_step is the time to converge with the CSR resident in HBM, and
time_to_converge_incl_h2d_ms the same from the host CSR.  The roofline
object is for the sweep kernel with the largest device time in the bandwidth
run (plain synchronous sweeps over the same graph: no colour classes), from
HIP events recorded by the library around every launch on its stream during
an untimed step; roofline_timed_config gives the same for the timed
configuration.  The same line carries the batched form (4,096 SBMs in one
batched run, against one-at-a-time runs) and the served form (a job mix under
Poisson arrivals: capacity, p50/p99 latency), each output checked against the
oracle's stored results; --form batched and --form served print those alone.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth


def workload(name):
    from paper_1410_1237_amd import graphs as G
    if name == "rmat_s24":
        return G.rmat24(), "R-MAT scale 24, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), unit weights, seed 3"
    if name == "rmat_s20":
        return G.rmat20(), "R-MAT scale 20, edge factor 16, (a,b,c,d)=(0.57,0.19,0.19,0.05), unit weights, seed 2"
    if name == "chunglu_8m":
        return G.chung_lu_8m(), "Chung-Lu, 8M vertices, 100M edges, exponent 2.1, max expected degree 50,000, weights U[1,100]"
    if name == "sbm_n1000":
        return G.sbm_1000(), "planted SBM 1,000 vertices, 10 blocks, p_in 0.10, p_out 0.002"
    raise SystemExit(f"unknown workload {name}")


HEURISTICS = {
    "full": dict(vf=1, color=1),               # VF + coloring + threshold cycling (1e-2 colored, 1e-6 final)
    "plain": dict(),                            # minimum-label synchronous sweeps only, theta 1e-6
}


def kernel_source_digest():
    h = hashlib.sha256()
    for f in ("sweep.hip", "lv.h"):
        with open(os.path.join(ROOT, "paper_1410_1237_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, wl, mode):
    """Per-launch HBM traffic of the dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            data = json.load(f)
        rec = data.get(f"{kernel}|{wl}|{mode}")
        if not rec or rec.get("source_digest") != kernel_source_digest():
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def cpu_info():
    """The host CPU model (from /proc/cpuinfo) and its logical core count."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model or platform.processor() or platform.machine(), "nproc": os.cpu_count()}


# sample graphs for the oracle's time to converge: the benched family at a
# size the serial oracle finishes in seconds
CPU_SAMPLES = {
    "rmat_s24": ("rmat_scale(20, 3)", lambda G: G.rmat_scale(20, 3)),
    "rmat_s20": ("rmat_scale(18, 2)", lambda G: G.rmat_scale(18, 2)),
    "chunglu_8m": ("chung_lu(500000, 2.1, 12500, 1.25e7, 6250000, wmax=100, seed=4)",
                   lambda G: G.chung_lu(500_000, 2.1, 12_500.0, 1.25e7, 6_250_000, wmax=100, seed=4)),
    "sbm_n1000": ("sbm_1000()", lambda G: G.sbm_1000()),
}


def cpu_baseline(workload_name, heuristics):
    """The serial oracle's time to converge, on one host core, on a smaller
    graph of the benched family with the same heuristics; GTEPS on the
    library's formula (CSR entries of every iteration's sweep / time).  The
    oracle's time on the full benched graph, where its golden record holds
    it, is reported beside it (measured when the golden was written)."""
    import oracle
    from paper_1410_1237_amd import graphs as G
    desc, make = CPU_SAMPLES[workload_name]
    g = make(G)
    O = oracle.default()
    t0 = time.time()
    r = O.run(g, oracle.Params(**HEURISTICS[heuristics]))
    dt = time.time() - t0
    entries = sum(p.iterations * p.nnz for p in r.phases)
    out = {"value": round(entries / dt / 1e9, 6), "unit": "GTEPS", "cores": 1, "kind": "oracle",
           "sample": f"serial oracle run to convergence on {desc} (n={g.n}, nnz={g.nnz}), heuristics "
                     f"{heuristics}: {len(r.phases)} phases, {entries} CSR entries swept in {dt:.1f} s on one core",
           "time_to_converge_s": round(dt, 2)}
    golden = os.path.join(ROOT, "tests", "golden", f"{workload_name}_{heuristics}.json")
    if os.path.exists(golden):
        with open(golden) as f:
            rec = json.load(f)
        out["full_workload_time_to_converge_s"] = rec.get("oracle_seconds")
        out["full_workload_note"] = ("the same oracle on the full benched graph, one core, measured when the "
                                     "golden record was written (not in this run)")
    out.update(cpu_info())
    return out


def _gen_many(fn, idx, threads):
    """Generates graphs fn(i) for i in idx on a thread pool (the generator
    releases the GIL)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, idx))


def _host_threads():
    return max(1, min(16, os.cpu_count() or 1))


def cpu_baseline_graphs(graphs, params, seconds_target=15.0, max_n=None):
    """The oracle's graphs/s: independent graphs of the sample spread over
    the host cores (still serial per graph), until about seconds_target;
    max_n leaves out graphs above that many vertices (one of those alone can
    take minutes on one core), which the sample then states."""
    import concurrent.futures as cf
    import oracle
    O = oracle.default()
    P = oracle.Params(**params)
    threads = _host_threads()
    if max_n is not None:
        graphs = [g for g in graphs if g.n <= max_n]
    done, t0 = 0, time.time()
    it = iter(graphs)
    with cf.ThreadPoolExecutor(max_workers=threads) as ex:
        running = set()
        for g in it:
            running.add(ex.submit(O.run, g, P))
            if len(running) >= threads:
                fin, running = cf.wait(running, return_when=cf.FIRST_COMPLETED)
                done += len(fin)
                if time.time() - t0 > seconds_target:
                    break
        fin, _ = cf.wait(running)
        done += len(fin)
    dt = time.time() - t0
    only = f" (jobs of at most {max_n} vertices)" if max_n is not None else ""
    out = {"value": round(done / dt, 2), "unit": "graphs/s", "cores": threads, "kind": "oracle",
           "sample": f"{done} graphs of the same mix{only}, serial oracle per graph, {threads} threads, {dt:.1f} s"}
    out.update(cpu_info())
    return out


def load_mix_golden(mix, count):
    """Per-graph oracle records of a mix (tests/golden), keyed by graph index."""
    path = os.path.join(ROOT, "tests", "golden", f"{mix}_x{count}_plain.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    return {r[0]: r for r in data["graphs"]}


def labels_sha16(labels):
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<i4").tobytes()).hexdigest()[:16]


def bench_batched(args):
    """Many planted-partition SBMs of uneven sizes in one disjoint-union CSR,
    run by the batched form; against the same graphs run one at a time."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")  # one generator thread per graph
    import numpy as np
    import torch
    from paper_1410_1237_amd import graphs as G
    from paper_1410_1237_amd import louvain as L

    t = time.time()
    gs = _gen_many(G.batch_sbm, range(args.graphs), _host_threads())
    goff, off, col, w = L.union_csr(gs)
    print(f"[bench] batched: {len(gs)} SBMs, n={int(goff[-1])} nnz={len(col)} generated in {time.time() - t:.1f}s",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    d_off = torch.from_numpy(off).to(dev)
    d_col = torch.from_numpy(col).to(dev)
    d_w = torch.from_numpy(w).to(dev) if w is not None else None
    labels = torch.empty(int(goff[-1]), dtype=torch.int32, device=dev)
    p = L.params()

    def step():
        b = L.Batch.from_union(goff, d_off, d_col, d_w)
        res = b.run(p, labels=labels, stats=False)
        b.close()
        return res

    for i in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        res = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gps = args.steps * len(gs) / elapsed

    # one at a time: sequential louvain_run per graph on one stream, CSR resident
    sample = list(range(0, len(gs), max(1, len(gs) // args.solo_sample)))[:args.solo_sample]
    dev_graphs = [(torch.from_numpy(gs[i].offsets).to(dev), torch.from_numpy(gs[i].cols).to(dev),
                   torch.from_numpy(gs[i].weights).to(dev) if gs[i].weights is not None else None) for i in sample]
    solo_labels = torch.empty(max(g.n for g in gs), dtype=torch.int32, device=dev)

    def solo(j):
        o, c, ww = dev_graphs[j]
        h = L.Graph.from_tensors(o, c, ww, validate=False)
        r = h.run(p, labels=solo_labels[:o.numel() - 1])
        h.close()
        return r

    solo(0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    solo_res = [solo(j) for j in range(len(sample))]
    torch.cuda.synchronize()
    solo_gps = len(sample) / (time.perf_counter() - t1)
    for j, i in enumerate(sample):  # identical outputs (exact modularity, communities)
        assert (solo_res[j].N, solo_res[j].D, solo_res[j].K) == (res[i].N, res[i].D, res[i].K), f"graph {i}"
    # every graph against the oracle's stored result (labels, K, exact Q)
    gold = load_mix_golden("batch_sbm", len(gs))
    checked = 0
    if gold is not None:
        lab = labels.cpu().numpy()
        for i, r in enumerate(res):
            rec = gold[i]
            assert (r.K, str(r.N), str(r.D)) == (rec[3], rec[4], rec[5]), f"graph {i} differs from the oracle"
            assert labels_sha16(lab[goff[i]:goff[i + 1]]) == rec[8], f"graph {i} labels differ from the oracle"
            checked += 1
    sizes = np.array([g.n for g in gs])
    out = {
        "metric": "batched graphs/s", "value": round(gps, 2), "unit": "graphs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"batch_sbm x{len(gs)}", "graphs": len(gs), "n_total": int(goff[-1]),
                   "nnz_total": int(len(col)), "n_min": int(sizes.min()), "n_median": int(np.median(sizes)),
                   "n_max": int(sizes.max()), "heuristics": "plain"},
        "one_at_a_time": {"value": round(solo_gps, 2), "unit": "graphs/s",
                          "sample": f"{len(sample)} graphs (every {max(1, len(gs) // args.solo_sample)}th), "
                                    "sequential louvain_run on one stream, CSR resident",
                          "batched_over_one_at_a_time": round(gps / solo_gps, 2)},
        "oracle_checked_graphs": checked,
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_graphs(gs, {}, args.cpu_seconds),
    }
    return out


def bench_served(args):
    """The request loop: a job mix of SBM and R-MAT graphs from 1e3 to 2e6
    vertices.  First all jobs at once (capacity), then Poisson arrivals at 80 %
    of that capacity: p50 / p99 latency (completion - submission) and
    completed graphs/s."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    import numpy as np
    import torch
    from paper_1410_1237_amd import graphs as G
    from paper_1410_1237_amd import louvain as L

    t = time.time()
    jobs = _gen_many(G.served_job, range(args.jobs), _host_threads())
    tot_n, tot_e = sum(g.n for g in jobs), sum(g.nnz for g in jobs)
    print(f"[bench] served: {len(jobs)} jobs, n={tot_n} nnz={tot_e} generated in {time.time() - t:.1f}s",
          file=sys.stderr, flush=True)
    p = L.params()
    torch.cuda.init()

    def run(rate):
        s = L.Server(p, solo_min_vertices=args.solo_min_vertices, max_inflight_batches=args.max_inflight)
        rng = np.random.default_rng(6)
        gaps = rng.exponential(1.0 / rate, size=len(jobs)) if rate else np.zeros(len(jobs))
        t0 = time.perf_counter()
        due = 0.0
        tickets = []
        for g, gap in zip(jobs, gaps):
            due += gap
            wait = due - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            tickets.append(s.submit(g, borrow=True))  # the job arrays outlive the server
        s.wait_all()
        infos = [s.poll(tk, labels=True) for tk in tickets]
        s.close()
        assert all(i.status == L.OK for i in infos)
        lat = np.array([i.t_done - i.t_submit for i in infos])
        span = max(i.t_done for i in infos) - min(i.t_submit for i in infos)
        return infos, lat, span

    run(0)  # warm-up
    infos, lat, span = run(0)
    capacity = len(jobs) / span
    rate = 0.8 * capacity
    infos, lat, span = run(rate)
    # one at a time: every job through louvain_init_csr (host CSR, as the
    # server receives it) + louvain_run, sequentially on one stream; each
    # result equals the job's result in the mix
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for j, g in enumerate(jobs):
        h = L.Graph.from_csr(g)
        r = h.run(p)
        h.close()
        assert (r.N, r.D, r.K) == (infos[j].N, infos[j].D, infos[j].K), f"job {j}"
    solo_gps = len(jobs) / (time.perf_counter() - t1)
    # every job against the oracle's stored result (labels, K, exact Q)
    gold = load_mix_golden("served", len(jobs))
    checked = 0
    if gold is not None:
        for j, inf in enumerate(infos):
            rec = gold[j]
            assert (inf.K, str(inf.N), str(inf.D)) == (rec[3], rec[4], rec[5]), f"job {j} differs from the oracle"
            assert labels_sha16(inf.labels) == rec[8], f"job {j} labels differ from the oracle"
            checked += 1
    out = {
        "metric": "served graphs/s", "value": round(len(jobs) / span, 2), "unit": "graphs/s", "n_gpus": 1,
        "steps": 1, "warmup": 1, "ms_per_step": round(span * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": f"served_job x{len(jobs)}", "jobs": len(jobs), "n_total": tot_n, "nnz_total": tot_e,
                   "arrivals": "Poisson", "rate_per_s": round(rate, 2), "capacity_per_s": round(capacity, 2),
                   "hbm_budget_bytes": 200 << 30, "heuristics": "plain",
                   "max_inflight_batches": L.louvain_server_config_default().max_inflight_batches
                   if args.max_inflight is None else args.max_inflight,
                   "solo_min_vertices": L.louvain_server_config_default().solo_min_vertices
                   if args.solo_min_vertices is None else args.solo_min_vertices, "submission": "borrowed"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 2),
                       "max": round(float(lat.max()) * 1e3, 2)},
        "batches": len({i.batch_id for i in infos}),
        "latency_split_ms_mean": {
            "queue": round(float(np.mean([i.t_admit - i.t_submit for i in infos])) * 1e3, 2),
            "host_pack": round(float(np.mean([i.t_packed - i.t_admit for i in infos])) * 1e3, 2),
            "to_device_and_check": round(float(np.mean([i.t_ready - i.t_packed for i in infos])) * 1e3, 2),
            "run": round(float(np.mean([i.t_done - i.t_ready for i in infos])) * 1e3, 2)},
        "one_at_a_time": {"value": round(solo_gps, 2), "unit": "graphs/s",
                          "sample": f"all {len(jobs)} jobs, sequential louvain_init_csr (host CSR) + louvain_run",
                          "capacity_over_one_at_a_time": round(capacity / solo_gps, 2)},
        "oracle_checked_jobs": checked,
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_graphs(jobs, {}, args.cpu_seconds,
                                                                             max_n=300_000),
    }
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat_s24")
    ap.add_argument("--heuristics", default="full", choices=sorted(HEURISTICS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled step after the timed ones")
    ap.add_argument("--no-forms", action="store_true",
                    help="single form only: leave out the batched and served figures of the default line")
    ap.add_argument("--form", default="single", choices=["single", "batched", "served"],
                    help="single graph (default); batched: many SBMs in one batched run; served: request loop")
    ap.add_argument("--graphs", type=int, default=4096, help="batched form: graphs in the batch")
    ap.add_argument("--jobs", type=int, default=128, help="served form: jobs")
    ap.add_argument("--max-inflight", type=int, default=None,
                    help="served form: concurrent batches (default: the library's)")
    ap.add_argument("--solo-min-vertices", type=int, default=None,
                    help="served form: jobs this large run alone (default: the library's)")
    ap.add_argument("--solo-sample", type=int, default=256, help="batched form: graphs timed one at a time")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the run, copy a buffer of this many MiB three times (a plain copy kernel of "
                         "known size, to calibrate HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path runs on a single MI355X (sharding across GPUs is "
              "described, not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.form == "batched":
        print(json.dumps(bench_batched(args)))
        return
    if args.form == "served":
        print(json.dumps(bench_served(args)))
        return

    # the batched (4,096 SBMs) and served (job mix) forms first, each in a
    # child process of its own (a fresh device and allocator state), each with
    # its one-at-a-time reference and the oracle's check of every output
    forms = None
    if not args.no_forms:
        def child(form):
            cmd = [sys.executable, os.path.abspath(__file__), "--form", form, "--steps", "3", "--warmup", "1",
                   "--cpu-seconds", str(args.cpu_seconds)]
            if args.no_cpu_baseline:
                cmd.append("--no-cpu-baseline")
            r = subprocess.run(cmd, stdout=subprocess.PIPE, text=True)
            if r.returncode != 0:
                raise SystemExit(f"bench.py --form {form} failed with status {r.returncode}")
            return json.loads(r.stdout.strip().splitlines()[-1])
        forms = (child("batched"), child("served"))

    import numpy as np
    import torch
    from paper_1410_1237_amd import louvain as L

    t_gen = time.time()
    g, desc = workload(args.workload)
    t_gen = time.time() - t_gen
    print(f"[bench] {args.workload}: n={g.n} nnz={g.nnz} generated in {t_gen:.1f}s", file=sys.stderr, flush=True)

    dev = torch.device("cuda:0")
    off = torch.from_numpy(g.offsets).to(dev)
    col = torch.from_numpy(g.cols).to(dev)
    w = torch.from_numpy(g.weights).to(dev) if g.weights is not None else None
    labels = torch.empty(g.n, dtype=torch.int32, device=dev)
    p = L.params(**HEURISTICS[args.heuristics])
    stream = torch.cuda.current_stream()

    def step(params, profile=False):
        gr = L.Graph.from_tensors(off, col, w, validate=False, stream=stream)
        if profile:
            gr.profile(True)
        res = gr.run(params, labels=labels)
        recs = gr.profile_records() if profile else None
        gr.close()
        return res, recs

    for i in range(args.warmup):
        res, _ = step(p)
        print(f"[bench] warmup {i}: {res.ms_total:.1f} ms K={res.K} q={res.q:.6f}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    entries = 0
    results = []
    for i in range(args.steps):
        res, _ = step(p)
        entries += res.sweep_entries
        results.append(res)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    gteps = entries / elapsed / 1e9
    last = results[-1]
    assert all(r.N == last.N and r.K == last.K for r in results), "steps disagree"
    # time to converge from the host CSR (H2D copy of offsets, columns and
    # weights inside the time), one untimed-loop step
    t_h = time.perf_counter()
    gh = L.Graph.from_csr(g, validate=False, stream=stream)
    res_h = gh.run(p, labels=labels)
    gh.close()
    torch.cuda.synchronize()
    ttc_h2d_ms = (time.perf_counter() - t_h) * 1e3
    assert res_h.N == last.N and res_h.K == last.K, "host-ingest step disagrees"

    def profiled(params):
        """One untimed step with HIP events around every launch on the
        library's stream: per-record launches, ms, algorithmic bytes."""
        res, recs = step(params, profile=True)
        out = {}
        for r in recs:
            if r["launches"]:
                out[r["name"]] = {k: r[k] for k in ("launches", "ms", "bytes", "entries")}
        return res, out

    def roofline_of(recs, run):
        sweep = {k: v for k, v in recs.items() if k.startswith("sweep")}
        if not sweep:
            return None
        name, r = max(sweep.items(), key=lambda kv: kv[1]["ms"])
        per_launch = r["bytes"] / r["launches"]
        avg_ms = r["ms"] / r["launches"]
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        tot_ms = sum(v["ms"] for v in sweep.values())
        tot_b = sum(v["bytes"] for v in sweep.values())
        traffic = load_traffic(name, args.workload, run)
        # the counters' bytes over the same launch time: how much of the peak
        # the kernel's actual (line-granular) traffic takes
        rate = traffic / (avg_ms * 1e-3) / 1e9 if traffic else None
        return {"bound": "hbm", "kernel": name, "run": run, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_GBps": round(rate, 1) if rate else None,
                "traffic_frac": round(rate / HBM_PEAK_GBS, 4) if rate else None,
                "launches": r["launches"], "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": round(per_launch),
                "all_sweep_kernels": {"ms": round(tot_ms, 3), "GBps": round(tot_b / (tot_ms * 1e-3) / 1e9, 1),
                                      "frac": round(tot_b / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}}

    kernels, roofline, roofline_timed = {}, None, None
    if not args.no_profile:
        # the bandwidth figure is taken on plain synchronous sweeps (no colour
        # classes), the timed configuration's own dominant kernel beside it
        res_t, recs_t = profiled(p)
        assert res_t.N == last.N and res_t.K == last.K, "profiled step disagrees"
        kernels = {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in recs_t.items()}
        roofline_timed = roofline_of(recs_t, args.heuristics)
        if args.heuristics == "plain":
            roofline = roofline_timed
        else:
            _, recs_p = profiled(L.params(**HEURISTICS["plain"]))
            roofline = roofline_of(recs_p, "plain")

    out = {
        "metric": "local-move GTEPS", "value": round(gteps, 4), "unit": "GTEPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": args.workload, "graph": desc, "n": g.n, "nnz": g.nnz,
                   "heuristics": args.heuristics, "params": {k: getattr(p, k) for k in ("vf", "color", "singlet_rule")},
                   "color_cutoff": p.color_cutoff, "theta_color": [p.theta_color.num, p.theta_color.den],
                   "theta_final": [p.theta_final.num, p.theta_final.den]},
        "time_to_converge_ms": round(ms_per_step, 3),
        "time_to_converge_incl_h2d_ms": round(ttc_h2d_ms, 3),
        "result": {"communities": last.K, "q": last.q, "phases": len(last.phases),
                   "iterations": sum(ph.iterations for ph in last.phases), "n_after_vf": last.n_vf,
                   "sweep_entries": last.sweep_entries, "lookahead_entries": last.lookahead_entries,
                   "phase_shape": [[ph.n, ph.nnz, int(ph.colored), ph.num_colors, ph.iterations] for ph in last.phases]},
        "time_split_ms": {"vf": round(last.ms_vf, 2), "color": round(last.ms_color, 2),
                          "sweep": round(last.ms_sweep, 2), "coarsen": round(last.ms_coarsen, 2)},
        "kernels": kernels,
        "roofline": roofline,
        "roofline_timed_config": roofline_timed,
        "cpu_baseline": None,
    }
    if args.copy_probe_mib:
        nb = args.copy_probe_mib << 20
        src = torch.empty(nb, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nb
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, args.heuristics)
        out["cpu_baseline"]["gpu_over_cpu"] = round(gteps / out["cpu_baseline"]["value"], 1)
    if forms:
        bt, sv = forms
        out["batched"] = {"graphs_per_s": bt["value"], "ms_per_batch": bt["ms_per_step"], "config": bt["config"],
                          "one_at_a_time_graphs_per_s": bt["one_at_a_time"]["value"],
                          "batched_over_one_at_a_time": bt["one_at_a_time"]["batched_over_one_at_a_time"],
                          "oracle_checked_graphs": bt["oracle_checked_graphs"], "cpu_baseline": bt["cpu_baseline"]}
        out["served"] = {"graphs_per_s": sv["value"], "capacity_graphs_per_s": sv["config"]["capacity_per_s"],
                         "rate_per_s": sv["config"]["rate_per_s"], "latency_ms": sv["latency_ms"],
                         "config": sv["config"], "one_at_a_time_graphs_per_s": sv["one_at_a_time"]["value"],
                         "capacity_over_one_at_a_time": sv["one_at_a_time"]["capacity_over_one_at_a_time"],
                         "oracle_checked_jobs": sv["oracle_checked_jobs"], "cpu_baseline": sv["cpu_baseline"]}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
