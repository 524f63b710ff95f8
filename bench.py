"""Exact minimum-cut throughput on one MI355X.

A step is one complete exact solve (every round of the contraction loop:
Padberg-Rinaldi tests, CAPFOREST scans, union-find, contraction, bound
updates, side) of the workload graph, already resident in HBM.  The
workload is a Chung-Lu power-law graph (n = 2^22, exponent 2.5, average
degree 32, unit weights) reduced to its 8-core and largest component.

Prints one JSON line: edges/s (undirected edges of the solved graph divided
by the solve time), the dominant kernel's roofline figures (event-timed on
the launch stream during the timed steps) and the CPU oracle's rate on a
bounded sample of the same workload family.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline():
    """Oracle (sequential NOI, one thread) on a smaller graph of the same
    recipe: Chung-Lu n = 2^19, exponent 2.5, average degree 32, 8-core, LCC."""
    import graphgen as gg
    import oracle
    g = gg.chung_lu_4m_8core(19)
    t0 = time.perf_counter()
    lam, side, rounds = oracle.noi(g, 1)
    dt = time.perf_counter() - t0
    return {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential NOI (O3) full solve of chung_lu n=2^19 8-core LCC "
                      f"(n={g.n}, m={g.m}, lambda={lam}, {rounds} rounds) in {dt:.2f} s"}


def batched_form(steps, warmup, loop=True):
    """The 4096-graph batch (planted clusters, n log-uniform in [64, 8192],
    2-16 clusters, intra degree U[8, 32], 1-4 inter edges per cluster pair,
    weights U[1, 100]) solved as one packed CSR, against a host loop of
    single-graph solves over the same graphs, already resident in HBM."""
    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))["batch_4096"]
    t0 = time.time()
    graphs = [gg.batch_graph(i) for i in range(gold["graphs"])]
    packed, vo, eo = gg.pack(graphs)
    log(f"batch: {len(graphs)} graphs, sum n={packed.n} sum m={packed.m} in {time.time() - t0:.1f}s")
    rp, col, w = mc.to_device(packed, "cuda:0")
    ref = np.asarray(gold["lambdas"], np.int64)
    # the autotuner picks the launch shapes on this batch (untimed)
    t0 = time.perf_counter()
    tuned, tune = mc.tune_batched(rp, col, w, vo, reps=2)
    tune["tuning_s"] = round(time.perf_counter() - t0, 2)
    log(f"batch tuned: threads {tune['sweep_threads']} groups {tune['sweep_groups']} sort tile "
        f"{tune['sort_tile']}: {tune['best_ms']:.1f} ms vs default {tune['default_ms']:.1f} ms "
        f"({tune['candidates']} shapes, {tune['tuning_s']} s)")
    for i in range(warmup):
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, opts=tuned)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, opts=tuned)
    torch.cuda.synchronize()
    dt_packed = (time.perf_counter() - t0) / steps
    packed_ok = bool(np.array_equal(lams, ref))
    s = sides.cpu().numpy()
    src = packed.src()
    cut = np.zeros(len(graphs), np.int64)
    gid = np.repeat(np.arange(len(graphs)), np.diff(vo))
    crossing = s[src] != s[packed.col]
    np.add.at(cut, gid[src[crossing]], packed.w[crossing].astype(np.int64))
    sides_ok = bool(np.array_equal(cut // 2, ref))
    log(f"batch packed: {dt_packed * 1e3:.1f} ms, {st['rounds']} rounds, lambdas equal: {packed_ok}, "
        f"side weights equal: {sides_ok}")
    out = {"graphs": len(graphs), "sum_n": packed.n, "sum_m": packed.m,
           "packed": {"ms": round(dt_packed * 1e3, 2), "edges_per_s": packed.m / dt_packed,
                      "rounds": st["rounds"], "steps": steps},
           "autotune": {k: (round(v, 2) if isinstance(v, float) else v) for k, v in tune.items()},
           "verified": {"lambdas_equal_oracle": packed_ok, "side_weights_equal": sides_ok}}
    if not loop:
        return out
    # the loop: one single-graph solve per graph, same device-resident CSRs
    dev = [mc.to_device(g, "cuda:0") for g in graphs]
    for g in dev[:16]:
        mc.mincut(*g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    looped = [mc.mincut(*g)[0] for g in dev]
    torch.cuda.synchronize()
    dt_loop = time.perf_counter() - t0
    loop_ok = bool(np.array_equal(np.asarray(looped), ref))
    log(f"batch looped: {dt_loop * 1e3:.1f} ms, lambdas equal: {loop_ok}")
    out["looped"] = {"ms": round(dt_loop * 1e3, 2), "edges_per_s": packed.m / dt_loop}
    out["speedup"] = round(dt_loop / dt_packed, 2)
    out["verified"]["lambdas_equal_oracle"] = packed_ok and loop_ok
    return out


def ablation():
    """Scan policies, rounds against time (every variant returns the same
    lambdas): the capped sweeps with ties at the cap batched (default),
    one-pop-at-a-time scans with an LDS hash map (scan_mode 2, small graphs),
    concurrent region scans (Algorithm 1, scan_mode 1, large graphs), and the
    triangle tests (default: from the second round; also without them and
    from the first round); on the 4096-graph batch and the Chung-Lu 2^22
    8-core."""
    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc
    out = {}

    def run(name, f, reps=2):
        f()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            lam, st = f()
        torch.cuda.synchronize()
        out[name] = {"ms": round((time.perf_counter() - t0) / reps * 1e3, 2), "rounds": st["rounds"],
                     "lambda": lam}
        log(f"ablation {name}: {out[name]}")

    graphs = [gg.batch_graph(i) for i in range(4096)]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda:0")

    def batch(**kw):
        def f():
            lams, _, st = mc.mincut_batched(rp, col, w, vo, want_side=False, **kw)
            return int(np.asarray(lams, np.int64).sum()), st
        return f
    run("batch_capped_sweeps", batch())
    run("batch_capped_sweeps_no_triangle_tests", batch(pr_triangle_deg=0))
    run("batch_capped_sweeps_triangle_tests_from_round_1", batch(pr_triangle_deg=-64))
    run("batch_one_pop_scans", batch(scan_mode=2))
    del rp, col, w
    g = gg.chung_lu_4m_8core(22)
    rp, col, w = mc.to_device(g, "cuda:0")

    def single(**kw):
        def f():
            lam, _, st = mc.mincut(rp, col, w, want_side=False, **kw)
            return lam, st
        return f
    run("chung_lu_capped_sweep", single())
    run("chung_lu_region_scans", single(scan_mode=1), reps=1)
    run("chung_lu_one_pop_hashed_small_graphs", single(scan_mode=2))
    return out


def rmat_form(steps):
    """R-MAT scale 24 (2^28 draws, (0.57, 0.19, 0.19, 0.05), multiplicity
    weights), 10-core, largest component, resident in HBM: exact solves."""
    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json"))).get("rmat_24_10core")
    t0 = time.time()
    g = gg.rmat_24_10core()
    log(f"rmat: n={g.n} m={g.m} generated in {time.time() - t0:.1f}s")
    rp, col, w = mc.to_device(g, "cuda:0")
    mc.mincut(rp, col, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lam, side, st = mc.mincut(rp, col, w)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    s = side.cpu().numpy()[: g.n].astype(bool)
    cut = int(g.w[s[g.src()] != s[g.col]].sum()) // 2
    out = {"n": g.n, "m": g.m, "ms": round(dt * 1e3, 3), "edges_per_s": g.m / dt, "rounds": st["rounds"],
           "lambda": lam, "oracle_lambda": gold["lambda"] if gold else None, "side_cut_weight": cut}
    log(f"rmat: {out}")
    return out


def served_form(requests, pool_size, lanes, seed=5):
    """Poisson arrivals of min-cut requests (Chung-Lu, exponent 2.5, average
    degree 16, n log-uniform in [2^10, 2^20], weights in [1, 50], largest
    component) drawn from a pool of generated graphs, served with continuous
    batching.  The capacity is measured closed-loop first; the open-loop
    runs arrive at 0.3 and 0.7 of it.  Latency = submit -> result on the host
    (host CSR in, upload included)."""
    import threading
    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc
    t0 = time.time()
    pool = [gg.served_request(i) for i in range(pool_size)]
    log(f"served: pool of {pool_size} requests, sum n={sum(g.n for g in pool)} "
        f"sum m={sum(g.m for g in pool)} in {time.time() - t0:.1f}s")
    alone = []
    for g in pool:
        rp, col, w = mc.to_device(g, "cuda:0")
        alone.append(mc.mincut(rp, col, w, want_side=False)[0])
    torch.cuda.synchronize()
    rng = np.random.default_rng(seed)
    order = rng.integers(0, pool_size, size=requests)
    mean_m = float(np.mean([pool[i].m for i in order]))

    # one long-lived server for every run; a first pass over the pool lets
    # each lane's buffers grow to their working size
    srv = mc.Server(lanes=lanes)
    warm = [srv.submit(g) for g in sorted(pool, key=lambda g: -g.nnz)]
    for t in warm:
        srv.wait(t, want_side=False)

    def run(rate):
        """rate None: everything submitted at once (closed loop)."""
        lat, ok = [], True
        tickets = [None] * requests
        ready = threading.Semaphore(0)

        def produce():
            gaps = rng.exponential(1.0 / rate, size=requests) if rate else np.zeros(requests)
            start = time.perf_counter()
            due = start
            for k in range(requests):
                due += gaps[k]
                d = due - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[k] = srv.submit(pool[order[k]])
                ready.release()

        t_start = time.perf_counter()
        th = threading.Thread(target=produce)
        th.start()
        for k in range(requests):
            ready.acquire()
            lam, _, l = srv.wait(tickets[k], want_side=False)
            ok = ok and lam == alone[order[k]]
            lat.append(l["total_ms"])
        t_end = time.perf_counter()
        th.join()
        lat = np.asarray(lat)
        span = t_end - t_start
        return {"requests": requests, "span_s": round(span, 3),
                "edges_per_s": float(sum(pool[i].m for i in order) / span),
                "requests_per_s": round(requests / span, 1),
                "p50_ms": round(float(np.percentile(lat, 50)), 3),
                "p99_ms": round(float(np.percentile(lat, 99)), 3),
                "same_as_alone": bool(ok)}

    cap = run(None)
    log(f"served closed loop: {cap}")
    # the same requests as a host loop of single-graph solves, each uploaded
    # from host memory like a served request
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(requests):
        g = pool[order[k]]
        rp, col, w = mc.to_device(g, "cuda:0")
        mc.mincut(rp, col, w)
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    looped = {"span_s": round(loop_s, 3), "edges_per_s": float(sum(pool[i].m for i in order) / loop_s)}
    log(f"looped single solves: {looped}")
    out = {"pool": pool_size, "lanes": lanes, "mean_m": round(mean_m), "closed_loop": cap,
           "looped": looped, "speedup_closed_loop": round(cap["edges_per_s"] / looped["edges_per_s"], 2)}
    for frac in (0.3, 0.7):
        r = run(frac * cap["requests_per_s"])
        r["rate_frac"] = frac
        log(f"served at {frac} of capacity: {r}")
        out[f"at_{frac}"] = r
    srv.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-log2", type=int, default=22)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--workload", choices=["chung_lu", "batched", "served"], default="chung_lu")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-rmat", action="store_true")
    ap.add_argument("--no-approx", action="store_true", help="skip the (2+eps)-approximation runs")
    ap.add_argument("--ablation", action="store_true",
                    help="print scan-policy ablations (rounds against time) instead of the bench line")
    ap.add_argument("--no-loop", action="store_true",
                    help="batched form: skip the loop of single solves (profiling the packed solve alone)")
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--pool", type=int, default=32)
    ap.add_argument("--lanes", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (the reference "
                         "kernel for scaling HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; graphs of the batched and served forms would "
              "shard across GPUs (independent graphs), but no multi-GPU path is implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        log(f"copied {x.numel() * 4} bytes three times")
        return
    if args.workload == "served":
        sv = served_form(args.requests, args.pool, args.lanes)
        out = {"metric": "served exact min-cut edges/s at 0.7 of capacity, p50/p99 latency, 1 GPU",
               "value": sv["at_0.7"]["edges_per_s"], "unit": "edges/s", "n_gpus": 1,
               "steps": args.requests, "warmup": 8, "ms_per_step": sv["at_0.7"]["p50_ms"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
               "data": "synthetic", "config": {"workload": "Poisson stream of Chung-Lu requests", **sv}}
        print(json.dumps(out), flush=True)
        return
    if args.ablation:
        ab = ablation()
        print(json.dumps({"ablation": ab}), flush=True)
        return
    if args.workload == "batched":
        b = batched_form(args.steps, args.warmup, loop=not args.no_loop)
        out = {"metric": "batched exact min-cut edges/s (sum of m / packed solve time) at 1 GPU",
               "value": b["packed"]["edges_per_s"], "unit": "edges/s", "n_gpus": 1,
               "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["packed"]["ms"],
               "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int64",
               "data": "synthetic", "config": {"workload": "batch of 4096 planted-cluster graphs", **b}}
        print(json.dumps(out), flush=True)
        return
    t0 = time.time()
    g = gg.chung_lu_4m_8core(args.n_log2)
    log(f"generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    rp, col, w = mc.to_device(g, "cuda:0")
    stream = torch.cuda.current_stream()

    opts = mc.options()
    for i in range(args.warmup):
        lam, side, st = mc.mincut(rp, col, w, opts=opts)
        log(f"warmup {i}: lambda={lam} rounds={st['rounds']} {st['ms']:.1f} ms "
            f"n_round={st['n_round']}")
    torch.cuda.synchronize()

    topts = mc.options(timing=1)
    mc.timing_reset()
    lams = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        lam, side, st = mc.mincut(rp, col, w, opts=topts)
        lams.append(lam)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1000.0 / args.steps
    value = g.m * args.steps / dt
    classes = mc.timing()
    log("kernel classes: " + ", ".join(f"{c['name']}={c['ms'] / args.steps:.2f}ms"
                                      for c in sorted(classes, key=lambda c: -c["ms"])))

    def rate(c):
        per_launch_s = c["ms"] / 1000.0 / c["launches"]
        per_launch_bytes = c["algo_bytes"] / c["launches"]
        return per_launch_bytes / per_launch_s / 1e9, per_launch_bytes

    dom = max(classes, key=lambda c: c["ms"])
    achieved, dom_bytes = rate(dom)
    # HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE counter runs of
    # this workload (scaled by the same counters on a plain copy), when the
    # summary is present; it is only valid for the build it was taken on
    measured = {}  # class -> counter bytes per launch of its main kernel
    tpath = os.path.join(ROOT, "profiles", f"hbm_traffic_chung_lu_2^{args.n_log2}_8core.txt")
    if os.path.exists(tpath):
        for line in open(tpath):
            f = line.split()
            if len(f) == 7 and f[0] == "traffic":
                measured[f[1]] = int(f[6])
    traffic = measured.get(dom["name"])

    def kernel_entry(c):
        e = {"ms_per_step": round(c["ms"] / args.steps, 3), "GBps": round(rate(c)[0], 1),
             "frac": round(rate(c)[0] / HBM_PEAK_GBS, 4)}
        if c["name"] in measured:
            # counter bytes (not algorithmic) over this run's event time
            e["traffic_GBps"] = round(measured[c["name"]] / (c["ms"] / 1000.0 / c["launches"]) / 1e9, 1)
        return e
    roofline = {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": traffic,
                "kernel": dom["name"], "avg_launch_ms": round(dom["ms"] / dom["launches"], 4),
                "launches_per_step": dom["launches"] / args.steps,
                "algo_bytes_per_launch": dom_bytes,
                "kernels": {c["name"]: kernel_entry(c) for c in sorted(classes, key=lambda c: -c["ms"])[:8]}}

    verified = None
    if not args.no_verify:
        gold_path = os.path.join(ROOT, "tests", "golden", "workloads.json")
        gold = json.load(open(gold_path)).get("chung_lu_4m_8core") if args.n_log2 == 22 else None
        s = side.cpu().numpy()[: g.n].astype(bool)
        src = g.src()
        cut = int(g.w[s[src] != s[g.col]].sum()) // 2
        verified = {"lambda": lams[0], "all_steps_equal": len(set(lams)) == 1,
                    "side_cut_weight": cut, "side_size": int(s.sum()),
                    "oracle_lambda": gold["lambda"] if gold else None}
        log(f"verify: {verified}")

    # Matula's (2+eps)-approximation on the same resident graph (the same
    # kernels with a lower contraction bound); its answer is a real cut
    approx = None
    if not args.no_approx:
        approx = []
        for ppm in (100_000, 250_000):
            mc.mincut(rp, col, w, approx_ppm=ppm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(3):
                lam_a, side_a, st_a = mc.mincut(rp, col, w, approx_ppm=ppm)
            torch.cuda.synchronize()
            dt_a = (time.perf_counter() - t0) / 3
            s_a = side_a.cpu().numpy()[: g.n].astype(bool)
            src = g.src()
            cut_a = int(g.w[s_a[src] != s_a[g.col]].sum()) // 2
            approx.append({"eps": ppm / 1e6, "ms": round(dt_a * 1e3, 2), "edges_per_s": g.m / dt_a,
                           "lambda": lam_a, "side_cut_weight": cut_a, "rounds": st_a["rounds"],
                           "exact_lambda": lams[0]})
            log(f"approx eps={ppm / 1e6}: {approx[-1]}")

    batched = None
    if not args.no_batched:
        batched = batched_form(max(1, min(args.steps, 3)), 1)
    served = None
    if not args.no_served:
        served = served_form(args.requests, args.pool, args.lanes)
    rmat = None
    if not args.no_rmat:
        rmat = rmat_form(max(1, min(args.steps, 3)))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline()
        log(f"cpu baseline: {cpu}")

    out = {"metric": "exact min-cut edges/s (m / solve time) at 1 GPU",
           "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64",
           "data": "synthetic",
           "config": {"workload": f"chung_lu n=2^{args.n_log2} exp2.5 avgdeg32 unit-weight "
                                  f"8-core LCC", "n": g.n, "m": g.m,
                      "rounds": st["rounds"], "verified": verified},
           "roofline": roofline, "cpu_baseline": cpu, "batched": batched, "served": served,
           "rmat_scale24": rmat, "matula_approx": approx}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
