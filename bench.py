"""Exact minimum-cut throughput on one MI355X.

A step is one complete exact solve (every round of the contraction loop:
Padberg-Rinaldi tests, CAPFOREST scans, union-find, contraction, bound
updates, side) of the workload graph, already resident in HBM.  The default
workload is the largest single-graph one: an R-MAT graph (scale 24, 2^28
edge draws, parameters 0.57/0.19/0.19/0.05, multiplicity weights) reduced to
its 10-core and largest component.

Prints one JSON line: edges/s (undirected edges of the solved graph divided
by the solve time), the dominant kernel's roofline figures (event-timed on
the launch stream during the timed steps), the CPU oracle's rate on a
bounded sample of the same recipe, and the other workloads (the planted
4096-vertex graph, the Chung-Lu 2^22 8-core, the 4096-graph batch, the
served stream) as extra keys.
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


def source_digest():
    """Digest of the kernel and library sources: a counter summary taken on
    other sources no longer describes the kernels."""
    import hashlib
    h = hashlib.blake2b(digest_size=8)
    d = os.path.join(ROOT, "paper_1808_05458_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".h", ".hip")):
            h.update(f.encode())
            h.update(open(os.path.join(d, f), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "mincut.h"), "rb").read())
    return h.hexdigest()


def golden():
    return json.load(open(os.path.join(ROOT, "tests", "golden", "workloads.json")))


def cpu_baseline(workload):
    """Oracle (sequential NOI, one thread) fully solving a smaller graph of
    the headline's recipe; the stored full-size oracle time is printed beside
    it (measured once when the expected values were written)."""
    import graphgen as gg
    import oracle
    if workload == "rmat":
        g, full_key, recipe = gg.rmat_24_10core(20, 24), "rmat_24_10core", "rmat scale 20 (2^24 draws) 10-core LCC"
    else:
        g, full_key, recipe = gg.chung_lu_4m_8core(19), "chung_lu_4m_8core", "chung_lu n=2^19 8-core LCC"
    t0 = time.perf_counter()
    lam, side, rounds = oracle.noi(g, 1)
    dt = time.perf_counter() - t0
    full = golden().get(full_key, {})
    return {"value": g.m / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"sequential NOI (O3) full solve of {recipe} (n={g.n}, m={g.m}, "
                      f"lambda={lam}, {rounds} rounds) in {dt:.2f} s",
            "full_size": {"graph": full_key, "m": full.get("m"), "oracle_seconds": full.get("oracle_seconds"),
                          "edges_per_s": (full["m"] / full["oracle_seconds"]) if full else None,
                          "note": "stored when the expected values were written (one thread, build host), "
                                  "not re-run here"}}


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
    from the first round), the priority-queue orders among equal keys
    (pq_order: 1 bucket queue, 2 bucket stack, 3 heap) and repeated visits
    of region scans (scan_visits); on the 4096-graph batch and the Chung-Lu
    2^22 8-core.  n_round: vertices at the start of each round."""
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
                     "n_round": list(st["n_round"][:min(st["rounds"], 8)]), "lambda": lam}
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
    for order, name in ((1, "bucket_queue"), (2, "bucket_stack"), (3, "heap")):
        run(f"batch_capped_sweeps_{name}", batch(pq_order=order))
        run(f"batch_one_pop_scans_{name}", batch(scan_mode=2, pq_order=order))
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
    for order, name in ((1, "bucket_queue"), (2, "bucket_stack"), (3, "heap")):
        run(f"chung_lu_region_scans_{name}", single(scan_mode=1, pq_order=order), reps=1)
    for k in (2, 3):
        run(f"chung_lu_region_scans_{k}_visits", single(scan_mode=1, scan_visits=k), reps=1)
    run("chung_lu_one_pop_hashed_small_graphs", single(scan_mode=2))
    return out


def served_form(requests, lanes, seed=5):
    """Poisson arrivals of distinct min-cut requests (Chung-Lu, exponent 2.5,
    average degree 16, n log-uniform in [2^10, 2^20], weights in [1, 50],
    largest component; request i is served_request(i)), served with
    continuous batching.  The capacity is measured closed-loop first; the
    open-loop runs arrive at 0.3 and 0.7 of it.  Latency = submit -> result
    on the host (host CSR in, upload included).  Every served lambda is
    compared with the same request solved alone (the loop of single solves)
    and, where stored, with the oracle's."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc
    t0 = time.time()
    with ThreadPoolExecutor(16) as ex:  # the generator releases the interpreter lock
        pool = list(ex.map(gg.served_request, range(requests)))
    sum_m = sum(g.m for g in pool)
    log(f"served: {requests} distinct requests, sum n={sum(g.n for g in pool)} sum m={sum_m} "
        f"in {time.time() - t0:.1f}s")
    gold = golden().get("served_2000")
    oracle_l = gold["lambdas"][:requests] if gold and gold["requests"] >= requests else None
    rng = np.random.default_rng(seed)

    # one long-lived server for every run; a first pass over the largest
    # requests lets each lane's buffers grow to their working size
    srv = mc.Server(lanes=lanes)
    warm = [srv.submit(g) for g in sorted(pool, key=lambda g: -g.nnz)[:4 * lanes]]
    for t in warm:
        srv.wait(t, want_side=False)

    def run(rate, ref):
        """rate None: everything submitted at once (closed loop)."""
        lat, lams = [], [None] * requests
        tickets = [None] * requests
        ready = threading.Semaphore(0)

        def produce():
            gaps = rng.exponential(1.0 / rate, size=requests) if rate else np.zeros(requests)
            due = time.perf_counter()
            for k in range(requests):
                due += gaps[k]
                d = due - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                tickets[k] = srv.submit(pool[k])
                ready.release()

        t_start = time.perf_counter()
        th = threading.Thread(target=produce)
        th.start()
        for k in range(requests):
            ready.acquire()
            lam, _, l = srv.wait(tickets[k], want_side=False)
            lams[k] = lam
            lat.append(l["total_ms"])
        t_end = time.perf_counter()
        th.join()
        lat = np.asarray(lat)
        span = t_end - t_start
        out = {"requests": requests, "span_s": round(span, 3), "edges_per_s": float(sum_m / span),
               "requests_per_s": round(requests / span, 1),
               "p50_ms": round(float(np.percentile(lat, 50)), 3),
               "p99_ms": round(float(np.percentile(lat, 99)), 3)}
        if ref is not None:
            out["same_as_alone"] = bool(lams == ref)
        if oracle_l is not None:
            out["same_as_oracle"] = bool(lams == oracle_l)
        return out, lams

    # the same requests as a host loop of single-graph solves, each uploaded
    # from host memory like a served request: the "alone" results
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alone = []
    for g in pool:
        rp, col, w = mc.to_device(g, "cuda:0")
        alone.append(mc.mincut(rp, col, w, want_side=False)[0])
    torch.cuda.synchronize()
    loop_s = time.perf_counter() - t0
    looped = {"span_s": round(loop_s, 3), "edges_per_s": float(sum_m / loop_s),
              "same_as_oracle": bool(oracle_l is not None and alone == oracle_l)}
    log(f"looped single solves: {looped}")
    cap, _ = run(None, alone)
    log(f"served closed loop: {cap}")
    out = {"requests": requests, "distinct": True, "lanes": lanes, "sum_m": sum_m,
           "mean_m": round(sum_m / requests), "closed_loop": cap, "looped": looped,
           "speedup_closed_loop": round(cap["edges_per_s"] / looped["edges_per_s"], 2)}
    for frac in (0.3, 0.7):
        r, _ = run(frac * cap["requests_per_s"], alone)
        r["rate_frac"] = frac
        log(f"served at {frac} of capacity: {r}")
        out[f"at_{frac}"] = r
    srv.close()
    return out


def solve_single(g, steps, warmup, gold_lambda, label):
    """Time `steps` exact solves of one resident graph.  A profile pass
    first (up to 3 solves, every kernel class event-timed on the solve
    stream) names the dominant class; the timed solves then record HIP
    events around that class's launches only, so the timed region pays for
    a few events per solve, not for every class's."""
    import torch
    import paper_1808_05458_amd as mc
    rp, col, w = mc.to_device(g, "cuda:0")
    for i in range(warmup):
        lam, side, st = mc.mincut(rp, col, w)
        log(f"{label} warmup {i}: lambda={lam} rounds={st['rounds']} {st['ms']:.1f} ms n_round={st['n_round']}")
    topts = mc.options(timing=1)
    prof_steps = max(1, min(steps, 3))
    mc.timing_focus(None)
    mc.timing_reset()
    for i in range(prof_steps):
        _, _, st_prof = mc.mincut(rp, col, w, opts=topts)
    torch.cuda.synchronize()
    classes = mc.timing()
    log(f"{label} kernel classes: " + ", ".join(f"{c['name']}={c['ms'] / prof_steps:.2f}ms"
                                               for c in sorted(classes, key=lambda c: -c["ms"])))
    dom_name = max(classes, key=lambda c: c["ms"])["name"]
    mc.timing_reset()
    mc.timing_focus(dom_name)
    lams = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        lam, side, st = mc.mincut(rp, col, w, opts=topts)
        lams.append(lam)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    dom = [c for c in mc.timing() if c["name"] == dom_name][0]
    mc.timing_focus(None)
    mc.timing_reset()
    s = side.cpu().numpy()[: g.n].astype(bool)
    cut = int(g.w[s[g.src()] != s[g.col]].sum()) // 2
    verified = {"lambda": lams[0], "all_steps_equal": len(set(lams)) == 1, "oracle_lambda": gold_lambda,
                "equals_oracle": gold_lambda is not None and all(x == gold_lambda for x in lams),
                "side_cut_weight": cut, "side_size": int(s.sum())}
    log(f"{label} verify: {verified}")
    # (the per-phase sweep counters are read back in the profile pass)
    sweep = {"big_batches": st_prof["sweep_big_batches"], "singles": st_prof["sweep_singles"],
             "batches": st_prof["sweep_batches"], "crossings": st_prof["sweep_cross"]}
    del rp, col, w
    return {"ms_per_step": dt * 1000.0 / steps, "value": g.m * steps / dt, "rounds": st["rounds"],
            "n_round": st["n_round"], "classes": classes, "prof_steps": prof_steps, "dominant": dom,
            "verified": verified, "sweep_phases": sweep}


def roofline_of(r, steps, traffic_file):
    """The dominant kernel (most device time per step in the profile pass)
    against HBM peak: algorithmic bytes per launch over its average launch
    time, both from the events of the timed region, plus the
    counter-measured bytes per launch when a summary taken on these sources
    exists.  Class fractions and the per-kernel table come from the profile
    pass (r["prof_steps"] solves, every class timed)."""
    classes, prof = r["classes"], r["prof_steps"]
    def rate(c):
        per_launch_s = c["ms"] / 1000.0 / c["launches"]
        per_launch_bytes = c["algo_bytes"] / c["launches"]
        return per_launch_bytes / per_launch_s / 1e9, per_launch_bytes

    measured, digest_ok = {}, False
    if os.path.exists(traffic_file):
        for line in open(traffic_file):
            f = line.split()
            if len(f) == 2 and f[0] == "source_digest":
                digest_ok = f[1] == source_digest()
            if len(f) == 6 and f[0] == "traffic":
                measured[f[1]] = int(f[5])
    if not digest_ok:
        measured = {}
    dom = r["dominant"]
    achieved, dom_bytes = rate(dom)

    def entry(c):
        e = {"ms_per_step": round(c["ms"] / prof, 3), "launches_per_step": c["launches"] / prof,
             "algo_GBps": round(rate(c)[0], 1), "frac": round(rate(c)[0] / HBM_PEAK_GBS, 5)}
        if c["name"] in measured:
            e["counter_bytes_per_launch"] = measured[c["name"]]
            e["counter_GBps"] = round(measured[c["name"]] / (c["ms"] / 1000.0 / c["launches"]) / 1e9, 1)
        return e
    # the hot path's kernel classes: algorithmic bytes of all their launches
    # over all their device time
    groups = {"capforest": ("k_sweep_seq", "k_sweep_tail", "k_sweep_big_relax", "k_sweep_big_pull",
                            "k_sweep_seg_bounds", "k_sweep_seg_relax", "k_sweep_seg_fallback", "k_sweep_big_mark",
                            "sweep_batch_prep", "sweep_rebuild", "k_sweep_unite", "k_small_sweep",
                            "capforest_region", "capforest_whole", "k_union_pairs"),
              "contraction": ("block_bits", "k_emit", "k_rs_hist", "k_rs_scatter", "merge_scan", "k_merge", "csr"),
              "padberg_rinaldi": ("k_pr_sample", "k_pr", "k_pr34")}
    class_frac = {}
    for gname, members in groups.items():
        cs = [c for c in classes if c["name"] in members]
        ms = sum(c["ms"] for c in cs)
        if ms > 0:
            gbps = sum(c["algo_bytes"] for c in cs) / (ms / 1000.0) / 1e9
            class_frac[gname] = {"ms_per_step": round(ms / prof, 3), "algo_GBps": round(gbps, 1),
                                 "frac": round(gbps / HBM_PEAK_GBS, 5)}
    return {"bound": "hbm", "achieved": round(achieved, 3), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 6), "traffic": measured.get(dom["name"]),
            "classes": class_frac,
            "kernel": dom["name"], "avg_launch_ms": round(dom["ms"] / dom["launches"], 4),
            "launches_per_step": dom["launches"] / steps, "algo_bytes_per_launch": dom_bytes,
            "traffic_source": os.path.relpath(traffic_file, ROOT) if measured else None,
            "kernels": {c["name"]: entry(c) for c in sorted(classes, key=lambda c: -c["ms"])[:10]}}


def planted_form(steps):
    """The planted-cluster graph (n = 4096, 8 clusters of 512): edges/s and
    rounds (its CSR fits in L2; latency-bound, so no HBM fraction)."""
    import graphgen as gg
    g = gg.planted_4096()
    r = solve_single(g, steps, 1, golden()["planted_4096"]["lambda"], "planted")
    return {"n": g.n, "m": g.m, "ms": round(r["ms_per_step"], 3), "edges_per_s": r["value"],
            "rounds": r["rounds"], "verified": r["verified"]}


def chung_lu_form(steps, approx=True):
    """The Chung-Lu 2^22 8-core: exact solves, its kernel classes, and
    Matula's (2+eps)-approximation on the same resident graph."""
    import torch
    import graphgen as gg
    import paper_1808_05458_amd as mc
    g = gg.chung_lu_4m_8core(22)
    r = solve_single(g, steps, 1, golden()["chung_lu_4m_8core"]["lambda"], "chung_lu")
    out = {"n": g.n, "m": g.m, "ms": round(r["ms_per_step"], 3), "edges_per_s": r["value"],
           "rounds": r["rounds"], "verified": r["verified"], "sweep_phases": r["sweep_phases"],
           "roofline": roofline_of(r, steps,
                                   os.path.join(ROOT, "profiles", "hbm_traffic_chung_lu_2^22_8core.txt"))}
    if approx:
        rp, col, w = mc.to_device(g, "cuda:0")
        out["matula_approx"] = []
        for ppm in (100_000, 250_000):
            mc.mincut(rp, col, w, approx_ppm=ppm)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(3):
                lam_a, side_a, st_a = mc.mincut(rp, col, w, approx_ppm=ppm)
            torch.cuda.synchronize()
            dt_a = (time.perf_counter() - t0) / 3
            s_a = side_a.cpu().numpy()[: g.n].astype(bool)
            cut_a = int(g.w[s_a[g.src()] != s_a[g.col]].sum()) // 2
            out["matula_approx"].append({"eps": ppm / 1e6, "ms": round(dt_a * 1e3, 2), "edges_per_s": g.m / dt_a,
                                         "lambda": lam_a, "side_cut_weight": cut_a, "rounds": st_a["rounds"],
                                         "exact_lambda": r["verified"]["lambda"]})
            log(f"approx eps={ppm / 1e6}: {out['matula_approx'][-1]}")
    return out


def _kernel_short(name):
    """rocprofv3's kernel name reduced to the timing-class name:
    'void mc::k_rs_scatter<16>(...)' -> 'k_rs_scatter'."""
    n = name.split("(")[0].replace("void ", "").strip()
    n = n.split("<")[0]
    return n.split("::")[-1]


def _db(path):
    import glob
    import sqlite3
    files = glob.glob(os.path.join(path, "**", "*.db"), recursive=True) if os.path.isdir(path) else [path]
    if len(files) != 1:
        raise SystemExit(f"expected one rocpd database under {path}, found {files}")
    return sqlite3.connect(files[0])


def summarize(args):
    """Text summaries of rocprofv3 output for profiles/: kernel statistics
    (--kernel-trace --stats), and HBM traffic per dispatch from a FETCH_SIZE
    run and a WRITE_SIZE run, each scaled by the same counter on a plain
    1 GiB device copy (bench.py --calibrate-copy)."""
    lines = [f"# {args.title}", "#", "# Commands (from /tmp with TMPDIR=/tmp; R = repository root):"]
    lines += [f"#   {c}" for c in args.command]
    if args.stats:
        c = _db(args.stats)
        rows = c.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                         "order by total_duration desc").fetchall()
        lines += ["#", "# Durations in microseconds (rocprofv3 top_kernels).", "",
                  "| kernel | calls | total us | avg us | % |", "|---|---:|---:|---:|---:|"]
        for name, calls, tot, avg, pct in rows[:args.top]:
            lines.append(f"| `{name.split('(')[0].replace('void ', '')}` | {calls} | {tot:.1f} | {avg:.1f} | {pct:.2f} |")
    if args.fetch:
        def per_kernel(path, counter):
            c = _db(path)
            out = {}
            for name, disp, val in c.execute(
                    "select kernel_name, dispatch_id, sum(value) from counters_collection where counter_name = ? "
                    "group by dispatch_id", (counter,)):
                k = _kernel_short(name)
                out.setdefault(k, []).append(val)
            return out
        cal_f = per_kernel(args.cal_fetch, "FETCH_SIZE")["__amd_rocclr_copyBuffer"]
        cal_w = per_kernel(args.cal_write, "WRITE_SIZE")["__amd_rocclr_copyBuffer"]
        copy_bytes = float(1 << 30)
        fs = copy_bytes / (np.median(cal_f) * 1024.0)
        ws = copy_bytes / (np.median(cal_w) * 1024.0)
        f = per_kernel(args.fetch, "FETCH_SIZE")
        w = per_kernel(args.write, "WRITE_SIZE")
        lines += ["#", f"# Calibration: __amd_rocclr_copyBuffer moving {int(copy_bytes)} bytes reads FETCH_SIZE "
                       f"{np.median(cal_f):.1f} KiB and WRITE_SIZE {np.median(cal_w):.1f} KiB per dispatch, so",
                  "# bytes = KiB * 1024 * scale with", f"fetch_scale {fs:.4f}", f"write_scale {ws:.4f}",
                  f"source_digest {source_digest()}",
                  "#", "# kernel dispatches fetch_KiB_per_dispatch write_KiB_per_dispatch bytes_per_dispatch(scaled)"]
        rank = sorted(f, key=lambda k: -sum(f[k]))
        for k in rank[:args.top]:
            fk = float(np.mean(f[k]))
            wk = float(np.mean(w.get(k, [0.0])))
            lines.append(f"traffic {k} {len(f[k])} {fk:.1f} {wk:.1f} {int(round(fk * 1024 * fs + wk * 1024 * ws))}")
    open(args.out, "w").write("\n".join(lines) + "\n")
    log(f"wrote {args.out}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["rmat", "chung_lu", "batched", "served"], default="rmat")
    ap.add_argument("--only", action="store_true",
                    help="the headline workload alone (no other workloads, no CPU baseline)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-planted", action="store_true")
    ap.add_argument("--no-chung-lu", action="store_true")
    ap.add_argument("--no-approx", action="store_true", help="skip the (2+eps)-approximation runs")
    ap.add_argument("--ablation", action="store_true",
                    help="print scan-policy ablations (rounds against time) instead of the bench line")
    ap.add_argument("--no-loop", action="store_true",
                    help="batched form: skip the loop of single solves (profiling the packed solve alone)")
    ap.add_argument("--requests", type=int, default=2000, help="distinct served requests")
    ap.add_argument("--lanes", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (the reference "
                         "kernel for scaling HBM traffic counters) and exit")
    ap.add_argument("--summarize", action="store_true",
                    help="write a profiles/ summary from rocprofv3 databases (no GPU work)")
    ap.add_argument("--stats", help="rocprofv3 --kernel-trace --stats output directory")
    ap.add_argument("--fetch", help="rocprofv3 --pmc FETCH_SIZE output directory")
    ap.add_argument("--write", help="rocprofv3 --pmc WRITE_SIZE output directory")
    ap.add_argument("--cal-fetch", help="FETCH_SIZE output of bench.py --calibrate-copy")
    ap.add_argument("--cal-write", help="WRITE_SIZE output of bench.py --calibrate-copy")
    ap.add_argument("--title", default="")
    ap.add_argument("--command", action="append", default=[])
    ap.add_argument("--top", type=int, default=30)
    ap.add_argument("--out")
    args = ap.parse_args()
    if args.summarize:
        summarize(args)
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only; graphs of the batched and served forms would "
              "shard across GPUs (independent graphs), but no multi-GPU path is implemented.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import graphgen as gg

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
        sv = served_form(args.requests, args.lanes)
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
    if args.workload == "rmat":
        g = gg.rmat_24_10core()
        gold_key, traffic_name = "rmat_24_10core", "hbm_traffic_rmat_24_10core.txt"
        workload = ("rmat scale 24, 2^28 draws (0.57, 0.19, 0.19, 0.05), multiplicity weights, "
                    "10-core, largest component")
    else:
        g = gg.chung_lu_4m_8core(22)
        gold_key, traffic_name = "chung_lu_4m_8core", "hbm_traffic_chung_lu_2^22_8core.txt"
        workload = "chung_lu n=2^22 exp2.5 avgdeg32 unit-weight 8-core LCC"
    log(f"generated {g.name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    r = solve_single(g, args.steps, args.warmup, golden().get(gold_key, {}).get("lambda"), args.workload)
    roofline = roofline_of(r, args.steps, os.path.join(ROOT, "profiles", traffic_name))
    n, m = g.n, g.m
    del g
    extra = {}
    if not args.only:
        if not args.no_planted:
            extra["planted_4096"] = planted_form(args.steps)
        if not args.no_chung_lu and args.workload != "chung_lu":
            extra["chung_lu_2^22_8core"] = chung_lu_form(max(1, min(args.steps, 5)), approx=not args.no_approx)
        if not args.no_batched:
            extra["batched"] = batched_form(max(1, min(args.steps, 3)), 1)
        if not args.no_served:
            extra["served"] = served_form(args.requests, args.lanes)
    cpu = None
    if not args.only and not args.no_cpu_baseline:
        cpu = cpu_baseline(args.workload)
        log(f"cpu baseline: {cpu}")
    out = {"metric": "exact min-cut edges/s (m / solve time) at 1 GPU",
           "value": r["value"], "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
           "config": {"workload": workload, "n": n, "m": m, "rounds": r["rounds"], "n_round": r["n_round"],
                      "verified": r["verified"], "sweep_phases": r["sweep_phases"]},
           "roofline": roofline, "cpu_baseline": cpu, **extra}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
