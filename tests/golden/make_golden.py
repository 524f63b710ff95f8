"""Write the expected minimum cuts of the workload graphs.

Calls only the generators (inputs) and the CPU oracle (sequential NOI, O3);
nothing here touches the GPU library.  Each entry records the graph's size
and a digest of its CSR so a drifting generator is caught, plus lambda and
the oracle's wall time.

    python tests/golden/make_golden.py planted_4096 chung_lu_4m_8core ...
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "workloads.json")

RECIPES = {
    "planted_4096": gg.planted_4096,
    "chung_lu_4m_8core": gg.chung_lu_4m_8core,
    "chung_lu_2^19_8core": lambda: gg.chung_lu_4m_8core(19),
    "rmat_24_10core": gg.rmat_24_10core,
    "rmat_20_10core": lambda: gg.rmat_24_10core(20, 24),
    "bridged_8cores_2^21_k3": lambda: gg.bridged_8cores(21, 3),
}


def digest(g) -> str:
    h = hashlib.blake2b(digest_size=16)
    for a in (g.row_ptr, g.col, g.w):
        h.update(a.tobytes())
    return h.hexdigest()


# batches: every graph's lambda, in graph order
BATCHES = {
    "batch_4096": (4096, gg.batch_graph),
}


def batch_entry(count, make):
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.time()
    graphs = [make(i) for i in range(count)]
    packed, vo, eo = gg.pack(graphs)
    print(f"  {count} graphs: sum n={packed.n} sum m={packed.m} in {time.time() - t0:.1f}s", flush=True)
    t0 = time.time()
    # the oracle releases the interpreter lock inside its C routines
    with ThreadPoolExecutor(max(1, os.cpu_count() or 1)) as ex:
        res = list(ex.map(lambda g: oracle.noi(g, 1), graphs))
    for g, (lam, side, _) in zip(graphs, res):
        assert oracle.cut_value(g, side) == lam
    return {"graphs": count, "n": packed.n, "m": packed.m, "nnz": packed.nnz,
            "digest": digest(packed), "lambdas": [r[0] for r in res],
            "oracle": "noi (O3), seed 1, one graph per thread",
            "oracle_seconds": round(time.time() - t0, 2)}


# request streams: every request's lambda, computed one request at a time
# per thread (the whole stream is too large to hold at once)
STREAMS = {
    "served_2000": (2000, gg.served_request),
}


def stream_entry(count, make):
    from concurrent.futures import ThreadPoolExecutor
    t0 = time.time()

    def one(i):
        g = make(i)
        lam, side, _ = oracle.noi(g, 1)
        assert oracle.cut_value(g, side) == lam
        return lam, g.n, g.m
    with ThreadPoolExecutor(max(1, os.cpu_count() or 1)) as ex:
        res = list(ex.map(one, range(count)))
    return {"requests": count, "lambdas": [r[0] for r in res], "n": [r[1] for r in res],
            "m": [r[2] for r in res], "oracle": "noi (O3), seed 1, one request per thread",
            "oracle_seconds": round(time.time() - t0, 2)}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name in STREAMS:
            data[name] = stream_entry(*STREAMS[name])
            json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
            continue
        if name in BATCHES:
            data[name] = batch_entry(*BATCHES[name])
            json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)
            continue
        t0 = time.time()
        g = RECIPES[name]()
        tg = time.time() - t0
        print(f"{name}: n={g.n} m={g.m} generated in {tg:.1f}s", flush=True)
        t0 = time.time()
        lam, side, rounds = oracle.noi(g, 1)
        to = time.time() - t0
        cut = oracle.cut_value(g, side)
        assert cut == lam, (cut, lam)
        print(f"  lambda={lam} rounds={rounds} oracle {to:.1f}s", flush=True)
        data[name] = {"n": g.n, "m": g.m, "nnz": g.nnz, "digest": digest(g), "lambda": lam,
                      "oracle": "noi (O3), seed 1", "oracle_seconds": round(to, 2),
                      "oracle_rounds": rounds}
        json.dump(data, open(OUT, "w"), indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["planted_4096"])
