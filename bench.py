"""Benchmark of the encrypted decision-forest evaluation on one MI355X.

Workload (default): 64 random unbalanced trees of maximum depth 8, 32
features, 16-bit values, 10 classes, with the thresholds, the reshuffle and
level diagonals and the masks encrypted under the data owner's key (45 GiB of
ciphertexts resident in HBM), ring N = 32768 with 11 data primes and 4 special
primes; all 256 encrypted queries of the workload (64 query groups of 4) per
step, in batched calls of 16 groups.  A step is the complete Algorithm 1 on
every query: comparison, reshuffle, level products with masks, product tree,
switch to q_0.  Encrypted queries are resident in device memory before the
timed region starts.  Inputs are synthetic (the pinned generator).

Prints one JSON line: throughput (encrypted queries/s), per-step latency
percentiles, the roofline of the dominant kernel (its per-launch time taken
with HIP events on the stream it runs on; against HBM bandwidth and, for an
encrypted model's MatMul inner sums, against the fp64 pipe's rate of exact
modular products), the unbatched path's rate on one group of the same
workload (batched / plain), the CPU oracle's throughput on a bounded sample
(single thread and one process per core), and extra lines for the batched
32-tree workload (1024 queries per step) and the one-query 16-tree workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--batch G] [--groups N] [--no-cpu-baseline] [--no-extras] [--no-plain]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "encrypted queries/sec + p50/p99 latency per forest; NTT/keyswitch HBM GB/s"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


KIND_NAMES = {0: "ntt_fwd_rows", 1: "ntt_fwd_cols", 2: "ntt_inv_rows", 3: "ntt_inv_cols", 4: "ks_inner_rot",
              5: "bconv_colpass", 6: "elementwise", 7: "ntt_fwd_rows_moddown", 8: "ntt_fwd_rows_modswitch",
              9: "matmul_inner", 10: "ntt_inv_rows_gather", 15: "ks_inner_relin", 16: "ks_inner_giant"}
KERNEL_KINDS = (0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 15, 16)
STAGE_NAMES = ("comparison", "reshuffle", "levels", "aggregation")
# kernel of each class (for the counter runs); class 6 is a family of small kernels and is not a roofline
# (name patterns for rocprofv3's kernel filter: class 7 is the ModDown finishes, alone and merged with the switch)
KIND_KERNELS = {0: "ntt_rowreg4_kernel<false>", 2: "ntt_rowreg4_kernel<true>", 4: "ks_inner2",
                5: "ntt_bridge_kernel", 7: "ntt_rowfwd_finish_kernel<[13]>", 8: "ntt_rowfwd_finish_kernel<2>",
                9: "mm_inner", 10: "ntt_rowinv_gather_kernel", 15: "ks_inner_rows", 16: "ks_inner_gsum"}


def measured_traffic(kind: str, workload: str):
    """HBM bytes per launch of the roofline kernel from the committed counter runs
    (profiles/hbm_bytes_<kind>_<workload>.json, written by paper_2104_09583_amd.pmc_traffic);
    None when there is none or the kernels' source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_bytes_{kind}_{workload}.json")
    src = os.path.join(ROOT, "paper_2104_09583_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != doc["kernels_hip_sha256"]:
            return None
    return doc["bytes_per_dispatch"]


def _dry_ct(level, npolys=2):
    """Stand-in ciphertext of the schedule's dry run: only its level and component count."""
    from oracle.bgv import Ciphertext
    return Ciphertext([None] * npolys, level)


class _DryBGV:
    """Runs the oracle's evaluation schedule (circuit.Evaluator) without arithmetic and records every
    operation it would perform as (name, level[, size]): the operation counts of one query group, taken
    from the schedule code itself."""

    def __init__(self, sc):
        self.N, self.t, self.L = sc.N, sc.t, sc.L
        self.ops = {}

    def _rec(self, *key):
        self.ops[key] = self.ops.get(key, 0) + 1

    def data_idx(self, level):
        return list(range(level + 1))

    # model and query set-up (not part of an evaluation)
    def encode(self, slots):
        return None

    def encrypt_slots(self, keys, slots, seed, obj, level=None):
        return _dry_ct(self.L if level is None else level)

    # the operations the evaluation performs
    def modswitch(self, ct):
        self._rec("modswitch", ct.level, len(ct.polys))
        return _dry_ct(ct.level - 1, len(ct.polys))

    def modswitch_to(self, ct, level):
        while ct.level > level:
            ct = self.modswitch(ct)
        return ct

    def _bin(self, name, a, b):
        lv = min(a.level, b.level)
        a, b = self.modswitch_to(a, lv), self.modswitch_to(b, lv)
        self._rec(name, lv, max(len(a.polys), len(b.polys)))
        return _dry_ct(lv, max(len(a.polys), len(b.polys)))

    def add(self, a, b):
        return self._bin("add", a, b)

    def sub(self, a, b):
        return self._bin("sub", a, b)

    def tensor(self, a, b):
        self._bin("tensor", a, b)
        return _dry_ct(min(a.level, b.level), 3)

    def mul(self, a, b, keys):
        lv = min(a.level, b.level)
        self.modswitch_to(a, lv), self.modswitch_to(b, lv)
        self._rec("mul", lv)
        return _dry_ct(lv - 1)

    def relinearize(self, ct, keys):
        self._rec("relin", ct.level)
        return _dry_ct(ct.level)

    def mul_int(self, a, k):
        self._rec("mul_int", a.level)
        return _dry_ct(a.level, len(a.polys))

    def add_plain(self, a, m):
        self._rec("add_plain", a.level)
        return _dry_ct(a.level, len(a.polys))

    def mul_plain(self, a, m):
        self._rec("mul_plain", a.level)
        return _dry_ct(a.level, len(a.polys))

    def rotate_hoisted(self, ct, rs, keys):
        nz = [r for r in rs if r % (self.N // 2)]
        if nz:
            self._rec("rot_hoisted", ct.level, len(nz))
        return {r: _dry_ct(ct.level) for r in rs}

    def rotate_sum(self, items, keys):
        lv = items[0][0].level
        self._rec("rotate_sum", lv, sum(1 for _, r in items if r % (self.N // 2)), len(items))
        return _dry_ct(lv)

    # plaintext-model inner sums (rows of residues)
    def ntt(self, a, idx):
        self._rec("ntt", len(idx))

    def intt(self, a, idx):
        self._rec("intt", len(idx))

    def plain_ntt(self, m, level):
        self._rec("plain_ntt", level)

    def pmul_ntt(self, a, b, idx):
        self._rec("pmul", len(idx))

    def padd(self, a, b, idx):
        return None


def _time_ops(sc, keys, ops, seed, reps=1):
    """Seconds of each recorded operation (by name and level) on the oracle, on fresh encryptions."""
    from oracle import bgv as B
    rng = np.random.default_rng(5)
    cache = {}

    def ct(level, npolys=2, obj=0):
        k = (level, npolys, obj)
        if k not in cache:
            v = rng.integers(0, 2, size=(2, sc.N // 2))
            c = sc.encrypt_slots(keys, v, seed, 10_000 + 100 * level + obj, level)
            cache[k] = c if npolys == 2 else sc.tensor(c, ct(level, 2, obj + 1))
        return cache[k]

    pt = sc.encode(rng.integers(0, 2, size=(2, sc.N // 2)))

    def best(f):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            f()
            ts.append(time.perf_counter() - t0)
        return min(ts)

    rows = {}
    for key in ops:
        name, lv = key[0], key[1]
        if name in ("modswitch", "add", "sub", "tensor"):
            np_ = key[2]
            a, b = ct(lv, np_ if name != "tensor" else 2), ct(lv, np_ if name != "tensor" else 2, 1)
            f = {"modswitch": lambda: sc.modswitch(a), "add": lambda: sc.add(a, b), "sub": lambda: sc.sub(a, b),
                 "tensor": lambda: sc.tensor(a, b)}[name]
            rows[key] = best(f)
        elif name == "mul":
            a, b = ct(lv), ct(lv, 2, 1)
            rows[key] = best(lambda: sc.mul(a, b, keys))
        elif name == "relin":
            a = ct(lv, 3)
            rows[key] = best(lambda: sc.relinearize(a, keys))
        elif name == "mul_int":
            a = ct(lv)
            rows[key] = best(lambda: sc.mul_int(a, 2))
        elif name == "add_plain":
            a = ct(lv)
            rows[key] = best(lambda: sc.add_plain(a, pt))
        elif name == "mul_plain":
            a = ct(lv)
            rows[key] = best(lambda: sc.mul_plain(a, pt))
        elif name == "plain_ntt":
            rows[key] = best(lambda: sc.plain_ntt(pt, lv))
        elif name in ("ntt", "intt", "pmul"):
            idx = list(range(lv))
            x = np.zeros((lv, sc.N), dtype=np.uint64)
            f = {"ntt": lambda: sc.ntt(x, idx), "intt": lambda: sc.intt(x, idx),
                 "pmul": lambda: sc.pmul_ntt(x, x, idx)}[name]
            rows[key] = best(f)
    # rotations: the hoisted set costs one ModUp plus a per-rotation part; a rotation sum a per-term part
    # plus the final ModDowns; both are fitted from one and two rotations at each level
    for lv in sorted({k[1] for k in ops if k[0] in ("rot_hoisted", "rotate_sum")}):
        a = ct(lv)
        t1 = best(lambda: sc.rotate_hoisted(a, [1], keys))
        t2 = best(lambda: sc.rotate_hoisted(a, [1, 2], keys))
        s1 = best(lambda: sc.rotate_sum([(a, 1)], keys))
        s2 = best(lambda: sc.rotate_sum([(a, 1), (a, 2)], keys))
        rows[("rot_each", lv)], rows[("rot_base", lv)] = t2 - t1, 2 * t1 - t2
        rows[("rsum_each", lv)], rows[("rsum_base", lv)] = s2 - s1, 2 * s1 - s2
    return rows


def _group_seconds(ops, rows):
    total = 0.0
    for key, n in ops.items():
        name, lv = key[0], key[1]
        if name == "rot_hoisted":
            total += n * (rows[("rot_base", lv)] + key[2] * rows[("rot_each", lv)])
        elif name == "rotate_sum":
            total += n * (rows[("rsum_base", lv)] + key[2] * rows[("rsum_each", lv)])
        else:
            total += n * rows[key]
    return total


def _cpu_sample(w, text, seed, reps=1):
    """One query group of the workload on the oracle: every operation of the evaluation schedule counted
    by a dry run of the oracle's own schedule code, each distinct (operation, level) timed once on the
    oracle, the group's time = sum of count x time.  Returns (seconds per group, sampled seconds, counts)."""
    from oracle import bgv as B
    from oracle import circuit as CI
    from oracle import compiler as OC
    from oracle import nt

    ch = w.chain
    sc = B.BGV(nt.make_chain(ch["log_n"], 65537, ch["n_data_primes"], ch["q0_max"], ch["data_max"],
                             ch["alpha"], ch["special_max"]))
    oc = OC.compile_forest(text, w.shape.n_features, w.shape.precision)
    pl = CI.make_plan(oc, sc.N, sc.L, fold=w.fold, encrypted_model=w.encrypted_model, n1_R=w.n1[0], n1_L=w.n1[1])
    dry = _DryBGV(sc)
    X = CI.encrypt_queries(dry, None, pl, np.zeros((1, oc.n_features), dtype=np.uint32), seed, 0)
    model = CI.encrypt_model(dry, None, pl, seed) if w.encrypted_model else CI.encode_model(dry, pl)
    CI.Evaluator(dry, None, pl).run(X, model)
    keys = sc.keygen(seed, rotations=[1, 2])            # untimed set-up
    t0 = time.perf_counter()
    rows = _time_ops(sc, keys, dry.ops, seed, reps)
    sampled = time.perf_counter() - t0
    return _group_seconds(dry.ops, rows), sampled, dry.ops


def _cpu_worker(args):
    name, text, seed = args
    from paper_2104_09583_amd import synth
    sec, sampled, _ = _cpu_sample(synth.WORKLOADS[name], text, seed)
    return sec, sampled


def cpu_baseline(w, text, queries, seed, all_cores: bool = True):
    """The oracle on a bounded sample of the workload: per query group, the operation counts of its whole
    evaluation (a dry run of the oracle's schedule) times the oracle's measured time of each distinct
    operation and level.  Single thread, and the same sample in one process per host core at once
    (all-core throughput: the sum of the processes' rates)."""
    import multiprocessing as mp
    from oracle import compiler as OC
    oc = OC.compile_forest(text, w.shape.n_features, w.shape.precision)
    qpg = min(w.n_queries, (1 << w.log_n) // oc.W)      # queries per group (slot blocks per ciphertext)
    log("cpu baseline: single thread")
    sec, sampled, ops = _cpu_sample(w, text, seed)
    n_ops = sum(ops.values())
    out = {"value": qpg / sec, "unit": "queries/s", "cores": 1, "kind": "oracle",
           "sample": (f"one query group ({qpg} queries): the {n_ops} operations of its evaluation counted by a dry "
                      f"run of the oracle's schedule, each distinct operation and level ({len(ops)} kinds) timed once "
                      f"on the oracle ({sampled:.1f}s of CPU work), group time = sum of count x time = {sec:.1f}s "
                      "(extrapolated), single thread"),
           "seconds_per_group": round(sec, 2)}
    if all_cores:
        # one process per core of this host's share, at most 16 (forked before the GPU is touched)
        P = max(1, min(16, len(os.sched_getaffinity(0))))
        log(f"cpu baseline: {P} processes at once")
        ctx = mp.get_context("fork")
        t0 = time.perf_counter()
        with ctx.Pool(P) as pool:
            res = pool.map(_cpu_worker, [(w.name, text, seed)] * P)
        wall = time.perf_counter() - t0
        rate = sum(qpg / s for s, _ in res)
        out["all_cores"] = {"value": rate, "unit": "queries/s", "cores": P, "nproc": P,
                            "sample": f"the same sample in {P} processes at once ({wall:.1f}s wall); rate = sum of "
                                      "the processes' extrapolated rates",
                            "seconds_per_group_mean": round(sum(s for s, _ in res) / P, 2)}
    # for context: the plaintext forest walk on the same queries (no encryption), one thread
    from oracle import forest as F
    _, trees = F.parse_forest(text)
    t0 = time.perf_counter()
    for x in queries:
        F.evaluate(trees, list(x))
    walk = time.perf_counter() - t0
    out["plain_forest"] = {"value": len(queries) / walk, "unit": "queries/s", "cores": 1,
                           "sample": f"the oracle's plaintext tree walk over the workload's {len(queries)} queries"}
    return out


def serve_bench(args):
    """Serving: Poisson arrivals of one-query requests against the three resident forests of the mix,
    the forest of each request drawn uniformly; swept offered rates from 0.25x to 1.25x the measured
    batched capacity; per forest p50/p99 latency (submission to result on the device, measured by
    the server) and the achieved request rate per offered rate."""
    import threading

    import torch

    from paper_2104_09583_amd import copse as C
    from paper_2104_09583_amd import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    members = [synth.WORKLOADS[n] for n in synth.SERVE_MIX]
    ch = members[0].chain
    assert all(m.chain == ch for m in members)
    seed = synth.crypto_seed("COPSE-cfg-5")
    ctx = C.Context(**ch)
    stream = torch.cuda.Stream()
    ctx.set_stream(stream.cuda_stream)
    comps, texts = [], []
    for m in members:
        text, _, _ = synth.workload_inputs(m)
        texts.append(text)
        comps.append(C.forest_compile(text, m.shape.n_features, m.shape.precision, m.log_n))
    rots = sorted(set(r for _, meta in comps for r in C.compiled_rotations(meta)))
    t0 = time.perf_counter()
    keys = ctx.keygen(seed, rots)
    evk = ctx.export_eval(keys)
    models = [ctx.model_encode(cp) for cp, _ in comps]
    log(f"keys and models {time.perf_counter() - t0:.1f}s; keys {keys.nbytes() / 2**30:.2f} GiB, models "
        f"{sum(md.nbytes() for md in models) / 2**30:.2f} GiB")
    max_batch = args.batch if args.batch > 1 else 8
    srv = C.Server(ctx, 240 << 30, max_batch=max_batch)
    mids = [srv.add_model(md, evk) for md in models]
    rng = np.random.default_rng(12345)
    n_req = args.requests

    def make_requests(n, salt):
        out = []
        for r in range(n):
            mi = int(rng.integers(0, len(members)))
            m = members[mi]
            q = synth.gen_queries(1, m.shape.n_features, m.shape.precision, 10_000 * salt + r)
            out.append((mi, ctx.query_encrypt(keys, comps[mi][1], q, seed, group=10_000 * salt + r)))
        return out

    def run(reqs, rate):
        """Submit reqs at Poisson times of the given rate (requests/s); one waiter per request."""
        gaps = rng.exponential(1.0 / rate, size=len(reqs)) if rate > 0 else np.zeros(len(reqs))
        tickets = [None] * len(reqs)
        done_t = [0.0] * len(reqs)
        lock = threading.Lock()
        ready = threading.Condition(lock)

        def waiter(i):
            with lock:
                while tickets[i] is None:
                    ready.wait()
            srv.wait(tickets[i], 600000)
            done_t[i] = time.perf_counter()

        ths = [threading.Thread(target=waiter, args=(i,)) for i in range(len(reqs))]
        for th in ths:
            th.start()
        start = time.perf_counter()
        t_next = start
        rejected = 0
        for i, (mi, cts) in enumerate(reqs):
            t_next += gaps[i]
            while True:
                now = time.perf_counter()
                if now < t_next:
                    time.sleep(t_next - now)
                try:
                    tk = srv.submit(mids[mi], cts)
                    break
                except C.CopseError as e:
                    if e.code != C.COPSE_ENOMEM:
                        raise
                    rejected += 1          # memory budget full: retry shortly
                    t_next = time.perf_counter() + 0.001
            with lock:
                tickets[i] = tk
                ready.notify_all()
        for th in ths:
            th.join()
        span = max(done_t) - start
        lat = [srv.latency_ms(t) for t in tickets]
        per = {}
        for k, m in enumerate(members):
            ls = [lat[i] for i, (mi, _) in enumerate(reqs) if mi == k]
            per[m.name] = {"n": len(ls), "p50_ms": round(percentile(ls, 50), 3),
                           "p99_ms": round(percentile(ls, 99), 3)}
        return {"offered_rps": round(rate, 2), "achieved_rps": round(len(reqs) / span, 2),
                "span_s": round(span, 3), "rejected_submits": rejected, "per_forest": per}

    # warmup, then the capacity: a burst of requests submitted at once (the server batches them)
    run(make_requests(3 * max_batch, 1), 0.0)
    cap = run(make_requests(n_req, 2), 0.0)
    peak = cap["achieved_rps"]
    log(f"burst capacity {peak:.1f} requests/s")
    sweep = []
    for frac in args.rates:
        res = run(make_requests(n_req, 3 + len(sweep)), frac * peak)
        res["offered_frac"] = frac
        sweep.append(res)
        log(f"rate {frac:.2f}x: offered {res['offered_rps']} achieved {res['achieved_rps']} "
            + " ".join(f"{k}: p50 {v['p50_ms']} p99 {v['p99_ms']}" for k, v in res["per_forest"].items()))
    srv.close()
    # headline: the highest offered rate the server keeps up with (achieved >= 95% of offered)
    kept = [r for r in sweep if r["achieved_rps"] >= 0.95 * r["offered_rps"]]
    best = max(kept, key=lambda r: r["achieved_rps"]) if kept else cap
    out = {
        "metric": METRIC,
        "value": best["achieved_rps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": n_req,
        "warmup": 3 * max_batch,
        "ms_per_step": round(1000.0 / best["achieved_rps"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "c5_serve_mix", "forests": list(synth.SERVE_MIX), "queries_per_request": 1,
                   "max_batch": max_batch, "requests_per_rate": n_req, "arrivals": "poisson",
                   "N": 1 << ch["log_n"], "data_primes": ch["n_data_primes"], "model": "plaintext"},
        "latency_ms": best["per_forest"],
        "burst": cap,
        "sweep": sweep,
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(out))


def micro_bench(args):
    """Table 6 microbenchmarks: per forest, the median time of each stage of one evaluation
    (comparison, reshuffle, levels, aggregation) over the timed steps, one encrypted query."""
    import torch

    from paper_2104_09583_amd import copse as C
    from paper_2104_09583_amd import synth

    assert torch.cuda.is_available(), "bench needs a GPU"
    stream = torch.cuda.Stream()
    ctxs = {}
    results = {}
    for i, mf in enumerate(synth.TABLE6):
        ch = synth.micro_chain(mf)
        key = tuple(sorted(ch.items()))
        if key not in ctxs:
            ctxs[key] = C.Context(**ch)
            ctxs[key].set_stream(stream.cuda_stream)
        ctx = ctxs[key]
        text = synth.gen_forest_exact(mf, 600 + i)
        seed = synth.crypto_seed(f"COPSE-micro-{mf.name}")
        comp, meta = C.forest_compile(text, mf.n_features, mf.precision, ch["log_n"])
        keys = ctx.keygen(seed, C.compiled_rotations(meta))
        evk = ctx.export_eval(keys)
        model = ctx.model_encode(comp)
        q = synth.gen_queries(1, mf.n_features, mf.precision, 700 + i)
        qct = ctx.query_encrypt(keys, meta, q, seed, group=0)
        for _ in range(args.warmup):
            ctx.evaluate(model, evk, qct)
        ctx.sync()
        per_stage = {n: [] for n in STAGE_NAMES}
        totals = []
        ctx.profile_enable(True)
        for _ in range(args.steps):
            for k in range(C.PROF_KINDS):
                ctx.profile_read(k, reset=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            ctx.evaluate(model, evk, qct)
            e1.record(stream)
            e1.synchronize()
            totals.append(e0.elapsed_time(e1))
            for j, n in enumerate(STAGE_NAMES):
                per_stage[n].append(ctx.profile_read(C.PROF_STAGES[j])["ms"])
        ctx.profile_enable(False)
        results[mf.name] = {"max_depth": mf.max_depth, "precision": mf.precision, "trees": len(mf.branches),
                            "branches": sum(mf.branches), "b": meta.b, "q": meta.q, "d": meta.d,
                            "median_ms": round(percentile(totals, 50), 3),
                            "stages_median_ms": {n: round(percentile(v, 50), 3) for n, v in per_stage.items()}}
        log(mf.name, results[mf.name])
        for h in (qct, model, evk, keys, comp):
            h.close()
    # the paper's trends, as measured ratios
    r = results
    trends = {
        "comparison_depth6_over_depth4": round(r["depth6"]["stages_median_ms"]["comparison"] /
                                               r["depth4"]["stages_median_ms"]["comparison"], 3),
        "levels_depth6_over_depth4": round(r["depth6"]["stages_median_ms"]["levels"] /
                                           r["depth4"]["stages_median_ms"]["levels"], 3),
        "levels_width677_over_width55": round(r["width677"]["stages_median_ms"]["levels"] /
                                              r["width55"]["stages_median_ms"]["levels"], 3),
        "reshuffle_width677_over_width55": round(r["width677"]["stages_median_ms"]["reshuffle"] /
                                                 r["width55"]["stages_median_ms"]["reshuffle"], 3),
        "comparison_prec16_over_prec8": round(r["prec16"]["stages_median_ms"]["comparison"] /
                                              r["prec8"]["stages_median_ms"]["comparison"], 3),
    }
    tot = sum(v["median_ms"] for v in results.values())
    out = {"metric": METRIC, "value": round(1000.0 * len(results) / tot, 3), "unit": "queries/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot / len(results), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "f2_table6", "forests": [m.name for m in synth.TABLE6], "features": 2,
                      "labels": 3, "queries_per_step": 1, "path": "single group, eager, stage events"},
           "per_forest": results, "trends": trends, "roofline": None, "cpu_baseline": None}
    print(json.dumps(out))


# exact modular product-accumulate on the fp64 pipe: h = a b, l = fma(a, b, -h), k = rint(h / q) (a product and a
# rounding), r = fma(-k, q, h) + l, acc += r: 7 fp64 instructions; MI355X issues 256 CUs x 4 SIMDs x 16 fp64
# lanes per clock at 2.4 GHz = 3.93e13 lane-instructions/s (78.6 TFLOP/s counting an fma as two flops)
FP64_LANE_INSTR_PER_S = 256 * 4 * 16 * 2.4e9
MODMUL_INSTR = 7
MODMUL_PEAK_T = FP64_LANE_INSTR_PER_S / MODMUL_INSTR / 1e12


def _matmul_modmuls(meta, encrypted, G, levels):
    """Algorithmic modular products of the MatMul inner sums of one evaluation of G query groups: per nonzero
    diagonal, baby step, group, coefficient and limb, 2 (plaintext diagonal: c0 d, c1 d) or 3 (encrypted
    diagonal: the tensor's a0 b0, a1 b1 and (a0 + a1)(b0 + b1)).  Every diagonal counts for an encrypted
    model (its zero diagonals are encrypted too); for a plaintext model `levels` gives the nonzero counts."""
    N = 1 << meta.log_n
    per = 3 if encrypted else 2
    return sum(n * per * G * nl * N for n, nl in levels)


def run_workload(w, args, steps, warmup, batch, n_groups, profile=True, plain_groups=0, check_labels=True):
    """Times `steps` steps of the workload on the GPU; a step evaluates n_groups query groups (every query of
    the workload by default) in calls of `batch` groups, with the encrypted queries resident in HBM."""
    import torch

    from paper_2104_09583_amd import copse as C
    from paper_2104_09583_amd import synth

    text, queries, seed = synth.workload_inputs(w)
    ch = dict(w.chain)
    if args.server_rep:
        ch["n_data_primes"] += 1   # the replication product takes one level
    n1_r = args.n1_r or w.n1[0]
    n1_l = args.n1_l or w.n1[1]
    log("workload", w.name, "chain", ch)
    t0 = time.perf_counter()
    ctx = C.Context(**ch)
    stream = torch.cuda.Stream()
    ctx.set_stream(stream.cuda_stream)
    if args.server_rep:
        comp, meta = C.forest_compile_ex(
            text, w.shape.n_features, w.shape.precision, w.log_n, fold=w.fold, n1_R=n1_r, n1_L=n1_l,
            server_replication=True,
            privacy_seed=synth.crypto_seed(f"COPSE-shuffle-{w.seed_index}") if args.result_pad >= 0 else None,
            n_pad=max(0, args.result_pad))
    elif args.result_pad < 0:
        comp, meta = C.forest_compile(text, w.shape.n_features, w.shape.precision, w.log_n, fold=w.fold,
                                      n1_R=n1_r, n1_L=n1_l)
    else:
        # result privacy: shuffled result slots and codebook, padded with never-selected labels
        comp, meta = C.forest_compile_private(text, w.shape.n_features, w.shape.precision, w.log_n,
                                              synth.crypto_seed(f"COPSE-shuffle-{w.seed_index}"), args.result_pad,
                                              fold=w.fold, n1_R=n1_r, n1_L=n1_l)
    rots = C.compiled_rotations(meta)
    keys = ctx.keygen(seed, rots)
    evk = ctx.export_eval(keys)
    log(f"keygen {time.perf_counter() - t0:.1f}s ({len(rots)} rotation keys, {keys.nbytes() / 2**30:.2f} GiB)")
    t1 = time.perf_counter()
    model = ctx.model_encode(comp, keys, encrypt=True, seed=seed) if w.encrypted_model else ctx.model_encode(comp)
    log(f"model encode {time.perf_counter() - t1:.1f}s ({model.nbytes() / 2**30:.2f} GiB)")
    qs = meta.queries_per_ct
    n_groups = n_groups or -(-w.n_queries // qs)        # 0: every query of the workload
    batch = min(batch or (w.batch if not args.plain else 1), n_groups)
    qsets = []
    for g in range(n_groups):
        qi = queries[(g * qs) % len(queries):][:qs]
        qsets.append(qi if len(qi) else queries[:qs])
    groups = [ctx.query_encrypt(keys, meta, qsets[g], seed, group=g) for g in range(n_groups)]
    queries_per_step = sum(len(q) for q in qsets)
    log(f"{n_groups} query groups ({queries_per_step} queries) resident, {batch} per call")

    ex = None
    if args.graph:
        t2 = time.perf_counter()
        ex = ctx.exec_create(model, evk, batch)
        log(f"captured evaluation of {batch} group(s) in {time.perf_counter() - t2:.1f}s")

    def call(gs, eager=False):
        if args.plain:
            return [ctx.evaluate_plain(model, evk, g) for g in gs]
        if ex is not None and not eager and len(gs) == batch:
            return ex.run(gs)
        if len(gs) == 1:
            return [ctx.evaluate(model, evk, gs[0])]
        return ctx.evaluate_batch(model, evk, gs)

    def step(eager=False, keep=False):
        out = []
        for g0 in range(0, n_groups, batch):
            r = call(groups[g0:g0 + batch], eager)
            if keep:
                out.extend(r)
        return out

    # the first warmup's results: every query's decrypted labels against the oracle's plain forest walk (part of
    # the CPU-baseline leg: skipped with it)
    res = step(keep=True)
    labels_ok = None
    if check_labels:
        from oracle import forest as F
        _, trees = F.parse_forest(text)
        book = C.compiled_codebook(comp)
        oracle_book = F.codebook(trees)
        for q, r in zip(qsets, res):
            bits = ctx.decrypt_labels(keys, meta, r, len(q))
            for x, b in zip(q, bits):
                plain = F.evaluate(trees, list(x))
                if args.result_pad < 0:
                    assert list(b) == list(plain), "decrypted labels differ from plain evaluation"
                else:
                    assert sorted(book[s] for s in range(len(book)) if b[s]) == \
                        sorted(oracle_book[i] for i in range(len(plain)) if plain[i]), "decrypted labels differ"
        labels_ok = queries_per_step
    del res
    for _ in range(max(0, warmup - 1)):
        step()
    ctx.sync()
    torch.cuda.synchronize()

    prof = None
    per_step = []
    if profile:
        ctx.profile_enable(True)
        for k in range(C.PROF_KINDS):
            ctx.profile_read(k, reset=True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        # per-kernel timings need one event pair per launch: this loop runs the same schedule eagerly
        for _ in range(steps):
            with torch.cuda.stream(stream):
                ev0.record(stream)
            step(eager=True)
            with torch.cuda.stream(stream):
                ev1.record(stream)
            ev1.synchronize()
            per_step.append(ev0.elapsed_time(ev1))
        ctx.sync()
        torch.cuda.synchronize()
        prof = {k: ctx.profile_read(k) for k in range(C.PROF_KINDS)}
        ctx.profile_enable(False)
    # Headline: an unprofiled loop, bracketed by device synchronization, timed on the host clock.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        step()
        e1.record(stream)
    ctx.sync()
    torch.cuda.synchronize()
    wall_clean = time.perf_counter() - wall1
    lat = [e0.elapsed_time(e1) for e0, e1 in evs]
    ms_per_step = wall_clean * 1000.0 / steps

    plain = None
    if plain_groups:
        # the unbatched path on the same slot layout: one group per call, one homomorphic operation per launch
        ctx.evaluate_plain(model, evk, groups[0])
        ctx.sync()
        t3 = time.perf_counter()
        for g in range(plain_groups):
            ctx.evaluate_plain(model, evk, groups[g])
        ctx.sync()
        pms = (time.perf_counter() - t3) * 1000.0 / plain_groups
        plain = {"ms_per_group": round(pms, 3), "queries_per_s": round(qs / (pms / 1000.0), 3),
                 "groups_timed": plain_groups}

    out = {"ctx": ctx, "meta": meta, "queries_per_step": queries_per_step, "n_groups": n_groups, "batch": batch, "ms_per_step": ms_per_step,
           "lat": lat, "per_step": per_step, "prof": prof, "plain": plain, "labels_checked": labels_ok,
           "chain": ch, "model_bytes": model.nbytes(), "keys_bytes": keys.nbytes()}
    for h in groups:
        h.close()
    for h in (ex, model, evk, keys, comp):
        if h is not None:
            h.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c4_encmodel_64x_d8")
    ap.add_argument("--batch", type=int, default=0,
                    help="query groups evaluated together per call (0: the workload's choice)")
    ap.add_argument("--groups", type=int, default=0,
                    help="query groups per step (0: every query of the workload)")
    ap.add_argument("--plain", action="store_true",
                    help="the unbatched path: each group alone, one homomorphic operation per call")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the c3 and c2 lines of the default run")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the unbatched comparison leg of the default run (counter runs: the timed steps' "
                         "launches are then the run's last)")
    ap.add_argument("--graph", action="store_true",
                    help="replay the captured evaluation (HIP graph) instead of launching eagerly; on this "
                         "ROCm stack a replay costs about 1 us more per kernel than the eager launches")
    ap.add_argument("--n1-r", type=int, default=0, help="baby steps of the reshuffle product (0: compiler default)")
    ap.add_argument("--n1-l", type=int, default=0, help="baby steps of the level products (0: compiler default)")
    ap.add_argument("--result-pad", type=int, default=-1,
                    help="result privacy: shuffle the result slots and pad them with this many labels (-1: off)")
    ap.add_argument("--server-rep", action="store_true",
                    help="queries hold each feature once and the server replicates them (one more prime)")
    ap.add_argument("--requests", type=int, default=240, help="serving mix: requests per offered rate")
    ap.add_argument("--rates", type=float, nargs="*", default=[0.25, 0.5, 0.75, 1.0, 1.25],
                    help="serving mix: offered rates as fractions of the burst capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is query-group "
              "data parallelism with no exchange, not built here", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c5_serve_mix":
        return serve_bench(args)
    if args.workload == "f2_table6":
        return micro_bench(args)

    from paper_2104_09583_amd import synth

    w = synth.WORKLOADS[args.workload]
    text, queries, seed = synth.workload_inputs(w)
    # the oracle's CPU baseline first, before anything touches the GPU (its all-core leg forks processes)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, text, queries, seed)
        log(f"cpu baseline {cpu['value']:.5f} queries/s single thread")

    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    from paper_2104_09583_amd import copse as C

    headline_default = args.workload == "c4_encmodel_64x_d8" and not (args.plain or args.graph)
    check = not args.no_cpu_baseline
    r = run_workload(w, args, args.steps, args.warmup, args.batch, args.groups,
                     plain_groups=1 if headline_default and not args.no_plain else 0, check_labels=check)
    meta, prof, per_step = r["meta"], r["prof"], r["per_step"]
    n_groups, batch = r["n_groups"], r["batch"]
    steps = args.steps

    # roofline of the dominant kernel (the class with the largest total time among the single-kernel
    # classes): algorithmic bytes (or modular products) per launch / average launch time, from the profiled loop
    cands = [k for k in KIND_KERNELS if prof[k]["launches"] > 0]
    dom = max(cands, key=lambda k: prof[k]["ms"])
    p = prof[dom]
    avg_ms = p["ms"] / max(1, p["launches"])
    bytes_per_launch = p["bytes"] / max(1, p["launches"])
    achieved = bytes_per_launch / (avg_ms / 1000.0) / 1e9 if avg_ms > 0 else 0.0
    hbm = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(KIND_NAMES[dom], w.name)}
    roofline = dict(hbm)
    if KIND_NAMES[dom] == "matmul_inner" and w.encrypted_model:
        # an encrypted model's inner sums: modular products on the fp64 pipe against the same launch time
        nl_r = r["chain"]["n_data_primes"] - (1 + math.ceil(math.log2(meta.precision)))   # dec level + 1
        mods = _matmul_modmuls(meta, True, n_groups, [(meta.q, nl_r), (meta.d * meta.b, nl_r - 1)])
        mods_per_launch = mods * steps / max(1, p["launches"])
        alu_t = mods_per_launch / (avg_ms / 1000.0) / 1e12
        alu = {"bound": "alu", "achieved": round(alu_t, 3), "peak": round(MODMUL_PEAK_T, 3), "unit": "Tmodmul/s",
               "frac": round(alu_t / MODMUL_PEAK_T, 4), "traffic": hbm["traffic"],
               "modmuls_per_launch": round(mods_per_launch)}
        roofline = dict(alu) if alu["frac"] >= hbm["frac"] else dict(hbm)
        roofline["hbm"] = hbm
        roofline["alu"] = alu
    roofline.update({"kernel": KIND_KERNELS[dom], "class": KIND_NAMES[dom], "avg_launch_ms": round(avg_ms, 5),
                     "algorithmic_bytes_per_launch": round(bytes_per_launch),
                     "share_of_step": round(p["ms"] / sum(per_step), 3)})
    kernels = {KIND_NAMES[k]: {"launches_per_step": prof[k]["launches"] / steps,
                               "ms_per_step": round(prof[k]["ms"] / steps, 3),
                               "avg_launch_us": round(1000 * prof[k]["ms"] / max(1, prof[k]["launches"]), 2),
                               "algorithmic_bytes_per_launch": round(prof[k]["bytes"] / max(1, prof[k]["launches"])),
                               "achieved_GBps": round(prof[k]["bytes"] / max(1e-9, prof[k]["ms"]) / 1e6, 1)}
               for k in KERNEL_KINDS if prof[k]["launches"] > 0}
    stages = {STAGE_NAMES[j]: round(prof[k]["ms"] / steps, 3)
              for j, k in enumerate(C.PROF_STAGES) if prof[k]["launches"] > 0}
    ms_per_step = r["ms_per_step"]
    value = r["queries_per_step"] / (ms_per_step / 1000.0)
    # reference copy of known size for the byte counters of a separate --pmc run
    r["ctx"].calib_copy(256 << 20)
    r["ctx"].sync()
    r["ctx"].close()

    extra = {}
    if r["plain"]:
        extra["plain_path"] = dict(r["plain"], workload=w.name)
        extra["batched_over_plain"] = round(value / r["plain"]["queries_per_s"], 2)
    if headline_default and not args.no_extras:
        for name, plain_g, stx in (("c3_batched_32x_d6", 1, 3), ("c2_forest16_d5", 0, 20)):
            wx = synth.WORKLOADS[name]
            rx = run_workload(wx, args, stx, 2, 0, 0, profile=False, plain_groups=plain_g, check_labels=check)
            vx = rx["queries_per_step"] / (rx["ms_per_step"] / 1000.0)
            e = {"value": round(vx, 3), "unit": "queries/s", "ms_per_step": round(rx["ms_per_step"], 3),
                 "steps": stx, "queries_per_step": rx["queries_per_step"], "query_groups_per_step": rx["n_groups"],
                 "groups_per_call": rx["batch"],
                 "latency_ms": {"p50": round(percentile(rx["lat"], 50), 3),
                                "p99": round(percentile(rx["lat"], 99), 3)},
                 "labels_checked": rx["labels_checked"]}
            if rx["plain"]:
                e["plain_path"] = rx["plain"]
                e["batched_over_plain"] = round(vx / rx["plain"]["queries_per_s"], 2)
            extra[name] = e
            rx["ctx"].close()
            log(name, e)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "trees": w.shape.n_trees, "max_depth": w.shape.max_depth,
                   "features": w.shape.n_features, "precision": w.shape.precision, "classes": w.shape.n_classes,
                   "queries_per_step": r["queries_per_step"], "query_groups_per_step": n_groups,
                   "groups_per_call": batch,
                   "path": "plain (one group per call, one operation per launch)" if args.plain else
                           ("batched" if batch > 1 else "single group") + (", captured graph" if args.graph else ", eager"),
                   "N": 1 << w.log_n, "data_primes": r["chain"]["n_data_primes"], "special_primes": r["chain"]["alpha"],
                   "model": "plaintext" if not w.encrypted_model else "encrypted",
                   "model_GiB": round(r["model_bytes"] / 2**30, 2), "keys_GiB": round(r["keys_bytes"] / 2**30, 2),
                   "b": meta.b, "m": meta.m, "q": meta.q, "d": meta.d, "W": meta.block_w,
                   "result_pad": args.result_pad, "server_replication": bool(args.server_rep),
                   "n1_R": meta.n1_R, "n1_L": meta.n1_L},
        "labels_checked": r["labels_checked"],
        "latency_ms": {"p50": round(percentile(r["lat"], 50), 3), "p99": round(percentile(r["lat"], 99), 3),
                       "profiled_mean": round(sum(per_step) / len(per_step), 3)},
        "roofline": roofline,
        "kernels": kernels,
        "stages_ms_per_step": stages,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
