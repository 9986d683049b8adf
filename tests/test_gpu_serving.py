"""Serving loop on the GPU: requests for resident models submitted in a mix,
also while earlier batches are on the device, are batched as they arrive and
run on two device lanes at once; every result is bit-identical to evaluating
that request alone (and, for the full-size serving forests, to the stored
oracle result), labels equal plain evaluation, and admission refuses what does
not fit the device-memory budget."""
import math
import sys
import threading

import numpy as np
import pytest

from oracle import circuit as CI
from oracle import compiler as OC
from oracle import forest as F
from paper_2104_09583_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def test_serving_mix_matches_alone():
    from paper_2104_09583_amd import copse as C
    shapes = [synth.ForestShape(3, 4, 0.7, 3, 4, 3), synth.ForestShape(2, 3, 0.9, 3, 4, 2)]
    texts = [synth.gen_forest_text(s, 70 + i) for i, s in enumerate(shapes)]
    need = 0
    for s, t in zip(shapes, texts):
        oc = OC.compile_forest(t, s.n_features, s.precision)
        need = max(need, CI.seccomp_depth(s.precision) + 2 + math.ceil(math.log2(oc.d)))
    log_n = 11
    ctx = C.Context(log_n, need + 1, 1 << 49, 1 << 42, 3, 1 << 49)
    seed = b"\x61" * 32
    comps = [C.forest_compile(t, s.n_features, s.precision, log_n) for s, t in zip(shapes, texts)]
    rots = sorted(set(r for _, m in comps for r in C.compiled_rotations(m)))
    keys = ctx.keygen(seed, rots)
    evk = ctx.export_eval(keys)
    models = [ctx.model_encode(cp) for cp, _ in comps]
    srv = C.Server(ctx, 64 << 30, max_batch=4)
    mids = [srv.add_model(m, evk) for m in models]
    # requests: (model, query set)
    reqs = []
    for r in range(10):
        mi = r % 2
        meta = comps[mi][1]
        q = synth.gen_queries(meta.queries_per_ct, shapes[mi].n_features, shapes[mi].precision, 3000 + r)
        reqs.append((mi, q))
    cts = [ctx.query_encrypt(keys, comps[mi][1], q, seed, group=r) for r, (mi, q) in enumerate(reqs)]
    say("submitting", len(reqs), "requests")
    tickets = [None] * len(reqs)

    def submit(lo, hi):
        for r in range(lo, hi):
            tickets[r] = srv.submit(mids[reqs[r][0]], cts[r])

    ths = [threading.Thread(target=submit, args=(0, 5)), threading.Thread(target=submit, args=(5, 10))]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    results = [srv.wait(t, 120000) for t in tickets]
    lat = [srv.latency_ms(t) for t in tickets]
    assert all(x > 0 for x in lat)
    srv.close()
    say("comparing with single evaluations")
    for r, (mi, q) in enumerate(reqs):
        alone = ctx.evaluate(models[mi], evk, ctx.query_encrypt(keys, comps[mi][1], q, seed, group=r))
        ea, eb = ctx.export(alone)[0], ctx.export(results[r])[0]
        assert all((a == b).all() for a, b in zip(ea["polys"], eb["polys"]))
        _, trees = F.parse_forest(texts[mi])
        bits = ctx.decrypt_labels(keys, comps[mi][1], results[r], len(q))
        assert (bits == np.array([F.evaluate(trees, list(x)) for x in q])).all()


def test_serving_admission_budget():
    from paper_2104_09583_amd import copse as C
    shape = synth.ForestShape(2, 3, 0.9, 3, 4, 2)
    text = synth.gen_forest_text(shape, 5)
    oc = OC.compile_forest(text, 3, 4)
    need = CI.seccomp_depth(4) + 2 + math.ceil(math.log2(oc.d))
    ctx = C.Context(11, need + 1, 1 << 49, 1 << 42, 3, 1 << 49)
    comp, meta = C.forest_compile(text, 3, 4, 11)
    keys = ctx.keygen(b"\x62" * 32, C.compiled_rotations(meta))
    model = ctx.model_encode(comp)
    tiny = C.Server(ctx, 1 << 20, max_batch=2)
    with pytest.raises(C.CopseError) as e:
        tiny.add_model(model, keys)
    assert e.value.code == C.COPSE_ENOMEM
    tiny.close()
    srv = C.Server(ctx, model.nbytes() + keys.nbytes() + (1 << 20), max_batch=2)
    mid = srv.add_model(model, keys)
    q = ctx.query_encrypt(keys, meta, synth.gen_queries(1, 3, 4, 1), b"\x62" * 32)
    with pytest.raises(C.CopseError) as e:
        srv.submit(mid, q)
    assert e.value.code == C.COPSE_ENOMEM
    srv.close()


def _digest(polys):
    import hashlib
    h = hashlib.sha256()
    for p in polys:
        h.update(np.ascontiguousarray(p, dtype="<u8").tobytes())
    return h.hexdigest()


def test_serving_full_size_mix_with_arrivals_during_gpu_work():
    """The three resident serving forests (8 trees of depth 4, 32 of depth 6, 64 of depth 8), each with its
    owner's keys; one-query requests submitted by one thread with gaps while waiter threads drive the device,
    so that requests arrive while batches of other forests run.  The golden query of each forest (query group
    0 of its workload) equals the stored oracle result; every request equals its evaluation alone."""
    import json
    import os
    import time
    from paper_2104_09583_amd import copse as C
    names = synth.SERVE_MIX
    ws = [synth.WORKLOADS[n] for n in names]
    ctx = C.Context(**ws[0].chain)
    srv = C.Server(ctx, 200 << 30, max_batch=4)
    forests = []
    for w in ws:
        text, queries, seed = synth.workload_inputs(w)
        comp, meta = C.forest_compile(text, w.shape.n_features, w.shape.precision, w.log_n)
        keys = ctx.keygen(seed, C.compiled_rotations(meta))
        evk = ctx.export_eval(keys)
        model = ctx.model_encode(comp)
        with open(os.path.join(os.path.dirname(__file__), "golden", f"{w.name}.json")) as f:
            gold = json.load(f)
        forests.append(dict(w=w, text=text, queries=queries, seed=seed, meta=meta, keys=keys, evk=evk,
                            model=model, gold=gold, mid=srv.add_model(model, evk)))
        say("resident", w.name, "model GiB", round(model.nbytes() / 2**30, 2))
    rng = np.random.default_rng(77)
    reqs = []
    for fi, fo in enumerate(forests):
        w = fo["w"]
        reqs.append((fi, fo["queries"][:1], 0))                       # the golden query
        for r in range(3):
            reqs.append((fi, synth.gen_queries(1, w.shape.n_features, w.shape.precision, 4000 + 10 * fi + r),
                         1 + r))
    order = rng.permutation(len(reqs))
    cts = {i: ctx.query_encrypt(forests[reqs[i][0]]["keys"], forests[reqs[i][0]]["meta"], reqs[i][1],
                                forests[reqs[i][0]]["seed"], group=reqs[i][2]) for i in range(len(reqs))}
    ctx.sync()
    tickets = {}
    results = {}
    lock = threading.Lock()
    ready = threading.Condition(lock)

    def waiter(i):
        with lock:
            while i not in tickets:
                ready.wait()
        results[i] = srv.wait(tickets[i], 300000)

    ths = [threading.Thread(target=waiter, args=(i,)) for i in range(len(reqs))]
    for th in ths:
        th.start()
    say("submitting", len(reqs), "requests with gaps")
    for k, i in enumerate(order):
        t = srv.submit(forests[reqs[i][0]]["mid"], cts[i])
        with lock:
            tickets[i] = t
            ready.notify_all()
        time.sleep(0.004 if k % 3 else 0.0)
    for th in ths:
        th.join()
    lat = [srv.latency_ms(tickets[i]) for i in range(len(reqs))]
    assert all(x > 0 for x in lat)
    srv.close()
    say("comparing", len(reqs), "results")
    for i, (fi, q, group) in enumerate(reqs):
        fo = forests[fi]
        got = ctx.export(results[i])[0]
        if group == 0:
            assert got["level"] == fo["gold"]["level"]
            assert _digest(got["polys"]) == fo["gold"]["sha256"], fo["w"].name
        alone = ctx.evaluate(fo["model"], fo["evk"], ctx.query_encrypt(fo["keys"], fo["meta"], q, fo["seed"],
                                                                        group=group))
        ea = ctx.export(alone)[0]
        assert all((a == b).all() for a, b in zip(ea["polys"], got["polys"])), (fo["w"].name, group)
        _, trees = F.parse_forest(fo["text"])
        bits = ctx.decrypt_labels(fo["keys"], fo["meta"], results[i], 1)
        assert (bits == np.array([F.evaluate(trees, list(x)) for x in q])).all()
