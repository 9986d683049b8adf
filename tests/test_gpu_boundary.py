"""Boundary checks through the C ABI: handles made by another context (another ring or chain) are
refused with EINVAL before any kernel reads them, and decryption refuses a result that is not N-hot
(one label per tree, Section 4.1 "Classification Result")."""
import math
import sys

import numpy as np
import pytest

from oracle import circuit as CI
from oracle import compiler as OC
from oracle import forest as F
from paper_2104_09583_amd import synth

pytestmark = pytest.mark.gpu
T = 65537


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def two_contexts():
    from paper_2104_09583_amd import copse as C
    shape = synth.ForestShape(2, 3, 0.8, 3, 4, 2)
    text = synth.gen_forest_text(shape, 81)
    oc = OC.compile_forest(text, 3, 4)
    need = CI.seccomp_depth(4) + 2 + math.ceil(math.log2(max(2, oc.d)))
    out = []
    for log_n, extra in ((11, 1), (12, 2)):
        ctx = C.Context(log_n, need + extra, 1 << 49, 1 << 42, 3, 1 << 49)
        comp, meta = C.forest_compile(text, 3, 4, log_n)
        seed = bytes([90 + log_n]) * 32
        keys = ctx.keygen(seed, C.compiled_rotations(meta))
        model = ctx.model_encode(comp)
        q = synth.gen_queries(meta.queries_per_ct, 3, 4, 82)
        qct = ctx.query_encrypt(keys, meta, q, seed, group=0)
        out.append(dict(ctx=ctx, comp=comp, meta=meta, keys=keys, model=model, q=q, qct=qct, text=text))
    return C, out


def test_evaluate_refuses_handles_of_another_context(two_contexts):
    C, (a, b) = two_contexts
    say("cross-context handles")
    cases = [
        ("model", lambda: a["ctx"].evaluate(b["model"], a["keys"], a["qct"])),
        ("keys", lambda: a["ctx"].evaluate(a["model"], b["keys"], a["qct"])),
        ("query", lambda: a["ctx"].evaluate(a["model"], a["keys"], b["qct"])),
        ("batch query", lambda: a["ctx"].evaluate_batch(a["model"], a["keys"], [a["qct"], b["qct"]])),
        ("plain path keys", lambda: a["ctx"].evaluate_plain(a["model"], b["keys"], a["qct"])),
        ("decrypt keys", lambda: a["ctx"].decrypt_slots(b["keys"], a["qct"])),
        ("rotation keys", lambda: a["ctx"].rotate_many(b["keys"], a["qct"], [1])),
        ("query encrypt keys", lambda: a["ctx"].query_encrypt(b["keys"], a["meta"], a["q"], b"\x01" * 32)),
        ("export eval keys", lambda: a["ctx"].export_eval(b["keys"])),
    ]
    for name, f in cases:
        with pytest.raises(C.CopseError) as e:
            f()
        assert e.value.code == C.COPSE_EINVAL, name
    srv = C.Server(a["ctx"], 64 << 30, max_batch=2)
    with pytest.raises(C.CopseError) as e:
        srv.add_model(b["model"], a["keys"])
    assert e.value.code == C.COPSE_EINVAL
    mid = srv.add_model(a["model"], a["keys"])
    with pytest.raises(C.CopseError) as e:
        srv.submit(mid, b["ctx"].query_encrypt(b["keys"], b["meta"], b["q"], b"\x02" * 32))
    assert e.value.code == C.COPSE_EINVAL
    srv.close()
    # the context still evaluates correctly afterwards
    res = a["ctx"].evaluate(a["model"], a["keys"], a["qct"])
    _, trees = F.parse_forest(a["text"])
    bits = a["ctx"].decrypt_labels(a["keys"], a["meta"], res, len(a["q"]))
    assert (bits == np.array([F.evaluate(trees, list(x)) for x in a["q"]])).all()


def test_decrypt_refuses_a_result_that_is_not_n_hot(two_contexts):
    C, (a, _) = two_contexts
    ctx, meta = a["ctx"], a["meta"]
    res = ctx.evaluate(a["model"], a["keys"], a["qct"])
    bits = ctx.decrypt_labels(a["keys"], meta, res, len(a["q"]))
    assert (bits.sum(axis=1) == meta.n_trees).all()
    # set one more label of query 0: a valid 0/1 vector with n_trees + 1 ones
    j = int(np.flatnonzero(bits[0] == 0)[0])
    slots = np.zeros((2, ctx.N // 2), dtype=np.uint64)
    slots[0, j] = 1
    bad = ctx.op(None, C.OP_ADD_PLAIN, res, slots=slots)
    with pytest.raises(C.CopseError) as e:
        ctx.decrypt_labels(a["keys"], meta, bad, len(a["q"]))
    assert e.value.code == C.COPSE_ENOISE
