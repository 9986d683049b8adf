"""The autotuner's knobs change no bit: every committed tuned setting (paper_2104_09583_amd/tuning.json), and
each knob at the ends of its range, gives the same result ciphertexts as the built-in launch shapes, for a
plaintext and an encrypted model, one group and a batch of eight, on the ring of the fused passes.  (The
full-size parity tests run with the committed settings installed, as copse.Context does by default.)"""
import math
import sys

import numpy as np
import pytest

from oracle import circuit as CI
from oracle import compiler as OC
from paper_2104_09583_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.stderr, flush=True)


def _settings(C):
    out = [e["knobs"] for e in C.load_tuning()]
    out += [dict(mm_cap=4, mm_waves=4, ks_jobs=1, bridge_wgs=64, gsum_b=4),
            dict(mm_cap=32, mm_waves=8, ks_jobs=32, bridge_wgs=8192, gsum_b=8),
            dict(mm_cap=16, ks_jobs=7, bridge_wgs=2048)]
    return out


@pytest.mark.parametrize("enc", [False, True])
def test_tuned_launch_shapes_keep_the_bits(enc):
    from paper_2104_09583_amd import copse as C
    shape = synth.ForestShape(5, 4, 0.85, 3, 4, 3)
    text = synth.gen_forest_text(shape, 91)
    oc = OC.compile_forest(text, 3, 4)
    need = CI.seccomp_depth(4) + 2 + math.ceil(math.log2(oc.d))
    ctx = C.Context(13, need + 1, 1 << 49, 1 << 42, 3, 1 << 49, tuning=False)
    comp, meta = C.forest_compile(text, 3, 4, 13, n1_R=3, n1_L=3)
    kseed = b"\x71" * 32
    keys = ctx.keygen(kseed, C.compiled_rotations(meta))
    evk = ctx.export_eval(keys)
    model = ctx.model_encode(comp, keys if enc else None, encrypt=enc, seed=kseed if enc else None)
    groups = [ctx.query_encrypt(keys, meta, synth.gen_queries(meta.queries_per_ct, 3, 4, 950 + g), kseed, group=g)
              for g in range(8)]

    def run(knobs, G):
        ctx.set_tuning([dict(log_n=13, top_level=ctx.L, batch=[1, 64], model=-1, knobs=knobs)] if knobs else [])
        res = ctx.evaluate_batch(model, evk, groups[:G]) if G > 1 else [ctx.evaluate(model, evk, groups[0])]
        return [[p.copy() for p in ctx.export(r)[0]["polys"]] for r in res]

    for G in (1, 8):
        want = run(None, G)
        for knobs in _settings(C):
            say("enc", enc, "groups", G, "knobs", knobs)
            got = run(knobs, G)
            for g in range(G):
                assert all((a == b).all() for a, b in zip(got[g], want[g])), (knobs, g)


def test_tuning_entries_are_validated():
    from paper_2104_09583_amd import copse as C
    ctx = C.Context(12, 4, 1 << 49, 1 << 42, 2, 1 << 49, tuning=False)
    for bad in (dict(mm_cap=40), dict(mm_waves=6), dict(ks_jobs=64), dict(bridge_wgs=9), dict(gsum_b=2)):
        with pytest.raises(C.CopseError) as e:
            ctx.set_tuning([dict(log_n=12, top_level=3, batch=[1, 1], knobs=bad)])
        assert e.value.code == C.COPSE_EINVAL
    ctx.set_tuning([])
