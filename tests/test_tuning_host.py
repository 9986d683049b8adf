"""The autotuner's host side on the CPU: the committed choices (paper_2104_09583_amd/tuning.json) are
well-formed and inside the ranges copse_ctx_set_tuning accepts, every candidate the tuner tries is inside
them too, and saving an entry replaces the one with the same key.  (That tuned settings keep the bits is
the GPU test tests/test_gpu_tuning.py.)"""
import json

import pytest

from paper_2104_09583_amd import autotune as AT
from paper_2104_09583_amd import copse as C
from paper_2104_09583_amd import synth

# the ranges copse_ctx_set_tuning accepts (0: the built-in choice)
ACCEPT = {
    "mm_cap": lambda v: v == 0 or 4 <= v <= 32,
    "mm_waves": lambda v: v in (0, 4, 8),
    "ks_jobs": lambda v: v == 0 or 1 <= v <= 32,
    "bridge_wgs": lambda v: v == 0 or 64 <= v <= 8192,
    "gsum_b": lambda v: v in (0, 4, 8),
}


def test_knob_names_match_the_binding():
    assert set(ACCEPT) == set(C.TUNE_KNOBS)


def test_committed_choices_are_valid():
    entries = C.load_tuning()
    assert entries, "no committed tuning entries"
    keys = set()
    for e in entries:
        k = (e["log_n"], e["top_level"], tuple(e["batch"]), e["model"])
        assert k not in keys, f"two entries for {k}"
        keys.add(k)
        lo, hi = e["batch"]
        assert 1 <= lo <= hi
        assert e["model"] in (-1, 0, 1)
        for name, v in e["knobs"].items():
            assert name in ACCEPT and ACCEPT[name](v), (e["workload"], name, v)
        # the entry's key is its workload's ring, top data level and model kind
        w = synth.WORKLOADS[e["workload"]]
        assert e["log_n"] == w.log_n
        assert e["top_level"] == w.chain["n_data_primes"] - 1
        assert e["model"] == (1 if w.encrypted_model else 0)
        # the choice is the best the tuner saw, and it was one of its trials (or the built-in choice)
        assert e["ms_tuned"] <= e["ms_builtin"]
        assert not e["knobs"] or any(t["knobs"] == e["knobs"] for t in e["tried"])
        assert all(t["ms"] >= 0.99 * e["ms_tuned"] or t["knobs"] == e["knobs"] for t in e["tried"])


@pytest.mark.parametrize("enc", [False, True])
@pytest.mark.parametrize("G", [1, 2, 8, 16])
def test_candidates_are_accepted_values(enc, G):
    cands = AT.candidates(enc, G)
    for name, vals in cands.items():
        assert vals and all(ACCEPT[name](v) and v != 0 for v in vals), (name, vals)
    # batch-only knobs appear only with a batch; eight waves per workgroup need a multiple of 8
    assert ("gsum_b" in cands) == (G > 1)
    assert ("mm_waves" in cands) == (G > 1 and G % 8 == 0)


def test_save_replaces_the_entry_with_the_same_key(tmp_path):
    path = tmp_path / "tuning.json"
    base = dict(log_n=15, top_level=10, batch=[16, 16], model=1, workload="w", ms_builtin=2.0, ms_tuned=1.5,
                reps=3, tried=[])
    AT.save(dict(base, knobs={"mm_cap": 8}), str(path))
    AT.save(dict(base, batch=[8, 8], knobs={}), str(path))
    AT.save(dict(base, knobs={"ks_jobs": 16}), str(path))
    doc = json.loads(path.read_text())
    got = {tuple(e["batch"]): e["knobs"] for e in doc["entries"]}
    assert got == {(8, 8): {}, (16, 16): {"ks_jobs": 16}}
    assert [e["batch"] for e in doc["entries"]] == [[8, 8], [16, 16]]
