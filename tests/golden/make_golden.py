"""Writes tests/golden/<workload>.json: the oracle's result ciphertext of one
query group of a full-size workload (SHA-256 of its coefficient residues plus
a few sampled coefficients) and the plain forest labels.  Calls only oracle/
and the shared input generator.

    python tests/golden/make_golden.py c2_forest16_d5 [c3_batched_32x_d6 ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import bgv as B  # noqa: E402
from oracle import circuit as CI  # noqa: E402
from oracle import compiler as OC  # noqa: E402
from oracle import forest as F  # noqa: E402
from oracle import nt  # noqa: E402
from paper_2104_09583_amd import synth  # noqa: E402


def digest(polys):
    h = hashlib.sha256()
    for p in polys:
        h.update(np.ascontiguousarray(p, dtype="<u8").tobytes())
    return h.hexdigest()


def make(name: str, group: int = 0):
    w = synth.WORKLOADS[name]
    text, queries, seed = synth.workload_inputs(w)
    ch = w.chain
    sc = B.BGV(nt.make_chain(ch["log_n"], 65537, ch["n_data_primes"], ch["q0_max"], ch["data_max"], ch["alpha"],
                             ch["special_max"]))
    oc = OC.compile_forest(text, w.shape.n_features, w.shape.precision)
    pl = CI.make_plan(oc, sc.N, sc.L, fold=w.fold, encrypted_model=w.encrypted_model, n1_R=w.n1[0], n1_L=w.n1[1])
    t0 = time.time()
    keys = sc.keygen(seed, rotations=pl.rotations())
    nq = min(pl.layout.Qs, len(queries) - group * pl.layout.Qs)
    qs = queries[group * pl.layout.Qs:group * pl.layout.Qs + nq]
    X = CI.encrypt_queries(sc, keys, pl, qs, seed, group)
    model = CI.encrypt_model(sc, keys, pl, seed) if w.encrypted_model else CI.encode_model(sc, pl)
    out = CI.Evaluator(sc, keys, pl).run(X, model)
    res = out["result"]
    lab = CI.decrypt_labels(sc, keys, pl, res, nq)
    _, trees = F.parse_forest(text)
    want = np.array([F.evaluate(trees, list(x)) for x in qs])
    assert (lab == want).all()
    rng = np.random.default_rng(0)
    idx = sorted(int(i) for i in rng.choice(sc.N, 16, replace=False))
    rec = {
        "workload": name, "group": group, "n_queries": int(nq), "level": res.level,
        "sha256": digest(res.polys), "sample_index": idx,
        "sample_c0": [int(res.polys[0][0, i]) for i in idx], "sample_c1": [int(res.polys[1][0, i]) for i in idx],
        "labels": want.tolist(), "margin_bits": round(sc.margin_bits(keys, res), 2),
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print(name, rec["sha256"], rec["margin_bits"], rec["oracle_seconds"], flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:]:
        make(n)
