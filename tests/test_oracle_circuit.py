"""End-to-end pins of the oracle's encrypted Algorithm 1 at small ring sizes:
decrypted labels equal the plain forest evaluation (the definition), every
decrypted intermediate equals the plaintext slot simulator in every slot, and
operation counts follow the closed forms."""
import math

import numpy as np
import pytest

from oracle import bgv as B
from oracle import circuit as CI
from oracle import compiler as C
from oracle import forest as F
from oracle import nt
from oracle import slotsim as S
from paper_2104_09583_amd import synth

T = 65537


def _setup(seed, fold, enc, trees=3, depth=4, feats=3, prec=4, classes=3, log_n=8, split=0.7):
    shape = synth.ForestShape(trees, depth, split, feats, prec, classes)
    text = synth.gen_forest_text(shape, seed)
    c = C.compile_forest(text, feats, prec)
    need = CI.seccomp_depth(prec) + (1 if fold else 2) + (math.ceil(math.log2(c.d)) if c.d > 1 else 0)
    ch = nt.make_chain(log_n, T, n_data=need + 1, q0_max=1 << 49, data_max=1 << 40, alpha=3,
                       special_max=1 << 49)
    sc = B.BGV(ch)
    pl = CI.make_plan(c, sc.N, sc.L, fold=fold, encrypted_model=enc)
    assert pl.levels["labels"] == 0
    kseed = bytes([seed]) * 32
    keys = sc.keygen(kseed, rotations=pl.rotations())
    queries = synth.gen_queries(pl.layout.Qs, feats, prec, 50 + seed)
    X = CI.encrypt_queries(sc, keys, pl, queries, kseed, 0)
    model = CI.encrypt_model(sc, keys, pl, kseed) if enc else CI.encode_model(sc, pl)
    _, tr = F.parse_forest(text)
    return sc, keys, pl, queries, X, model, tr, c


@pytest.mark.parametrize("seed,fold,enc", [(1, False, False), (2, True, False), (3, False, True),
                                           (4, True, True), (5, False, False)])
def test_encrypted_algorithm_matches_definition_and_slots(seed, fold, enc):
    sc, keys, pl, queries, X, model, trees, c = _setup(seed, fold, enc)
    ev = CI.Evaluator(sc, keys, pl)
    out = ev.run(X, model)
    lab = CI.decrypt_labels(sc, keys, pl, out["result"], len(queries))
    want = np.array([F.evaluate(trees, list(x)) for x in queries])
    assert (lab == want).all()
    sim = S.run(c, queries, n_slots=sc.N, fold_reshuffle=fold, n1_R=pl.n1_R, n1_L=pl.n1_L)
    assert (sc.decrypt_slots(keys, out["dec"]) == sim["dec"]).all()
    if not fold:
        assert (sc.decrypt_slots(keys, out["branches"]) == sim["branches"]).all()
    for l in range(c.d):
        assert (sc.decrypt_slots(keys, out["levels"][l]) == sim["levels"][l]).all()
    assert (sc.decrypt_slots(keys, out["result"]) == sim["labels"]).all()
    assert sc.margin_bits(keys, out["result"]) > 10


def test_determinism_of_ciphertexts():
    sc, keys, pl, queries, X, model, trees, c = _setup(7, False, False)
    r1 = CI.Evaluator(sc, keys, pl).run(X, model)["result"]
    r2 = CI.Evaluator(sc, keys, pl).run(X, model)["result"]
    assert all((a == b).all() for a, b in zip(r1.polys, r2.polys))


def test_operation_counts_closed_form():
    """SecComp's products: every aligned block of two or more of the n = p - 1 equality bits
    (sum_s floor(n / 2^s)) plus popcount(i) merges for term i = 1..n (21 -> 16 for p = 8);
    MultAll uses d-1 products; with n1 = 1 (no baby steps) the rotation count is the paper's
    q + d b minus the d + 1 rotations by zero (Table 2)."""
    sc, keys, pl, queries, X, model, trees, c = _setup(8, False, False)
    p = c.precision
    n = p - 1
    blocks = sum(n >> s for s in range(1, n.bit_length() + 1))
    merges = sum(bin(i).count("1") for i in range(1, n + 1))
    ev = CI.Evaluator(sc, keys, pl)
    ev.seccomp(X, model)
    assert ev.counts["mul"] == blocks + merges
    ev2 = CI.Evaluator(sc, keys, pl)
    ev2.counts["mul"] = 0
    S.multall(list(range(c.d)), lambda a, b: ev2.counts.__setitem__("mul", ev2.counts["mul"] + 1) or 0)
    assert ev2.counts["mul"] == c.d - 1
    pl1 = CI.make_plan(c, sc.N, sc.L, n1_R=1, n1_L=1)
    rots = [r for r in pl1.rotations()]
    # distinct giant steps: 1..q-1 for R and 1..b-1 for the levels (shared keys)
    assert set(rots) == set(range(1, max(c.q, c.b)))
    n_rot_ops = (c.q - 1) + c.d * (c.b - 1)
    assert n_rot_ops == c.q + c.d * c.b - (c.d + 1)


def test_single_leaf_tree_and_full_block():
    """A tree that is a lone label always selects it; queries fill every block."""
    text = "a b c\nB 0 3 L 0 L 1\nL 2\n"
    c = C.compile_forest(text, 2, 2)
    ch = nt.make_chain(6, T, n_data=1 + CI.seccomp_depth(2) + 2 + 1, q0_max=1 << 49,
                       data_max=1 << 40, alpha=2, special_max=1 << 49)
    sc = B.BGV(ch)
    pl = CI.make_plan(c, sc.N, sc.L)
    keys = sc.keygen(b"\x21" * 32, rotations=pl.rotations())
    queries = np.array([[x, 0] for x in range(pl.layout.Qs)]) % 4
    X = CI.encrypt_queries(sc, keys, pl, queries, b"\x22" * 32, 3)
    out = CI.Evaluator(sc, keys, pl).run(X, CI.encode_model(sc, pl))
    lab = CI.decrypt_labels(sc, keys, pl, out["result"], len(queries))
    _, trees = F.parse_forest(text)
    assert (lab == np.array([F.evaluate(trees, list(x)) for x in queries])).all()


@pytest.mark.parametrize("seed,fold", [(11, False), (12, True)])
def test_server_replication_encrypted(seed, fold):
    """Queries holding each feature once; the server's replication product before the comparison
    (one more level): decrypted labels = tree walk, and every intermediate = the slot simulator."""
    shape = synth.ForestShape(3, 4, 0.7, 3, 4, 3)
    text = synth.gen_forest_text(shape, seed)
    c = C.server_replicated(C.compile_forest(text, 3, 4))
    need = 1 + CI.seccomp_depth(4) + (1 if fold else 2) + math.ceil(math.log2(c.d))
    sc = B.BGV(nt.make_chain(9, T, n_data=need + 1, q0_max=1 << 49, data_max=1 << 40, alpha=3,
                             special_max=1 << 49))
    pl = CI.make_plan(c, sc.N, sc.L, fold=fold)
    assert pl.server_rep and pl.levels["labels"] == 0 and pl.levels["top"] == sc.L - 1
    kseed = bytes([seed]) * 32
    keys = sc.keygen(kseed, rotations=pl.rotations())
    queries = synth.gen_queries(pl.layout.Qs, 3, 4, 70 + seed)
    X = CI.encrypt_queries(sc, keys, pl, queries, kseed, 0)
    out = CI.Evaluator(sc, keys, pl).run(X, CI.encode_model(sc, pl))
    _, trees = F.parse_forest(text)
    lab = CI.decrypt_labels(sc, keys, pl, out["result"], len(queries))
    assert (lab == np.array([F.evaluate(trees, list(x)) for x in queries])).all()
    sim = S.run(c, queries, n_slots=sc.N, fold_reshuffle=fold, n1_R=pl.n1_R, n1_L=pl.n1_L)
    assert (sc.decrypt_slots(keys, out["dec"]) == sim["dec"]).all()
    assert sc.margin_bits(keys, out["result"]) > 10
    with pytest.raises(ValueError):
        CI.make_plan(c, sc.N, sc.L, encrypted_model=True)
