"""Host-side checks of the GPU library that need no GPU: the shared object
loads and exports every declared symbol, and its SHAKE-256, samplers, prime
chain, slot encoder and forest compiler agree with independent
implementations (hashlib and the oracle)."""
import hashlib
import os
import re

import numpy as np
import pytest

from oracle import bgv as B
from oracle import circuit as CI
from oracle import compiler as OC
from oracle import nt, sampling
from paper_2104_09583_amd import copse as C
from paper_2104_09583_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "copse.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(copse_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = C.lib()
    names = declared_symbols()
    assert len(names) > 30
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.parametrize("n_in,n_out", [(0, 32), (3, 136), (135, 200), (136, 137), (137, 1000), (500, 64)])
def test_shake256_matches_hashlib(n_in, n_out):
    msg = bytes((i * 7 + 3) % 256 for i in range(n_in))
    assert C.shake256(msg, n_out) == hashlib.shake_256(msg).digest(n_out)


def test_samplers_match_oracle_streams():
    seed = bytes(range(32))
    q = nt.make_chain(15, 65537, 3, 1 << 48, 1 << 42, 2, 1 << 48).data[1]
    assert (C.sample(seed, "ksk.a", 5 * 256 + 1, 3, 0, q, 5000) ==
            sampling.uniform(seed, "ksk.a", 5 * 256 + 1, 3, q, 5000).astype(np.int64)).all()
    assert (C.sample(seed, "sk.s", 0, 0, 1, 0, 5000) == sampling.ternary(seed, "sk.s", 0, 5000)).all()
    assert (C.sample(seed, "enc.e0", 77, 0, 2, 0, 5000) == sampling.cbd21(seed, "enc.e0", 77, 5000)).all()


@pytest.mark.parametrize("name", sorted(synth.WORKLOADS))
def test_prime_chain_matches_oracle(name):
    ch = synth.WORKLOADS[name].chain
    lib_primes = C.chain_primes(**ch)
    o = nt.make_chain(ch["log_n"], 65537, ch["n_data_primes"], ch["q0_max"], ch["data_max"], ch["alpha"],
                      ch["special_max"])
    assert lib_primes == o.all_primes()
    assert o.total_bits() <= (438 if ch["log_n"] == 14 else 881)


def test_chain_errors():
    with pytest.raises(C.CopseError) as e:
        C.chain_primes(14, 9, 1 << 42, 1 << 60, 2, 1 << 44)
    assert e.value.code == C.COPSE_EINVAL
    with pytest.raises(C.CopseError):
        C.chain_primes(14, 9, 1 << 42, 1 << 33, 2, 1 << 44)   # not enough small primes


@pytest.mark.parametrize("log_n", [4, 8, 12])
def test_encoder_matches_oracle(log_n):
    ch = nt.make_chain(log_n, 65537, 2, 1 << 48, 1 << 42, 1, 1 << 48)
    sc = B.BGV(ch)
    rng = np.random.default_rng(log_n)
    slots = rng.integers(0, 65537, size=(2, sc.N // 2))
    got = C.encode(log_n, slots) % 65537
    assert (got == sc.encode(slots).astype(np.int64)).all()
    # centered lift range
    raw = C.encode(log_n, slots)
    assert raw.min() >= -32768 and raw.max() <= 32768


def _meta_vs_oracle(text, F, p, log_n, fold, n1=(0, 0)):
    ch, meta = C.forest_compile(text, F, p, log_n, fold=fold, n1_R=n1[0], n1_L=n1[1])
    oc = OC.compile_forest(text, F, p)
    assert (meta.K, meta.q, meta.b, meta.m, meta.d) == (oc.K, oc.q, oc.b, oc.m, oc.d)
    assert meta.block_w == oc.W and meta.queries_per_ct == (1 << log_n) // oc.W
    pl = CI.make_plan(oc, 1 << log_n, 40, fold=fold, n1_R=n1[0], n1_L=n1[1])
    assert (meta.n1_R, meta.n1_L) == (pl.n1_R, pl.n1_L)
    for given, got in zip(n1, (meta.n1_R, meta.n1_L)):
        assert given == 0 or got == given
    assert C.compiled_rotations(meta) == pl.rotations()
    depth = CI.seccomp_depth(p) + (1 if fold else 2) + (int(np.ceil(np.log2(oc.d))) if oc.d > 1 else 0)
    assert meta.depth == depth


@pytest.mark.parametrize("name", ["c1_plain_d3", "c2_forest16_d5", "c3_batched_32x_d6", "c5_serve_8x_d4"])
def test_compiler_matches_oracle_on_workloads(name):
    w = synth.WORKLOADS[name]
    text, _, _ = synth.workload_inputs(w)
    _meta_vs_oracle(text, w.shape.n_features, w.shape.precision, w.log_n, w.fold)
    _meta_vs_oracle(text, w.shape.n_features, w.shape.precision, w.log_n, not w.fold)


@pytest.mark.parametrize("name", [k for k, w in synth.WORKLOADS.items() if w.n1 != (0, 0)])
def test_workload_baby_steps_reach_both_sides(name):
    """A workload's measured baby-step split (where it is not the compiler's rule) is what the library
    compiles and what the oracle plans, so both evaluate the same schedule (the stored goldens rely on it)."""
    w = synth.WORKLOADS[name]
    text, _, _ = synth.workload_inputs(w)
    _meta_vs_oracle(text, w.shape.n_features, w.shape.precision, w.log_n, w.fold, w.n1)


@pytest.mark.parametrize("seed", range(6))
def test_compiler_matches_oracle_random(seed):
    shape = synth.ForestShape(1 + seed % 4, 3 + seed % 4, 0.6, 3 + seed, 6, 3)
    text = synth.gen_forest_text(shape, 40 + seed)
    _meta_vs_oracle(text, shape.n_features, shape.precision, 13, bool(seed % 2))


def test_compiler_errors():
    bad = {"": C.COPSE_EINVAL, "a b\nB 0 1 L 0": C.COPSE_EINVAL, "a\nL 3": C.COPSE_EINVAL,
           "a b\nX 1": C.COPSE_EINVAL, "a b\nL 0 L 1": C.COPSE_EINVAL, "a b\nL 0": C.COPSE_EINVAL,
           "a b\nB 5 1 L 0 L 1": C.COPSE_EINVAL, "a b\nB 0 999 L 0 L 1": C.COPSE_EINVAL,
           "a b\nB 0 x L 0 L 1": C.COPSE_EINVAL}
    for text, code in bad.items():
        with pytest.raises(C.CopseError) as e:
            C.forest_compile(text, 2, 8, 10)
        assert e.value.code == code, text
    # a forest whose query block does not fit one slot row
    w = synth.WORKLOADS["c2_forest16_d5"]
    text, _, _ = synth.workload_inputs(w)
    with pytest.raises(C.CopseError) as e:
        C.forest_compile(text, 16, 8, 10)
    assert e.value.code == C.COPSE_ECAPACITY


@pytest.mark.parametrize("seed,n_pad", [(0, 0), (1, 5), (2, 17)])
def test_private_compile_matches_oracle(seed, n_pad):
    """The library's shuffled and padded result layout equals the oracle's: slot count, block width
    and the codebook (which encodes the permutation and the padding labels)."""
    from oracle import compiler as OC
    from oracle import forest as F
    shape = synth.ForestShape(3, 5, 0.7, 4, 6, 5)
    text = synth.gen_forest_text(shape, 90 + seed)
    names, _ = F.parse_forest(text)
    key = bytes([seed + 1]) * 32
    comp, meta = C.forest_compile_private(text, 4, 6, 13, key, n_pad)
    oc = OC.privatize(OC.compile_forest(text, 4, 6), key, n_pad, len(names))
    assert meta.m == oc.m and meta.block_w == oc.W and meta.b == oc.b and meta.q == oc.q
    assert C.compiled_codebook(comp) == oc.codebook
    _, pmeta = C.forest_compile(text, 4, 6, 13)
    assert pmeta.m + n_pad == meta.m


@pytest.mark.parametrize("seed", range(3))
def test_server_replication_layout_matches_oracle(seed):
    """Server-side replication: block width, depth and rotations equal the oracle's (the query planes
    are compared bit for bit after encryption in the GPU tests)."""
    from oracle import circuit as CI
    from oracle import compiler as OC
    shape = synth.ForestShape(2 + seed, 4, 0.7, 3 + seed, 5, 3)
    text = synth.gen_forest_text(shape, 120 + seed)
    comp, meta = C.forest_compile_ex(text, shape.n_features, 5, 12, server_replication=True)
    oc = OC.server_replicated(OC.compile_forest(text, shape.n_features, 5))
    assert meta.server_rep == 1 and meta.block_w == oc.W and meta.n1_F == OC.bsgs_n1(shape.n_features)
    _, plain = C.forest_compile(text, shape.n_features, 5, 12)
    assert meta.depth == plain.depth + 1
    pl = CI.make_plan(oc, 1 << 12, 20)
    assert C.compiled_rotations(meta) == pl.rotations()
