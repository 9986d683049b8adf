"""Pins of the oracle's BGV against mathematics it does not itself use:
schoolbook negacyclic products, the automorphism's closed form, exact CRT,
brute-force evaluation of the transform definition, and round trips."""
import math
import random

import numpy as np
import pytest

from oracle import bgv as B
from oracle import nt
from oracle import sampling
from oracle import slotsim as S

T = 65537


def small_chain(log_n=6, n_data=5, alpha=2):
    return nt.make_chain(log_n, T, n_data=n_data, q0_max=1 << 49, data_max=1 << 40, alpha=alpha, special_max=1 << 49)


@pytest.fixture(scope="module")
def scheme():
    return B.BGV(small_chain())


@pytest.fixture(scope="module")
def keys(scheme):
    return scheme.keygen(b"\x07" * 32, rotations=[1, 2, 3, 5, 7, 16, 31])


def test_primes_and_chain():
    ch = small_chain()
    M = 2 * ch.n * T
    for p in ch.all_primes():
        assert p % M == 1 and p < 2 ** 50
        # trial division up to 2^20 as an independent partial check
        assert all(p % d for d in range(3, 1 << 12, 2))
    assert len(set(ch.all_primes())) == len(ch.all_primes())
    assert ch.data[1] > ch.data[2] > ch.data[3]
    # Miller-Rabin on known cases: Carmichael numbers and base-2 strong pseudoprimes
    for comp in [561, 1105, 1729, 2047, 3215031751, 3825123056546413051]:
        assert not nt.is_prime(comp)
    for pr in [2, 3, 65537, 2 ** 61 - 1, 1000000007, 18446744073709551557]:
        assert nt.is_prime(pr)


def test_transform_definition_and_schoolbook():
    rng = random.Random(1)
    q = small_chain().data[0]
    n = 16
    psi = nt.root_of_unity(2 * n, q)
    a = np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)
    b = np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)
    fa = B.ntt_fwd(a, q, psi)
    for i in range(n):
        assert int(fa[i]) == sum(int(a[j]) * pow(psi, (2 * i + 1) * j, q) for j in range(n)) % q
    assert (B.ntt_inv(fa, q, psi) == a).all()
    # product via transform == schoolbook negacyclic with Python ints
    prod = B.ntt_inv(B.mulmod_vec(fa, B.ntt_fwd(b, q, psi), q), q, psi)
    want = [0] * n
    for i in range(n):
        for j in range(n):
            k = i + j
            v = int(a[i]) * int(b[j])
            if k < n:
                want[k] += v
            else:
                want[k - n] -= v
    assert [int(x) for x in prod] == [w % q for w in want]
    assert (B.negacyclic_schoolbook(a, b, q) == prod).all()


@pytest.mark.parametrize("n", [64, 1024])
def test_transform_product_large(n):
    q = nt.make_chain(int(math.log2(n)), T, 2, 1 << 49, 1 << 45, 1, 1 << 49).data[1]
    psi = nt.root_of_unity(2 * n, q)
    rng = np.random.default_rng(n)
    a = rng.integers(0, q, n, dtype=np.uint64)
    b = rng.integers(0, q, n, dtype=np.uint64)
    prod = B.ntt_inv(B.mulmod_vec(B.ntt_fwd(a, q, psi), B.ntt_fwd(b, q, psi), q), q, psi)
    assert (prod == B.negacyclic_schoolbook(a, b, q)).all()


def test_automorphism_closed_form():
    q = small_chain().data[1]
    n = 32
    rng = random.Random(3)
    a = np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)
    for g in [3, 5, 25, 2 * n - 1, 77 % (2 * n)]:
        if g % 2 == 0:
            continue
        out = B.automorphism(a, g, q)
        # a(X^g): X^(ig) reduced with X^N = -1
        want = [0] * n
        for i in range(n):
            e = i * g
            sign = -1 if (e // n) % 2 else 1
            want[e % n] = (want[e % n] + sign * int(a[i])) % q
        assert [int(x) for x in out] == want
    # ring homomorphism
    b = np.array([rng.randrange(q) for _ in range(n)], dtype=np.uint64)
    ab = B.negacyclic_schoolbook(a, b, q)
    assert (B.automorphism(ab, 5, q) ==
            B.negacyclic_schoolbook(B.automorphism(a, 5, q), B.automorphism(b, 5, q), q)).all()


def test_encode_decode_and_rotation(scheme):
    rng = np.random.default_rng(2)
    v = rng.integers(0, T, size=(2, scheme.N // 2))
    m = scheme.encode(v)
    assert (scheme.decode(m) == v).all()
    for r in [1, 3, 7]:
        g = scheme.galois(r)
        rm = B.automorphism(m.astype(np.uint64), g, T)
        assert (scheme.decode(rm) == S.rot(v, r)).all()
    sw = B.automorphism(m.astype(np.uint64), 2 * scheme.N - 1, T)
    assert (scheme.decode(sw) == v[::-1]).all()
    # slotwise product = ring product mod t
    w = rng.integers(0, T, size=(2, scheme.N // 2))
    prod = B.negacyclic_schoolbook(m.astype(np.uint64), scheme.encode(w).astype(np.uint64), T)
    assert (scheme.decode(prod) == (v * w) % T).all()


def test_encode_matches_direct_evaluation():
    ch = nt.make_chain(4, T, 2, 1 << 49, 1 << 45, 1, 1 << 49)
    sc = B.BGV(ch)
    rng = np.random.default_rng(9)
    m = rng.integers(0, T, sc.N)
    slots = sc.decode(m)
    for r in range(2):
        for j in range(sc.N // 2):
            e = pow(5, j, 2 * sc.N) if r == 0 else (-pow(5, j, 2 * sc.N)) % (2 * sc.N)
            x = pow(sc.zeta, e, T)
            assert slots[r, j] == sum(int(m[i]) * pow(x, i, T) for i in range(sc.N)) % T


def test_fastbconv_is_exact_up_to_multiple_of_Q():
    ch = small_chain()
    qs = ch.data[:3]
    ps = ch.data[3:] + ch.special
    Q = math.prod(qs)
    rng = random.Random(4)
    xs = [rng.randrange(Q) for _ in range(40)]
    rows = np.array([[x % qi for x in xs] for qi in qs], dtype=np.uint64)
    out = B.fastbconv(rows, qs, ps)
    for c, x in enumerate(xs):
        for o, p in enumerate(ps):
            ok = [(x + u * Q) % p for u in range(len(qs))]
            assert int(out[o, c]) in ok


def test_samplers():
    seed = b"\x01" * 32
    s = sampling.ternary(seed, "sk.s", 0, 30000)
    assert set(np.unique(s)) <= {-1, 0, 1}
    assert all(abs((s == v).mean() - 1 / 3) < 0.02 for v in (-1, 0, 1))
    e = sampling.cbd21(seed, "x", 1, 30000)
    assert abs(e.mean()) < 0.1 and abs(e.var() - 10.5) < 0.6 and np.abs(e).max() <= 21
    q = small_chain().data[0]
    u = sampling.uniform(seed, "u", 2, 3, q, 30000)
    assert (u < q).all() and abs(u.astype(float).mean() / q - 0.5) < 0.02
    # streams differ by domain, object and limb
    assert (sampling.uniform(seed, "u", 2, 4, q, 100) != u[:100]).any()


def test_encrypt_decrypt_roundtrip(scheme, keys):
    rng = np.random.default_rng(5)
    v = rng.integers(0, T, size=(2, scheme.N // 2))
    ct = scheme.encrypt_slots(keys, v, b"\x09" * 32, obj=1)
    assert (scheme.decrypt_slots(keys, ct) == v).all()
    assert scheme.margin_bits(keys, ct) > 100


def test_homomorphic_ops(scheme, keys):
    rng = np.random.default_rng(6)
    seed = b"\x0a" * 32
    a = rng.integers(0, T, size=(2, scheme.N // 2))
    b = rng.integers(0, T, size=(2, scheme.N // 2))
    ca = scheme.encrypt_slots(keys, a, seed, 1)
    cb = scheme.encrypt_slots(keys, b, seed, 2)
    assert (scheme.decrypt_slots(keys, scheme.add(ca, cb)) == (a + b) % T).all()
    assert (scheme.decrypt_slots(keys, scheme.sub(ca, cb)) == (a - b) % T).all()
    assert (scheme.decrypt_slots(keys, scheme.mul_int(ca, 2)) == (2 * a) % T).all()
    ten = scheme.tensor(ca, cb)
    assert (scheme.decrypt_slots(keys, ten) == (a * b) % T).all()
    rel = scheme.relinearize(ten, keys)
    assert len(rel.polys) == 2 and (scheme.decrypt_slots(keys, rel) == (a * b) % T).all()
    ms = scheme.modswitch(rel)
    assert ms.level == rel.level - 1
    assert (scheme.decrypt_slots(keys, ms) == (a * b) % T).all()
    assert scheme.noise_bits(keys, ms) < scheme.noise_bits(keys, rel)
    pm = scheme.mul_plain(ca, scheme.encode(b))
    assert (scheme.decrypt_slots(keys, pm) == (a * b) % T).all()
    pa = scheme.add_plain(ca, scheme.encode(b))
    assert (scheme.decrypt_slots(keys, pa) == (a + b) % T).all()
    # mixed levels are equalized by modulus switching
    mix = scheme.add(ms, ca)
    assert mix.level == ms.level and (scheme.decrypt_slots(keys, mix) == (a * b + a) % T).all()


def test_modswitch_exact_division(scheme, keys):
    """c' = (c - delta)/q_l with delta = 0 mod t, checked with exact CRT."""
    rng = np.random.default_rng(7)
    v = rng.integers(0, T, size=(2, scheme.N // 2))
    ct = scheme.encrypt_slots(keys, v, b"\x0b" * 32, 3)
    ms = scheme.modswitch(ct)
    l = ct.level
    idx_hi, idx_lo = scheme.data_idx(l), scheme.data_idx(l - 1)
    Qh = math.prod(scheme.q(i) for i in idx_hi)
    Ql = Qh // scheme.q(l)
    for poly_hi, poly_lo in zip(ct.polys, ms.polys):
        hi = scheme.crt(poly_hi, idx_hi)
        lo = scheme.crt(poly_lo, idx_lo)
        for c, cp in zip(hi[:64], lo[:64]):
            delta = c - cp * scheme.q(l)
            # the difference is congruent to c mod Q_l-hat structure: delta = 0 mod t
            # and |delta| <= t q_l / 2 after reducing mod Q_l
            d = delta % Qh
            d = d - Qh if d > Qh // 2 else d
            assert d % T == 0 and abs(d) <= T * scheme.q(l) // 2 + T


def test_rotations(scheme, keys):
    rng = np.random.default_rng(8)
    v = rng.integers(0, T, size=(2, scheme.N // 2))
    ct = scheme.encrypt_slots(keys, v, b"\x0c" * 32, 4)
    rots = scheme.rotate_hoisted(ct, [1, 2, 5, 16, 31], keys)
    for r, c in rots.items():
        assert (scheme.decrypt_slots(keys, c) == S.rot(v, r)).all()
    single = scheme.rotate(ct, 5, keys)
    assert all((p == q).all() for p, q in zip(single.polys, rots[5].polys))


def test_rotate_sum(scheme, keys):
    """One ModDown for a sum of rotations: decrypts to the sum of the rotated messages (the same as
    the sum of single rotations), and with no rotated term it is the plain sum."""
    rng = np.random.default_rng(12)
    msgs = [rng.integers(0, T, size=(2, scheme.N // 2)) for _ in range(4)]
    cts = [scheme.encrypt_slots(keys, m, b"\x0e" * 32, 20 + i) for i, m in enumerate(msgs)]
    rs = [0, 2, 16, 31]
    out = scheme.rotate_sum(list(zip(cts, rs)), keys)
    want = sum(S.rot(m, r) for m, r in zip(msgs, rs)) % T
    assert (scheme.decrypt_slots(keys, out) == want).all()
    single = cts[0]
    for ct, r in zip(cts[1:], rs[1:]):
        single = scheme.add(single, scheme.rotate(ct, r, keys))
    assert (scheme.decrypt_slots(keys, single) == want).all()
    plain = scheme.rotate_sum([(cts[0], 0), (cts[1], 0)], keys)
    assert all((p == q).all() for p, q in zip(plain.polys, scheme.add(cts[0], cts[1]).polys))
    # a lower level, and the switch after it keeps the message
    low = scheme.rotate_sum([(scheme.modswitch_to(ct, 2), r) for ct, r in zip(cts, rs)], keys)
    assert (scheme.decrypt_slots(keys, scheme.modswitch(low)) == want).all()


def test_keyswitch_lower_level(scheme, keys):
    """The top-level key serves every lower level (dropped limbs removed)."""
    rng = np.random.default_rng(10)
    a = rng.integers(0, 2, size=(2, scheme.N // 2))
    ct = scheme.encrypt_slots(keys, a, b"\x0d" * 32, 5)
    ct = scheme.modswitch_to(ct, 2)
    r = scheme.rotate(ct, 3, keys)
    assert (scheme.decrypt_slots(keys, r) == S.rot(a, 3)).all()
    m = scheme.mul(ct, ct, keys)
    assert m.level == 1 and (scheme.decrypt_slots(keys, m) == a).all()


def test_determinism(scheme):
    k1 = scheme.keygen(b"\x11" * 32, rotations=[1])
    k2 = scheme.keygen(b"\x11" * 32, rotations=[1])
    assert (k1.pk_b == k2.pk_b).all() and (k1.rot[5].b[0] == k2.rot[5].b[0]).all()
    k3 = scheme.keygen(b"\x12" * 32, rotations=[1])
    assert (k1.pk_b != k3.pk_b).any()
