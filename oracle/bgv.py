"""BGV over an RNS prime chain: the oracle's scheme.  TEST INFRASTRUCTURE ONLY.

Ring Z_Q[X]/(X^N + 1) with plaintext modulus t, N slots (t = 1 mod 2N).
All polynomials are held in COEFFICIENT form, one row of N unsigned residues
per prime; the negacyclic transform of cbgv.c is used only inside products.
The paper relies on HElib's BGV (Section 5, "COPSE Runtime"); the scheme
below is the textbook RNS variant, with every choice that decides the bits of
a ciphertext fixed as follows (each is a reading, the paper is silent):

  slots      slot (r, j), r in {0,1}, j < N/2, is m(zeta^e) with
             e = 5^j (r = 0) or -5^j (r = 1) mod 2N, zeta = 3^((t-1)/2N) mod t;
             sigma_{5^k} then rotates each row left by k slots
  lift       plaintext coefficients in [0, t) are lifted centered into
             [-(t-1)/2, (t-1)/2] before reduction mod each prime
  keys       s ternary; pk = (-a s + t e, a) over Q_L; a key-switching key
             from s' has one pair per digit j of alpha consecutive data primes,
             (-a_j s + t e_j + g_j s', a_j) over P Q_L, g_j = P mod q_i for
             q_i in digit j and 0 elsewhere; lower levels drop limbs
  encrypt    (pk0 u + t e0 + m, pk1 u + t e1), u ternary, e0, e1 error
  modswitch  drop q_l: z = [c_l t^-1]_{q_l} centered, c'_i = (c_i - t z) q_l^-1
  key switch ModUp per digit by fast base conversion with y_i in [0, q_i),
             inner product with the key, ModDown: z_r = [y_r t^-1]_{p_r},
             fast base conversion P -> Q, out_i = (y_i - t z^_i) P^-1
  rotation   always hoisted form: ModUp(c1), sigma on every digit, inner
             product with the key of sigma(s), ModDown, plus sigma(c0)
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import nt, sampling

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_lib(force: bool = False) -> str:
    so = os.path.join(_HERE, "_cbgv.so")
    src = os.path.join(_HERE, "cbgv.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", so, src])
    return so


def lib():
    global _LIB
    if _LIB is None:
        L = ctypes.CDLL(build_lib())
        u64p = ctypes.POINTER(ctypes.c_uint64)
        sz, u64 = ctypes.c_size_t, ctypes.c_uint64
        L.oc_ntt_fwd.argtypes = [u64p, sz, u64, u64]
        L.oc_ntt_inv.argtypes = [u64p, sz, u64, u64]
        L.oc_mul.argtypes = [u64p, u64p, u64p, sz, u64]
        L.oc_mac.argtypes = [u64p, u64p, u64p, sz, u64]
        L.oc_mul_scalar.argtypes = [u64p, u64p, sz, u64, u64]
        L.oc_fastbconv.argtypes = [u64p, u64p, sz, sz, u64p, sz, u64p, u64p, u64p]
        L.oc_negacyclic_schoolbook.argtypes = [u64p, u64p, u64p, sz, u64]
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _u64(xs: Sequence[int]) -> np.ndarray:
    return np.ascontiguousarray(np.array([int(x) for x in xs], dtype=np.uint64))


# ---------------------------------------------------------------- primitives
def ntt_fwd(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    lib().oc_ntt_fwd(_p(out), out.shape[-1], q, psi)
    return out


def ntt_inv(a: np.ndarray, q: int, psi: int) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.uint64).copy()
    lib().oc_ntt_inv(_p(out), out.shape[-1], q, psi)
    return out


def mulmod_vec(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().oc_mul(_p(out), _p(a), _p(b), a.size, q)
    return out


def mulscalar(a: np.ndarray, s: int, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.empty_like(a)
    lib().oc_mul_scalar(_p(out), _p(a), a.size, q, s % q)
    return out


def negacyclic_schoolbook(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    out = np.empty_like(a)
    lib().oc_negacyclic_schoolbook(_p(out), _p(a), _p(b), a.size, q)
    return out


def fastbconv(x: np.ndarray, in_q: List[int], out_p: List[int]) -> np.ndarray:
    """Fast base conversion (rows of x are residues mod in_q)."""
    n = x.shape[1]
    Q = math.prod(in_q)
    qhat_inv = _u64([pow(Q // qi, -1, qi) for qi in in_q])
    qhat_mod = _u64([(Q // qi) % po for qi in in_q for po in out_p])
    out = np.empty((len(out_p), n), dtype=np.uint64)
    xin = np.ascontiguousarray(x, dtype=np.uint64)
    lib().oc_fastbconv(_p(out), _p(xin), n, len(in_q), _p(_u64(in_q)), len(out_p), _p(_u64(out_p)),
                       _p(qhat_inv), _p(qhat_mod))
    return out


def automorphism(a: np.ndarray, g: int, q: int) -> np.ndarray:
    """sigma_g: a(X) -> a(X^g) mod (X^N + 1, q) on one coefficient row."""
    n = a.shape[-1]
    i = np.arange(n, dtype=np.int64)
    pos = (i * g) % (2 * n)
    out = np.zeros_like(a)
    lo = pos < n
    out[pos[lo]] = a[lo]
    neg = a[~lo]
    out[pos[~lo] - n] = np.where(neg == 0, np.uint64(0), np.uint64(q) - neg)
    return out


# ---------------------------------------------------------------- containers
@dataclass
class Ciphertext:
    polys: List[np.ndarray]          # each [level+1, N] uint64, coefficient form
    level: int

    def copy(self) -> "Ciphertext":
        return Ciphertext([p.copy() for p in self.polys], self.level)


@dataclass
class KSKey:
    b: List[np.ndarray]              # per digit [L+1+alpha, N] coefficient form
    a: List[np.ndarray]
    b_ntt: List[np.ndarray] = field(default_factory=list)
    a_ntt: List[np.ndarray] = field(default_factory=list)


@dataclass
class Keys:
    s: np.ndarray                    # int64 ternary coefficients
    pk_b: np.ndarray                 # [L+1, N]
    pk_a: np.ndarray
    relin: Optional[KSKey] = None
    rot: Dict[int, KSKey] = field(default_factory=dict)   # Galois element -> key


RELIN_KEY_ID = 0


class BGV:
    """Scheme over one prime chain (see module docstring for every pin)."""

    def __init__(self, chain: nt.Chain):
        self.chain = chain
        self.N = chain.n
        self.t = chain.t
        self.L = chain.L
        self.alpha = chain.alpha
        self.primes = chain.all_primes()           # global prime index
        self.special_idx = list(range(self.L + 1, self.L + 1 + self.alpha))
        self.psi = [nt.root_of_unity(2 * self.N, q) for q in self.primes]
        self.zeta = nt.slot_root(self.t, self.N)
        self.P = math.prod(chain.special)
        # slot (r, j) -> natural evaluation index (e - 1) / 2
        N2 = self.N // 2
        e0 = np.array([pow(5, j, 2 * self.N) for j in range(N2)], dtype=np.int64)
        e1 = (2 * self.N - e0) % (2 * self.N)
        self.slot_index = np.stack([(e0 - 1) // 2, (e1 - 1) // 2])

    # ---- helpers over prime-index lists
    def q(self, i: int) -> int:
        return self.primes[i]

    def data_idx(self, level: int) -> List[int]:
        return list(range(level + 1))

    def ext_idx(self, level: int) -> List[int]:
        return self.data_idx(level) + self.special_idx

    def reduce_signed(self, v: np.ndarray, idx: List[int]) -> np.ndarray:
        v = np.asarray(v, dtype=np.int64)
        return np.stack([(v % self.q(i)).astype(np.uint64) for i in idx])

    def ntt(self, a: np.ndarray, idx: List[int]) -> np.ndarray:
        return np.stack([ntt_fwd(a[k], self.q(i), self.psi[i]) for k, i in enumerate(idx)])

    def intt(self, a: np.ndarray, idx: List[int]) -> np.ndarray:
        return np.stack([ntt_inv(a[k], self.q(i), self.psi[i]) for k, i in enumerate(idx)])

    def pmul_ntt(self, a: np.ndarray, b: np.ndarray, idx: List[int]) -> np.ndarray:
        return np.stack([mulmod_vec(a[k], b[k], self.q(i)) for k, i in enumerate(idx)])

    def padd(self, a, b, idx):
        qs = np.array([self.q(i) for i in idx], dtype=np.uint64)[:, None]
        return (a + b) % qs

    def psub(self, a, b, idx):
        qs = np.array([self.q(i) for i in idx], dtype=np.uint64)[:, None]
        return (a + qs - b) % qs

    def pneg(self, a, idx):
        qs = np.array([self.q(i) for i in idx], dtype=np.uint64)[:, None]
        return (qs - a) % qs

    def polymul(self, a: np.ndarray, b: np.ndarray, idx: List[int]) -> np.ndarray:
        return self.intt(self.pmul_ntt(self.ntt(a, idx), self.ntt(b, idx), idx), idx)

    def pscalar(self, a, s: int, idx):
        return np.stack([mulscalar(a[k], s, self.q(i)) for k, i in enumerate(idx)])

    def pauto(self, a, g: int, idx):
        return np.stack([automorphism(a[k], g, self.q(i)) for k, i in enumerate(idx)])

    # ---- encoding (slots <-> plaintext polynomial mod t)
    def encode(self, slots: np.ndarray) -> np.ndarray:
        ev = np.zeros(self.N, dtype=np.uint64)
        ev[self.slot_index.reshape(-1)] = (np.asarray(slots, dtype=np.int64) % self.t).reshape(-1)
        return ntt_inv(ev, self.t, self.zeta)

    def decode(self, m: np.ndarray) -> np.ndarray:
        ev = ntt_fwd(np.asarray(m, dtype=np.uint64) % np.uint64(self.t), self.t, self.zeta)
        return ev[self.slot_index].astype(np.int64)

    def lift(self, m: np.ndarray) -> np.ndarray:
        """Centered representative of plaintext coefficients in [0, t)."""
        m = np.asarray(m, dtype=np.int64)
        return np.where(m > (self.t - 1) // 2, m - self.t, m)

    # ---- keys
    def keygen(self, seed: bytes, rotations: Sequence[int] = (), relin: bool = True) -> Keys:
        N = self.N
        s = sampling.ternary(seed, "sk.s", 0, N)
        didx = self.data_idx(self.L)
        a = np.stack([sampling.uniform(seed, "pk.a", 0, i, self.q(i), N) for i in didx])
        e = sampling.cbd21(seed, "pk.e", 0, N)
        s_r = self.reduce_signed(s, didx)
        b = self.padd(self.pneg(self.polymul(a, s_r, didx), didx),
                      self.reduce_signed(self.t * e, didx), didx)
        keys = Keys(s=s, pk_b=b, pk_a=a)
        if relin:
            s2 = self.polymul(self.reduce_signed(s, self.ext_idx(self.L)),
                              self.reduce_signed(s, self.ext_idx(self.L)), self.ext_idx(self.L))
            keys.relin = self.ksk_gen(seed, s, s2, RELIN_KEY_ID)
        for r in rotations:
            g = self.galois(r)
            if g in keys.rot:
                continue
            sg = self.pauto(self.reduce_signed(s, self.ext_idx(self.L)), g, self.ext_idx(self.L))
            keys.rot[g] = self.ksk_gen(seed, s, sg, g)
        return keys

    def n_digits(self, level: int) -> int:
        return -(-(level + 1) // self.alpha)

    def digit(self, j: int, level: int) -> List[int]:
        return list(range(j * self.alpha, min((j + 1) * self.alpha, level + 1)))

    def ksk_gen(self, seed: bytes, s: np.ndarray, s_new: np.ndarray, key_id: int) -> KSKey:
        """Key switching s_new -> s; s_new given over P Q_L (all primes)."""
        idx = self.ext_idx(self.L)
        s_r = self.reduce_signed(s, idx)
        s_ntt = self.ntt(s_r, idx)
        key = KSKey([], [])
        for j in range(self.n_digits(self.L)):
            obj = key_id * 256 + j
            a = np.stack([sampling.uniform(seed, "ksk.a", obj, i, self.q(i), self.N) for i in idx])
            e = sampling.cbd21(seed, "ksk.e", obj, self.N)
            a_ntt = self.ntt(a, idx)
            b = self.padd(self.pneg(self.intt(self.pmul_ntt(a_ntt, s_ntt, idx), idx), idx),
                          self.reduce_signed(self.t * e, idx), idx)
            gadget_rows = self.digit(j, self.L)
            for k in gadget_rows:
                qi = self.q(k)
                b[k] = (b[k] + mulscalar(s_new[k], self.P % qi, qi)) % np.uint64(qi)
            key.b.append(b)
            key.a.append(a)
            key.b_ntt.append(self.ntt(b, idx))
            key.a_ntt.append(a_ntt)
        return key

    def galois(self, r: int) -> int:
        """Galois element of a left rotation by r slots within each row."""
        return pow(5, r % (self.N // 2), 2 * self.N)

    # ---- encryption
    def encrypt_poly(self, keys: Keys, m: np.ndarray, seed: bytes, obj: int, level: Optional[int] = None) -> Ciphertext:
        level = self.L if level is None else level
        idx = self.data_idx(level)
        N = self.N
        u = self.reduce_signed(sampling.ternary(seed, "enc.u", obj, N), idx)
        e0 = sampling.cbd21(seed, "enc.e0", obj, N)
        e1 = sampling.cbd21(seed, "enc.e1", obj, N)
        u_ntt = self.ntt(u, idx)
        c0 = self.intt(self.pmul_ntt(self.ntt(keys.pk_b[:level + 1], idx), u_ntt, idx), idx)
        c1 = self.intt(self.pmul_ntt(self.ntt(keys.pk_a[:level + 1], idx), u_ntt, idx), idx)
        c0 = self.padd(c0, self.reduce_signed(self.t * e0 + self.lift(m), idx), idx)
        c1 = self.padd(c1, self.reduce_signed(self.t * e1, idx), idx)
        return Ciphertext([c0, c1], level)

    def encrypt_slots(self, keys: Keys, slots, seed: bytes, obj: int, level=None) -> Ciphertext:
        return self.encrypt_poly(keys, self.encode(slots), seed, obj, level)

    def phase(self, keys: Keys, ct: Ciphertext) -> List[int]:
        """[c0 + c1 s (+ c2 s^2)]_{Q_l} as centered Python integers."""
        idx = self.data_idx(ct.level)
        s = self.reduce_signed(keys.s, idx)
        s_ntt = self.ntt(s, idx)
        acc = self.ntt(ct.polys[0], idx)
        spow = s_ntt
        for poly in ct.polys[1:]:
            acc = self.padd(acc, self.pmul_ntt(self.ntt(poly, idx), spow, idx), idx)
            spow = self.pmul_ntt(spow, s_ntt, idx)
        x = self.intt(acc, idx)
        return self.crt(x, idx)

    def crt(self, x: np.ndarray, idx: List[int]) -> List[int]:
        qs = [self.q(i) for i in idx]
        Q = math.prod(qs)
        tot = np.zeros(x.shape[1], dtype=object)
        for k, qi in enumerate(qs):
            Qh = Q // qi
            c = (Qh * pow(Qh, -1, qi)) % Q
            tot = tot + np.array([int(v) for v in x[k]], dtype=object) * c
        half = Q // 2
        return [int(v) % Q - Q if int(v) % Q > half else int(v) % Q for v in tot]

    def decrypt_poly(self, keys: Keys, ct: Ciphertext) -> np.ndarray:
        ph = self.phase(keys, ct)
        return np.array([v % self.t for v in ph], dtype=np.int64)

    def decrypt_slots(self, keys: Keys, ct: Ciphertext) -> np.ndarray:
        return self.decode(self.decrypt_poly(keys, ct))

    def noise_bits(self, keys: Keys, ct: Ciphertext) -> float:
        """log2 of the infinity norm of the phase (noise plus message)."""
        ph = self.phase(keys, ct)
        mx = max(abs(v) for v in ph)
        return math.log2(mx) if mx else 0.0

    def margin_bits(self, keys: Keys, ct: Ciphertext) -> float:
        Q = math.prod(self.q(i) for i in self.data_idx(ct.level))
        return math.log2(Q / 2) - self.noise_bits(keys, ct)

    # ---- homomorphic operations (all exact except the rounding ones)
    def modswitch(self, ct: Ciphertext) -> Ciphertext:
        l = ct.level
        if l == 0:
            raise ValueError("cannot switch below q_0")
        ql = self.q(l)
        tinv = pow(self.t, -1, ql)
        new = []
        idx = self.data_idx(l - 1)
        for poly in ct.polys:
            z = mulscalar(poly[l], tinv, ql).astype(np.int64)
            z = np.where(z > (ql - 1) // 2, z - ql, z)
            out = []
            for i in idx:
                qi = self.q(i)
                delta = mulscalar((z % qi).astype(np.uint64), self.t % qi, qi)
                diff = (poly[i] + np.uint64(qi) - delta) % np.uint64(qi)
                out.append(mulscalar(diff, pow(ql, -1, qi), qi))
            new.append(np.stack(out))
        return Ciphertext(new, l - 1)

    def modswitch_to(self, ct: Ciphertext, level: int) -> Ciphertext:
        while ct.level > level:
            ct = self.modswitch(ct)
        return ct

    def equalize(self, a: Ciphertext, b: Ciphertext):
        lv = min(a.level, b.level)
        return self.modswitch_to(a, lv), self.modswitch_to(b, lv)

    def add(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        a, b = self.equalize(a, b)
        idx = self.data_idx(a.level)
        n = max(len(a.polys), len(b.polys))
        out = []
        for k in range(n):
            if k < len(a.polys) and k < len(b.polys):
                out.append(self.padd(a.polys[k], b.polys[k], idx))
            else:
                out.append((a.polys[k] if k < len(a.polys) else b.polys[k]).copy())
        return Ciphertext(out, a.level)

    def neg(self, a: Ciphertext) -> Ciphertext:
        idx = self.data_idx(a.level)
        return Ciphertext([self.pneg(p, idx) for p in a.polys], a.level)

    def sub(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        return self.add(a, self.neg(b))

    def mul_int(self, a: Ciphertext, k: int) -> Ciphertext:
        idx = self.data_idx(a.level)
        return Ciphertext([self.pscalar(p, k, idx) for p in a.polys], a.level)

    def add_plain(self, a: Ciphertext, m: np.ndarray) -> Ciphertext:
        """Add a plaintext polynomial (coefficients mod t) to c0."""
        idx = self.data_idx(a.level)
        out = a.copy()
        out.polys[0] = self.padd(out.polys[0], self.reduce_signed(self.lift(m), idx), idx)
        return out

    def plain_ntt(self, m: np.ndarray, level: int) -> np.ndarray:
        idx = self.data_idx(level)
        return self.ntt(self.reduce_signed(self.lift(m), idx), idx)

    def mul_plain(self, a: Ciphertext, m: np.ndarray) -> Ciphertext:
        idx = self.data_idx(a.level)
        pt = self.plain_ntt(m, a.level)
        return Ciphertext([self.intt(self.pmul_ntt(self.ntt(p, idx), pt, idx), idx) for p in a.polys], a.level)

    def tensor(self, a: Ciphertext, b: Ciphertext) -> Ciphertext:
        a, b = self.equalize(a, b)
        idx = self.data_idx(a.level)
        a0, a1 = (self.ntt(p, idx) for p in a.polys)
        b0, b1 = (self.ntt(p, idx) for p in b.polys)
        d0 = self.pmul_ntt(a0, b0, idx)
        d1 = self.padd(self.pmul_ntt(a0, b1, idx), self.pmul_ntt(a1, b0, idx), idx)
        d2 = self.pmul_ntt(a1, b1, idx)
        return Ciphertext([self.intt(d, idx) for d in (d0, d1, d2)], a.level)

    # key switching
    def modup(self, d: np.ndarray, level: int) -> List[np.ndarray]:
        """Digits of d (coefficient form over Q_l), each extended to P Q_l."""
        ext = self.ext_idx(level)
        out = []
        for j in range(self.n_digits(level)):
            dig = self.digit(j, level)
            targets = [i for i in ext if i not in dig]
            conv = fastbconv(d[dig], [self.q(i) for i in dig], [self.q(i) for i in targets])
            full = np.zeros((len(ext), self.N), dtype=np.uint64)
            for row, i in enumerate(ext):
                full[row] = d[i] if i in dig else conv[targets.index(i)]
            out.append(full)
        return out

    def ks_inner(self, digits: List[np.ndarray], key: KSKey, level: int):
        ext = self.ext_idx(level)
        rows = self.data_idx(level) + [self.L + 1 + r for r in range(self.alpha)]
        acc0 = np.zeros((len(ext), self.N), dtype=np.uint64)
        acc1 = np.zeros_like(acc0)
        for j, dg in enumerate(digits):
            dn = self.ntt(dg, ext)
            acc0 = self.padd(acc0, self.pmul_ntt(dn, key.b_ntt[j][rows], ext), ext)
            acc1 = self.padd(acc1, self.pmul_ntt(dn, key.a_ntt[j][rows], ext), ext)
        return self.intt(acc0, ext), self.intt(acc1, ext)

    def moddown(self, y: np.ndarray, level: int) -> np.ndarray:
        didx = self.data_idx(level)
        nd = len(didx)
        sp = [self.q(i) for i in self.special_idx]
        z = np.stack([mulscalar(y[nd + r], pow(self.t, -1, p), p) for r, p in enumerate(sp)])
        zh = fastbconv(z, sp, [self.q(i) for i in didx])
        out = []
        for k, i in enumerate(didx):
            qi = self.q(i)
            delta = mulscalar(zh[k], self.t % qi, qi)
            diff = (y[k] + np.uint64(qi) - delta) % np.uint64(qi)
            out.append(mulscalar(diff, pow(self.P, -1, qi), qi))
        return np.stack(out)

    def keyswitch_digits(self, digits, key: KSKey, level: int):
        y0, y1 = self.ks_inner(digits, key, level)
        return self.moddown(y0, level), self.moddown(y1, level)

    def relinearize(self, ct: Ciphertext, keys: Keys) -> Ciphertext:
        assert len(ct.polys) == 3
        idx = self.data_idx(ct.level)
        k0, k1 = self.keyswitch_digits(self.modup(ct.polys[2], ct.level), keys.relin, ct.level)
        return Ciphertext([self.padd(ct.polys[0], k0, idx), self.padd(ct.polys[1], k1, idx)], ct.level)

    def mul(self, a: Ciphertext, b: Ciphertext, keys: Keys) -> Ciphertext:
        """Ciphertext product: tensor, relinearize, one modulus switch."""
        return self.modswitch(self.relinearize(self.tensor(a, b), keys))

    def rotate_hoisted(self, ct: Ciphertext, rs: Sequence[int], keys: Keys) -> Dict[int, Ciphertext]:
        """Left rotations of ct by every r in rs, sharing one ModUp of c1."""
        assert len(ct.polys) == 2
        idx = self.data_idx(ct.level)
        ext = self.ext_idx(ct.level)
        digits = None
        out = {}
        for r in rs:
            if r % (self.N // 2) == 0:
                out[r] = ct.copy()
                continue
            if digits is None:
                digits = self.modup(ct.polys[1], ct.level)
            g = self.galois(r)
            dg = [self.pauto(d, g, ext) for d in digits]
            k0, k1 = self.keyswitch_digits(dg, keys.rot[g], ct.level)
            out[r] = Ciphertext([self.padd(self.pauto(ct.polys[0], g, idx), k0, idx), k1], ct.level)
        return out

    def rotate(self, ct: Ciphertext, r: int, keys: Keys) -> Ciphertext:
        return self.rotate_hoisted(ct, [r], keys)[r]

    def rotate_sum(self, items: Sequence[Tuple[Ciphertext, int]], keys: Keys) -> Ciphertext:
        """sum_g rot(ct_g, r_g) with one ModDown: the key-switching inner products of the rotated
        terms are added in the extended basis P Q_l and brought down once; the sigma(c0) parts and the
        unrotated terms are added in Q_l.  A ModDown of a sum and the sum of ModDowns differ only in
        rounding, which is why both sides fix this form."""
        level = items[0][0].level
        assert all(ct.level == level and len(ct.polys) == 2 for ct, _ in items)
        idx = self.data_idx(level)
        ext = self.ext_idx(level)
        c0 = np.zeros((len(idx), self.N), dtype=np.uint64)
        c1 = np.zeros_like(c0)
        y0 = y1 = None
        for ct, r in items:
            if r % (self.N // 2) == 0:
                c0 = self.padd(c0, ct.polys[0], idx)
                c1 = self.padd(c1, ct.polys[1], idx)
                continue
            g = self.galois(r)
            digits = [self.pauto(d, g, ext) for d in self.modup(ct.polys[1], level)]
            a0, a1 = self.ks_inner(digits, keys.rot[g], level)
            y0 = a0 if y0 is None else self.padd(y0, a0, ext)
            y1 = a1 if y1 is None else self.padd(y1, a1, ext)
            c0 = self.padd(c0, self.pauto(ct.polys[0], g, idx), idx)
        if y0 is not None:
            c0 = self.padd(c0, self.moddown(y0, level), idx)
            c1 = self.padd(c1, self.moddown(y1, level), idx)
        return Ciphertext([c0, c1], level)
