"""Algorithm 1 over BGV ciphertexts: the canonical encrypted schedule.
TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper gives Algorithm 1 (Section 4.3) as SecComp -> MatMul(Reshuf) ->
per-level MatMul and XOR with the mask -> MultAll, and Tables 1-2 (Section 6)
count its operations.  Every ciphertext bit also depends on where modulus
switches and relinearizations happen; this module fixes that schedule (a
reading: the paper relies on HElib's automatic choices):

  * a binary operation on ciphertexts at different levels first switches the
    higher one down, one prime at a time;
  * a sum of several terms switches every term to the lowest level first,
    then adds (modulus switching does not commute with addition);
  * ciphertext product = tensor, relinearize, one modulus switch;
  * a layer of plaintext products is followed by one modulus switch;
  * MatMul: hoisted baby rotations of the input, per giant group the sum of
    products with pre-rotated diagonals (ciphertext diagonals: tensor sums
    relinearized once per group), a giant rotation, the sum over groups, one
    modulus switch; all-zero plaintext diagonals and unused baby rotations
    are skipped (this changes no bit, 0 * x = 0 exactly);
  * the level mask is added after the MatMul's modulus switch;
  * MultAll pairs (0,1), (2,3), ... and carries an odd last element up;
  * the result is switched down to q_0.

Comparison circuit with plaintext thresholds (per bit k, one plaintext
product and one plaintext addition, then a modulus switch):
    eq_k = x_k * (2 th_k - 1) + (1 - th_k),   lt_k = x_k * (-th_k) + th_k.
With encrypted thresholds: u_k = x_k * Th_k (ciphertext product), then
    eq_k = 2 u_k - x_k - Th_k + 1,  lt_k = Th_k - u_k.
Both equal the slot formulas of slotsim.seccomp_slots.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import slotsim as S
from .bgv import BGV, Ciphertext, Keys
from .compiler import Compiled, bsgs_n1, extended_reshuffle, generalized_diagonal

OBJ_QUERY = 1
OBJ_THRESH = 2
OBJ_RDIAG = 3
OBJ_LDIAG = 4
OBJ_MASK = 5


def obj_id(kind: int, a: int = 0, b: int = 0) -> int:
    """Encryption object id: kind in the top byte, then two fields."""
    return (kind << 56) | (a << 32) | b


@dataclass
class Plan:
    c: Compiled
    layout: S.Layout
    n1_R: int
    n1_L: int
    fold: bool
    encrypted_model: bool
    L: int
    levels: Dict[str, int] = field(default_factory=dict)
    n1_F: int = 1
    server_rep: bool = False

    def rotations(self) -> List[int]:
        rs = set()
        if self.server_rep:
            n = self.c.n_features
            rs |= set(range(1, self.n1_F))
            rs |= {g * self.n1_F for g in range(1, -(-n // self.n1_F))}
        if not self.fold:
            n = self.c.q
            rs |= set(range(1, self.n1_R))
            rs |= {g * self.n1_R for g in range(1, -(-n // self.n1_R))}
        n = self.c.q if self.fold else self.c.b
        rs |= set(range(1, self.n1_L))
        rs |= {g * self.n1_L for g in range(1, -(-n // self.n1_L))}
        return sorted(rs)


def seccomp_depth(p: int) -> int:
    """Levels the comparison takes: the plaintext layer's switch, then ceil(log2 p) product rounds."""
    return 1 + math.ceil(math.log2(p))


def make_plan(c: Compiled, N: int, L: int, fold: bool = False, encrypted_model: bool = False,
              n1_R: int = 0, n1_L: int = 0) -> Plan:
    lay = S.Layout(N, c.W)
    n1_R = n1_R or bsgs_n1(c.q)
    n1_L = n1_L or bsgs_n1(c.q if fold else c.b)
    pl = Plan(c, lay, n1_R, n1_L, fold, encrypted_model, L)
    # server-side replication: one plaintext product (and its switch) before the comparison
    pl.server_rep = bool(c.meta.get("server_rep", False))
    if pl.server_rep and encrypted_model:
        raise ValueError("server-side replication is for a server-held (plaintext) model")
    pl.n1_F = bsgs_n1(c.n_features)
    top = L - 1 if pl.server_rep else L
    dec = top - seccomp_depth(c.precision)
    br = dec if fold else dec - 1
    lvl = br - 1
    final = lvl - math.ceil(math.log2(c.d)) if c.d > 1 else lvl
    pl.levels = dict(top=top, dec=dec, branches=br, levels=lvl, labels=final)
    if final < 0:
        raise ValueError(f"circuit needs {L - final} levels, chain has {L}")
    return pl


# ------------------------------------------------------------------ model
@dataclass
class PlainModel:
    E: List[np.ndarray]        # per bit: encode(2 th - 1)
    C: List[np.ndarray]        # encode(1 - th)
    G: List[np.ndarray]        # encode(-th)
    TH: List[np.ndarray]       # encode(th)
    rdiag: "Diagonals"                  # [] when the reshuffle is folded
    ldiag: List["Diagonals"]
    masks: List[np.ndarray]
    rep: object = field(default_factory=list)   # replication diagonals (Diagonals) or []


@dataclass
class EncModel:
    TH: List[Ciphertext]
    rdiag: "Diagonals"
    ldiag: List["Diagonals"]
    masks: List[Ciphertext]


class Diagonals:
    """The pre-rotated generalized diagonals of one MatMul matrix (Section 4.1, "Matrix
    Multiplication"), each encoded or encrypted when it is read and then dropped.

    Entry k is exactly what a list of every encoded (encrypted) diagonal would hold at k, so the
    evaluation sees the same values; only no whole model is held at once (an encrypted model of the
    64-tree, depth-8 shape is tens of GB).  A plaintext entry is None when the diagonal is all zero
    (the product with it is skipped); an encrypted model hides its sparsity, so every entry is a
    ciphertext."""

    def __init__(self, A: np.ndarray, layout: S.Layout, n1: int, t: int, make, encrypted: bool):
        self.A = A % t
        self.layout, self.n1, self.make, self.encrypted = layout, n1, make, encrypted

    def __len__(self) -> int:
        return self.A.shape[1]

    def present(self, k: int) -> bool:
        return self.encrypted or bool(generalized_diagonal(self.A, k).any())

    def slots(self, k: int) -> np.ndarray:
        return S.prerotated_diagonal(self.A, self.layout, self.n1, k)

    def __getitem__(self, k: int):
        if not 0 <= k < len(self):
            raise IndexError(k)
        return self.make(k, self.slots(k)) if self.present(k) else None


def _present(diags, k: int) -> bool:
    if isinstance(diags, Diagonals):
        return diags.present(k)
    return diags[k] is not None


def encode_model(sc: BGV, pl: Plan) -> PlainModel:
    c, t = pl.c, sc.t
    tp = S.threshold_planes(c, pl.layout)
    E = [sc.encode((2 * th - 1) % t) for th in tp]
    Cc = [sc.encode((1 - th) % t) for th in tp]
    G = [sc.encode((-th) % t) for th in tp]
    TH = [sc.encode(th) for th in tp]

    def plain(A, n1):
        return Diagonals(A, pl.layout, n1, t, lambda k, slots: sc.encode(slots), False)
    if pl.fold:
        rdiag = []
        ldiag = [plain(c.Lfold[l] @ c.R, pl.n1_L) for l in range(c.d)]
    else:
        rdiag = plain(extended_reshuffle(c), pl.n1_R)
        ldiag = [plain(c.Lfold[l], pl.n1_L) for l in range(c.d)]
    masks = [sc.encode(pl.layout.replicate(mk)) for mk in c.masks]
    rep = []
    if pl.server_rep:
        from .compiler import replication_matrix
        rep = plain(replication_matrix(c), pl.n1_F)
    return PlainModel(E, Cc, G, TH, rdiag, ldiag, masks, rep)


def encrypt_model(sc: BGV, keys: Keys, pl: Plan, seed: bytes) -> EncModel:
    """Model owner encrypts thresholds, diagonals and masks under the data
    owner's key, each at the level where the schedule consumes it; diagonal i
    of level l has object id (OBJ_LDIAG, l, i), of the reshuffle (OBJ_RDIAG, 0, i)."""
    c, t = pl.c, sc.t
    lv = pl.levels
    tp = S.threshold_planes(c, pl.layout)
    TH = [sc.encrypt_slots(keys, th, seed, obj_id(OBJ_THRESH, 0, k), pl.L) for k, th in enumerate(tp)]

    def enc(A, n1, kind, a, level):
        return Diagonals(A, pl.layout, n1, t,
                         lambda k, slots: sc.encrypt_slots(keys, slots, seed, obj_id(kind, a, k), level), True)
    if pl.fold:
        rdiag = []
        ldiag = [enc(c.Lfold[l] @ c.R, pl.n1_L, OBJ_LDIAG, l, lv["dec"]) for l in range(c.d)]
    else:
        rdiag = enc(extended_reshuffle(c), pl.n1_R, OBJ_RDIAG, 0, lv["dec"])
        ldiag = [enc(c.Lfold[l], pl.n1_L, OBJ_LDIAG, l, lv["branches"]) for l in range(c.d)]
    masks = [sc.encrypt_slots(keys, pl.layout.replicate(mk), seed, obj_id(OBJ_MASK, 0, l), lv["levels"])
             for l, mk in enumerate(c.masks)]
    return EncModel(TH, rdiag, ldiag, masks)


def encrypt_queries(sc: BGV, keys: Keys, pl: Plan, queries: np.ndarray, seed: bytes, group: int) -> List[Ciphertext]:
    planes = S.query_planes(pl.c, pl.layout, queries)
    return [sc.encrypt_slots(keys, pk, seed, obj_id(OBJ_QUERY, group, k), pl.L) for k, pk in enumerate(planes)]


# ------------------------------------------------------------------ evaluation
class Evaluator:
    def __init__(self, sc: BGV, keys: Keys, pl: Plan):
        self.sc, self.keys, self.pl = sc, keys, pl
        self.counts = dict(mul=0, relin=0, rot=0, modswitch=0, ptmul=0, tensor=0)

    # level-aware helpers
    def mul(self, a, b):
        self.counts["mul"] += 1
        return self.sc.mul(a, b, self.keys)

    def sum_all(self, terms: List[Ciphertext]) -> Ciphertext:
        lv = min(t.level for t in terms)
        terms = [self.sc.modswitch_to(t, lv) for t in terms]
        out = terms[0]
        for t in terms[1:]:
            out = self.sc.add(out, t)
        return out

    def seccomp(self, X: List[Ciphertext], model) -> Ciphertext:
        sc = self.sc
        p = len(X)
        eq: Dict[int, Ciphertext] = {}
        lt: Dict[int, Ciphertext] = {}
        if isinstance(model, PlainModel):
            for k in range(p):
                if k >= 1:
                    eq[k] = sc.modswitch(sc.add_plain(sc.mul_plain(X[k], model.E[k]), model.C[k]))
                lt[k] = sc.modswitch(sc.add_plain(sc.mul_plain(X[k], model.G[k]), model.TH[k]))
        else:
            one = np.zeros(sc.N, dtype=np.int64)
            one[0] = 1
            for k in range(p):
                u = self.mul(X[k], model.TH[k])
                xs = sc.modswitch(X[k])
                ts = sc.modswitch(model.TH[k])
                if k >= 1:
                    eq[k] = sc.add_plain(sc.sub(sc.sub(sc.mul_int(u, 2), xs), ts), one)
                lt[k] = sc.sub(ts, u)
        # the terms lt_k * prod_{j > k} eq_j in ceil(log2 p) rounds of products (slotsim's plan); each
        # round first switches all its operands to the lowest level among them, so it runs at one level
        val = {}
        for m in range(p - 1):
            val[frozenset([("e", m)])] = eq[p - 1 - m]
            val[frozenset([("l", m)])] = lt[p - 2 - m]
        rounds, terms = S.seccomp_product_plan(p - 1)
        for rnd in rounds:
            lv = min(min(val[a].level, val[b].level) for _, a, b in rnd)
            for k, a, b in rnd:
                val[k] = self.mul(sc.modswitch_to(val[a], lv), sc.modswitch_to(val[b], lv))
        return self.sum_all([lt[p - 1]] + [val[terms[i]] for i in range(p - 1)])

    def matmul(self, v: Ciphertext, diags: list, n1: int) -> Ciphertext:
        sc = self.sc
        n = len(diags)
        n2 = -(-n // n1)
        used = sorted({k % n1 for k in range(n) if _present(diags, k)})
        baby = sc.rotate_hoisted(v, used, self.keys)
        idx = sc.data_idx(v.level)
        enc = diags.encrypted if isinstance(diags, Diagonals) else any(isinstance(d, Ciphertext) for d in diags)
        baby_ntt = {}
        if not enc:
            for j, ct in baby.items():
                baby_ntt[j] = [sc.ntt(pp, idx) for pp in ct.polys]
        parts = []
        for g in range(n2):
            terms = [(j, diags[g * n1 + j]) for j in range(n1)
                     if g * n1 + j < n and _present(diags, g * n1 + j)]
            if not terms:
                continue
            if enc:
                inner = None
                for j, D in terms:
                    tt = sc.tensor(baby[j], D)
                    inner = tt if inner is None else sc.add(inner, tt)
                inner = sc.relinearize(inner, self.keys)
            else:
                acc0 = np.zeros((len(idx), sc.N), dtype=np.uint64)
                acc1 = np.zeros_like(acc0)
                for j, D in terms:
                    pt = sc.plain_ntt(D, v.level)
                    acc0 = sc.padd(acc0, sc.pmul_ntt(baby_ntt[j][0], pt, idx), idx)
                    acc1 = sc.padd(acc1, sc.pmul_ntt(baby_ntt[j][1], pt, idx), idx)
                inner = Ciphertext([sc.intt(acc0, idx), sc.intt(acc1, idx)], v.level)
            parts.append((inner, g * n1))
        # giant steps: the rotated inner sums added with one ModDown (BGV.rotate_sum), then one switch
        return sc.modswitch(sc.rotate_sum(parts, self.keys))

    def add_mask(self, ct: Ciphertext, mask) -> Ciphertext:
        if isinstance(mask, Ciphertext):
            return self.sc.add(ct, mask)
        return self.sc.add_plain(ct, mask)

    def run(self, X: List[Ciphertext], model) -> Dict[str, object]:
        sc, pl = self.sc, self.pl
        if pl.server_rep:
            # each plane: the replication product (hoisted babies, giants, one switch)
            X = [self.matmul(x, model.rep, pl.n1_F) for x in X]
        dec = self.seccomp(X, model)
        assert dec.level == pl.levels["dec"], (dec.level, pl.levels)
        levels = []
        branches = None
        if pl.fold:
            for l in range(pl.c.d):
                levels.append(self.add_mask(self.matmul(dec, model.ldiag[l], pl.n1_L), model.masks[l]))
        else:
            branches = self.matmul(dec, model.rdiag, pl.n1_R)
            for l in range(pl.c.d):
                levels.append(self.add_mask(self.matmul(branches, model.ldiag[l], pl.n1_L), model.masks[l]))
        labels = S.multall(levels, self.mul)
        result = sc.modswitch_to(labels, 0)
        return dict(dec=dec, branches=branches, levels=levels, labels=labels, result=result)


def decrypt_labels(sc: BGV, keys: Keys, pl: Plan, result: Ciphertext, n_queries: int) -> np.ndarray:
    slots = sc.decrypt_slots(keys, result)
    return np.stack([pl.layout.extract(slots, k, pl.c.m) for k in range(n_queries)])
