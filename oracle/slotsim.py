"""Algorithm 1 on plaintext slot vectors mod t, with the exact packed layout.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

This is the arithmetic the encrypted circuit performs, one slot at a time,
with rotations realized as cyclic left shifts of each of the two slot rows
(a left rotation by r moves the value of slot j + r into slot j).

Steps, in the order of the paper's Algorithm 1 (Section 4.3):
  1. SecComp (Section 4.1, "Integer Comparison"): per-slot x < theta over the
     p transposed bit-planes (Section 4.1, "Representing Non-integral
     Values").  The paper only cites this primitive; the circuit used here
     (reading) is the standard most-significant-bit-first comparison:
        eq_k = 1 - x_k - th_k + 2 x_k th_k,  lt_k = th_k - x_k th_k,
        S_k  = prod_{j>k} eq_j  (a Kogge-Stone prefix product),
        dec  = lt_{p-1} + sum_{k<p-1} lt_k S_k.
  2. Reshuffle: Branches = MatMul(R_ext, dec) (Section 4.2, "Reshuffling
     Matrix"; MatMul of Section 4.1, "Matrix Multiplication").
  3. Levels: LvlRes_l = MatMul(L'_l, Branches) + mask_l, where
     L'_l = diag(1 - 2 mask_l) L_l folds the XOR with the mask
     (a xor c = c + (1 - 2c) a on bits).  Reading: the level products read
     the reshuffled vector, as the prose of Section 4.3 says.
  4. MultAll: balanced product tree over the d level vectors.
MatMul uses the baby-step/giant-step form of the diagonal method:
  out = sum_g rot( sum_j rot(d_{g n1 + j}, -g n1) * rot(v, j), g n1 ),
which equals the plain sum_k d_k * rot(v, k).
"""
from __future__ import annotations

from typing import List

import numpy as np

from .compiler import (Compiled, bsgs_n1, extended_reshuffle, generalized_diagonal,
                       replicate_features)


class Layout:
    """Slot geometry: N slots as 2 rows of N/2; blocks of W slots per query."""

    def __init__(self, n_slots: int, W: int):
        self.N = n_slots
        self.row = n_slots // 2
        self.W = W
        if W > self.row:
            raise ValueError("block width exceeds a slot row")
        self.blocks_per_row = self.row // W
        self.Qs = 2 * self.blocks_per_row

    def block_origin(self, k: int):
        return k // self.blocks_per_row, (k % self.blocks_per_row) * self.W

    def place(self, per_block: List[np.ndarray]) -> np.ndarray:
        """Put one length-<=W vector into each block; the rest stays 0."""
        out = np.zeros((2, self.row), dtype=np.int64)
        for k, vec in enumerate(per_block):
            r, c0 = self.block_origin(k)
            out[r, c0:c0 + len(vec)] = vec
        return out

    def replicate(self, vec: np.ndarray, n_blocks: int = None) -> np.ndarray:
        n_blocks = self.Qs if n_blocks is None else n_blocks
        return self.place([vec] * n_blocks)

    def extract(self, slots: np.ndarray, k: int, length: int) -> np.ndarray:
        r, c0 = self.block_origin(k)
        return slots[r, c0:c0 + length]


def rot(v: np.ndarray, r: int) -> np.ndarray:
    """Left rotation of each slot row by r (slot j receives slot j + r)."""
    return np.roll(v, -r, axis=1)


def query_planes(c: Compiled, lay: Layout, queries: np.ndarray) -> List[np.ndarray]:
    """p bit-plane slot vectors; plane k holds bit k of the replicated,
    cyclically extended features (slot s of a block holds padded position
    s mod q for s < B_in).  k = p-1 is the most significant bit."""
    planes = []
    server_rep = c.meta.get("server_rep", False)
    for k in range(c.precision):
        per_block = []
        for x in queries:
            if server_rep:
                # each feature once, cyclically extended with period F (server-side replication)
                ext = np.array(list(x), dtype=np.int64)[np.arange(c.B_in + c.n_features - 1) % c.n_features]
            else:
                rep = np.array(replicate_features(list(x), c.K), dtype=np.int64)
                ext = rep[np.arange(c.B_in) % c.q]
            per_block.append((ext >> k) & 1)
        planes.append(lay.place(per_block))
    return planes


def threshold_planes(c: Compiled, lay: Layout) -> List[np.ndarray]:
    thr = np.array(c.thresholds_padded, dtype=np.int64)
    ext = thr[np.arange(c.B_in) % c.q]
    return [lay.replicate((ext >> k) & 1) for k in range(c.precision)]


def kogge_stone_prefix(seq: List, mul) -> List:
    """Inclusive prefix products pre[i] = seq[0] * ... * seq[i] in
    ceil(log2 len) rounds; round with stride s multiplies i by i - s."""
    cur = list(seq)
    s = 1
    while s < len(cur):
        nxt = list(cur)
        for i in range(s, len(cur)):
            nxt[i] = mul(cur[i], cur[i - s])
        cur = nxt
        s *= 2
    return cur


def seccomp_product_plan(n: int):
    """Products that form t_i = l_i * e_0 * e_1 * ... * e_i for every i < n in ceil(log2(n + 1))
    rounds, with the comparison's e_m = eq_{p-1-m} and l_i = lt_{p-2-i} (n = p - 1), so that
    t_i = lt_k * prod_{j > k} eq_j for k = p - 2 - i.

    Every value is named by the set of leaves it multiplies: ('e', m) and ('l', i).  The e's are
    combined in aligned blocks [j 2^s, (j + 1) 2^s), block s from two blocks s - 1 (depth s); the
    factors of t_i are the aligned blocks that tile [0, i], left to right (sizes falling), then
    l_i; they are multiplied from the right end (the last two into one) until one is left.  A
    product's depth is one more than its deeper operand; since the blocks' sizes are distinct
    powers of two, t_i ends at depth ceil(log2(i + 2)).  Products with the same leaf set are made
    once.

    Returns (rounds, terms): rounds[d] lists (key, a, b) of the products of depth d + 1 in the order
    they were first needed; terms[i] is the key of t_i."""
    depth = {}
    order = []

    def leaf(kind, idx):
        k = frozenset([(kind, idx)])
        depth[k] = 0
        return k

    def prod(a, b):
        k = a | b
        if k not in depth:
            depth[k] = max(depth[a], depth[b]) + 1
            order.append((k, a, b))
        return k

    def block(s, j):
        if s == 0:
            return leaf("e", j)
        return prod(block(s - 1, 2 * j), block(s - 1, 2 * j + 1))

    terms = []
    for i in range(n):
        factors = []
        start = 0
        while start <= i:
            size = 1
            while start % (2 * size) == 0 and start + 2 * size <= i + 1:
                size *= 2
            factors.append(block(size.bit_length() - 1, start // size))
            start += size
        factors.append(leaf("l", i))
        while len(factors) > 1:
            b = factors.pop()
            a = factors.pop()
            factors.append(prod(a, b))
        terms.append(factors[0])
    n_rounds = max((depth[k] for k in terms), default=0)
    rounds = [[(k, a, b) for k, a, b in order if depth[k] == d + 1] for d in range(n_rounds)]
    return rounds, terms


def seccomp_slots(xp: List[np.ndarray], tp: List[np.ndarray], t: int) -> np.ndarray:
    p = len(xp)
    eq = [(1 - xp[k] - tp[k] + 2 * xp[k] * tp[k]) % t for k in range(p)]
    lt = [(tp[k] - xp[k] * tp[k]) % t for k in range(p)]
    val = {}
    for m in range(p - 1):
        val[frozenset([("e", m)])] = eq[p - 1 - m]
        val[frozenset([("l", m)])] = lt[p - 2 - m]
    rounds, terms = seccomp_product_plan(p - 1)
    for rnd in rounds:
        for k, a, b in rnd:
            val[k] = (val[a] * val[b]) % t
    dec = lt[p - 1].copy()
    for i in range(p - 1):
        dec = (dec + val[terms[i]]) % t
    return dec


def prerotated_diagonal(A: np.ndarray, lay: Layout, n1: int, k: int) -> np.ndarray:
    """Diagonal k = g n1 + j of A, placed at block offsets g n1 .. g n1 + rows - 1
    (that is rot(d_k, -g n1) inside every block)."""
    rows, n = A.shape
    g = k // n1
    vec = np.zeros(g * n1 + rows, dtype=np.int64)
    vec[g * n1:] = generalized_diagonal(A, k)
    return lay.replicate(vec)


def prerotated_diagonals(A: np.ndarray, lay: Layout, n1: int) -> List[np.ndarray]:
    """Every pre-rotated diagonal of A (see prerotated_diagonal)."""
    return [prerotated_diagonal(A, lay, n1, k) for k in range(A.shape[1])]


def matmul_bsgs(v: np.ndarray, diags: List[np.ndarray], n1: int, t: int) -> np.ndarray:
    n = len(diags)
    n2 = -(-n // n1)
    baby = [rot(v, j) for j in range(n1)]
    out = np.zeros_like(v)
    for g in range(n2):
        inner = np.zeros_like(v)
        for j in range(n1):
            k = g * n1 + j
            if k < n:
                inner = (inner + diags[k] * baby[j]) % t
        out = (out + rot(inner, g * n1)) % t
    return out


def matmul_plain(v: np.ndarray, A: np.ndarray, lay: Layout, t: int) -> np.ndarray:
    """The plain diagonal method sum_k d_k * rot(v, k) (no baby/giant split)."""
    rows, n = A.shape
    out = np.zeros_like(v)
    for k in range(n):
        dk = lay.replicate(generalized_diagonal(A, k))
        out = (out + dk * rot(v, k)) % t
    return out


def multall(vs: List, mul) -> object:
    cur = list(vs)
    while len(cur) > 1:
        nxt = [mul(cur[2 * i], cur[2 * i + 1]) for i in range(len(cur) // 2)]
        if len(cur) % 2:
            nxt.append(cur[-1])
        cur = nxt
    return cur[0]


def run(c: Compiled, queries: np.ndarray, n_slots: int, t: int = 65537,
        fold_reshuffle: bool = False, n1_R: int = 0, n1_L: int = 0) -> dict:
    """Algorithm 1 over slot vectors; returns every stage for inspection."""
    lay = Layout(n_slots, c.W)
    if len(queries) > lay.Qs:
        raise ValueError("more queries than blocks")
    xp = query_planes(c, lay, queries)
    if c.meta.get("server_rep", False):
        from .compiler import replication_matrix
        n1_F = bsgs_n1(c.n_features)
        rd = prerotated_diagonals(replication_matrix(c), lay, n1_F)
        xp = [matmul_bsgs(x, rd, n1_F, t) for x in xp]
    tp = threshold_planes(c, lay)
    dec = seccomp_slots(xp, tp, t)
    Rext = extended_reshuffle(c)
    n1_R = n1_R or bsgs_n1(c.q)
    n1_L = n1_L or (bsgs_n1(c.q) if fold_reshuffle else bsgs_n1(c.b))
    masks = [lay.replicate(mk) for mk in c.masks]
    lvl = []
    if fold_reshuffle:
        branches = None
        for l in range(c.d):
            A = c.Lfold[l] @ c.R          # m x q: level selection composed with R
            lvl.append((matmul_bsgs(dec, prerotated_diagonals(A % t, lay, n1_L), n1_L, t)
                        + masks[l]) % t)
    else:
        branches = matmul_bsgs(dec, prerotated_diagonals(Rext, lay, n1_R), n1_R, t)
        for l in range(c.d):
            lvl.append((matmul_bsgs(branches, prerotated_diagonals(c.Lfold[l] % t, lay, n1_L),
                                    n1_L, t) + masks[l]) % t)
    labels = multall(lvl, lambda a, b: (a * b) % t)
    per_query = [lay.extract(labels, k, c.m).copy() for k in range(len(queries))]
    return dict(planes=xp, thresholds=tp, dec=dec, branches=branches, levels=lvl,
                labels=labels, per_query=per_query, layout=lay)
