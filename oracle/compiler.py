"""Forest compiler: the vectorizable structures of Section 4.2.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's definitions in its order:
  * node level = branches on the longest path down to a label, counting the
    node itself; a label has level 0 (Section 4.1, "Properties of nodes");
  * multiplicity kappa_f, maximum multiplicity K, branching b and quantized
    branching q = K * F (Section 4.1, "Properties of models");
  * padded threshold vector: thresholds grouped by feature, each group padded
    with sentinels S = 0 up to K entries (Section 4.2, "Padded Threshold
    Vector"); within a group, branches in ascending preorder index (reading:
    the paper does not fix the order);
  * reshuffling matrix R (b x q): R[i][j] = 1 iff padded slot j holds branch i
    (Section 4.2, "Reshuffling Matrix");
  * level matrices L_l (m x b) and masks (Section 4.2, "Level Matrices",
    "Level Masks").  For label i and level l the selected branch is the
    ancestor at level exactly l; else the ancestor with the greatest level
    below l ("the highest branch not exceeding that level"); else (reading:
    every ancestor lies above l) the label's parent.  mask = 0 when the label
    lies under the true (right) child of the selected branch, 1 otherwise;
  * generalized diagonals d_k[j] = A[j][(j + k) mod n] (Section 4.1, "Matrix
    Representation"; the printed formula is garbled, this is its reading).

Slot layout (reading; the paper leaves the packing unstated): the query's
replicated feature vector is cyclically extended inside a block of W slots so
that both matrix products can read rotated inputs without wrap-around:
B_in = m + b + q - 2 padded positions are used, W = next power of two >= B_in.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .forest import Branch, Leaf, Node, codebook, parse_forest, tree_of_label


@dataclass
class Compiled:
    n_features: int
    precision: int
    branches: List[Branch]
    labels: List[Leaf]
    level_of_branch: List[int]
    kappa: List[int]
    K: int
    q: int
    b: int
    m: int
    d: int
    padded: List[Optional[int]]          # padded slot -> branch index or None (sentinel)
    thresholds_padded: List[int]          # threshold per padded slot (sentinel = 0)
    R: np.ndarray                         # b x q
    L: List[np.ndarray]                   # d matrices, m x b
    masks: List[np.ndarray]               # d vectors, length m
    Lfold: List[np.ndarray]               # d signed matrices (1 - 2 mask) * L, entries in {-1,0,1}
    selected: List[List[Optional[int]]]   # [level-1][label] -> selected branch index
    codebook: List[int]
    tree_of_label: List[int]
    n_trees: int
    B_in: int = 0
    W: int = 0
    meta: dict = field(default_factory=dict)


def next_pow2(x: int) -> int:
    p = 1
    while p < x:
        p <<= 1
    return p


def bsgs_n1(n: int) -> int:
    """Baby-step count n1 = 2^ceil(log2 sqrt(n)) (at least 1)."""
    if n <= 1:
        return 1
    return 1 << math.ceil(math.log2(math.sqrt(n)) - 1e-12)


def compile_forest(text: str, n_features: int, precision: int) -> Compiled:
    _, trees = parse_forest(text)
    return compile_trees(trees, n_features, precision)


def compile_trees(trees: List[Node], n_features: int, precision: int) -> Compiled:
    branches: List[Branch] = []
    labels: List[Leaf] = []
    parent_of_label: List[List[Branch]] = []   # ancestors root..parent per label
    side_of_label: List[List[int]] = []        # 1 if label is in right subtree of that ancestor
    levels: dict = {}

    def level(n: Node) -> int:
        if isinstance(n, Leaf):
            return 0
        if id(n) not in levels:
            levels[id(n)] = 1 + max(level(n.left), level(n.right))
        return levels[id(n)]

    def walk(n: Node, anc: List[Branch], side: List[int]) -> None:
        if isinstance(n, Leaf):
            labels.append(n)
            parent_of_label.append(list(anc))
            side_of_label.append(list(side))
            return
        branches.append(n)
        walk(n.left, anc + [n], side + [0])
        walk(n.right, anc + [n], side + [1])

    for t in trees:
        walk(t, [], [])
    b, m = len(branches), len(labels)
    if b == 0:
        raise ValueError("forest has no branches")
    for i, br in enumerate(branches):
        assert br.index == i
        if not 0 <= br.feature < n_features:
            raise ValueError(f"feature {br.feature} out of range")
        if br.threshold >= (1 << precision):
            raise ValueError(f"threshold {br.threshold} needs more than {precision} bits")
    lvl = [level(br) for br in branches]
    d = max(level(t) for t in trees)

    kappa = [0] * n_features
    for br in branches:
        kappa[br.feature] += 1
    K = max(kappa)
    q = K * n_features

    padded: List[Optional[int]] = []
    for f in range(n_features):
        group = [br.index for br in branches if br.feature == f]   # ascending preorder
        padded.extend(group + [None] * (K - len(group)))
    thr_pad = [0 if j is None else branches[j].threshold for j in padded]

    R = np.zeros((b, q), dtype=np.int64)
    for col, br_idx in enumerate(padded):
        if br_idx is not None:
            R[br_idx, col] = 1

    L_mats, masks, folds, selected = [], [], [], []
    for l in range(1, d + 1):
        Lm = np.zeros((m, b), dtype=np.int64)
        mk = np.zeros(m, dtype=np.int64)
        sel_l: List[Optional[int]] = []
        for i in range(m):
            anc = parent_of_label[i]
            side = side_of_label[i]
            if not anc:                       # a tree that is a single label
                sel_l.append(None)
                mk[i] = 1
                continue
            choice = None
            for a_pos, a in enumerate(anc):
                if lvl[a.index] == l:
                    choice = a_pos
            if choice is None:
                below = [a_pos for a_pos, a in enumerate(anc) if lvl[a.index] < l]
                if below:
                    choice = max(below, key=lambda ap: lvl[anc[ap].index])
                else:
                    choice = len(anc) - 1     # parent
            br = anc[choice]
            Lm[i, br.index] = 1
            mk[i] = 0 if side[choice] == 1 else 1
            sel_l.append(br.index)
        L_mats.append(Lm)
        masks.append(mk)
        folds.append((1 - 2 * mk)[:, None] * Lm)
        selected.append(sel_l)

    c = Compiled(
        n_features=n_features, precision=precision, branches=branches, labels=labels,
        level_of_branch=lvl, kappa=kappa, K=K, q=q, b=b, m=m, d=d, padded=padded,
        thresholds_padded=thr_pad, R=R, L=L_mats, masks=masks, Lfold=folds,
        selected=selected, codebook=codebook(trees), tree_of_label=tree_of_label(trees),
        n_trees=len(trees))
    c.B_in = m + b + q - 2
    c.W = next_pow2(c.B_in)
    return c


class _Draws:
    """Sequential bounded draws from one SHAKE-256 stream: an 8-byte little-endian word masked to
    bitlen(bound) bits, accepted if below bound (the uniform sampler of the key material)."""

    def __init__(self, seed: bytes, domain: str):
        from .sampling import stream
        self._get = lambda n: stream(seed, domain, 0, 0, n)
        self._buf = self._get(4096)
        self._pos = 0

    def word(self) -> int:
        if self._pos + 8 > len(self._buf):
            self._buf = self._get(2 * len(self._buf))
        w = int.from_bytes(self._buf[self._pos:self._pos + 8], "little")
        self._pos += 8
        return w

    def below(self, bound: int) -> int:
        mask = (1 << bound.bit_length()) - 1
        while True:
            w = self.word() & mask
            if w < bound:
                return w


def privatize(c: Compiled, seed: bytes, n_pad: int, n_classes: int) -> Compiled:
    """Result privacy (Section 7.2.2, "Returning classification bitvectors"): the server shuffles the
    result bitvector and the codebook by one random permutation and pads both with n_pad extra labels
    that are never selected.  Folded into the level products: slot s of every level matrix, mask and
    the codebook takes original row arr[s], where arr is the identity on m + n_pad rows shuffled by
    Fisher-Yates (for i from m + n_pad - 1 down to 1: swap arr[i] with arr[j], j drawn below i + 1);
    a row arr[s] >= m is a padding row (all-zero matrix row, mask 0: its level results and product
    are 0) whose codebook label is drawn below n_classes (the forest's label count), in increasing
    arr[s] order,
    after the permutation.  All draws come from the SHAKE-256 stream of domain "res.perm"."""
    import copy
    if n_pad < 0:
        raise ValueError("negative padding")
    m, mp = c.m, c.m + n_pad
    dr = _Draws(seed, "res.perm")
    arr = list(range(mp))
    for i in range(mp - 1, 0, -1):
        j = dr.below(i + 1)
        arr[i], arr[j] = arr[j], arr[i]
    pad_label = [dr.below(n_classes) for _ in range(n_pad)]
    out = copy.copy(c)
    out.m = mp
    out.L = [np.stack([A[r] if r < m else np.zeros(c.b, dtype=np.int64) for r in arr]) for A in c.L]
    out.masks = [np.array([mk[r] if r < m else 0 for r in arr], dtype=np.int64) for mk in c.masks]
    out.Lfold = [(1 - 2 * mk)[:, None] * A for A, mk in zip(out.L, out.masks)]
    out.selected = [[sel[r] if r < m else None for r in arr] for sel in c.selected]
    out.codebook = [c.codebook[r] if r < m else pad_label[r - m] for r in arr]
    out.tree_of_label = [c.tree_of_label[r] if r < m else -1 for r in arr]
    out.meta = dict(c.meta, perm=list(arr))
    out.B_in = mp + c.b + c.q - 2
    out.W = next_pow2(out.B_in)
    return out


def server_replicated(c: Compiled) -> Compiled:
    """Server-side feature replication (Section 7.2.1, "Feature padding": the alternative to Diane replicating her features):
    the query holds each feature once, cyclically extended with period F (block slot s < B_in + F - 1
    holds feature s mod F), so that no multiplicity is revealed; the server maps it onto the padded
    layout by one plaintext matrix product with replication_matrix(c).  The block must hold the
    longer input: W = next power of two >= B_in + F - 1."""
    import copy
    out = copy.copy(c)
    out.meta = dict(c.meta, server_rep=True)
    out.W = next_pow2(c.B_in + c.n_features - 1)
    return out


def replication_matrix(c: Compiled) -> np.ndarray:
    """Rep (B_in x F): Rep[s][f] = 1 iff padded slot s mod q belongs to feature f (slot j of the
    padded vector holds feature j div K, Section 4.2)."""
    Rep = np.zeros((c.B_in, c.n_features), dtype=np.int64)
    s = np.arange(c.B_in)
    Rep[s, (s % c.q) // c.K] = 1
    return Rep


def generalized_diagonal(A: np.ndarray, k: int) -> np.ndarray:
    """d_k[j] = A[j][(j + k) mod n], j < rows (Section 4.1)."""
    rows, n = A.shape
    j = np.arange(rows)
    return A[j, (j + k) % n]


def extended_reshuffle(c: Compiled) -> np.ndarray:
    """R_ext ((m + b - 1) x q): row j is R[j mod b], so the reshuffled output
    is already the period-b cyclic extension the level products read."""
    rows = c.m + c.b - 1
    return c.R[np.arange(rows) % c.b]


def replicate_features(x: List[int], K: int) -> List[int]:
    """Diane's replicated feature vector [x0]*K + [x1]*K + ... (Section 3.3, Step 0)."""
    out: List[int] = []
    for v in x:
        out.extend([int(v)] * K)
    return out
