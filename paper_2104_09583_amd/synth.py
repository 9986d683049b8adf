"""Seeded synthetic workload generators (forests, queries, crypto seeds).

This module is shared by the CPU oracle and the GPU library's tests and
benchmark.  It holds *no* arithmetic of the method: it only draws random
forest shapes, thresholds, labels and feature values with numpy's PCG64
generator and writes them in the serialized forest format (paper, Section 5,
"Input Representation": one line of label names, then one line per tree in
preorder; a leaf carries its label index, a branch its feature index,
threshold, then its left and right subtrees).

Generator pin (the shapes of the evaluated workloads):
  * the root of every tree is a branch;
  * a node at depth k with 1 <= k < max_depth is a branch with probability
    ``split_prob``, otherwise a leaf; a node at depth max_depth is a leaf;
  * a branch draws feature ~ U[0, F) and threshold ~ U[0, 2^p);
    a leaf draws label ~ U[0, C);
  * nodes are drawn in preorder (self, left subtree, right subtree);
  * query features are drawn ~ U[0, 2^p).

Token grammar of one tree line: ``B <feature> <threshold> <left> <right>`` or
``L <label>``; indices are 0-based.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class ForestShape:
    n_trees: int
    max_depth: int
    split_prob: float
    n_features: int
    precision: int
    n_classes: int


@dataclass(frozen=True)
class Workload:
    """One evaluated configuration: forest shape, query count, ring size."""
    name: str
    shape: ForestShape
    n_queries: int
    log_n: int
    encrypted_model: bool
    seed_index: int
    notes: str = ""
    chain: dict = field(default_factory=dict)
    fold: bool = False
    # baby steps of the reshuffle and level products (0: the compiler's square-root rule); a measured
    # choice where it beats the rule on the GPU
    n1: tuple = (0, 0)
    # query groups evaluated together per batched call when every group of the workload is timed
    batch: int = 1


def _gen_tree(rng: np.random.Generator, shape: ForestShape, depth: int, out: list) -> None:
    is_branch = depth == 0 or (depth < shape.max_depth and rng.random() < shape.split_prob)
    if depth >= shape.max_depth:
        is_branch = False
    if is_branch:
        f = int(rng.integers(0, shape.n_features))
        thr = int(rng.integers(0, 1 << shape.precision))
        out.extend(["B", str(f), str(thr)])
        _gen_tree(rng, shape, depth + 1, out)
        _gen_tree(rng, shape, depth + 1, out)
    else:
        out.extend(["L", str(int(rng.integers(0, shape.n_classes)))])


def gen_forest_text(shape: ForestShape, seed: int) -> str:
    """Serialized random forest of the given shape (deterministic in ``seed``)."""
    rng = np.random.default_rng(seed)
    lines = [" ".join(f"c{i}" for i in range(shape.n_classes))]
    for _ in range(shape.n_trees):
        toks: list = []
        _gen_tree(rng, shape, 0, toks)
        lines.append(" ".join(toks))
    return "\n".join(lines) + "\n"


def gen_queries(n_queries: int, n_features: int, precision: int, seed: int) -> np.ndarray:
    """Uniform unsigned feature vectors, shape [n_queries, n_features], uint32."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 1 << precision, size=(n_queries, n_features), dtype=np.uint64).astype(np.uint32)


def crypto_seed(label: str) -> bytes:
    """32-byte seed for all randomness of one workload's keys and ciphertexts."""
    return hashlib.shake_256(label.encode("ascii")).digest(32)


# The five evaluated workloads.  Depth/feature/precision/class counts follow
# the configuration list of the benchmark; ``seed_index`` i gives forest seed
# i, query seed 100 + i and crypto seed SHAKE-256("COPSE-cfg-i").
# Prime-chain parameters (see the library's copse_params): number of data
# primes, exclusive bounds for q_0, the other data primes and the special
# primes, and alpha = special primes = primes per key-switching digit.
#   N=16384: 8 data primes, total log2(PQ) ~ 394 <= 438 (HE-standard bound
#            for 128-bit security); the reshuffle is folded into the level
#            products to fit the circuit in that chain.
#   N=32768: 10 (p = 8) or 11 (p = 16) data primes, log2(PQ) ~ 617-659 <= 881.
# Each chain has exactly the levels the circuit takes: the comparison (1 + ceil(log2 p)), the
# reshuffle (unless folded), the level products and the product tree over d levels.
CHAIN_16K = dict(log_n=14, n_data_primes=8, q0_max=1 << 42, data_max=388736063996,   # 2^38.5
                 alpha=2, special_max=1 << 44)
CHAIN_32K_P8 = dict(log_n=15, n_data_primes=10, q0_max=1 << 48, data_max=1 << 42, alpha=4,
                    special_max=1 << 48)
CHAIN_32K_P16 = dict(log_n=15, n_data_primes=11, q0_max=1 << 48, data_max=1 << 42, alpha=4,
                     special_max=1 << 48)

WORKLOADS = {
    "c1_plain_d3": Workload(
        "c1_plain_d3", ForestShape(1, 3, 1.0, 4, 8, 2), 1, 14, False, 1,
        "one complete binary tree of depth 3, one query, N=16384", CHAIN_16K, True),
    "c2_forest16_d5": Workload(
        "c2_forest16_d5", ForestShape(16, 5, 0.7, 16, 8, 4), 1, 15, False, 2,
        "16 random unbalanced trees, max depth 5, one query, N=32768", CHAIN_32K_P8, n1=(16, 0)),
    "c3_batched_32x_d6": Workload(
        "c3_batched_32x_d6", ForestShape(32, 6, 0.7, 16, 8, 8), 1024, 15, False, 3,
        "1024 queries against 32 trees of max depth 6, N=32768", CHAIN_32K_P8, n1=(0, 16), batch=16),
    "c4_encmodel_64x_d8": Workload(
        "c4_encmodel_64x_d8", ForestShape(64, 8, 0.7, 32, 16, 10), 256, 15, True, 4,
        "encrypted model and queries, 64 trees max depth 8, 16-bit, N=32768", CHAIN_32K_P16, n1=(0, 128),
        batch=16),
    "c5_serve_8x_d4": Workload(
        "c5_serve_8x_d4", ForestShape(8, 4, 0.7, 16, 8, 4), 1, 15, False, 5,
        "serving mix member: 8 trees of depth 4", CHAIN_32K_P16),
    "c5_serve_32x_d6": Workload(
        "c5_serve_32x_d6", ForestShape(32, 6, 0.7, 16, 8, 8), 1, 15, False, 6,
        "serving mix member: 32 trees of depth 6", CHAIN_32K_P16),
    "c5_serve_64x_d8": Workload(
        "c5_serve_64x_d8", ForestShape(64, 8, 0.7, 32, 16, 10), 1, 15, False, 7,
        "serving mix member: 64 trees of depth 8, plaintext model", CHAIN_32K_P16),
}


def workload_inputs(w: Workload):
    """(forest_text, queries[n, F], crypto_seed) for a workload."""
    s = w.shape
    text = gen_forest_text(s, w.seed_index)
    queries = gen_queries(w.n_queries, s.n_features, s.precision, 100 + w.seed_index)
    return text, queries, crypto_seed(f"COPSE-cfg-{w.seed_index}")


# The serving mix: resident forests of the three sizes, one query per request, each request's
# forest drawn uniformly (all three share the N = 32768, 16-bit-capable chain).
SERVE_MIX = ("c5_serve_8x_d4", "c5_serve_32x_d6", "c5_serve_64x_d8")


# ---------------------------------------------------------------- microbenchmark forests (Table 6)
# Eight forests over 2 features and 3 labels that differ in one property at a time: maximum depth
# (depth4/5/6), branch count and tree count (width55, width78, width677: the digits of the name are the
# branches per tree) and threshold precision (prec8/16).  "# of branches" 15 over 2 trees is split
# 7 + 8 (the width78 split).
@dataclass(frozen=True)
class MicroForest:
    name: str
    branches: tuple        # branches per tree
    max_depth: int
    precision: int
    n_features: int = 2
    n_classes: int = 3


TABLE6 = (
    MicroForest("depth4", (7, 8), 4, 8),
    MicroForest("depth5", (7, 8), 5, 8),
    MicroForest("depth6", (7, 8), 6, 8),
    MicroForest("width55", (5, 5), 5, 8),
    MicroForest("width78", (7, 8), 5, 8),
    MicroForest("width677", (6, 7, 7), 5, 8),
    MicroForest("prec8", (7, 8), 5, 8),
    MicroForest("prec16", (7, 8), 5, 16),
)


def gen_forest_exact(mf: MicroForest, seed: int) -> str:
    """A random forest with exactly ``mf.branches[i]`` branches in tree i and maximum depth exactly
    ``mf.max_depth`` (branches at depths 0 .. max_depth - 1, leaves at depth <= max_depth).

    Tree 0 first grows a chain of ``max_depth`` branches from its root (its direction at each step
    drawn uniformly); every tree then turns uniformly drawn leaves above the maximum depth into
    branches until it has its branch count.  Features ~ U[0, F), thresholds ~ U[0, 2^p), labels
    ~ U[0, C), drawn in preorder when the tree is written out."""
    rng = np.random.default_rng(seed)
    if mf.branches[0] < mf.max_depth:
        raise ValueError("the first tree must hold the chain to the maximum depth")
    lines = [" ".join(f"c{i}" for i in range(mf.n_classes))]
    for t, nb in enumerate(mf.branches):
        if nb > (1 << mf.max_depth) - 1:
            raise ValueError("more branches than a tree of that depth holds")
        # node: [is_branch, left, right, depth]; node 0 is the root
        nodes = [[False, -1, -1, 0]]

        def grow(i):
            nodes[i][0] = True
            d = nodes[i][3]
            nodes[i][1] = len(nodes)
            nodes.append([False, -1, -1, d + 1])
            nodes[i][2] = len(nodes)
            nodes.append([False, -1, -1, d + 1])

        count = 0
        if t == 0:
            cur = 0
            for _ in range(mf.max_depth):
                grow(cur)
                count += 1
                cur = nodes[cur][1 + int(rng.integers(0, 2))]
        else:
            grow(0)
            count = 1
        while count < nb:
            leaves = [i for i, n in enumerate(nodes) if not n[0] and n[3] < mf.max_depth]
            grow(leaves[int(rng.integers(0, len(leaves)))])
            count += 1
        toks: list = []

        def emit(i):
            if nodes[i][0]:
                toks.extend(["B", str(int(rng.integers(0, mf.n_features))),
                             str(int(rng.integers(0, 1 << mf.precision)))])
                emit(nodes[i][1])
                emit(nodes[i][2])
            else:
                toks.extend(["L", str(int(rng.integers(0, mf.n_classes)))])

        emit(0)
        lines.append(" ".join(toks))
    return "\n".join(lines) + "\n"


def micro_chain(mf: MicroForest) -> dict:
    """The N = 32768 chain of the configured workloads with enough levels for the forest."""
    return CHAIN_32K_P16 if mf.precision > 8 else CHAIN_32K_P8
