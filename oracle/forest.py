"""Plain decision-forest evaluation: the definition of the result.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Paper, Section 2.1: a branch compares one feature with a threshold and
descends into the left child when the decision is false and the right child
when it is true; Section 4.1 indexes branches and labels of the whole forest
in preorder; Section 4.1 "Classification Result": one output slot per label
node, holding 1 iff that label is the one its tree selects (an N-hot vector).
Reading taken where the paper is silent: the decision at a branch is the
strict comparison x_f < threshold (tie -> false, go left).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Tuple, Union


@dataclass
class Leaf:
    label: int                 # class index (codebook entry)
    index: int = -1            # forest-wide preorder label index


@dataclass
class Branch:
    feature: int
    threshold: int
    left: "Node"
    right: "Node"
    index: int = -1            # forest-wide preorder branch index


Node = Union[Leaf, Branch]


class ParseError(ValueError):
    pass


def parse_forest(text: str) -> Tuple[List[str], List[Node]]:
    """Parse the serialized format (Section 5, "Input Representation").

    First line: label names.  Then one line per tree, preorder tokens
    ``B f thr <left> <right>`` or ``L label``.
    """
    lines = [ln for ln in text.splitlines() if ln.strip()]
    if not lines:
        raise ParseError("empty forest text")
    names = lines[0].split()
    trees: List[Node] = []
    for ln in lines[1:]:
        toks = ln.split()
        pos = 0

        def rec() -> Node:
            nonlocal pos
            if pos >= len(toks):
                raise ParseError("truncated tree")
            tag = toks[pos]
            if tag == "L":
                if pos + 1 >= len(toks):
                    raise ParseError("truncated leaf")
                lab = int(toks[pos + 1])
                pos += 2
                if not 0 <= lab < len(names):
                    raise ParseError(f"label {lab} out of range")
                return Leaf(lab)
            if tag == "B":
                if pos + 2 >= len(toks):
                    raise ParseError("truncated branch")
                f, thr = int(toks[pos + 1]), int(toks[pos + 2])
                if f < 0 or thr < 0:
                    raise ParseError("negative feature or threshold")
                pos += 3
                left = rec()
                right = rec()
                return Branch(f, thr, left, right)
            raise ParseError(f"bad token {tag!r}")

        t = rec()
        if pos != len(toks):
            raise ParseError("trailing tokens on tree line")
        trees.append(t)
    if not trees:
        raise ParseError("forest has no trees")
    index_forest(trees)
    return names, trees


def index_forest(trees: List[Node]) -> Tuple[int, int]:
    """Assign forest-wide preorder indices to branches and labels (Section 4.1)."""
    nb = 0
    nl = 0

    def rec(n: Node) -> None:
        nonlocal nb, nl
        if isinstance(n, Leaf):
            n.index = nl
            nl += 1
        else:
            n.index = nb
            nb += 1
            rec(n.left)
            rec(n.right)

    for t in trees:
        rec(t)
    return nb, nl


def decision(x: List[int], br: Branch) -> int:
    """The branch decision: 1 iff x[f] < threshold (true -> right child)."""
    return 1 if x[br.feature] < br.threshold else 0


def evaluate(trees: List[Node], x: List[int]) -> List[int]:
    """N-hot output over all label nodes: walk each tree from its root."""
    n_labels = sum(count_leaves(t) for t in trees)
    out = [0] * n_labels
    for t in trees:
        n = t
        while isinstance(n, Branch):
            n = n.right if decision(x, n) else n.left
        out[n.index] = 1
    return out


def evaluate_path_product(trees: List[Node], x: List[int]) -> List[int]:
    """Second formulation: each label is the product over its ancestors of
    the decision (if the label lies in the true/right subtree) or of one
    minus it (false/left), as in the polynomial representation of trees
    described among the paper's related work (Section 2.3)."""
    out: List[int] = []

    def rec(n: Node, acc: int) -> None:
        if isinstance(n, Leaf):
            out.append(acc)
            return
        d = decision(x, n)
        rec(n.left, acc * (1 - d))
        rec(n.right, acc * d)

    for t in trees:
        rec(t, 1)
    return out


def count_leaves(n: Node) -> int:
    return 1 if isinstance(n, Leaf) else count_leaves(n.left) + count_leaves(n.right)


def codebook(trees: List[Node]) -> List[int]:
    """Class label of each output slot (label node), in preorder."""
    out: List[int] = []

    def rec(n: Node) -> None:
        if isinstance(n, Leaf):
            out.append(n.label)
        else:
            rec(n.left)
            rec(n.right)

    for t in trees:
        rec(t)
    return out


def tree_of_label(trees: List[Node]) -> List[int]:
    """Tree id of each label node (used to check one 1 per tree)."""
    out: List[int] = []
    for ti, t in enumerate(trees):
        out.extend([ti] * count_leaves(t))
    return out


def plurality(trees: List[Node], bits: List[int], n_classes: int) -> Optional[int]:
    """Client-side vote over the per-tree labels (Section 7.2)."""
    cb = codebook(trees)
    votes = [0] * n_classes
    for slot, bit in enumerate(bits):
        if bit:
            votes[cb[slot]] += 1
    if not any(votes):
        return None
    return max(range(n_classes), key=lambda c: (votes[c], -c))
