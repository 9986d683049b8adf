"""The microbenchmark forests of Table 6: exact branch counts per tree, exact maximum depth, two
features, three labels, thresholds within the precision."""
import pytest

from oracle import forest as F
from paper_2104_09583_amd import synth


def _walk(n, depth, acc):
    if isinstance(n, F.Leaf):
        acc["leaf_depth"] = max(acc["leaf_depth"], depth)
        acc["labels"].add(n.label)
        return
    acc["branches"] += 1
    acc["branch_depth"] = max(acc["branch_depth"], depth)
    acc["features"].add(n.feature)
    acc["max_thr"] = max(acc["max_thr"], n.threshold)
    _walk(n.left, depth + 1, acc)
    _walk(n.right, depth + 1, acc)


@pytest.mark.parametrize("i", range(len(synth.TABLE6)))
def test_table6_forest_shape(i):
    mf = synth.TABLE6[i]
    labels, trees = F.parse_forest(synth.gen_forest_exact(mf, 600 + i))
    assert len(labels) == 3 and len(trees) == len(mf.branches)
    deepest = 0
    for t, nb in zip(trees, mf.branches):
        acc = dict(branches=0, branch_depth=0, leaf_depth=0, features=set(), labels=set(), max_thr=0)
        _walk(t, 0, acc)
        assert acc["branches"] == nb
        assert acc["leaf_depth"] <= mf.max_depth
        assert acc["features"] <= {0, 1}
        assert acc["max_thr"] < (1 << mf.precision)
        assert acc["labels"] <= {0, 1, 2}
        deepest = max(deepest, acc["branch_depth"] + 1)
    assert deepest == mf.max_depth


def test_table6_names_encode_branches():
    by = {m.name: m for m in synth.TABLE6}
    assert by["width55"].branches == (5, 5)
    assert by["width78"].branches == (7, 8)
    assert by["width677"].branches == (6, 7, 7)
    assert {by[n].max_depth for n in ("depth4", "depth5", "depth6")} == {4, 5, 6}
    assert by["prec16"].precision == 16 and by["prec8"].precision == 8
