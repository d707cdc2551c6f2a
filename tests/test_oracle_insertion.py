"""Pins of the oracle's online insertion (Algorithm 2's insertion loop, oracle/insertion.py):
a sequence worked by hand, invariants that any correct tree satisfies, the special case in
in which no node is ever split (then the result is the bulk tree of all points), and
planted mistakes that the hand-worked sequence must catch."""
import json
import os
import sys
import types

import numpy as np
import pytest

import oracle
from oracle import insertion as ins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "insertion.py")


def _golden():
    with open(os.path.join(ROOT, "tests", "golden", "insert_sequence.json")) as f:
        return json.load(f)


def _as_dicts(leaves, with_ids=True):
    out = []
    for x in leaves:
        d = dict(depth=[int(v) for v in x.depth], prefix=[int(v) for v in x.prefix])
        if with_ids:
            d["ids"] = [int(v) for v in x.ids]
        out.append(d)
    return out


def _golden_holds(mod):
    g = _golden()
    codes = np.array(g["codes"], dtype=np.uint8)
    t = mod.bulk_tree(codes[g["resident"]], g["Nr"], g["max_size"])
    for call, exp in zip(g["calls"], g["after"]):
        mod.insert_points(t, codes, call)
        if _as_dicts(t.leaves()) != exp["leaves"]:
            return False
        empty = [x for x in t.leaves(keep_empty=True) if not x.ids and not (x.depth == 1).all()]
        if _as_dicts(empty, with_ids=False) != exp["empty"]:
            return False
    return True


def test_hand_worked_sequence():
    assert _golden_holds(ins)


def test_hand_worked_bulk_tree_differs():
    g = _golden()
    codes = np.array(g["codes"], dtype=np.uint8)[:8]
    b = oracle.build_tree(codes, g["Nr"], g["max_size"])
    got = [dict(depth=[int(v) for v in b.leaf_depth[i]], prefix=[int(v) for v in b.leaf_prefix[i]],
                ids=[int(v) for v in b.perm[b.leaf_start[i]:b.leaf_start[i] + b.leaf_count[i]]])
           for i in range(b.nl)]
    assert got == g["bulk_of_first_eight"]
    assert got != g["after"][0]["leaves"]


def _region_holds(node, code_row, bits):
    return all((int(code_row[j]) >> (bits - int(node.depth[j]))) == int(node.prefix[j])
               for j in range(len(code_row)))


def _check_invariants(t, codes, ids_present):
    bits, K = t.bits, t.K
    flat = t.flatten()
    # every point exactly once, ids ascending inside every leaf
    assert sorted(flat.perm.tolist()) == sorted(ids_present)
    for i in range(flat.nl):
        seg = flat.perm[flat.leaf_start[i]:flat.leaf_start[i] + flat.leaf_count[i]]
        assert np.all(np.diff(seg) > 0)
    # a leaf holds more than max_size points only when it is fully refined; its region
    # holds its points' codes
    for x in t.leaves():
        if len(x.ids) > t.max_size:
            assert np.all(x.depth == bits)
        for z in x.ids:
            assert _region_holds(x, codes[z], bits)
    # the complete leaves (empty ones and unused first-layer nodes included) tile the code
    # space: region sizes add up to Nr^K
    cover = sum(2 ** int(np.sum(bits - x.depth)) for x in t.leaves(keep_empty=True))
    cover += (2 ** K - len(t.roots)) * 2 ** (K * (bits - 1))
    assert cover == t.Nr ** K
    # brute force: the leaf found by descent is the only complete leaf whose region holds
    # the code
    rng = np.random.default_rng(0)
    for _ in range(20):
        c = rng.integers(0, t.Nr, size=K)
        hits = [x for x in t.leaves(keep_empty=True) if _region_holds(x, c, bits)]
        key = sum(((int(c[j]) >> (bits - 1)) & 1) << (K - 1 - j) for j in range(K))
        if key in t.roots:
            assert len(hits) == 1 and hits[0] is t.leaf_of(c)
        else:
            assert not hits


def _clustered_codes(rng, n, K, Nr, dup_frac=0.3):
    """Codes with clusters and exact duplicates, so that splits leave empty children."""
    centres = rng.integers(0, Nr, size=(4, K))
    c = centres[rng.integers(0, 4, size=n)] + rng.integers(-2, 3, size=(n, K))
    c = np.clip(c, 0, Nr - 1)
    dup = rng.random(n) < dup_frac
    c[dup] = centres[0]
    return c.astype(np.uint8)


@pytest.mark.parametrize("K,Nr,max_leaf,n0,m", [(2, 4, 2, 20, 30), (3, 8, 3, 100, 200),
                                                (4, 16, 4, 300, 300), (5, 256, 8, 500, 700)])
def test_insertion_invariants(K, Nr, max_leaf, n0, m):
    rng = np.random.default_rng(K * 100 + max_leaf)
    codes = _clustered_codes(rng, n0 + m, K, Nr)
    t = ins.bulk_tree(codes[:n0], Nr, max_leaf)
    _check_invariants(t, codes, list(range(n0)))
    ins.insert_points(t, codes, range(n0, n0 + m // 2))
    _check_invariants(t, codes, list(range(n0 + m // 2)))
    ins.insert_points(t, codes, range(n0 + m // 2, n0 + m))
    _check_invariants(t, codes, list(range(n0 + m)))


@pytest.mark.parametrize("K,Nr,max_leaf", [(2, 4, 2), (3, 8, 5), (4, 256, 16), (8, 256, 4)])
def test_bulk_trie_flattens_to_the_bulk_tree(K, Nr, max_leaf):
    rng = np.random.default_rng(7 * K + max_leaf)
    codes = _clustered_codes(rng, 400, K, Nr)
    a = ins.bulk_tree(codes, Nr, max_leaf).flatten()
    b = oracle.build_tree(codes, Nr, max_leaf)
    for f in ("perm", "leaf_start", "leaf_count", "leaf_depth", "leaf_prefix"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))


def _internal(t):
    n = 0
    for r in t.roots.values():
        stack = [r]
        while stack:
            x = stack.pop()
            if x.split >= 0:
                n += 1
                stack.extend(x.kids)
    return n


def test_without_any_split_insertion_equals_the_bulk_tree_of_all_points():
    """When no node is ever split (no first-layer node reaches max_size points while a
    point arrives), both forms keep every point in its first-layer node, so the trees
    coincide; a single overflow makes the sequential form split where the bulk one may
    not (or on another dimension)."""
    rng = np.random.default_rng(3)
    quiet = 0
    for trial in range(80):
        K, Nr, max_leaf = 3, 8, 6
        n0, m = int(rng.integers(2, 20)), int(rng.integers(1, 20))
        codes = rng.integers(0, Nr, size=(n0 + m, K)).astype(np.uint8)
        t = ins.bulk_tree(codes[:n0], Nr, max_leaf)
        ins.insert_points(t, codes, range(n0, n0 + m))
        if _internal(t):
            continue
        quiet += 1
        a, b = t.flatten(), oracle.build_tree(codes, Nr, max_leaf)
        for f in ("perm", "leaf_start", "leaf_count", "leaf_depth", "leaf_prefix"):
            np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    assert quiet >= 10


def test_insertion_in_one_call_or_several_is_the_same():
    rng = np.random.default_rng(11)
    codes = _clustered_codes(rng, 600, 4, 16)
    one = ins.insert_points(ins.bulk_tree(codes[:200], 16, 4), codes, range(200, 600))
    many = ins.bulk_tree(codes[:200], 16, 4)
    for a in range(200, 600, 37):
        ins.insert_points(many, codes, range(a, min(a + 37, 600)))
    x, y = one.flatten(), many.flatten()
    for f in ("perm", "leaf_start", "leaf_count", "leaf_depth", "leaf_prefix"):
        np.testing.assert_array_equal(getattr(x, f), getattr(y, f))


def test_from_an_empty_index_without_splits_every_point_sits_in_its_first_layer_node():
    rng = np.random.default_rng(5)
    codes = rng.integers(0, 16, size=(50, 3)).astype(np.uint8)
    t = ins.insert_points(ins.DETree(3, 16, 1000), codes, range(50))
    flat = t.flatten()
    key = oracle.first_layer_key(codes, 4)
    assert flat.nl == len(np.unique(key))
    assert np.all(flat.leaf_depth == 1)
    for i in range(flat.nl):
        seg = flat.perm[flat.leaf_start[i]:flat.leaf_start[i] + flat.leaf_count[i]]
        assert len(set(key[seg].tolist())) == 1


# ---------------------------------------------------------------- planted mistakes
MUTATIONS = {
    # the split rule also counts the point being inserted
    "counts_new_point": ("""        target = self.leaf_of(codes_i[z])
        while len(target.ids) >= self.max_size:
            if not self.split(target, codes_i):""",
                         """        target = self.leaf_of(codes_i[z])
        while len(target.ids) >= self.max_size:
            target.ids.append(int(z))
            ok = self.split(target, codes_i)
            for kid in target.kids:
                if int(z) in kid.ids:
                    kid.ids.remove(int(z))
            if target.split < 0:
                target.ids.remove(int(z))
            if not ok:"""),
    # split only when the leaf holds more than max_size points
    "strict_size": ("        while len(target.ids) >= self.max_size:\n",
                    "        while len(target.ids) > self.max_size:\n"),
    # empty children dropped: a split that would leave one child empty refines the node in
    # place instead, so the empty region is lost
    "drops_empty": [("""            kids.append(Node(dep, pre, [z for z in node.ids if self._bit(codes_i[z], node, j) == b]))
        node.split, node.kids, node.ids = j, tuple(kids), []""",
                     """            kids.append(Node(dep, pre, [z for z in node.ids if self._bit(codes_i[z], node, j) == b]))
        if not kids[0].ids or not kids[1].ids:
            full = kids[0] if kids[0].ids else kids[1]
            node.depth, node.prefix = full.depth, full.prefix
            return True
        node.split, node.kids, node.ids = j, tuple(kids), []"""),
                    ("""            target = target.kids[self._bit(codes_i[z], target, target.split)]""",
                     """            if target.split >= 0:
                target = target.kids[self._bit(codes_i[z], target, target.split)]""")],
}


def _mutant(name):
    src = open(SRC).read()
    pairs = MUTATIONS[name]
    for old, new in (pairs if isinstance(pairs, list) else [pairs]):
        assert src.count(old) == 1, name   # the anchor must still match the oracle's source
        src = src.replace(old, new)
    mod = types.ModuleType(f"oracle.insertion_mutant_{name}")
    mod.__file__ = SRC
    mod.__package__ = "oracle"
    sys.modules[mod.__name__] = mod
    try:
        exec(compile(src, SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_the_hand_worked_sequence(name):
    try:
        holds = _golden_holds(_mutant(name))
    except Exception:   # a mutant that breaks the loop outright is caught too
        holds = False
    assert not holds, name
