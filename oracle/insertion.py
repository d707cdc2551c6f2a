"""CPU oracle for online insertion into a resident DE-Tree. TEST INFRASTRUCTURE ONLY.

Plain Python restatement of the insertion loop of Algorithm 2 (Create Index): every point
is placed in the leaf of the tree whose region holds its encoded representation, and a
leaf that is full is split, repeatedly, until the point finds room. The library never
calls this module and shares no code with it.

Readings (the paper gives the loop, not these details):

* The resident tree before any insertion is the bulk tree of ``detlsh.build_tree`` with
  the empty children of its splits kept as (empty) leaves, and with all 2^K first-layer
  nodes present from the start (Algorithm 2 creates them before the first point), empty
  ones as empty leaves. Empty leaves hold no points, so they never appear in the
  flattened tree that queries use, but a later point may land in one.
* Points are inserted one at a time in ascending id order. The target is split while it
  holds max_size points or more (the loop condition of Algorithm 2) and some dimension is
  still unrefined; the split dimension follows the node-split rule of the indexing phase
  (the most even division of the points the node holds, ties to the smallest dimension)
  over the points already in the node, not counting the point being inserted. A fully
  refined target takes the point whatever its size.
* Inside a leaf, ids stay ascending; leaves are numbered depth first (first-layer nodes
  by ascending key, the bit-0 child before the bit-1 child), as in the bulk tree.
"""
from __future__ import annotations

import math

import numpy as np

from .detlsh import Tree, choose_split, first_layer_key


class Node:
    """A node of one DE-Tree: a leaf (split < 0, ids = its points) or an internal node
    split on dimension ``split`` into kids (bit-0 child, bit-1 child)."""
    __slots__ = ("depth", "prefix", "split", "kids", "ids")

    def __init__(self, depth, prefix, ids=None):
        self.depth = np.asarray(depth, dtype=np.int64)
        self.prefix = np.asarray(prefix, dtype=np.int64)
        self.split = -1
        self.kids = ()
        self.ids = [] if ids is None else list(ids)


class DETree:
    """One DE-Tree as a trie: root's 2^K first-layer children, created on first use."""

    def __init__(self, K: int, Nr: int, max_size: int):
        self.K, self.Nr, self.max_size = K, Nr, max_size
        self.bits = int(round(math.log2(Nr)))
        self.roots: dict[int, Node] = {}

    def first_layer(self, key: int) -> Node:
        if key not in self.roots:
            prefix = [(key >> (self.K - 1 - j)) & 1 for j in range(self.K)]
            self.roots[key] = Node(np.ones(self.K, dtype=np.int64), prefix)
        return self.roots[key]

    def _bit(self, code_row, node: Node, j: int) -> int:
        """The next unrefined bit of dimension j of a code row below this node."""
        return (int(code_row[j]) >> (self.bits - 1 - int(node.depth[j]))) & 1

    def split(self, node: Node, codes_i: np.ndarray) -> bool:
        """SplitNode: divide a leaf in two on the dimension the split rule picks over the
        points it holds; False when every dimension is fully refined."""
        ids = np.asarray(node.ids, dtype=np.int64)
        j = choose_split(codes_i[ids].reshape(len(ids), self.K), node.depth, self.bits)
        if j < 0:
            return False
        kids = []
        for b in (0, 1):
            dep = node.depth.copy()
            dep[j] += 1
            pre = node.prefix.copy()
            pre[j] = 2 * pre[j] + b
            kids.append(Node(dep, pre, [z for z in node.ids if self._bit(codes_i[z], node, j) == b]))
        node.split, node.kids, node.ids = j, tuple(kids), []
        return True

    def leaf_of(self, code_row) -> Node:
        """The leaf whose region holds a code row."""
        key = 0
        for j in range(self.K):
            key |= ((int(code_row[j]) >> (self.bits - 1)) & 1) << (self.K - 1 - j)
        node = self.first_layer(key)
        while node.split >= 0:
            node = node.kids[self._bit(code_row, node, node.split)]
        return node

    def insert(self, z: int, codes_i: np.ndarray) -> None:
        """Algorithm 2's loop body for one point: find the target leaf, split it while it
        is full, then add the point."""
        target = self.leaf_of(codes_i[z])
        while len(target.ids) >= self.max_size:
            if not self.split(target, codes_i):
                break
            target = target.kids[self._bit(codes_i[z], target, target.split)]
        target.ids.append(int(z))

    def leaves(self, keep_empty: bool = False):
        """Leaves in depth-first order (first-layer keys ascending, bit-0 child first)."""
        out = []
        for key in sorted(self.roots):
            stack = [self.roots[key]]
            while stack:
                node = stack.pop()
                if node.split >= 0:
                    stack.append(node.kids[1])
                    stack.append(node.kids[0])
                elif node.ids or keep_empty:
                    out.append(node)
        return out

    def flatten(self) -> Tree:
        """The tree as the queries see it: non-empty leaves, depth first, ids ascending."""
        lv = self.leaves()
        counts = np.array([len(x.ids) for x in lv], dtype=np.int64)
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
        perm = (np.concatenate([np.asarray(x.ids, dtype=np.int64) for x in lv])
                if lv else np.zeros(0, dtype=np.int64))
        depth = np.array([x.depth for x in lv], dtype=np.int64).reshape(-1, self.K)
        prefix = np.array([x.prefix for x in lv], dtype=np.int64).reshape(-1, self.K)
        return Tree(perm, starts, counts, depth, prefix)


def bulk_tree(codes_i: np.ndarray, Nr: int, max_leaf: int) -> DETree:
    """The bulk tree of ``detlsh.build_tree`` as a trie whose empty children are kept:
    a node with more than max_leaf points and an unrefined dimension is split by the
    node-split rule over all its points."""
    n, K = codes_i.shape
    t = DETree(K, Nr, max_leaf)
    key = first_layer_key(codes_i, t.bits)
    for k in np.unique(key):
        root = t.first_layer(int(k))
        root.ids = [int(z) for z in np.nonzero(key == k)[0]]   # ascending ids
        stack = [root]
        while stack:
            node = stack.pop()
            if len(node.ids) > max_leaf and t.split(node, codes_i):
                stack.extend(node.kids)
    return t


def insert_points(tree: DETree, codes_i: np.ndarray, ids) -> DETree:
    """Insert the given points, in ascending id order, into a resident tree (in place)."""
    for z in sorted(int(v) for v in ids):
        tree.insert(z, codes_i)
    return tree
