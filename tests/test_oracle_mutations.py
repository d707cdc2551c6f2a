"""The oracle's query pins have teeth: each plausible mistake below, planted in a copy of the
oracle's source on the CPU, makes the hand-worked query golden (tests/golden/
query_control_flow.json, Algorithm 5 with the Section 6.2.2 admission order) fail.

  ordinal   admitted leaves taken in leaf-ordinal order instead of ascending (LB, ordinal)
  per_tree  stop rule A checked once per tree instead of after every admitted leaf
  r_not_cr  stop rule B compared with r instead of c*r
"""
import json
import os
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "detlsh.py")

MUTATIONS = {
    "ordinal": ("            adm = adm[np.lexsort((adm, lb2[adm]))]\n", ""),
    "per_tree": ("""                if n_s >= T:
                    return _finish(cand, cdist, k, rho + 1, "A", leaves, r, trace)
        if n_s >= k:""", """            if n_s >= T:
                return _finish(cand, cdist, k, rho + 1, "A", leaves, r, trace)
        if n_s >= k:"""),
    "r_not_cr": ("""            if np.partition(alld, k - 1)[k - 1] <= c * r:
                return _finish(cand, cdist, k, rho + 1, "B", leaves, r, trace)""",
                 """            if np.partition(alld, k - 1)[k - 1] <= r:
                return _finish(cand, cdist, k, rho + 1, "B", leaves, r, trace)"""),
}


def _mutant(name):
    src = open(SRC).read()
    old, new = MUTATIONS[name]
    assert src.count(old) == 1, name   # the anchor must still match the oracle's source
    mod = types.ModuleType(f"detlsh_mutant_{name}")
    mod.__file__ = SRC
    sys.modules[mod.__name__] = mod    # dataclasses look the module up by name
    try:
        exec(compile(src.replace(old, new), SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    return mod


def _golden_holds(mod):
    """True if every optimised case of the hand-worked golden holds for module `mod`."""
    with open(os.path.join(ROOT, "tests", "golden", "query_control_flow.json")) as f:
        g = json.load(f)
    X = np.array(g["points"], dtype=np.float32)
    idx = mod.build_index(X, np.eye(2, dtype=np.float32), np.arange(len(X)), g["L"], g["K"],
                          g["Nr"], g["max_leaf"], B=np.array(g["B"], dtype=np.float64))
    for cs in g["optimised"]:
        res = mod.query(idx, X, np.array(g["q"], dtype=np.float32), cs["k"], cs["c"], cs["beta"],
                        cs["r_min"], cs["eps"])
        if [list(t) for t in res.trace] != cs["trace"]:
            return False
        if not np.array_equal(res.cand, cs["cand"]):
            return False
        if (res.stop, res.rounds, res.leaves) != (cs["stop"], cs["rounds"], cs["leaves"]):
            return False
        if not np.array_equal(res.ids, cs["ids"]):
            return False
    return True


def test_unmutated_copy_passes():
    """The copy mechanism itself: the unchanged source passes the golden."""
    mod = types.ModuleType("detlsh_copy")
    mod.__file__ = SRC
    sys.modules[mod.__name__] = mod
    try:
        exec(compile(open(SRC).read(), SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules[mod.__name__]
    assert _golden_holds(mod)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_fails_the_golden(name):
    assert not _golden_holds(_mutant(name)), name
