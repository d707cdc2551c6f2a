"""CPU checks of the comparison used by the GPU parity tests (tests/parity.py): it accepts
the oracle's own results, and rejects results with a planted mistake (a wrong candidate,
a wrong stop rule, a wrong neighbour, a wrong distance) unless a near tie explains it."""
import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import workloads as wl
from parity import compare_batch, set_hashes


@pytest.fixture(scope="module")
def case():
    w = wl.SMALL_MIXTURE.scaled(n=3000)
    X, A = w.data(), w.proj()
    idx = oracle.build_index(X, A, w.sample(), w.L, w.K, w.Nr, 32)
    Q = w.queries(8)
    eps = oracle.epsilon(w.K, w.L)
    return X, idx, Q, eps


def _as_gpu(X, idx, Q, eps, k, c, beta, r_min):
    """Outputs shaped like the library's, taken from the oracle itself."""
    ids = np.zeros((len(Q), k), dtype=np.int64)
    dists = np.zeros((len(Q), k), dtype=np.float32)
    st = np.zeros((len(Q), 10), dtype=np.int64)
    cands = []
    for qi, q in enumerate(Q):
        r = oracle.query(idx, X, q, k, c, beta, r_min, eps)
        ids[qi], dists[qi] = r.ids, r.dists
        hs, hm = set_hashes(r.cand)
        st[qi, :6] = (r.rounds, r.n_cand, {"A": 1, "B": 2}[r.stop], r.leaves, hs, hm)
        cands.append(np.sort(r.cand))
    return ids, dists, st, cands


def test_oracle_results_pass(case):
    X, idx, Q, eps = case
    ids, dists, st, cands = _as_gpu(X, idx, Q, eps, 10, 1.5, 0.05, 2.0)
    same, band, _ = compare_batch(X, idx, Q, range(len(Q)), ids, dists, st, 10, 1.5, 0.05, 2.0,
                                  eps, "clean", cands=cands)
    assert same == len(Q) and band == 0


@pytest.mark.parametrize("plant", ["candidate", "stop", "neighbour", "distance", "hash"])
def test_planted_mistakes_are_rejected(case, plant):
    X, idx, Q, eps = case
    ids, dists, st, cands = _as_gpu(X, idx, Q, eps, 10, 1.5, 0.05, 2.0)
    use_cands = cands
    if plant == "candidate":
        missing = np.setdiff1d(np.arange(len(X)), cands[3])[0]
        cands[3] = np.sort(np.concatenate([cands[3][1:], [missing]]))
    elif plant == "stop":
        st[3, 2] = 3 - st[3, 2]
    elif plant == "neighbour":
        ids[3, 4] = ids[3, 4] + 1
    elif plant == "distance":
        dists[3, 0] *= 1.001
    else:   # without the exported set, a wrong id is caught by the two hashes
        st[3, 4] += 1
        use_cands = None
    with pytest.raises(AssertionError):
        compare_batch(X, idx, Q, range(len(Q)), ids, dists, st, 10, 1.5, 0.05, 2.0, eps,
                      plant, cands=use_cands)
