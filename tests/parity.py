"""Comparison of libpdet query results with the FP64 oracle (test infrastructure).

Used by the GPU parity tests and by ``__graft_entry__.smoke()``. A query of the GPU
batch is compared with the oracle's query on the same inputs:

* candidate set S: element by element when the GPU exported it (pdet_query_candidates),
  else by size and two 32-bit sums of the ids;
* control flow: stop rule, rounds, admitted leaves;
* results: identical ids (except at an exact distance tie at the k boundary), FP32
  distances within 1e-6 relative of the oracle's FP64 distances.

A query that differs must be explained by an FP32-vs-FP64 near tie (the band of the
design's readings): a leaf lower bound within 1e-5 relative of a radius threshold
(eps r)^2 that the query used, or the k-th distance within 1e-5 relative of c*r. Every
difference is classified; an unexplained one fails.
"""
from __future__ import annotations

import numpy as np

import oracle

U32 = 2.0 ** -24
BAND = 1e-5
STOP_CODE = {"A": 1, "B": 2}
QS_ROUNDS, QS_NCAND, QS_STOP, QS_LEAVES, QS_HSUM, QS_HMIX = 0, 1, 2, 3, 4, 5


def mix32(h):
    h = np.asarray(h).astype(np.uint64) & 0xFFFFFFFF
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & 0xFFFFFFFF
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & 0xFFFFFFFF
    h ^= h >> 16
    return h


def set_hashes(ids):
    """(sum of ids, sum of mix32(id)) mod 2^32 as signed int32, as qstats words 4 and 5."""
    ids = np.asarray(ids, dtype=np.uint64)
    hs = int(ids.sum() & 0xFFFFFFFF)
    hm = int(mix32(ids).sum() & 0xFFFFFFFF)
    to32 = lambda v: v - (1 << 32) if v >= (1 << 31) else v
    return to32(hs), to32(hm)


def proj_bound(X, A):
    """Error bound of an FP32 dot product of length d, per (point, column)."""
    d = X.shape[1]
    return 1.01 * (d + 1) * U32 * (np.abs(X.astype(np.float64)) @ np.abs(A.astype(np.float64)))


def near_threshold(idx_or, q, rounds, r_min, c, eps):
    """True if some leaf bound of q lies within BAND of a radius threshold it used."""
    qp = np.asarray(q, dtype=np.float64) @ idx_or.A
    t2 = np.array([(eps * r) ** 2 for r in oracle.radius_ladder(r_min, c, rounds + 1)])
    for i in range(idx_or.L):
        lo, hi = idx_or.boxes[i]
        lb2 = oracle.lower_bound_sq(qp[i * idx_or.K:(i + 1) * idx_or.K], lo, hi)
        if np.any(np.abs(lb2[:, None] - t2[None, :]) <= BAND * t2[None, :]):
            return True
    return False


def near_stop_b(X, q, cand, k, rounds, r_min, c):
    """True if the k-th distance in S lies within BAND of c*r for a round it ran."""
    if len(cand) < k:
        return False
    dd = np.sort(np.sqrt(((X[cand].astype(np.float64) - np.asarray(q, dtype=np.float64)) ** 2)
                         .sum(axis=1)))
    kth = dd[k - 1]
    return any(abs(kth - c * r) <= BAND * c * r for r in oracle.radius_ladder(r_min, c, rounds + 1))


def compare_batch(X, idx_or, Q, sel, ids, dists, st, k, c, beta, r_min, eps, label,
                  cands=None, k_of=None, off_of=None, log=print):
    """Compare GPU results of queries `sel` of batch Q with the oracle run one by one.

    ids / dists are [nq][k] (uniform k) or flat CSR with k_of(q) / off_of(q); st is the
    qstats array; cands[q], if given, is the sorted GPU candidate set of query q (all of it
    when its |S| fits the export). Returns (identical, banded, results by query)."""
    n_same = n_band = 0
    results = {}
    for qi in sel:
        q = Q[qi]
        kq = k if k_of is None else k_of(qi)
        cq = c if np.isscalar(c) else c[qi]
        res = oracle.query(idx_or, X, q, kq, cq, beta, r_min, eps)
        results[qi] = res
        if cands is not None and len(cands[qi]) == st[qi, QS_NCAND]:
            same_set = np.array_equal(cands[qi], np.sort(res.cand))
        else:
            hs, hm = set_hashes(res.cand)
            same_set = (st[qi, QS_NCAND] == res.n_cand and st[qi, QS_HSUM] == hs
                        and st[qi, QS_HMIX] == hm)
        same_flow = (st[qi, QS_STOP] == STOP_CODE[res.stop] and st[qi, QS_ROUNDS] == res.rounds
                     and st[qi, QS_LEAVES] == res.leaves)
        if off_of is None:
            gi, gd = ids[qi], dists[qi]
        else:
            gi, gd = ids[off_of(qi):off_of(qi) + kq], dists[off_of(qi):off_of(qi) + kq]
        if same_set and same_flow:
            if not np.array_equal(gi, res.ids):
                # allowed only at an exact distance tie at the k boundary
                dk = res.dists[kq - 1]
                dall = np.sqrt(((X[res.cand].astype(np.float64) - q) ** 2).sum(1))
                tie = np.sum(np.abs(dall - dk) <= 1e-12 * max(dk, 1e-300)) > 1
                assert tie, (label, qi, gi, res.ids)
            np.testing.assert_allclose(gd, res.dists, rtol=1e-6)
            n_same += 1
            continue
        rounds = max(res.rounds, int(st[qi, QS_ROUNDS]))
        banded = (near_threshold(idx_or, q, rounds, r_min, cq, eps)
                  or near_stop_b(X, q, res.cand, kq, rounds, r_min, cq))
        assert banded, (label, qi, st[qi], res.n_cand, res.stop, res.rounds, res.leaves)
        n_band += 1
    log(f"[query {label}] identical={n_same}/{len(sel)} banded={n_band}")
    return n_same, n_band, results
