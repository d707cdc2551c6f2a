"""GPU parity at full size: sift-like-1M-d128 (below) and normed-10M-d256 (further down).

sift-like-1M-d128: n = 1,000,000, d = 128, L = 4, K = 16, 256 regions, 10,000 queries, k = 50,
c = 1.5. It runs in the launch configuration the benchmark times: one batch of all 10,000
queries, beta = 0.001, with r_min and the resolved rounds set by the autotuner on the first
256 queries.

  projection     4,096 sampled rows within the FP32 dot-product error bound;
  breakpoints    all 64 columns within that bound (the oracle sorts the 100,000 sampled
                 values of each column);
  codes          all 64M coordinates bit-exact outside the 1e-5 band (banded ones counted);
  trees          the oracle's trees built on the GPU's codes equal the GPU's trees exactly;
  queries        200 sampled queries of the batch, plus its first and last, against the
                 oracle run one by one on the GPU's breakpoints and codes: same candidate
                 set, stop rule, rounds, leaves and ids, distances within 1e-6 relative,
                 except where a leaf bound lies within 1e-5 of a radius threshold (counted);
  low precision  BF16 and FP8 verification with an FP32 rescore of the top 4k on the same
                 sampled queries: recall@k against the oracle's ids, and each returned
                 distance equal to the exact distance of the returned id.
"""
import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl
from test_gpu_parity import (Case, check_breakpoints, check_codes, check_trees,
                             compare_queries, proj_bound)

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BETA = 0.001
N_SAMPLED = 200


@pytest.fixture(scope="module")
def full():
    w = wl.SIFT_LIKE_1M
    cs = Case(w.data(), w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf,
              lowp=("bf16", "fp8"))
    Q = w.queries()
    Qd = torch.from_numpy(Q).cuda()
    t = cs.idx.autotune(Qd[:256].contiguous(), k=w.k, c=w.c, beta=BETA)
    print(f"[full] autotune {t}", flush=True)
    rng = np.random.default_rng(2603)
    sel = sorted(set(rng.choice(len(Q), N_SAMPLED, replace=False).tolist()) | {0, len(Q) - 1})
    return w, cs, Q, Qd, t, sel


def test_full_projection_sampled_rows(full):
    w, cs, Q, Qd, t, sel = full
    rows = np.sort(np.random.default_rng(7).choice(len(cs.X), 4096, replace=False))
    P = cs.idx.project(cs.Xd[torch.from_numpy(rows).cuda()].contiguous()).cpu().numpy()
    err = np.abs(P.astype(np.float64) - cs.H[rows])
    bound = proj_bound(cs.X[rows], cs.A)
    assert np.all(err <= bound), float((err / bound).max())


def test_full_breakpoints_codes_trees(full):
    w, cs, Q, Qd, t, sel = full
    check_breakpoints(cs)
    check_codes(cs)
    check_trees(cs)


def test_full_batch_sampled_queries_fp32(full):
    w, cs, Q, Qd, t, sel = full
    print(f"[full fp32] nq={len(Q)} beta={BETA} r_min={t['r_min']:.6g} "
          f"rounds_resolved={t['rounds_resolved']}", flush=True)
    ids, dists, st = cs.idx.query(Qd, k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], eps=cs.eps,
                                  stats=True)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    compare_queries(cs, cs.stepwise_oracle(), Q, sel, ids, dists, st, w.k, w.c, BETA,
                    t["r_min"], "full fp32", allow_frac=0.02)
    # every query of the batch: ids distinct, distances ascending and exact for its ids
    assert np.all(np.diff(dists, axis=1) >= 0)
    assert all(len(set(r)) == w.k for r in ids[::97])
    exact = np.sqrt(((cs.X[ids[::97]].astype(np.float64)
                      - Q[::97, None, :].astype(np.float64)) ** 2).sum(-1))
    np.testing.assert_allclose(dists[::97], exact, rtol=1e-6)


def test_full_batch_order_does_not_change_results(full):
    """Every query of the batch gives the same candidate set, stop rule, rounds, leaves and
    ids when the batch runs in reverse order, so that each query shares its bound tiles and
    waves with other queries (a query's search must not depend on its neighbours)."""
    w, cs, Q, Qd, t, sel = full
    kw = dict(k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], eps=cs.eps, stats=True)
    ids, _, st = cs.idx.query(Qd, **kw)
    rids, _, rst = cs.idx.query(torch.flip(Qd, [0]).contiguous(), **kw)
    ids, st = ids.cpu().numpy(), st.cpu().numpy()
    rids, rst = rids.cpu().numpy()[::-1], rst.cpu().numpy()[::-1]
    words = [pdet.QSTAT[f] for f in ("rounds", "ncand", "stop", "leaves", "hsum", "hmix")]
    bad = np.nonzero((st[:, words] != rst[:, words]).any(axis=1) | (ids != rids).any(axis=1))[0]
    assert len(bad) == 0, (len(bad), bad[:10].tolist())


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_full_batch_low_precision_recall(full, prec):
    w, cs, Q, Qd, t, sel = full
    ids, dists = cs.idx.query(Qd, k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], eps=cs.eps,
                              precision=prec,
                              rescore=4)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    idx_or = cs.stepwise_oracle()
    hit = 0
    for qi in sel:
        res = oracle.query(idx_or, cs.X, Q[qi], w.k, w.c, BETA, t["r_min"], cs.eps)
        hit += len(set(ids[qi].tolist()) & set(res.ids.tolist()))
        exact = np.sqrt(((cs.X[ids[qi]].astype(np.float64)
                          - Q[qi].astype(np.float64)) ** 2).sum(-1))
        np.testing.assert_allclose(dists[qi], exact, rtol=1e-6)
    recall = hit / (w.k * len(sel))
    print(f"[full {prec}] recall@{w.k} vs oracle on {len(sel)} sampled queries: {recall:.4f}",
          flush=True)
    assert recall >= 0.95


# ---------------------------------------------------------------------------------------
# normed-10M-d256 (serving form): n = 10,000,000, d = 256, unit-norm rows of a 4,096-centre
# mixture; L = 4, K = 16, 256 regions; k = 10, c = 1.5. The oracle cannot build this index in
# test time, so it checks what it can compute one by one (sampled projections and codes,
# every interior breakpoint from the sample's order statistics, brute-force kNN of sampled
# queries) and properties that hold at any size (each tree's perm is a permutation whose
# leaf counts sum to n; returned distances are the exact distances of the returned ids).
SERVE_BETA = 0.001


@pytest.fixture(scope="module")
def serving10m():
    w = wl.NORMED_10M_D256
    X = w.data()
    A, sid = w.proj(), w.sample()
    print(f"\n[10M] n={len(X)} d={X.shape[1]} n_sample={len(sid)}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf, lowp=("fp8",))
    torch.cuda.synchronize()
    Q = w.queries(2048)
    Qd = torch.from_numpy(Q).cuda()
    t = idx.autotune(Qd[:256].contiguous(), k=w.k, c=w.c, beta=SERVE_BETA)
    print(f"[10M] autotune {t}", flush=True)
    return w, X, A, sid, Xd, idx, Q, Qd, t


def test_10m_sampled_projection_codes_and_breakpoints(serving10m):
    w, X, A, sid, Xd, idx, Q, Qd, t = serving10m
    rng = np.random.default_rng(11)
    rows = np.sort(rng.choice(len(X), 100_000, replace=False))
    H = oracle.project(X[rows], A)
    P = idx.project(Xd[torch.from_numpy(rows).cuda()].contiguous()).cpu().numpy()
    bound = proj_bound(X[rows], A)
    assert np.all(np.abs(P.astype(np.float64) - H) <= bound)
    # interior breakpoints: exact order statistics of the FP64 sample projections, within
    # the FP32 projection bound of the sampled rows
    Hs = oracle.project(X[sid], A)
    B_or = oracle.breakpoints(Hs, w.Nr, Hs.min(axis=0), Hs.max(axis=0))
    B_gpu = idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
    E_s = proj_bound(X[sid], A).max(axis=0)
    assert np.all(np.abs(B_gpu[:, 1:-1] - B_or[:, 1:-1]) <= E_s[:, None] + 1e-30)
    # codes of the sampled rows: the oracle's encoding on the GPU's breakpoints, exact
    # except within 1e-5 of the column range of a breakpoint
    codes = idx.export(pdet.X_CODES)[:, rows, :w.K]
    ref = oracle.encode(H, B_gpu, w.L, w.K)
    mism = codes != ref
    banded = np.zeros_like(mism)
    for i in range(w.L):
        for j in range(w.K):
            col = i * w.K + j
            inner = B_gpu[col, 1:-1]
            h = H[:, col]
            pos = np.searchsorted(inner, h)
            near = np.minimum(np.abs(h - inner[np.clip(pos - 1, 0, len(inner) - 1)]),
                              np.abs(h - inner[np.clip(pos, 0, len(inner) - 1)]))
            banded[i, :, j] = near <= 1e-5 * (B_gpu[col, -1] - B_gpu[col, 0])
    print(f"[10M codes] sampled coords={mism.size} mismatched={int(mism.sum())} "
          f"banded={int(banded.sum())}", flush=True)
    assert not (mism & ~banded).any()


def test_10m_trees_are_partitions(serving10m):
    w, X, A, sid, Xd, idx, Q, Qd, t = serving10m
    n = len(X)
    for i in range(w.L):
        perm = idx.export(pdet.X_PERM, i)
        cnt = idx.export(pdet.X_LEAF_COUNT, i)
        start = idx.export(pdet.X_LEAF_START, i)
        assert np.array_equal(np.sort(perm), np.arange(n, dtype=np.int32))
        assert int(cnt.astype(np.int64).sum()) == n and np.all(cnt > 0)
        assert np.array_equal(start[1:], np.cumsum(cnt)[:-1]) and start[0] == 0


def _exact_knn(X, Q, k, chunk=1 << 20):
    """Brute-force kNN in FP64: the norm form over chunks picks 4k candidates, the
    difference form ranks them."""
    q64 = Q.astype(np.float64)
    best = [np.empty(0, np.int64) for _ in Q]
    for s in range(0, len(X), chunk):
        C = X[s:s + chunk].astype(np.float64)
        d2 = (C * C).sum(1)[None, :] - 2.0 * (q64 @ C.T) + (q64 * q64).sum(1)[:, None]
        part = np.argpartition(d2, 4 * k, axis=1)[:, :4 * k] + s
        best = [np.concatenate([b, p]) for b, p in zip(best, part)]
    ids = []
    for qi, b in enumerate(best):
        dd = np.sqrt(((X[b].astype(np.float64) - q64[qi]) ** 2).sum(1))
        o = np.lexsort((b, dd))[:k]
        ids.append(b[o])
    return np.array(ids)


@pytest.mark.parametrize("prec", ["fp32", "fp8"])
def test_10m_batch_recall_and_exact_distances(serving10m, prec):
    # A larger beta only moves stop rule A later, so its candidate set contains the smaller
    # beta's: every true neighbour found at beta = 0.001 is still returned at beta = 0.01.
    w, X, A, sid, Xd, idx, Q, Qd, t = serving10m
    sel = np.arange(0, len(Q), 256)
    exact = _exact_knn(X, Q[sel], w.k)
    found = {}
    for beta in (SERVE_BETA, 10 * SERVE_BETA):
        ids, dists = idx.query(Qd, k=w.k, c=w.c, beta=beta, r_min=t["r_min"], precision=prec,
                               rescore=4)
        ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
        assert np.all(np.diff(dists, axis=1) >= 0)
        got = np.sqrt(((X[ids[sel]].astype(np.float64)
                        - Q[sel, None, :].astype(np.float64)) ** 2).sum(-1))
        np.testing.assert_allclose(dists[sel], got, rtol=1e-6)
        found[beta] = [set(ids[q].tolist()) & set(e.tolist()) for q, e in zip(sel, exact)]
        rec = np.mean([len(f) / w.k for f in found[beta]])
        print(f"[10M {prec}] beta={beta} recall@{w.k} vs brute force on {len(sel)} queries: "
              f"{rec:.3f}", flush=True)
    if prec == "fp32":
        for small, large in zip(found[SERVE_BETA], found[10 * SERVE_BETA]):
            assert small <= large
