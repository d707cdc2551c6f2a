"""GPU checks at full size on sift-like-100M-d128 (the batching form's workload).

n = 100,000,000 points, d = 128, integer-valued coordinates of a 1,000-centre mixture (51 GB
resident); L = 4, K = 16, 256 regions, a 10% sample (10M rows); 10,000 queries, beta = 0.001,
with r_min and the resolved rounds set by the autotuner on the first 256 queries, as in the
benchmark. The oracle cannot build this index in test time, so it checks what it computes
one by one, and properties that hold at any size:

  projection     50,000 sampled rows within the FP32 dot-product error bound;
  breakpoints    8 of the 64 columns: every interior breakpoint against the exact order
                 statistics of the 10M FP64 sample projections, within that bound;
  codes          the sampled rows' codes equal the oracle's encoding on the GPU's
                 breakpoints, except within 1e-5 of the column range of a breakpoint;
  trees          each tree's perm is a permutation of the n ids and its leaf counts tile it;
  leaf ordinals  every point's leaf in every tree (scattered over three id windows at this
                 size, read back through tree 0's leaf rows) is the leaf holding it in that
                 tree's permutation;
  queries        the FP32 batch runs on capped leaf lists (2,048 slots); 64 of its queries
                 run again on full-capacity slots and give identical ids, distances and
                 statistics; returned distances equal the FP64 distances of the returned ids;
  batching       the HIP-graph plan of the batch with k in {1, 10, 100}, c in {1.2, 1.5, 2.0}
                 and BF16 verification with an FP32 rescore of the top 4k equals the eager
                 call, and its distances are the exact ones of its ids.
"""
import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl
from test_gpu_parity import proj_bound

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BETA = 0.001


@pytest.fixture(scope="module")
def xl():
    torch.cuda.empty_cache()
    pdet.release_cache()
    w = wl.SIFT_LIKE_100M
    print(f"\n[100M] generating n={w.n} d={w.d}", flush=True)
    X = w.data(threads=16)
    A, sid = w.proj(), w.sample()
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf, lowp=("bf16",))
    torch.cuda.synchronize()
    Q = w.queries()
    Qd = torch.from_numpy(Q).cuda()
    t = idx.autotune(Qd[:256].contiguous(), k=w.k, c=w.c, beta=BETA)
    print(f"[100M] built; autotune {t}", flush=True)
    yield w, X, A, sid, Xd, idx, Q, Qd, t
    idx.close()
    del Xd
    torch.cuda.empty_cache()
    pdet.release_cache()


def test_100m_leaf_ordinals_match_every_tree(xl):
    w, X, A, sid, Xd, idx, Q, Qd, t = xl
    for j in range(w.L):
        perm = idx.export(pdet.X_PERM, j)
        cnt = idx.export(pdet.X_LEAF_COUNT, j)
        want = np.empty(w.n, dtype=np.int32)
        want[perm] = np.repeat(np.arange(len(cnt), dtype=np.int32), cnt)
        got = idx.export(pdet.X_LEAF_OF, j)
        bad = np.flatnonzero(got != want)
        assert bad.size == 0, f"tree {j}: {bad.size} ids, first {bad[:5]} (windows of 2^25 ids)"


def test_100m_sampled_projection_codes_and_breakpoints(xl):
    w, X, A, sid, Xd, idx, Q, Qd, t = xl
    rng = np.random.default_rng(13)
    rows = np.sort(rng.choice(len(X), 50_000, replace=False))
    H = oracle.project(X[rows], A)
    P = idx.project(Xd[torch.from_numpy(rows).cuda()].contiguous()).cpu().numpy()
    assert np.all(np.abs(P.astype(np.float64) - H) <= proj_bound(X[rows], A))
    B_gpu = idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
    # interior breakpoints of 8 columns (every tree, two dimensions each) from the exact
    # order statistics of the 10M-row sample
    cols = np.array([i * w.K + j for i in range(w.L) for j in (0, w.K - 1)])
    Xs = X[sid]
    Hs = oracle.project(Xs, A[:, cols])
    B_or = oracle.breakpoints(Hs, w.Nr, Hs.min(axis=0), Hs.max(axis=0))
    E_s = proj_bound(Xs, A[:, cols]).max(axis=0)
    assert np.all(np.abs(B_gpu[cols, 1:-1] - B_or[:, 1:-1]) <= E_s[:, None] + 1e-30)
    del Xs, Hs
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
    print(f"[100M codes] sampled coords={mism.size} mismatched={int(mism.sum())} "
          f"banded={int(banded.sum())}", flush=True)
    assert not (mism & ~banded).any()


def test_100m_trees_are_partitions(xl):
    w, X, A, sid, Xd, idx, Q, Qd, t = xl
    n = len(X)
    for i in range(w.L):
        perm = idx.export(pdet.X_PERM, i)
        assert np.array_equal(np.bincount(perm, minlength=n), np.ones(n, np.int64)), i
        del perm
        cnt = idx.export(pdet.X_LEAF_COUNT, i)
        start = idx.export(pdet.X_LEAF_START, i)
        assert int(cnt.astype(np.int64).sum()) == n and np.all(cnt > 0)
        assert np.array_equal(start[1:], np.cumsum(cnt)[:-1]) and start[0] == 0


def _exact_dists(X, Q, ids):
    return np.sqrt(((X[ids].astype(np.float64) - Q[:, None, :].astype(np.float64)) ** 2).sum(-1))


def test_100m_capped_batch_equals_full_capacity(xl):
    w, X, A, sid, Xd, idx, Q, Qd, t = xl
    pdet.set_timing(True)
    try:
        ids, dists, st = idx.query(Qd, k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], stats=True)
        tm = pdet.get_timing()
        print(f"[100M batch] launches={tm['query_main_launches']} "
              f"answered again={tm['query_retried']}", flush=True)
        # capped lists: 2,048 slots per launch, then 16 full-capacity slots per retry launch
        again = tm["query_retried"]
        assert tm["query_main_launches"] == (len(Q) + 2047) // 2048 + (again + 15) // 16
        sel = np.arange(0, len(Q), len(Q) // 64)[:64]
        idx.set_list_cap(1 << 30)   # every leaf fits: full-capacity slots
        f_ids, f_d, f_st = idx.query(Qd[torch.from_numpy(sel).cuda()].contiguous(), k=w.k,
                                     c=w.c, beta=BETA, r_min=t["r_min"], stats=True)
    finally:
        idx.set_list_cap(0)
        pdet.set_timing(False)
    keep = [0, 1, 2, 3, 4, 5, 7, 8, 9]    # word 6 is the query's device time
    s = torch.from_numpy(sel).cuda()
    assert torch.equal(ids[s], f_ids) and torch.equal(dists[s], f_d)
    assert torch.equal(st[s][:, keep], f_st[:, keep])
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    assert np.all(np.diff(dists, axis=1) >= 0)
    np.testing.assert_allclose(dists[sel], _exact_dists(X, Q[sel], ids[sel]), rtol=1e-6)


def test_100m_uneven_bf16_plan_equals_eager(xl):
    w, X, A, sid, Xd, idx, Q, Qd, t = xl
    rng = np.random.default_rng(7)
    ks = rng.choice([1, 10, 100], size=len(Q)).astype(np.int32)
    cs = rng.choice([1.2, 1.5, 2.0], size=len(Q))
    kw = dict(k=0, beta=BETA, r_min=t["r_min"], k_per_query=ks, c_per_query=cs,
              precision="bf16", rescore=4)
    plan = idx.plan(Qd, **kw)
    e_ids, e_d = idx.query(Qd, **kw)
    plan.launch()
    torch.cuda.synchronize()
    assert torch.equal(plan.ids, e_ids) and torch.equal(plan.dists, e_d)
    plan.close()
    # flat rows in query order: each query's distances are the exact ones of its ids
    off = np.concatenate([[0], np.cumsum(ks)])
    e_ids, e_d = e_ids.cpu().numpy(), e_d.cpu().numpy()
    for q in range(0, len(Q), 97):
        got = e_ids[off[q]:off[q + 1]]
        ok = got >= 0
        d64 = np.sqrt(((X[got[ok]].astype(np.float64) - Q[q].astype(np.float64)) ** 2).sum(-1))
        np.testing.assert_allclose(e_d[off[q]:off[q + 1]][ok], d64, rtol=1e-6)
