"""GPU parity of online insertion (pdet_insert, Algorithm 2's insertion loop) against the
oracle's sequential insertion (oracle/insertion.py), step by step:
  codes   the indexed rows' codes are unchanged; the new rows' codes equal the oracle's
          encoding with the GPU's breakpoints outside the usual 1e-5 band;
  outer   the outer breakpoints are the column extremes over all rows (FP32 bound);
  trees   the oracle's resident bulk tree of the GPU's old codes, with the GPU's new codes
          inserted in row order (in the same calls), equals the GPU's trees exactly: leaf
          order, sizes, node ids, point sets per leaf;
  queries after insertion, the oracle's query on those trees gives the GPU's results.
"""
import types

import numpy as np
import pytest

import oracle
from oracle import insertion as ins
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl
from parity import proj_bound
from test_gpu_parity import run_and_compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _gpu_tree(idx, i, K):
    gs = idx.export(pdet.X_LEAF_START, i)
    gc = idx.export(pdet.X_LEAF_COUNT, i)
    gh = idx.export(pdet.X_LEAF_HIDX, i)[:, :K]
    gp = idx.export(pdet.X_PERM, i)
    return gs, gc, gh, gp


def _check_tree(idx, i, K, flat, label):
    gs, gc, gh, gp = _gpu_tree(idx, i, K)
    assert len(gs) == flat.nl, (label, i, len(gs), flat.nl)
    np.testing.assert_array_equal(gs, flat.leaf_start, err_msg=f"{label} tree {i} starts")
    np.testing.assert_array_equal(gc, flat.leaf_count, err_msg=f"{label} tree {i} counts")
    np.testing.assert_array_equal(gh, flat.hidx(), err_msg=f"{label} tree {i} node ids")
    leaf_of_pos = np.repeat(np.arange(flat.nl), flat.leaf_count)
    np.testing.assert_array_equal(gp[np.lexsort((gp, leaf_of_pos))],
                                  flat.perm[np.lexsort((flat.perm, leaf_of_pos))],
                                  err_msg=f"{label} tree {i} point sets")


class Grown:
    """An index built on the first n0 rows of X, grown by the given calls, with the oracle's
    trees (bulk tree of the GPU's old codes, then sequential insertion) kept alongside."""

    def __init__(self, X, A, n0, K, L, Nr, max_leaf, sample_ids=None, lowp=(), label=""):
        self.X, self.A, self.K, self.L, self.Nr, self.max_leaf = X, A, K, L, Nr, max_leaf
        self.label = label
        self.Xd = torch.from_numpy(X).cuda()
        sid = np.arange(n0) if sample_ids is None else sample_ids
        print(f"\n[insert {label}] build n0={n0} d={X.shape[1]} K={K} L={L} Nr={Nr} "
              f"max_leaf={max_leaf}", flush=True)
        self.idx = pdet.Index(self.Xd[:n0].contiguous(), A, sid, K, L, Nr, max_leaf, lowp=lowp)
        torch.cuda.synchronize()
        self.n = n0
        self.B0 = self.idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
        codes = np.ascontiguousarray(self.idx.export(pdet.X_CODES)[:, :, :K])
        self.trees = [ins.bulk_tree(codes[i], Nr, max_leaf) for i in range(L)]
        self.codes = codes

    def grow(self, n1):
        print(f"[insert {self.label}] rows {self.n}..{n1 - 1}", flush=True)
        self.idx.insert(self.Xd[:n1].contiguous())
        torch.cuda.synchronize()
        codes = np.ascontiguousarray(self.idx.export(pdet.X_CODES)[:, :, :self.K])
        assert codes.shape[1] == n1
        np.testing.assert_array_equal(codes[:, :self.n], self.codes, err_msg="old codes moved")
        self.codes = codes
        for i in range(self.L):
            ins.insert_points(self.trees[i], codes[i], range(self.n, n1))
        self.n = n1

    def check_codes_and_breakpoints(self):
        n = self.n
        B = self.idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
        # interior breakpoints stay as built; outer ones are the extremes over all rows
        np.testing.assert_array_equal(B[:, 1:-1], self.B0[:, 1:-1])
        H = oracle.project(self.X[:n], self.A)
        E = proj_bound(self.X[:n], self.A).max(axis=0)
        assert np.all(np.abs(B[:, 0] - H.min(axis=0)) <= E + 1e-30)
        assert np.all(np.abs(B[:, -1] - H.max(axis=0)) <= E + 1e-30)
        codes_or = oracle.encode(H, B, self.L, self.K)
        bad = 0
        for i in range(self.L):
            for j in range(self.K):
                col = i * self.K + j
                mism = self.codes[i, :, j] != codes_or[i, :, j]
                if not mism.any():
                    continue
                inner = B[col, 1:-1]
                h = H[mism, col]
                gap = np.min(np.abs(h[:, None] - inner[None, :]), axis=1)
                rng = B[col, -1] - B[col, 0]
                bad += int(np.sum(gap > 1e-5 * rng))
        assert bad == 0, bad
        return B

    def check_trees(self):
        for i in range(self.L):
            _check_tree(self.idx, i, self.K, self.trees[i].flatten(), self.label)

    def oracle_index(self, B):
        trees = [t.flatten() for t in self.trees]
        boxes = [oracle.leaf_boxes(t, B[i * self.K:(i + 1) * self.K], self.Nr)
                 for i, t in enumerate(trees)]
        return oracle.Index(self.n, self.X.shape[1], self.L, self.K, self.Nr,
                            np.asarray(self.A, dtype=np.float64), B, self.codes, trees, boxes)


def _dup_data(rng, n, d, n_dup_vectors=5, dup_frac=0.35):
    X = rng.standard_normal((n, d)).astype(np.float32)
    X += (rng.integers(0, 4, size=(n, 1)) * 3.0).astype(np.float32)
    dup = rng.random(n) < dup_frac
    base = rng.standard_normal((n_dup_vectors, d)).astype(np.float32)
    X[dup] = base[rng.integers(0, n_dup_vectors, size=int(dup.sum()))]
    return X


def test_insert_mixture_two_calls_trees_and_queries():
    w = wl.SMALL_MIXTURE
    X, A = w.data(), w.proj()
    g = Grown(X, A, 8000, w.K, w.L, w.Nr, w.max_leaf, label="mixture")
    for n1 in (9000, 10000):
        g.grow(n1)
        B = g.check_codes_and_breakpoints()
        g.check_trees()
    assert g.idx.info()["n"] == 10000
    cs = types.SimpleNamespace(X=X, idx=g.idx, eps=oracle.epsilon(w.K, w.L), max_leaf=w.max_leaf)
    run_and_compare(cs, g.oracle_index(B), w.queries(), w.k, w.c, 0.1, 4.0, "after insert")


@pytest.mark.parametrize("n0,n1,K,L,Nr,max_leaf,calls", [
    (3000, 4500, 8, 2, 16, 8, 3),     # duplicates: empty children and fully refined leaves
    (64, 2064, 6, 2, 8, 4, 2),        # almost empty resident index: mostly Algorithm 2 alone
    (2000, 2600, 16, 3, 256, 16, 4),  # full K and Nr, small leaves
])
def test_insert_duplicates_and_small_leaves(n0, n1, K, L, Nr, max_leaf, calls):
    rng = np.random.default_rng(n0 + K)
    d = 16
    X = _dup_data(rng, n1, d)
    A = rng.standard_normal((d, L * K)).astype(np.float32)
    label = f"dup n0={n0} K={K} Nr={Nr} max_leaf={max_leaf}"
    g = Grown(X, A, n0, K, L, Nr, max_leaf, label=label)
    g.check_trees()   # the resident bulk trees
    for c in range(1, calls + 1):
        g.grow(n0 + (n1 - n0) * c // calls)
        g.check_codes_and_breakpoints()
        g.check_trees()
    # stored empty leaves must exist for these inputs to mean something
    empties = sum(len([x for x in t.leaves(keep_empty=True) if not x.ids]) for t in g.trees)
    print(f"[insert {label}] oracle empty leaves {empties}", flush=True)


def test_insert_queries_on_duplicates():
    rng = np.random.default_rng(17)
    d, K, L, Nr, max_leaf = 16, 8, 2, 16, 8
    X = _dup_data(rng, 5000, d)
    A = rng.standard_normal((d, L * K)).astype(np.float32)
    g = Grown(X, A, 3000, K, L, Nr, max_leaf, label="dup queries")
    g.grow(5000)
    B = g.check_codes_and_breakpoints()
    g.check_trees()
    Q = X[rng.integers(0, 5000, size=40)] + 0.05 * rng.standard_normal((40, d)).astype(np.float32)
    cs = types.SimpleNamespace(X=X, idx=g.idx, eps=oracle.epsilon(K, L), max_leaf=max_leaf)
    run_and_compare(cs, g.oracle_index(B), np.ascontiguousarray(Q), 5, 1.5, 0.05, 0.5,
                    "dup after insert")


def test_insert_keeps_low_precision_copies_whole():
    w = wl.SMALL_MIXTURE
    X, A = w.data(), w.proj()
    g = Grown(X, A, 6000, w.K, w.L, w.Nr, w.max_leaf, lowp=("bf16", "fp8"), label="lowp")
    g.grow(10000)
    Q = torch.from_numpy(X[9000:9100]).cuda()   # inserted points are their own neighbours
    ids32, d32 = g.idx.query(Q, k=10, c=1.5, beta=0.1, r_min=4.0, eps=oracle.epsilon(w.K, w.L))
    assert np.array_equal(ids32.cpu().numpy()[:, 0], np.arange(9000, 9100))
    for prec in ("bf16", "fp8"):
        ids, dd = g.idx.query(Q, k=10, c=1.5, beta=0.1, r_min=4.0,
                              eps=oracle.epsilon(w.K, w.L), precision=prec)
        ids, dd = ids.cpu().numpy(), dd.cpu().numpy()
        assert np.array_equal(ids[:, 0], np.arange(9000, 9100)), prec
        # re-ranked distances are the exact float32 distances of the returned ids
        ref = np.sqrt(((X[ids].astype(np.float64) - X[9000:9100, None, :]) ** 2).sum(-1))
        assert np.allclose(dd, ref, rtol=1e-5, atol=1e-5), prec


def test_insert_refusals_leave_the_index_unchanged():
    w = wl.SMALL_MIXTURE
    X, A = w.data(), w.proj()
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd[:5000].contiguous(), A, np.arange(5000), w.K, w.L, w.Nr, w.max_leaf)
    perm0 = idx.export(pdet.X_PERM, 0)
    Q = Xd[:20].contiguous()
    before = idx.query(Q, k=5, c=1.5, beta=0.1, r_min=4.0, eps=oracle.epsilon(w.K, w.L))
    # non-finite values in the new rows
    bad = Xd[:6000].clone()
    bad[5500, 3] = float("nan")
    print("\n[insert refusals] non-finite rows", flush=True)
    with pytest.raises(pdet.PdetError) as e:
        idx.insert(bad)
    assert e.value.status == pdet.PDET_EINVAL
    assert idx.info()["n"] == 5000
    np.testing.assert_array_equal(idx.export(pdet.X_PERM, 0), perm0)
    # a live plan
    plan = idx.plan(Q, k=5, c=1.5, beta=0.1, r_min=4.0, eps=oracle.epsilon(w.K, w.L))
    with pytest.raises(pdet.PdetError):
        idx.insert(Xd[:6000].contiguous())
    plan.close()
    # same row count: only the data pointer changes
    idx.insert(Xd[:5000].contiguous())
    after = idx.query(Q, k=5, c=1.5, beta=0.1, r_min=4.0, eps=oracle.epsilon(w.K, w.L))
    assert np.array_equal(before[0].cpu().numpy(), after[0].cpu().numpy())
    # the outer breakpoints did not keep the refused rows' extremes
    idx.insert(Xd[:6000].contiguous())
    B = idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
    H = oracle.project(X[:6000], A)
    E = proj_bound(X[:6000], A).max(axis=0)
    assert np.all(np.abs(B[:, 0] - H.min(axis=0)) <= E + 1e-30)
