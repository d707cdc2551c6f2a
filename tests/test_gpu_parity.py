"""GPU parity: libpdet (HIP, through the C ABI) against the FP64 CPU oracle.

Checked step by step so that a mismatch names its step:
  projection  within the FP32 dot-product error bound (d+1) u sum|x_t a_t|;
  breakpoints within that bound (order statistics are 1-Lipschitz);
  codes       bit-exact except coordinates within 1e-5 of the column range of a breakpoint
              (counted and reported);
  trees       the oracle's tree built on the GPU's codes equals the GPU tree exactly
              (leaf order, sizes, node ids; point sets per leaf);
  queries     the oracle's query run on the GPU's breakpoints, codes and trees gives the
              same candidate set (size and two hashes), stop rule, rounds, admitted leaves,
              ids, and distances within 1e-9 relative (FP64 accumulation on both sides);
              a difference is allowed only where a leaf bound lies within 1e-5 of a radius
              threshold or the k-th distance within 1e-5 of c*r.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from parity import BAND, compare_batch, near_stop_b, near_threshold, proj_bound, set_hashes  # noqa: E402


class Case:
    def __init__(self, X, A, sid, K, L, Nr, max_leaf, lowp=(), encoding="dynamic"):
        self.X, self.A, self.sid = X, A, sid
        self.K, self.L, self.Nr, self.max_leaf = K, L, Nr, max_leaf
        self.Xd = torch.from_numpy(X).cuda()
        print(f"\n[case] n={len(X)} d={X.shape[1]} K={K} L={L} Nr={Nr} max_leaf={max_leaf} "
              f"encoding={encoding}", flush=True)
        self.idx = pdet.Index(self.Xd, A, sid, K, L, Nr, max_leaf, lowp=lowp, encoding=encoding)
        torch.cuda.synchronize()
        self.H = oracle.project(X, A)
        make = oracle.static_breakpoints if encoding == "static" else oracle.breakpoints
        self.B_or = make(self.H[sid], Nr, self.H.min(axis=0), self.H.max(axis=0))
        self.B_gpu = self.idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
        self.codes_gpu = np.ascontiguousarray(self.idx.export(pdet.X_CODES)[:, :, :K])
        # the oracle's own eps (Eq. 2 / Lemma 3), passed to both sides
        self.eps = oracle.epsilon(K, L)
        self._stepwise = None

    def stepwise_oracle(self):
        """Oracle index on the GPU's breakpoints and codes."""
        if self._stepwise is None:
            self._stepwise = oracle.build_index(self.X, self.A, self.sid, self.L, self.K,
                                                self.Nr, self.max_leaf, B=self.B_gpu,
                                                codes=self.codes_gpu)
        return self._stepwise


def check_projection(cs, rows=2000):
    m = min(rows, len(cs.X))
    P = cs.idx.project(cs.Xd[:m]).cpu().numpy().astype(np.float64)
    bound = proj_bound(cs.X[:m], cs.A)
    err = np.abs(P - cs.H[:m])
    assert np.all(err <= bound), float((err / bound).max())


def check_breakpoints(cs):
    E_s = proj_bound(cs.X[cs.sid], cs.A).max(axis=0)
    E_all = proj_bound(cs.X, cs.A).max(axis=0)
    Bo, Bg = cs.B_or, cs.B_gpu
    assert np.all(np.abs(Bg[:, 1:-1] - Bo[:, 1:-1]) <= E_s[:, None] + 1e-30)
    assert np.all(np.abs(Bg[:, [0, -1]] - Bo[:, [0, -1]]) <= E_all[:, None] + 1e-30)


def check_codes(cs):
    codes_or = oracle.encode(cs.H, cs.B_or, cs.L, cs.K)
    mism = cs.codes_gpu != codes_or
    banded = np.zeros_like(mism)
    for i in range(cs.L):
        for j in range(cs.K):
            col = i * cs.K + j
            inner = cs.B_or[col, 1:-1]
            h = cs.H[:, col]
            pos = np.searchsorted(inner, h)
            lo = np.abs(h - inner[np.clip(pos - 1, 0, len(inner) - 1)])
            hi = np.abs(h - inner[np.clip(pos, 0, len(inner) - 1)])
            rng = cs.B_or[col, -1] - cs.B_or[col, 0]
            banded[i, :, j] = np.minimum(lo, hi) <= BAND * rng
    bad = mism & ~banded
    print(f"[codes] coords={mism.size} banded={int(banded.sum())} "
          f"mismatched={int(mism.sum())} (all banded: {not bad.any()})", flush=True)
    assert not bad.any(), np.argwhere(bad)[:10]


def check_trees(cs):
    for i in range(cs.L):
        t = oracle.build_tree(cs.codes_gpu[i], cs.Nr, cs.max_leaf)
        gs = cs.idx.export(pdet.X_LEAF_START, i)
        gc = cs.idx.export(pdet.X_LEAF_COUNT, i)
        gh = cs.idx.export(pdet.X_LEAF_HIDX, i)[:, :cs.K]
        gp = cs.idx.export(pdet.X_PERM, i)
        assert len(gs) == t.nl, (i, len(gs), t.nl)
        np.testing.assert_array_equal(gs, t.leaf_start)
        np.testing.assert_array_equal(gc, t.leaf_count)
        np.testing.assert_array_equal(gh, t.hidx())
        leaf_of_pos = np.repeat(np.arange(t.nl), t.leaf_count)
        np.testing.assert_array_equal(gp[np.lexsort((gp, leaf_of_pos))], t.perm)


def run_and_compare(cs, idx_or, Q, k, c, beta, r_min, label, allow_frac=0.0):
    """One GPU batch with candidate export, every query compared with the oracle."""
    Qd = torch.from_numpy(Q).cuda()
    cap = min(len(cs.X), int(np.ceil(beta * len(cs.X))) + k + 8 * cs.max_leaf + 64)
    print(f"[query {label}] nq={len(Q)} k={k} c={c} beta={beta} r_min={r_min} eps={cs.eps}",
          flush=True)
    ids, dists, st, cands = cs.idx.query_candidates(Qd, cap, k=k, c=c, beta=beta, r_min=r_min,
                                                    eps=cs.eps)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    compare_queries(cs, idx_or, Q, range(len(Q)), ids, dists, st, k, c, beta, r_min, label,
                    allow_frac, cands=cands)
    return ids, dists, st


def compare_queries(cs, idx_or, Q, sel, ids, dists, st, k, c, beta, r_min, label,
                    allow_frac=0.0, cands=None):
    """GPU results of the queries `sel` of batch Q against the oracle run one by one; every
    difference must be a classified near tie, and at most allow_frac of them (at least 1)."""
    sel = list(sel)
    n_same, n_band, results = compare_batch(cs.X, idx_or, Q, sel, ids, dists, st, k, c, beta,
                                            r_min, cs.eps, label, cands=cands,
                                            log=lambda m: print(m, flush=True))
    assert len(sel) - n_same <= max(1, allow_frac * len(sel))
    if cands is not None:
        whole = sum(len(cands[q]) == st[q, 1] for q in sel)
        print(f"[query {label}] candidate sets compared element by element: {whole}/{len(sel)}",
              flush=True)
    return results


# --------------------------------------------------------------------------- cases
@pytest.fixture(scope="module")
def mixture():
    w = wl.SMALL_MIXTURE
    return w, Case(w.data(), w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf,
                   lowp=("bf16", "fp8"))


@pytest.fixture(scope="module")
def ragged():
    # n not a multiple of any tile, d not a multiple of 4, K < 16, L = 3, Nr = 16
    w = wl.SMALL_MIXTURE.scaled(n=3001, d=37, K=5, L=3, Nr=16, max_leaf=7)
    X = w.data()
    A = wl.projection_matrix(37, 3, 5, seed=77)
    sid = wl.sample_ids(len(X), 600, 78)
    return w, Case(X, A, sid, 5, 3, 16, 7)


def test_projection_within_fp32_bound(mixture, ragged):
    check_projection(mixture[1])
    check_projection(ragged[1])


def test_breakpoints_within_bound(mixture, ragged):
    check_breakpoints(mixture[1])
    check_breakpoints(ragged[1])


def test_codes_exact_outside_band(mixture, ragged):
    check_codes(mixture[1])
    check_codes(ragged[1])


def test_trees_equal_oracle_on_gpu_codes(mixture, ragged):
    check_trees(mixture[1])
    check_trees(ragged[1])


@pytest.mark.parametrize("beta,r_min", [(0.1, 4.0), (0.02, 1.0), (1.0, 6.0), (0.05, 0.05)])
def test_query_stepwise_mixture(mixture, beta, r_min):
    w, cs = mixture
    _, _, st = run_and_compare(cs, cs.stepwise_oracle(), w.queries(), w.k, w.c, beta, r_min,
                               f"mixture b={beta}")
    if r_min <= 0.05:
        # small first radii run past the rounds the batched bound kernel resolves (5),
        # so the per-query refinement of the open leaves is exercised
        assert st[:, pdet.QSTAT["rounds"]].max() > 6



def test_query_stepwise_past_the_lds_hash(mixture):
    # k = 1000 and c = 1.05 keep stop rule B from firing early: every query admits more than
    # 1024 leaves (the LDS hash holds 512), so its dedupe state moves to the dense round table in
    # device memory (and is restored for the slot's next query)
    w, cs = mixture
    Q = w.queries(20)
    _, _, st = run_and_compare(cs, cs.stepwise_oracle(), Q, 1000, 1.05, 1.0, 1.0, "dense")
    assert st[:, pdet.QSTAT["leaves"]].min() > 1024
    # the same slots with the queries reversed: a table left dirty by the first call
    # would mark other queries' leaves as admitted
    run_and_compare(cs, cs.stepwise_oracle(), np.ascontiguousarray(Q[::-1]), 1000, 1.05, 1.0,
                    1.0, "dense reversed")


# r_min = 1000 admits every leaf in round 0: the stop tree then has more leaves than one
# ordering pass takes and the counted-prefix selection runs
@pytest.mark.parametrize("beta,r_min,k,c", [(0.05, 2.0, 7, 1.5), (0.3, 0.5, 1, 2.0),
                                            (0.0, 3.0, 30, 1.2), (0.3, 1000.0, 10, 1.5)])
def test_query_stepwise_ragged(ragged, beta, r_min, k, c):
    w, cs = ragged
    run_and_compare(cs, cs.stepwise_oracle(), w.queries(40), k, c, beta, r_min,
                    f"ragged k={k}")


def _first_layer_nodes_with_changed_codes(codes_a, codes_b, bits):
    """Per tree, the first-layer keys of the points whose codes differ between two builds."""
    out = []
    for i in range(codes_a.shape[0]):
        diff = np.nonzero(np.any(codes_a[i] != codes_b[i], axis=1))[0]
        keys = set()
        for codes in (codes_a[i], codes_b[i]):
            keys |= set(oracle.first_layer_key(codes[diff], bits).tolist())
        out.append(keys)
    return out


def test_query_end_to_end_against_oracle_from_scratch(mixture):
    """Oracle built from its own FP64 projections and breakpoints. Every query must give
    the oracle's candidate set, control flow and ids, unless the difference is explained
    (and counted): the query admitted a leaf of a first-layer node whose points' codes
    differ (all such codes are banded, see the code test), or a leaf bound / k-th
    distance lies in the band of a threshold (FP32 vs FP64 breakpoints)."""
    w, cs = mixture
    idx_or = oracle.build_index(cs.X, cs.A, cs.sid, w.L, w.K, w.Nr, w.max_leaf)
    step = cs.stepwise_oracle()
    Q = w.queries()
    Qd = torch.from_numpy(Q).cuda()
    cap = len(cs.X)
    ids, dists, st, cands = cs.idx.query_candidates(Qd, cap, k=w.k, c=w.c, beta=w.beta,
                                                    r_min=4.0, eps=cs.eps)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    changed = _first_layer_nodes_with_changed_codes(idx_or.codes, cs.codes_gpu,
                                                    int(np.log2(w.Nr)))
    same = by_codes = by_band = 0
    for qi, q in enumerate(Q):
        res = oracle.query(idx_or, cs.X, q, w.k, w.c, w.beta, 4.0, cs.eps)
        if np.array_equal(cands[qi], np.sort(res.cand)) and st[qi, 2] == {"A": 1, "B": 2}[res.stop] \
                and st[qi, 0] == res.rounds and st[qi, 3] == res.leaves:
            np.testing.assert_array_equal(ids[qi], res.ids)
            np.testing.assert_allclose(dists[qi], res.dists, rtol=1e-6)
            same += 1
            continue
        # the GPU equals the oracle on its own breakpoints and codes
        rs = oracle.query(step, cs.X, q, w.k, w.c, w.beta, 4.0, cs.eps)
        assert np.array_equal(cands[qi], np.sort(rs.cand)), qi
        touched = False
        for index, r in ((idx_or, res), (step, rs)):
            for rho, i, leaf, _, _ in r.trace:
                t = index.trees[i]
                o = t.perm[t.leaf_start[leaf]]
                key = int(oracle.first_layer_key(index.codes[i][o:o + 1], int(np.log2(w.Nr)))[0])
                touched = touched or key in changed[i]
        if touched:
            by_codes += 1
            continue
        rounds = max(res.rounds, rs.rounds)
        assert (near_threshold(idx_or, q, rounds, 4.0, w.c, cs.eps)
                or near_threshold(step, q, rounds, 4.0, w.c, cs.eps)
                or near_stop_b(cs.X, q, res.cand, w.k, rounds, 4.0, w.c)), qi
        by_band += 1
    print(f"[end-to-end] identical {same}/{len(Q)}; explained by banded codes {by_codes}, "
          f"by a threshold near tie {by_band}", flush=True)
    assert same + by_codes + by_band == len(Q)


def test_exact_knn_when_everything_is_admitted(mixture):
    """beta = 1 and a first radius covering every point: S = D, output = exact kNN."""
    w, cs = mixture
    Q = w.queries(30)
    ids, dists, st = cs.idx.query(torch.from_numpy(Q).cuda(), k=25, c=1.5, beta=1.0,
                                  r_min=1e4, eps=cs.eps, stats=True)
    ex_ids, ex_d = oracle.knn_exact(cs.X, Q, 25)
    np.testing.assert_array_equal(ids.cpu().numpy(), ex_ids)
    np.testing.assert_allclose(dists.cpu().numpy(), ex_d, rtol=1e-6)
    st = st.cpu().numpy()
    assert np.all(st[:, pdet.QSTAT["ncand"]] == len(cs.X)) and np.all(st[:, 2] == 2)


def test_batch_composition_does_not_change_results(mixture):
    w, cs = mixture
    Q = torch.from_numpy(w.queries()).cuda()
    ids_b, d_b = cs.idx.query(Q, k=10, c=1.5, beta=0.05, r_min=3.0)
    for sel in ([3], [17, 5], list(range(40, 47))):
        ids_s, d_s = cs.idx.query(Q[sel].contiguous(), k=10, c=1.5, beta=0.05, r_min=3.0)
        assert torch.equal(ids_s, ids_b[sel]) and torch.equal(d_s, d_b[sel])


def test_per_query_k_and_c(mixture):
    w, cs = mixture
    Q = w.queries(24)
    rng = np.random.default_rng(3)
    ks = rng.choice([1, 10, 100], size=len(Q)).astype(np.int32)
    cc = rng.choice([1.2, 1.5, 2.0], size=len(Q))
    ids, dists = cs.idx.query(torch.from_numpy(Q).cuda(), k=0, beta=0.05, r_min=3.0,
                              eps=cs.eps, k_per_query=ks, c_per_query=cc)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    idx_or = cs.stepwise_oracle()
    off = 0
    for qi, q in enumerate(Q):
        res = oracle.query(idx_or, cs.X, q, int(ks[qi]), float(cc[qi]), 0.05, 3.0, cs.eps)
        np.testing.assert_array_equal(ids[off:off + ks[qi]], res.ids)
        off += ks[qi]


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_low_precision_forms_recall_and_rescored_distances(mixture, prec):
    """Recall against the float32 path, exact re-ranked distances, and the same stop rule
    and round as the float32 path (stop rule B counts the kept candidates by their exact
    distance): the queries that stop elsewhere are counted and must be rare."""
    w, cs = mixture
    Q = torch.from_numpy(w.queries()).cuda()
    i32, d32, s32 = cs.idx.query(Q, k=10, c=1.5, beta=0.1, r_min=4.0, eps=cs.eps, stats=True)
    il, dl, sl = cs.idx.query(Q, k=10, c=1.5, beta=0.1, r_min=4.0, eps=cs.eps, precision=prec,
                              rescore=4, stats=True)
    i32, il, dl = i32.cpu().numpy(), il.cpu().numpy(), dl.cpu().numpy()
    s32, sl = s32.cpu().numpy(), sl.cpu().numpy()
    rec = np.mean([len(np.intersect1d(a, b)) / 10 for a, b in zip(il, i32)])
    moved = int(np.sum((s32[:, 0] != sl[:, 0]) | (s32[:, 2] != sl[:, 2])))
    print(f"[{prec}] recall vs fp32 path = {rec:.4f}; queries stopping in another round or "
          f"by another rule than fp32: {moved}/{len(Q)}", flush=True)
    assert rec >= 0.95
    assert moved <= max(1, len(Q) // 20)
    # distances of returned ids are exact (re-ranked from float32 data)
    ex = np.sqrt(((cs.X[il].astype(np.float64) - w.queries()[:, None, :]) ** 2).sum(-1))
    np.testing.assert_allclose(dl, ex, rtol=1e-6)
    # with beta = 1 stop rule B decides every query: its round must match the float32 path
    _, _, b32 = cs.idx.query(Q, k=10, c=1.5, beta=1.0, r_min=0.5, eps=cs.eps, stats=True)
    _, _, bl = cs.idx.query(Q, k=10, c=1.5, beta=1.0, r_min=0.5, eps=cs.eps, precision=prec,
                            rescore=4, stats=True)
    b32, bl = b32.cpu().numpy(), bl.cpu().numpy()
    assert np.all(b32[:, 2] == 2)
    moved_b = int(np.sum(b32[:, 0] != bl[:, 0]))
    print(f"[{prec}] stop rule B rounds differing from fp32: {moved_b}/{len(Q)}", flush=True)
    assert moved_b <= max(1, len(Q) // 20)


def test_duplicates_make_a_fully_refined_leaf():
    rng = np.random.default_rng(9)
    X = rng.standard_normal((700, 16)).astype(np.float32)
    X[100:400] = X[100]
    A = wl.projection_matrix(16, 2, 8, seed=3)
    cs = Case(X, A, np.arange(700), 8, 2, 64, 20)
    check_codes(cs)
    check_trees(cs)
    counts = cs.idx.export(pdet.X_LEAF_COUNT, 0)
    assert counts.max() >= 300
    Q = rng.standard_normal((10, 16)).astype(np.float32)
    run_and_compare(cs, cs.stepwise_oracle(), Q, 5, 1.5, 0.1, 0.3, "duplicates")


def test_tiny_index_k_equals_n():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((16, 3)).astype(np.float32)
    A = wl.projection_matrix(3, 1, 1, seed=5)
    cs = Case(X, A, np.arange(16), 1, 1, 2, 1)
    check_trees(cs)
    Q = rng.standard_normal((4, 3)).astype(np.float32)
    ids, dists = cs.idx.query(torch.from_numpy(Q).cuda(), k=16, c=2.0, beta=0.0, r_min=0.01)
    ex_ids, ex_d = oracle.knn_exact(X, Q, 16)
    np.testing.assert_array_equal(ids.cpu().numpy(), ex_ids)


def test_minimum_sample_one_point_per_region():
    w = wl.SMALL_MIXTURE.scaled(n=2000, L=1)
    X = w.data()
    A = wl.projection_matrix(128, 1, 16, seed=8)
    sid = wl.sample_ids(2000, 256, 9)              # m = floor(256/256) = 1
    cs = Case(X, A, sid, 16, 1, 256, 32)
    check_breakpoints(cs)
    check_codes(cs)
    check_trees(cs)
    run_and_compare(cs, cs.stepwise_oracle(), w.queries(20), 5, 1.5, 0.1, 3.0, "m=1")
