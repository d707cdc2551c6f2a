"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a hand-worked
example from the paper's text (``tests/golden``), a closed form, an invariant
the paper proves or states, or an independent brute-force construction.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2603_24920_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


# ---------------------------------------------------------------- projection
def test_projection_of_basis_vectors_gives_hash_vectors():
    """Eq. 1: h(e_t) = a . e_t = a[t]; column i*K+j of A is a_ij."""
    d, L, K = 12, 3, 4
    A = wl.projection_matrix(d, L, K, seed=5)
    H = oracle.project(np.eye(d, dtype=np.float32), A)
    np.testing.assert_array_equal(H, A.astype(np.float64))
    x = np.zeros((1, d), dtype=np.float32)
    x[0, 3], x[0, 7] = 2.0, -1.0
    np.testing.assert_allclose(oracle.project(x, A)[0], 2.0 * A[3].astype(np.float64) - A[7],
                               rtol=0, atol=1e-12)


def test_lemma1_projected_distance_ratio_is_chi2():
    """Lemma 1: s'^2 / s^2 ~ chi2(K) over the random choice of the K hash vectors."""
    d, K, trials = 32, 16, 4000
    rng = np.random.default_rng(11)
    o1, o2 = rng.standard_normal(d), rng.standard_normal(d) * 3
    s2 = ((o1 - o2) ** 2).sum()
    ratios = np.empty(trials)
    X = np.stack([o1, o2]).astype(np.float32)
    for t in range(trials):
        A = wl.projection_matrix(d, 1, K, seed=1000 + t)
        H = oracle.project(X, A)
        ratios[t] = ((H[0] - H[1]) ** 2).sum() / ((X[0].astype(np.float64) - X[1]) ** 2).sum()
    assert abs(s2 - ((X[0].astype(np.float64) - X[1]) ** 2).sum()) < 1e-3 * s2
    p = stats.kstest(ratios, stats.chi2(K).cdf).pvalue
    assert p > 1e-3, p
    # Lemma 2 at the level used by the method: Pr[s' > s*eps] = alpha1
    eps = oracle.epsilon(K, 4)
    frac = np.mean(ratios > eps * eps)
    assert abs(frac - math.exp(-1 / 4)) < 4 * math.sqrt(0.25 / trials)


# --------------------------------------------------------------- breakpoints
def test_breakpoints_and_codes_hand_example():
    g = golden("breakpoints_ranks.json")
    col = np.array(g["column"], dtype=np.float64)[:, None]
    B = oracle.breakpoints(col, g["Nr"], col.min(axis=0), col.max(axis=0))
    np.testing.assert_array_equal(B[0], np.array(g["breakpoints"], dtype=np.float64))
    codes = oracle.encode(col, B, 1, 1)[0, :, 0]
    np.testing.assert_array_equal(codes, g["codes"])
    np.testing.assert_array_equal(np.bincount(codes, minlength=g["Nr"]), g["region_counts"])


@pytest.mark.parametrize("n,Nr", [(10_000, 256), (1000, 16), (777, 8)])
def test_region_counts_closed_form_when_sample_is_everything(n, Nr):
    """With ns = n and distinct values, regions hold exactly m-1, m (Nr-2 times) and
    n-(Nr-1)m+1 points, m = floor(n/Nr) (breakpoint formula of the encoding phase)."""
    rng = np.random.default_rng(n)
    H = rng.standard_normal((n, 3)) * rng.uniform(1, 50, size=3)
    B = oracle.breakpoints(H, Nr, H.min(axis=0), H.max(axis=0))
    codes = oracle.encode(H, B, 1, 3)[0]
    m = n // Nr
    want = [m - 1] + [m] * (Nr - 2) + [n - (Nr - 1) * m + 1]
    for j in range(3):
        np.testing.assert_array_equal(np.bincount(codes[:, j], minlength=Nr), want)


def test_encode_ties_and_extremes():
    """Algorithm 1's closed interval is read as: a value equal to a breakpoint goes up."""
    B = np.array([[-1.0, 0.0, 1.0, 2.0, 3.0]])          # Nr = 4, interior 0,1,2
    h = np.array([[-1.0], [-0.5], [0.0], [0.5], [1.0], [2.0], [2.5], [3.0]])
    np.testing.assert_array_equal(oracle.encode(h, B, 1, 1)[0, :, 0], [0, 0, 1, 1, 2, 3, 3, 3])


def test_sampled_regions_near_equal_frequency():
    """Sampled breakpoints give regions of near-equal mass over the full data."""
    w = wl.SMALL_MIXTURE.scaled(n=20_000)
    X = w.data()
    A = w.proj()
    H = oracle.project(X, A)
    ids = wl.sample_ids(len(X), 8192, 7)
    Nr = 16
    B = oracle.breakpoints(H[ids], Nr, H.min(axis=0), H.max(axis=0))
    codes = oracle.encode(H, B, w.L, w.K)
    m = len(ids) // Nr
    # expected full-data share of each region from the sample's rank layout
    share = np.array([m - 1] + [m] * (Nr - 2) + [len(ids) - (Nr - 1) * m + 1]) / len(ids)
    for i in range(w.L):
        for j in range(0, w.K, 5):
            cnt = np.bincount(codes[i, :, j], minlength=Nr)
            chi = ((cnt - share * len(X)) ** 2 / (share * len(X))).sum()
            assert stats.chi2(Nr - 1).sf(chi / 3.5) > 1e-4, (i, j, cnt)


# ---------------------------------------------------------------- DE-Tree
def test_tree_hand_example_split():
    g = golden("isax_split.json")
    codes = np.array(g["codes"], dtype=np.uint8)
    t = oracle.build_tree(codes, g["Nr"], g["max_leaf"])
    assert t.nl == len(g["leaves"])
    for ell, want in enumerate(g["leaves"]):
        ids = t.perm[t.leaf_start[ell]:t.leaf_start[ell] + t.leaf_count[ell]]
        np.testing.assert_array_equal(ids, want["ids"])
        np.testing.assert_array_equal(t.hidx()[ell], want["hidx"])


def _brute_tree(codes, bits, max_leaf):
    """Independent construction of the DE-Tree leaves from the definitions, using code
    bit strings and recursion; returns [(ids tuple, path strings)] in depth-first order."""
    n, K = codes.shape
    strs = [["{:0{}b}".format(int(c), bits) for c in row] for row in codes]

    def rec(ids, pref):
        if not ids:
            return []
        if len(ids) <= max_leaf or all(len(p) == bits for p in pref):
            return [(tuple(sorted(ids)), tuple(pref))]
        best = None
        for j in range(K):
            if len(pref[j]) == bits:
                continue
            ones = sum(strs[o][j][len(pref[j])] == "1" for o in ids)
            score = abs(ones - (len(ids) - ones))
            if best is None or score < best[0]:
                best = (score, j)
        j = best[1]
        out = []
        for b in "01":
            sub = [o for o in ids if strs[o][j][len(pref[j])] == b]
            p2 = list(pref)
            p2[j] = pref[j] + b
            out += rec(sub, p2)
        return out

    groups = {}
    for o in range(n):
        groups.setdefault(tuple(s[0] for s in strs[o]), []).append(o)
    leaves = []
    for key in sorted(groups):
        leaves += rec(groups[key], list(key))
    return leaves


@pytest.mark.parametrize("n,K,Nr,max_leaf,seed", [(300, 3, 8, 4, 0), (500, 4, 16, 7, 1),
                                                   (200, 2, 4, 3, 2), (400, 5, 256, 10, 3)])
def test_tree_matches_brute_force_construction(n, K, Nr, max_leaf, seed):
    rng = np.random.default_rng(seed)
    # clustered codes so that splits go deep and duplicates occur
    base = rng.integers(0, Nr, size=(8, K))
    codes = np.clip(base[rng.integers(0, 8, n)] + rng.integers(-1, 2, size=(n, K)), 0, Nr - 1)
    codes = codes.astype(np.uint8)
    bits = int(math.log2(Nr))
    t = oracle.build_tree(codes, Nr, max_leaf)
    brute = _brute_tree(codes, bits, max_leaf)
    assert t.nl == len(brute)
    for ell, (ids, pref) in enumerate(brute):
        got = t.perm[t.leaf_start[ell]:t.leaf_start[ell] + t.leaf_count[ell]]
        np.testing.assert_array_equal(got, ids)
        np.testing.assert_array_equal(t.leaf_depth[ell], [len(p) for p in pref])
        np.testing.assert_array_equal(t.leaf_prefix[ell], [int(p, 2) for p in pref])


def test_tree_partition_invariants():
    rng = np.random.default_rng(4)
    n, K, Nr, max_leaf = 5000, 16, 256, 32
    codes = rng.integers(0, Nr, size=(n, K)).astype(np.uint8)
    codes[:200] = codes[0]                     # 200 identical points: a fully refined leaf
    t = oracle.build_tree(codes, Nr, max_leaf)
    np.testing.assert_array_equal(np.sort(t.perm), np.arange(n))
    assert t.leaf_start[0] == 0 and np.all(t.leaf_start[1:] == t.leaf_start[:-1] + t.leaf_count[:-1])
    for ell in range(t.nl):
        ids = t.perm[t.leaf_start[ell]:t.leaf_start[ell] + t.leaf_count[ell]]
        dep, pre = t.leaf_depth[ell], t.leaf_prefix[ell]
        assert np.all(codes[ids].astype(np.int64) >> (8 - dep) == pre)
        assert len(ids) <= max_leaf or np.all(dep == 8)
    assert t.leaf_count.max() == 200


# ---------------------------------------------------------------- bounds
def test_bound_example_from_the_paper_figure():
    g = golden("bound_example.json")
    tr = oracle.Tree(np.array([0]), np.array([0]), np.array([1]), np.array([g["depth"]]),
                     np.array([g["prefix"]]))
    lo, hi = oracle.leaf_boxes(tr, np.array(g["B"], dtype=np.float64), g["Nr"])
    q = np.array(g["q"], dtype=np.float64)
    assert oracle.lower_bound_sq(q, lo, hi)[0] == g["lb_sq"]
    assert oracle.upper_bound_sq(q, lo, hi)[0] == g["ub_sq"]


def test_lower_bound_never_exceeds_projected_distance():
    w = wl.SMALL_MIXTURE.scaled(n=3000)
    X, A = w.data(), w.proj()
    idx = oracle.build_index(X, A, w.sample(), w.L, w.K, w.Nr, 16)
    Q = w.queries(20)
    H = oracle.project(X, A)
    for q in Q:
        qp = q.astype(np.float64) @ idx.A
        for i in range(w.L):
            t = idx.trees[i]
            lo, hi = idx.boxes[i]
            lb2 = oracle.lower_bound_sq(qp[i * w.K:(i + 1) * w.K], lo, hi)
            ub2 = oracle.upper_bound_sq(qp[i * w.K:(i + 1) * w.K], lo, hi)
            leaf_of = np.empty(len(X), dtype=np.int64)
            for ell in range(t.nl):
                leaf_of[t.perm[t.leaf_start[ell]:t.leaf_start[ell] + t.leaf_count[ell]]] = ell
            true2 = ((H[:, i * w.K:(i + 1) * w.K] - qp[i * w.K:(i + 1) * w.K]) ** 2).sum(axis=1)
            assert np.all(lb2[leaf_of] <= true2 * (1 + 1e-12) + 1e-9)
            assert np.all(ub2[leaf_of] >= true2 * (1 - 1e-12) - 1e-9)
    # a point's own projection lies in its leaf box: LB = 0
    for i in range(w.L):
        t, (lo, hi) = idx.trees[i], idx.boxes[i]
        o = t.perm[t.leaf_start[5]]
        assert oracle.lower_bound_sq(H[o, i * w.K:(i + 1) * w.K], lo, hi)[5] == 0.0


# ---------------------------------------------------------------- parameters
def _chi2_sf_even(x, K):
    """Closed-form chi2 survival function for even K: exp(-x/2) sum_{i<K/2} (x/2)^i / i!."""
    return math.exp(-x / 2) * sum((x / 2) ** i / math.factorial(i) for i in range(K // 2))


@pytest.mark.parametrize("L", [1, 2, 4, 8, 16])
def test_epsilon_solves_eq2(L):
    K = 16
    eps = oracle.epsilon(K, L)
    assert abs(_chi2_sf_even(eps * eps, K) - math.exp(-1 / L)) < 1e-12


def test_theoretical_beta_and_l4_values():
    """Lemma 3 at K=16, L=4: eps = 3.388515; beta(c=1.5) = 2 - 2 alpha2^4 with
    alpha2 = sf(eps^2/c^2)."""
    K, L = 16, 4
    eps = oracle.epsilon(K, L)
    assert abs(eps - 3.388515) < 1e-6
    for c in (1.2, 1.5, 2.0):
        a2 = _chi2_sf_even(eps * eps / (c * c), K)
        assert abs(oracle.theoretical_beta(K, L, c) - (2 - 2 * a2 ** L)) < 1e-12
    assert abs(oracle.theoretical_beta(K, L, 1.5) - 0.0380) < 5e-5
    # Pr[E1] >= 1 - alpha1^L = 1 - 1/e at L = -1/ln(alpha1)
    assert abs(1 - math.exp(-1 / L) ** L - (1 - 1 / math.e)) < 1e-15


# ---------------------------------------------------------------- query
@pytest.fixture(scope="module")
def small_index():
    w = wl.SMALL_MIXTURE.scaled(n=4000)
    X, A = w.data(), w.proj()
    idx = oracle.build_index(X, A, w.sample(), w.L, w.K, w.Nr, 32)
    return w, X, idx


def test_query_reduces_to_exact_knn_when_everything_is_admitted(small_index):
    """With T > n and a first radius covering every point, S = D and the answer is the
    exact kNN (Definition 2 with c -> 1)."""
    w, X, idx = small_index
    Q = w.queries(10)
    ids_x, d_x = oracle.knn_exact(X, Q, 10)
    eps = oracle.epsilon(w.K, w.L)
    big = 1e6
    for q, ie, de in zip(Q, ids_x, d_x):
        res = oracle.query(idx, X, q, 10, 1.5, 1.0, big, eps)
        assert res.stop == "B" and res.n_cand == len(X) and res.rounds == 1
        np.testing.assert_array_equal(res.ids, ie)
        np.testing.assert_allclose(res.dists, de, rtol=1e-15)


def _leaf_lb2(idx, q):
    """Per point and tree: squared LB of the leaf holding the point."""
    qp = np.asarray(q, dtype=np.float64) @ idx.A
    out = np.empty((idx.L, idx.n))
    for i in range(idx.L):
        t, (lo, hi) = idx.trees[i], idx.boxes[i]
        lb2 = oracle.lower_bound_sq(qp[i * idx.K:(i + 1) * idx.K], lo, hi)
        for ell in range(t.nl):
            out[i, t.perm[t.leaf_start[ell]:t.leaf_start[ell] + t.leaf_count[ell]]] = lb2[ell]
    return out


def _leaf_keys(idx, q, i):
    """(LB^2, leaf ordinal) of every leaf of tree i for query q."""
    qp = np.asarray(q, dtype=np.float64) @ idx.A
    lo, hi = idx.boxes[i]
    return oracle.lower_bound_sq(qp[i * idx.K:(i + 1) * idx.K], lo, hi)


def test_candidate_set_closed_form(small_index):
    """S is the union over the admitted prefix of (round, tree) steps: before step
    (rho, i), o is in S iff LB_{i'}(o) <= (eps r_rho)^2 for some i' < i, or
    LB_{i'}(o) <= (eps r_{rho-1})^2 for some i'. Within a step the admitted leaves are
    the qualifying leaves in ascending (LB^2, ordinal) order (Section 6.2.2), all of them
    unless stop rule A fires; stop rule A fires on the first leaf that lifts |S| to T
    (the cut is minimal); stop rule B fires in the first round whose k-th distance in S
    is within c*r (Algorithm 5), never earlier."""
    w, X, idx = small_index
    eps = oracle.epsilon(w.K, w.L)
    Q = w.queries(12)
    k, c = 10, 1.5
    for beta, r_min in ((0.05, 2.0), (0.2, 4.0), (0.01, 1.0), (0.0, 0.5)):
        T = math.ceil(beta * len(X)) + k
        for q in Q:
            res = oracle.query(idx, X, q, k, c, beta, r_min, eps)
            lb = _leaf_lb2(idx, q)
            S = set(res.cand.tolist())
            assert len(S) == res.n_cand
            ladder = list(oracle.radius_ladder(r_min, c, res.rounds))
            t2 = [(eps * r) ** 2 for r in ladder]
            if res.stop == "B":
                want = set(np.nonzero(lb.min(axis=0) <= t2[-1])[0].tolist())
                assert S == want
                assert len(S) < T
            else:
                assert len(S) >= T
                before = lb.min(axis=0) <= (t2[-2] if len(t2) > 1 else -1.0)
                assert set(np.nonzero(before)[0].tolist()) <= S
                within = set(np.nonzero(lb.min(axis=0) <= t2[-1])[0].tolist())
                assert S <= within
                # minimal cut: without the last admitted leaf's new points |S| < T
                assert len(S) - res.trace[-1][4] < T
            # the trace accounts for S exactly
            assert sum(t[4] for t in res.trace) == len(S) and len(res.trace) == res.leaves
            # admission per step: a prefix (all of it except at the stop cut) of the step's
            # qualifying leaves sorted by (LB^2, ordinal)
            steps = {}
            for rho, i, leaf, l2, nn in res.trace:
                steps.setdefault((rho, i), []).append((leaf, l2))
            last = (res.trace[-1][0], res.trace[-1][1]) if res.trace else None
            for rho in range(res.rounds):
                for i in range(w.L):
                    keys = _leaf_keys(idx, q, i)
                    lo_t = t2[rho - 1] if rho > 0 else -1.0
                    qual = np.nonzero((keys <= t2[rho]) & (keys > lo_t))[0]
                    qual = [int(x) for x in qual[np.lexsort((qual, keys[qual]))]]
                    got = [leaf for leaf, _ in steps.get((rho, i), [])]
                    for leaf, l2 in steps.get((rho, i), []):
                        assert l2 == keys[leaf]
                    if res.stop == "A" and (rho, i) == last:
                        assert got == qual[:len(got)] and len(got) >= 1
                    elif res.stop == "A" and (rho, i) > last:
                        assert got == []
                    else:
                        assert got == qual, (rho, i)
            # stop rule B never held at the end of an earlier round, and holds at the end
            # of the last round when it is the rule that fired
            Xq = np.sqrt(((X.astype(np.float64) - q.astype(np.float64)) ** 2).sum(axis=1))
            for rho in range(res.rounds):
                ids_rho = [t for t in res.trace if t[0] <= rho]
                n_rho = sum(t[4] for t in ids_rho)
                members = res.cand[:n_rho]
                if rho < res.rounds - 1 or res.stop == "B":
                    holds = len(members) >= k and np.sort(Xq[members])[k - 1] <= c * ladder[rho]
                    assert holds == (rho == res.rounds - 1 and res.stop == "B"), (rho, res.stop)
            # results are the top-k of S by (distance, id)
            cand = np.array(sorted(S))
            dd = np.sqrt(((X[cand].astype(np.float64) - q.astype(np.float64)) ** 2).sum(axis=1))
            o = np.lexsort((cand, dd))[:10]
            np.testing.assert_array_equal(res.ids, cand[o])


def _golden_index():
    g = golden("query_control_flow.json")
    X = np.array(g["points"], dtype=np.float32)
    A = np.eye(2, dtype=np.float32)
    B = np.array(g["B"], dtype=np.float64)
    idx = oracle.build_index(X, A, np.arange(len(X)), g["L"], g["K"], g["Nr"], g["max_leaf"], B=B)
    return g, X, idx


def test_golden_trees_and_bounds():
    g, X, idx = _golden_index()
    q = np.array(g["q"])
    for i, want in enumerate(g["trees"]):
        t = idx.trees[i]
        assert t.nl == len(want["leaves"])
        for ell, ids in enumerate(want["leaves"]):
            np.testing.assert_array_equal(t.perm[t.leaf_start[ell]:t.leaf_start[ell] + t.leaf_count[ell]],
                                          ids)
        np.testing.assert_array_equal(t.hidx()[:, 0], want["hidx"])
        np.testing.assert_array_equal(_leaf_keys(idx, q, i), want["lb_sq"])


@pytest.mark.parametrize("case", range(3))
def test_golden_optimised_query_control_flow(case):
    """Admission order by LB (Section 6.2.2), the leaf where |S| reaches ceil(beta n)+k,
    and the round where stop rule B fires, against hand-worked values."""
    g, X, idx = _golden_index()
    cs = g["optimised"][case]
    res = oracle.query(idx, X, np.array(g["q"], dtype=np.float32), cs["k"], cs["c"], cs["beta"],
                       cs["r_min"], cs["eps"])
    assert [list(t) for t in res.trace] == cs["trace"], cs["label"]
    np.testing.assert_array_equal(res.cand, cs["cand"])
    assert (res.stop, res.rounds, res.leaves) == (cs["stop"], cs["rounds"], cs["leaves"])
    np.testing.assert_array_equal(res.ids, cs["ids"])
    np.testing.assert_allclose(res.dists ** 2, cs["dists_sq"], rtol=1e-15)


def test_golden_literal_range_query():
    """Algorithm 3: LB pruning, whole leaves when UB <= r', per-point filter otherwise."""
    g, X, idx = _golden_index()
    q = np.array(g["q"], dtype=np.float64)
    for cs in g["range_literal"]:
        i = cs["tree"]
        ids, examined, whole = oracle.range_query_literal(idx, X, i, q[i:i + 1], cs["r_prime"])
        np.testing.assert_array_equal(ids, cs["ids"], err_msg=cs["label"])
        assert (examined, whole) == (cs["examined"], cs["whole"]), cs["label"]


def test_golden_rc_ann_query():
    """Algorithm 4: stop at beta*n + 1 with the closest point of S, else the closest point
    within c*r, else nothing."""
    g, X, idx = _golden_index()
    for cs in g["rc_ann"]:
        oid, dist, n_c, trees = oracle.rc_ann_query(idx, X, np.array(g["q"]), cs["c"], cs["r"],
                                                    cs["beta"], cs["eps"])
        assert (oid, n_c, trees) == (cs["id"], cs["n_cand"], cs["trees"]), cs["label"]
        if cs["dist"] is None:
            assert dist is None
        else:
            assert abs(dist - cs["dist"]) < 1e-15


def test_golden_literal_query():
    """Algorithm 5 as printed: literal range queries re-run every round, stop rule A per tree."""
    g, X, idx = _golden_index()
    for cs in g["literal"]:
        res = oracle.query_literal(idx, X, np.array(g["q"]), cs["k"], cs["c"], cs["beta"],
                                   cs["r_min"], cs["eps"])
        assert [list(t) for t in res.trace] == cs["trace"], cs["label"]
        np.testing.assert_array_equal(res.cand, cs["cand"])
        assert (res.stop, res.rounds) == (cs["stop"], cs["rounds"])
        np.testing.assert_array_equal(res.ids, cs["ids"])
        np.testing.assert_allclose(res.dists ** 2, cs["dists_sq"], rtol=1e-15)


def test_literal_range_query_is_the_projected_ball(small_index):
    """Every point of a leaf lies between the leaf's bounds, so Algorithm 3 returns exactly
    the points whose projected distance to q' is smaller than r' (ties have measure zero
    on this data): checked against brute force in the projected space."""
    w, X, idx = small_index
    H = oracle.project(X, idx.A)
    for q in w.queries(6):
        qp = q.astype(np.float64) @ idx.A
        for i in range(w.L):
            sl = slice(i * w.K, (i + 1) * w.K)
            d2 = ((H[:, sl] - qp[sl]) ** 2).sum(axis=1)
            for rp in np.quantile(np.sqrt(d2), [0.001, 0.01, 0.1]):
                ids, examined, whole = oracle.range_query_literal(idx, X, i, qp[sl], rp)
                np.testing.assert_array_equal(ids, np.nonzero(d2 < rp * rp)[0])
                assert examined <= idx.trees[i].nl and whole <= examined


def test_literal_query_candidates_within_the_relaxed_ones(small_index):
    """Per round and tree the literal range query takes a subset of the points of the
    leaves the relaxed admission takes whole (LB <= eps*r), and the literal stop rule A is
    checked per tree: before the tree where it fires, |S| < T."""
    w, X, idx = small_index
    eps = oracle.epsilon(w.K, w.L)
    for q in w.queries(5):
        for beta, r_min in ((0.05, 2.0), (0.01, 1.0)):
            lit = oracle.query_literal(idx, X, q, 10, 1.5, beta, r_min, eps)
            T = math.ceil(beta * len(X)) + 10
            lb = _leaf_lb2(idx, q)
            t2 = (eps * lit.radius) ** 2
            within = set(np.nonzero(lb.min(axis=0) <= t2)[0].tolist())
            assert set(lit.cand.tolist()) <= within
            sizes = np.cumsum([t[4] for t in lit.trace])
            if lit.stop == "A":
                assert sizes[-1] >= T and np.all(sizes[:-1] < T)
            else:
                assert np.all(sizes < T)


def test_candidate_set_grows_with_radius(small_index):
    """S_{r} is contained in S_{c r} (proof of Theorem 2): with no stop rule A the
    candidate set at a later termination radius contains the earlier one."""
    w, X, idx = small_index
    eps = oracle.epsilon(w.K, w.L)
    q = w.queries(1)[0]
    prev = set()
    for r_min in (0.5, 0.75, 1.125, 1.6875):
        lb = _leaf_lb2(idx, q)
        cur = set(np.nonzero(lb.min(axis=0) <= (eps * r_min) ** 2)[0].tolist())
        assert prev <= cur
        prev = cur


@pytest.mark.slow
def test_theorem2_success_probability():
    """Theorem 2: with the theoretical beta of Lemma 3 and r_min below every exact
    neighbour distance, each returned o_i is within c^2 of o*_i with probability at
    least 1/2 - 1/e. Checked with a 99% binomial lower confidence bound."""
    w = wl.SMALL_MIXTURE.scaled(n=2000)
    X, A = w.data(), w.proj()
    idx = oracle.build_index(X, A, w.sample(), w.L, w.K, w.Nr, 32)
    Q = w.queries(300)
    k, c = 5, 1.5
    ids_x, d_x = oracle.knn_exact(X, Q, k)
    eps = oracle.epsilon(w.K, w.L)
    beta = oracle.theoretical_beta(w.K, w.L, c)
    r_min = 0.5 * d_x[:, 0].min()
    ok = 0
    for q, de in zip(Q, d_x):
        res = oracle.query(idx, X, q, k, c, beta, r_min, eps)
        ok += bool(np.all(res.dists <= c * c * de * (1 + 1e-12)))
    lo = stats.beta.ppf(0.01, ok, len(Q) - ok + 1) if ok else 0.0
    assert lo >= 0.5 - 1 / math.e, (ok, lo)
