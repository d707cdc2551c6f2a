"""Pins of the oracle's parameter and schedule functions (Section 5.2) and of the static
encoding variant (Section 3.1), against closed forms, textbook values and the query loop."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2603_24920_amd import workloads as wl


def test_static_breakpoints_are_normal_quantiles():
    """Static iSAX breakpoints: equal-mass N(0,1) quantiles, here on a column normalised to
    mean 10 and standard deviation 3. Phi^-1(0.75) = 0.6744897501960817 (textbook value)."""
    col = np.array([7.0, 13.0] * 50)[:, None]          # mean 10, population std 3
    B = oracle.static_breakpoints(col, 4, col.min(axis=0), col.max(axis=0))
    q75 = 0.6744897501960817
    np.testing.assert_allclose(B[0], [7.0, 10 - 3 * q75, 10.0, 10 + 3 * q75, 13.0], rtol=0,
                               atol=1e-12)


def test_static_breakpoints_equalise_gaussian_columns_only():
    """On Gaussian columns the static scheme gives near-equal region counts; on a skewed
    column (exponential) it does not, while the dynamic scheme does (the contrast the
    encoding phase draws)."""
    rng = np.random.default_rng(3)
    n, Nr = 40_000, 16
    G = rng.normal(5.0, 2.0, size=(n, 1))
    E = rng.exponential(1.0, size=(n, 1))
    for H, gaussian in ((G, True), (E, False)):
        Bs = oracle.static_breakpoints(H, Nr, H.min(axis=0), H.max(axis=0))
        Bd = oracle.breakpoints(H, Nr, H.min(axis=0), H.max(axis=0))
        cs = np.bincount(oracle.encode(H, Bs, 1, 1)[0, :, 0], minlength=Nr)
        cd = np.bincount(oracle.encode(H, Bd, 1, 1)[0, :, 0], minlength=Nr)
        chi_s = ((cs - n / Nr) ** 2 / (n / Nr)).sum()
        chi_d = ((cd - n / Nr) ** 2 / (n / Nr)).sum()
        assert stats.chi2(Nr - 1).sf(chi_d) > 0.5            # dynamic: equal by construction
        if gaussian:
            assert stats.chi2(Nr - 1).sf(chi_s) > 1e-3
        else:
            assert stats.chi2(Nr - 1).sf(chi_s) < 1e-12


@pytest.fixture(scope="module")
def small():
    w = wl.SMALL_MIXTURE.scaled(n=3000)
    X, A = w.data(), w.proj()
    idx = oracle.build_index(X, A, w.sample(), w.L, w.K, w.Nr, 32)
    return w, X, idx


def test_candidate_count_is_the_closed_form_union(small):
    """|S| at radius r = #points whose leaf in some tree has LB <= eps r (per point)."""
    w, X, idx = small
    eps = oracle.epsilon(w.K, w.L)
    for q in w.queries(4):
        qp = q.astype(np.float64) @ idx.A
        lbp = np.empty((w.L, len(X)))
        for i in range(w.L):
            t, (lo, hi) = idx.trees[i], idx.boxes[i]
            lb2 = oracle.lower_bound_sq(qp[i * w.K:(i + 1) * w.K], lo, hi)
            leaf_of = np.repeat(np.arange(t.nl), t.leaf_count)
            lbp[i, t.perm] = lb2[leaf_of]
        for r in (0.5, 1.0, 2.0, 4.0):
            assert oracle.candidate_count(idx, q, r, eps) == int(np.sum(lbp.min(axis=0) <= (eps * r) ** 2))


def test_magic_r_min_is_the_round_where_stop_rule_a_fires(small):
    """The magic r_min (Section 5.2.1) on the grid r0*c^j: a query started at r0 that stops
    by rule A in round rho has magic index j = rho (|S| first reaches beta n + k there)."""
    w, X, idx = small
    eps = oracle.epsilon(w.K, w.L)
    k, c, beta, r0 = 10, 1.5, 0.05, 0.05
    seen = 0
    for q in w.queries(20):
        res = oracle.query(idx, X, q, k, c, beta, r0, eps)
        j, r = oracle.magic_r_min(idx, q, k, beta, c, eps, r0)
        T = math.ceil(beta * len(X)) + k
        assert oracle.candidate_count(idx, q, r, eps) >= T
        if j > 0:
            assert oracle.candidate_count(idx, q, r / c, eps) < T
        if res.stop == "A":
            assert j == res.rounds - 1
            seen += 1
        else:
            assert j >= res.rounds - 1      # stop rule B came first
    assert seen > 0


def test_autotune_radius_is_one_step_below_the_median_terminating_radius(small):
    w, X, idx = small
    eps = oracle.epsilon(w.K, w.L)
    pilots = w.queries(9)
    r0 = oracle.autotune_first_radius(idx.B, w.K, w.L)
    rounds = sorted(oracle.query(idx, X, q, 10, 1.5, 0.05, r0, eps).rounds for q in pilots)
    r = oracle.autotune_r_min(idx, X, pilots, 10, 1.5, 0.05, eps, r0)
    assert r == pytest.approx(r0 * 1.5 ** max(0, rounds[4] - 2), rel=1e-12)
    rng = np.sort(idx.B[:, -1] - idx.B[:, 0])
    assert r0 == pytest.approx(1e-4 * rng[len(rng) // 2] / eps, rel=1e-15)


def test_theoretical_beta_per_c():
    b = oracle.theoretical_beta_for(16, 4, [1.2, 1.5, 2.0])
    np.testing.assert_allclose(b, [oracle.theoretical_beta(16, 4, c) for c in (1.2, 1.5, 2.0)],
                               rtol=0, atol=0)
    assert b[0] > b[1] > b[2] > 0          # beta falls as c grows (Figure "betal", Lemma 3)
