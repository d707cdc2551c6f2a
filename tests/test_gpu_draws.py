"""Builds that leave the projection and the sample to the library (Eq. 1 entries and the
sampled ids of the encoding phase, Section 3.1, drawn from a seed), and the build's check
for non-finite data."""
import numpy as np
import pytest

from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl
from test_gpu_parity import Case, check_breakpoints, check_codes, check_trees, run_and_compare

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SEED, FRAC = 20260314, 0.2


@pytest.fixture(scope="module")
def drawn():
    # 16 regions: the sample (ceil(0.2 n) = 2,000 ids, above the Nr^2 floor) is a strict subset
    w = wl.SMALL_MIXTURE.scaled(Nr=16)
    X = w.data()
    Xd = torch.from_numpy(X).cuda()
    print(f"\n[drawn] n={len(X)} d={X.shape[1]} K={w.K} L={w.L} seed={SEED} frac={FRAC}",
          flush=True)
    idx = pdet.Index(Xd, None, None, w.K, w.L, w.Nr, w.max_leaf, sample_frac=FRAC, seed=SEED)
    torch.cuda.synchronize()
    A, sid = pdet.draw_params(len(X), X.shape[1], w.L, w.K, w.Nr, FRAC, SEED)
    cs = Case(X, A, sid, w.K, w.L, w.Nr, w.max_leaf)
    return w, idx, cs


def test_drawn_parameters_are_the_exported_ones(drawn):
    w, idx, cs = drawn
    np.testing.assert_array_equal(idx.export(pdet.X_PROJ), cs.A)
    np.testing.assert_array_equal(idx.export(pdet.X_SAMPLE), cs.sid)
    assert idx.info()["n_sample"] == len(cs.sid) == int(np.ceil(FRAC * len(cs.X)))
    # a build given the parameters exports them unchanged
    np.testing.assert_array_equal(cs.idx.export(pdet.X_PROJ), cs.A)
    np.testing.assert_array_equal(cs.idx.export(pdet.X_SAMPLE), cs.sid)


def test_drawn_build_equals_the_build_given_its_draws(drawn):
    w, idx, cs = drawn
    np.testing.assert_array_equal(idx.export(pdet.X_BREAKPOINTS), cs.B_gpu.astype(np.float32))
    np.testing.assert_array_equal(idx.export(pdet.X_CODES)[:, :, :w.K], cs.codes_gpu)
    for t in range(w.L):
        for what in (pdet.X_LEAF_START, pdet.X_LEAF_COUNT, pdet.X_LEAF_HIDX):
            np.testing.assert_array_equal(idx.export(what, t), cs.idx.export(what, t))
    check_breakpoints(cs)
    check_codes(cs)
    check_trees(cs)


def test_drawn_build_queries_match_the_oracle(drawn):
    w, idx, cs = drawn
    own = cs.idx
    cs.idx = idx
    try:
        run_and_compare(cs, cs.stepwise_oracle(), w.queries(), w.k, w.c, 0.1, 4.0, "drawn")
    finally:
        cs.idx = own


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
def test_build_rejects_non_finite_data(bad):
    rng = np.random.default_rng(5)
    X = rng.standard_normal((3000, 32)).astype(np.float32)
    X[1777, 9] = bad
    Xd = torch.from_numpy(X).cuda()
    print(f"\n[non-finite] value={bad} n=3000 d=32", flush=True)
    with pytest.raises(pdet.PdetError) as e:
        pdet.Index(Xd, None, None, K=8, L=2, Nr=16, max_leaf=32, sample_frac=0.5, seed=1)
    assert e.value.status == pdet.PDET_EINVAL and "non-finite" in str(e.value)
    # the library is still usable afterwards
    X[1777, 9] = 0.0
    idx = pdet.Index(torch.from_numpy(X).cuda(), None, None, K=8, L=2, Nr=16, max_leaf=32,
                     sample_frac=0.5, seed=1)
    ids, dists = idx.query(torch.from_numpy(X[:4]).cuda(), k=1, c=1.5, beta=1.0, r_min=1.0,
                               eps=pdet.epsilon(8, 2))
    assert np.array_equal(ids.cpu().numpy()[:, 0], np.arange(4))
