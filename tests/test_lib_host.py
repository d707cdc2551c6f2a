"""Host-side checks of libpdet: it loads, exports every symbol pdet.h declares, and its
host logic (parameter checks, eps from Eq. 2) is right. No GPU compute is called."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "pdet.h")) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(pdet_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    syms = declared_symbols()
    assert set(syms) == set(pdet.EXPORTED), syms
    L = pdet.lib()
    for s in syms:
        assert hasattr(L, s), s


@pytest.mark.parametrize("K,L", [(16, 4), (16, 1), (16, 16), (8, 2), (5, 3), (1, 1)])
def test_epsilon_matches_eq2(K, L):
    assert abs(pdet.epsilon(K, L) - oracle.epsilon(K, L)) < 1e-9 * oracle.epsilon(K, L)


def test_epsilon_invalid():
    assert math.isnan(pdet.epsilon(0, 4))


def _params(**kw):
    proj = np.zeros((8, 64), dtype=np.float32)
    ids = np.arange(256, dtype=np.int64)
    base = dict(K=16, L=4, Nr=256, max_leaf=128, proj=proj.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                sample_ids=ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_sample=256,
                lowp_copies=0)
    base.update(kw)
    return pdet.BuildParams(**base), (proj, ids)


@pytest.mark.parametrize("kw,n,d", [
    (dict(K=17), 1000, 8), (dict(K=0), 1000, 8), (dict(L=0), 1000, 8), (dict(L=17), 1000, 8),
    (dict(Nr=100), 1000, 8), (dict(Nr=512), 1000, 8), (dict(Nr=1), 1000, 8),
    (dict(max_leaf=0), 1000, 8), (dict(n_sample=100), 1000, 8), (dict(n_sample=2000), 1000, 8),
    (dict(lowp_copies=8), 1000, 8), ({}, 0, 8), ({}, 1000, 0),
])
def test_build_rejects_invalid_arguments_before_touching_the_device(kw, n, d):
    p, keep = _params(**kw)
    h = ctypes.c_void_p(1234)
    st = pdet.lib().pdet_build(ctypes.c_void_p(4096), n, d, ctypes.byref(p), None, ctypes.byref(h))
    assert st == pdet.PDET_EINVAL
    assert h.value is None
    assert pdet.lib().pdet_last_error()


def test_build_rejects_sizes_beyond_the_packed_leaf_ids():
    p, keep = _params()
    h = ctypes.c_void_p()
    st = pdet.lib().pdet_build(ctypes.c_void_p(4096), 1 << 28, 8, ctypes.byref(p), None,
                               ctypes.byref(h))
    assert st == pdet.PDET_EUNSUPPORTED and h.value is None


def test_build_rejects_out_of_range_sample_ids():
    p, keep = _params()
    keep[1][7] = 5000
    h = ctypes.c_void_p()
    st = pdet.lib().pdet_build(ctypes.c_void_p(4096), 1000, 8, ctypes.byref(p), None, ctypes.byref(h))
    assert st == pdet.PDET_EINVAL and b"sample id" in pdet.lib().pdet_last_error()


def test_null_handles_are_rejected():
    q = pdet.QueryParams(10, 1.5, None, None, 0.1, 1.0, 0.0, 0, 4)
    assert pdet.lib().pdet_query(None, None, 1, ctypes.byref(q), None, None, None, None) == pdet.PDET_EINVAL
    assert pdet.lib().pdet_info(None, None) == pdet.PDET_EINVAL
    assert pdet.lib().pdet_export(None, 0, 0, None, 0) == pdet.PDET_EINVAL
    assert pdet.lib().pdet_reserve(None, 16, None) == pdet.PDET_EINVAL
    assert pdet.lib().pdet_set_list_cap(None, 0) == pdet.PDET_EINVAL
    pdet.release_cache()   # nothing cached on a host without a device: no device call
    pdet.lib().pdet_free(None)


def test_threaded_generation_reproduces_the_serial_draw(monkeypatch):
    """Chunks carry their own generators: drawing them on several threads gives the same
    rows as one thread (large workloads are generated this way)."""
    from paper_2603_24920_amd import workloads as wl
    monkeypatch.setattr(wl, "CHUNK_ROWS", 1000)
    w = wl.SIFT_LIKE_100M.scaled(n=7_500)
    seen = []
    a = w.data()
    b = w.data(threads=4, progress=lambda done, total: seen.append((done, total)))
    assert np.array_equal(a, b)
    assert seen[-1] == (8, 8) and len(seen) == 8


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; --gpus 2 exits with status 2 and says why, before it
    imports torch or touches a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


@pytest.mark.parametrize("L", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("c", [1.2, 1.5, 2.0])
def test_theoretical_beta_matches_lemma3(L, c):
    """The library's theoretical beta (Lemma 3) against the oracle's (SciPy chi2)."""
    want = oracle.theoretical_beta(16, L, c)
    assert abs(pdet.theoretical_beta(16, L, c) - want) <= 1e-9 * max(want, 1e-12)


def test_theoretical_beta_invalid():
    assert math.isnan(pdet.theoretical_beta(16, 4, 1.0))
    assert math.isnan(pdet.theoretical_beta(0, 4, 1.5))


def test_normal_quantile_matches_scipy():
    """The static encoding's Phi^-1 (bisection + Newton on erfc) against SciPy's ppf at the
    quantiles it uses (u / Nr) and in the tails."""
    from scipy.stats import norm
    ps = [u / 256 for u in range(1, 256)] + [1e-12, 1e-6, 0.3, 0.7, 1 - 1e-6]
    for p in ps:
        want = norm.ppf(p)
        got = pdet.normal_quantile(p)
        assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (p, got, want)
    assert pdet.normal_quantile(0.5) == 0.0
    for bad in (0.0, 1.0, -0.5, 2.0, float("nan")):
        assert math.isnan(pdet.normal_quantile(bad))


def test_build_rejects_unknown_encoding():
    p, keep = _params(encoding=2)
    h = ctypes.c_void_p()
    st = pdet.lib().pdet_build(ctypes.c_void_p(4096), 1000, 8, ctypes.byref(p), None,
                               ctypes.byref(h))
    assert st == pdet.PDET_EINVAL and b"encoding" in pdet.lib().pdet_last_error()


def test_draw_params_is_seeded_and_has_the_stated_shapes():
    p1, s1 = pdet.draw_params(100000, 64, 4, 16, Nr=64, sample_frac=0.1, seed=7)
    p2, s2 = pdet.draw_params(100000, 64, 4, 16, Nr=64, sample_frac=0.1, seed=7)
    p3, s3 = pdet.draw_params(100000, 64, 4, 16, Nr=64, sample_frac=0.1, seed=8)
    assert p1.shape == (64, 64) and p1.dtype == np.float32
    assert np.array_equal(p1, p2) and np.array_equal(s1, s2)
    assert not np.array_equal(p1, p3) and not np.array_equal(s1, s3)
    # min(n, max(ceil(frac * n), Nr^2)) distinct ids, ascending, in range
    assert len(s1) == 10000
    assert np.all(np.diff(s1) > 0) and s1[0] >= 0 and s1[-1] < 100000
    _, s = pdet.draw_params(100000, 8, 1, 1, Nr=256, sample_frac=0.01, seed=1)
    assert len(s) == 256 * 256
    _, s = pdet.draw_params(1000, 8, 1, 1, Nr=256, sample_frac=0.5, seed=1)
    assert np.array_equal(s, np.arange(1000))
    _, s = pdet.draw_params(5000, 8, 1, 1, Nr=2, sample_frac=1.0, seed=3)
    assert np.array_equal(s, np.arange(5000))


def test_drawn_projection_entries_are_standard_normal():
    # Eq. 1 asks for i.i.d. N(0, 1) entries: Kolmogorov-Smirnov against the normal law
    from scipy import stats
    proj, _ = pdet.draw_params(1000, 512, 16, 16, seed=11)
    v = proj.astype(np.float64).ravel()
    assert stats.kstest(v, "norm").pvalue > 1e-3
    assert abs(v.mean()) < 0.01 and abs(v.var() - 1.0) < 0.01
    # neighbouring entries (the two outputs of one Box-Muller pair) are uncorrelated
    assert abs(np.corrcoef(v[0::2], v[1::2])[0, 1]) < 0.01


def test_drawn_sample_is_uniform_over_the_ids():
    # every id is drawn with probability m / n; over 400 seeds the counts follow a binomial law
    n, m, runs = 2000, 100, 400
    hits = np.zeros(n)
    for seed in range(runs):
        _, s = pdet.draw_params(n, 4, 1, 1, Nr=8, sample_frac=m / n, seed=seed)
        assert len(s) == m and len(np.unique(s)) == m
        hits[s] += 1
    from scipy import stats
    expect = runs * m / n
    chi2 = ((hits - expect) ** 2 / expect).sum()
    assert stats.chi2.sf(chi2, n - 1) > 1e-3
    # halves of the id range are drawn equally often (no bias toward the Floyd tail)
    assert abs(hits[: n // 2].sum() - hits[n // 2:].sum()) < 4 * math.sqrt(runs * m)


def test_draw_params_rejects_invalid_arguments():
    L = pdet.lib()
    m = ctypes.c_int64()
    for args in [(0, 8, 1, 1, 256, 0.1), (1000, 0, 1, 1, 256, 0.1), (1000, 8, 17, 1, 256, 0.1),
                 (1000, 8, 1, 0, 256, 0.1), (1000, 8, 1, 1, 1, 0.1), (1000, 8, 1, 1, 256, 0.0),
                 (1000, 8, 1, 1, 256, 1.5), (1000, 8, 1, 1, 256, float("nan"))]:
        assert L.pdet_draw_params(*args, 0, None, None, ctypes.byref(m)) == pdet.PDET_EINVAL, args


def test_build_without_sample_ids_needs_a_sample_fraction():
    p, keep = _params(sample_ids=None, n_sample=0, sample_frac=0.0)
    h = ctypes.c_void_p(1234)
    st = pdet.lib().pdet_build(ctypes.c_void_p(4096), 1000, 8, ctypes.byref(p), None, ctypes.byref(h))
    assert st == pdet.PDET_EINVAL


def test_insert_rejects_null_arguments_before_touching_the_device():
    L = pdet.lib()
    assert L.pdet_insert(None, ctypes.c_void_p(4096), 10, None) == pdet.PDET_EINVAL
