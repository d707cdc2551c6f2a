"""GPU parity of the literal query forms (Algorithm 5 with the literal DET Range Query of
Algorithm 3, and the (r,c)-ANN query of Algorithm 4) against the oracle on the GPU's
breakpoints and codes. Per query: |S| and two sums of its ids, the stop rule, the rounds
and the ids and distances must equal the oracle's; a difference is allowed only where a leaf
bound or a point's projected distance lies within 1e-5 relative of a threshold eps*r the
query used (FP32 hash values against the oracle's FP64 ones), or the k-th distance within
1e-5 of c*r, and is counted."""
import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl
from parity import BAND, near_stop_b, set_hashes

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lit():
    w = wl.SMALL_MIXTURE
    X, A, sid = w.data(), w.proj(), w.sample()
    print(f"\n[literal] n={len(X)} d={X.shape[1]}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf)
    B = idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
    codes = np.ascontiguousarray(idx.export(pdet.X_CODES)[:, :, :w.K])
    ref = oracle.build_index(X, A, sid, w.L, w.K, w.Nr, w.max_leaf, B=B, codes=codes)
    H = oracle.project(X, A)
    return w, X, idx, ref, H, oracle.epsilon(w.K, w.L)


def near_literal(ref, H, q, radii, eps):
    """A leaf bound or a projected distance within BAND of some (eps r)^2 used."""
    qp = np.asarray(q, dtype=np.float64) @ ref.A
    t2 = np.array([(eps * r) ** 2 for r in radii])
    for i in range(ref.L):
        sl = slice(i * ref.K, (i + 1) * ref.K)
        lo, hi = ref.boxes[i]
        for v in (oracle.lower_bound_sq(qp[sl], lo, hi), oracle.upper_bound_sq(qp[sl], lo, hi),
                  ((H[:, sl] - qp[sl]) ** 2).sum(axis=1)):
            if np.any(np.abs(v[:, None] - t2[None, :]) <= BAND * t2[None, :]):
                return True
    return False


@pytest.mark.parametrize("k,c,beta,r_min", [(10, 1.5, 0.05, 2.0), (5, 2.0, 0.2, 0.5),
                                            (20, 1.2, 0.0, 3.0)])
def test_literal_query_equals_oracle(lit, k, c, beta, r_min):
    w, X, idx, ref, H, eps = lit
    Q = w.queries(40)
    ids, dists, st = idx.query_literal(torch.from_numpy(Q).cuda(), k=k, c=c, beta=beta,
                                       r_min=r_min, eps=eps)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    same = band = 0
    for qi, q in enumerate(Q):
        res = oracle.query_literal(ref, X, q, k, c, beta, r_min, eps)
        hs, hm = set_hashes(res.cand)
        ok = (st[qi, 1] == res.n_cand and st[qi, 4] == hs and st[qi, 5] == hm
              and st[qi, 2] == {"A": 1, "B": 2}[res.stop] and st[qi, 0] == res.rounds
              and st[qi, 3] == res.leaves)
        if ok:
            np.testing.assert_array_equal(ids[qi], res.ids)
            np.testing.assert_allclose(dists[qi], res.dists, rtol=1e-6)
            same += 1
            continue
        radii = list(oracle.radius_ladder(r_min, c, max(res.rounds, int(st[qi, 0])) + 1))
        assert near_literal(ref, H, q, radii, eps) or near_stop_b(
            X, q, res.cand, k, len(radii), r_min, c), (qi, st[qi], res.n_cand, res.stop, res.rounds)
        band += 1
    print(f"[literal k={k}] identical {same}/{len(Q)}, banded {band}", flush=True)
    assert same >= len(Q) - max(1, len(Q) // 10)


@pytest.mark.parametrize("r,beta", [(1.5, 0.05), (4.0, 0.01), (0.3, 0.5)])
def test_rc_ann_equals_oracle(lit, r, beta):
    w, X, idx, ref, H, eps = lit
    Q = w.queries(40)
    c = 1.5
    ids, dists, st = idx.rc_ann(torch.from_numpy(Q).cuda(), r, c=c, beta=beta, eps=eps)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    same = band = nones = 0
    for qi, q in enumerate(Q):
        oid, od, n_c, trees = oracle.rc_ann_query(ref, X, q, c, r, beta, eps)
        want = -1 if oid is None else oid
        nones += oid is None
        if ids[qi] == want and st[qi, 1] == n_c:
            if oid is not None:
                assert abs(dists[qi] - od) <= 1e-6 * od
            else:
                assert np.isinf(dists[qi]) and st[qi, 2] == 0
            same += 1
            continue
        assert near_literal(ref, H, q, [r], eps) or (oid is not None and abs(od - c * r) <= BAND * c * r), qi
        band += 1
    print(f"[rc-ann r={r}] identical {same}/{len(Q)} (none: {nones}), banded {band}", flush=True)
    assert same >= len(Q) - max(1, len(Q) // 10)
