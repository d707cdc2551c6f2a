"""GPU parity at full benchmark size: sift-like-1M-d128.

Workload: n = 1,000,000, d = 128, L = 4, K = 16, 256 regions, 10,000 queries, k = 50,
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
    ids, dists, st = cs.idx.query(Qd, k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], stats=True)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    compare_queries(cs, cs.stepwise_oracle(), Q, sel, ids, dists, st, w.k, w.c, BETA,
                    t["r_min"], "full fp32", allow_frac=0.02)
    # every query of the batch: ids distinct, distances ascending and exact for its ids
    assert np.all(np.diff(dists, axis=1) >= 0)
    assert all(len(set(r)) == w.k for r in ids[::97])
    exact = np.sqrt(((cs.X[ids[::97]].astype(np.float64)
                      - Q[::97, None, :].astype(np.float64)) ** 2).sum(-1))
    np.testing.assert_allclose(dists[::97], exact, rtol=1e-6)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_full_batch_low_precision_recall(full, prec):
    w, cs, Q, Qd, t, sel = full
    ids, dists = cs.idx.query(Qd, k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], precision=prec,
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
