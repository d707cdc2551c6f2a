"""GPU parity on the precision-form workload shape: the normed 256-centre mixture at
d = 960 with n reduced to 250,000 (d kept), 1,000 queries, k = 10, c = 1.5, beta = 0.02,
r_min from the autotuner.

  codes, trees  bit-exact outside the band / equal to the oracle's trees on the GPU's codes
  FP32          60 sampled queries (and the batch's first and last) against the oracle on the
                GPU's breakpoints and codes: candidate sets element by element, control
                flow, ids, distances
  BF16 / FP8    verification with an FP32 re-rank of the top 4k: recall@10 against the
                oracle's ids on the same queries, every returned distance exact for its id
"""
import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import workloads as wl
from test_gpu_parity import Case, check_codes, check_trees, compare_queries

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

BETA = 0.02


@pytest.fixture(scope="module")
def d960():
    w = wl.NORMED_1M_D960.scaled(n=250_000)
    cs = Case(w.data(), w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf,
              lowp=("bf16", "fp8"))
    Q = w.queries()
    Qd = torch.from_numpy(Q).cuda()
    t = cs.idx.autotune(Qd[:256].contiguous(), k=w.k, c=w.c, beta=BETA)
    print(f"[d960] autotune {t}", flush=True)
    rng = np.random.default_rng(960)
    sel = sorted(set(rng.choice(len(Q), 60, replace=False).tolist()) | {0, len(Q) - 1})
    return w, cs, Q, Qd, t, sel


def test_d960_codes_and_trees(d960):
    w, cs, Q, Qd, t, sel = d960
    check_codes(cs)
    check_trees(cs)


def test_d960_fp32_sampled_queries(d960):
    w, cs, Q, Qd, t, sel = d960
    cap = int(np.ceil(BETA * len(cs.X))) + w.k + 16 * cs.max_leaf
    ids, dists, st, cands = cs.idx.query_candidates(Qd, cap, k=w.k, c=w.c, beta=BETA,
                                                    r_min=t["r_min"], eps=cs.eps)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    compare_queries(cs, cs.stepwise_oracle(), Q, sel, ids, dists, st, w.k, w.c, BETA,
                    t["r_min"], "d960 fp32", allow_frac=0.05, cands=cands)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
def test_d960_low_precision_recall_and_exact_distances(d960, prec):
    w, cs, Q, Qd, t, sel = d960
    ids, dists = cs.idx.query(Qd, k=w.k, c=w.c, beta=BETA, r_min=t["r_min"], eps=cs.eps,
                              precision=prec, rescore=4)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    idx_or = cs.stepwise_oracle()
    hit = 0
    for qi in sel:
        res = oracle.query(idx_or, cs.X, Q[qi], w.k, w.c, BETA, t["r_min"], cs.eps)
        hit += len(set(ids[qi].tolist()) & set(res.ids.tolist()))
        exact = np.sqrt(((cs.X[ids[qi]].astype(np.float64) - Q[qi].astype(np.float64)) ** 2)
                        .sum(-1))
        np.testing.assert_allclose(dists[qi], exact, rtol=1e-6)
    recall = hit / (w.k * len(sel))
    print(f"[d960 {prec}] recall@{w.k} against the oracle's ids on {len(sel)} queries: "
          f"{recall:.4f}", flush=True)
    assert recall >= 0.9
