"""GPU tests of the batching and serving forms and of the radius-schedule autotuner.

* autotune: the tuned schedule is used when r_min <= 0 and matches an explicit call; the
  number of rounds the batched bound kernel resolves never changes a result (checked
  against the oracle for 1 and 8 resolved rounds).
* plans: a HIP-graph replay of a batch with uneven k and c equals the eager call, replay
  after replay, with eager work in between, and after the query buffer is rewritten.
* serving: each result is the same alone and in a mix of concurrently submitted requests,
  and equals the batched call.
"""
import threading

import numpy as np
import pytest

import oracle
from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

from parity import compare_batch  # noqa: E402


@pytest.fixture(scope="module")
def env():
    w = wl.SMALL_MIXTURE
    X, A, sid = w.data(), w.proj(), w.sample()
    print(f"\n[forms] n={len(X)} d={X.shape[1]}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf, lowp=("bf16", "fp8"))
    Q = w.queries()
    return w, X, A, sid, idx, Q, torch.from_numpy(Q).cuda()


def uneven(nq, seed=5):
    rng = np.random.default_rng(seed)
    return (rng.choice([1, 10, 100], size=nq).astype(np.int32),
            rng.choice([1.2, 1.5, 2.0], size=nq).astype(np.float64))


def test_autotune_sets_schedule_and_auto_radius_matches(env):
    w, X, A, sid, idx, Q, Qd = env
    t = idx.autotune(Qd[:64].contiguous(), k=w.k, c=w.c, beta=w.beta)
    print(f"[autotune] {t}", flush=True)
    assert t["r_min"] > 0 and 1 <= t["rounds_resolved"] <= 8
    a_ids, a_d = idx.query(Qd, k=w.k, c=w.c, beta=w.beta, r_min=0.0)
    e_ids, e_d = idx.query(Qd, k=w.k, c=w.c, beta=w.beta, r_min=t["r_min"])
    assert torch.equal(a_ids, e_ids) and torch.equal(a_d, e_d)


@pytest.mark.parametrize("rounds", [1, 8])
def test_rounds_resolved_never_changes_results(env, rounds):
    """Every query against the oracle on the GPU's breakpoints and codes (candidate sets
    element by element); any difference must be a classified near tie."""
    w, X, A, sid, idx, Q, Qd = env
    idx.set_tuning(0.5, rounds)
    eps = oracle.epsilon(w.K, w.L)
    ids, dists, st, cands = idx.query_candidates(Qd, len(X), k=w.k, c=w.c, beta=0.05,
                                                 r_min=0.5, eps=eps)
    ids, dists, st = ids.cpu().numpy(), dists.cpu().numpy(), st.cpu().numpy()
    B = idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
    codes = np.ascontiguousarray(idx.export(pdet.X_CODES)[:, :, :w.K])
    ref = oracle.build_index(X, A, sid, w.L, w.K, w.Nr, w.max_leaf, B=B, codes=codes)
    n_same, n_band, _ = compare_batch(X, ref, Q, range(len(Q)), ids, dists, st, w.k, w.c, 0.05,
                                      0.5, eps, f"rounds={rounds}", cands=cands,
                                      log=lambda m: print(m, flush=True))
    assert n_same + n_band == len(Q) and n_band <= 1
    if rounds == 1:   # the per-query refinement of open leaves runs
        assert st[:, pdet.QSTAT["rounds"]].max() > 2


def test_plan_replays_equal_eager_calls(env):
    w, X, A, sid, idx, Q, Qd = env
    ks, cs = uneven(len(Q))
    Qbuf = Qd.clone()
    plan = idx.plan(Qbuf, k=0, beta=0.05, r_min=3.0, k_per_query=ks, c_per_query=cs,
                    stats=True)
    e_ids, e_d, e_st = idx.query(Qd, k=0, beta=0.05, r_min=3.0, k_per_query=ks,
                                 c_per_query=cs, stats=True)
    for rep in range(3):
        plan.ids.fill_(-7)
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(plan.ids, e_ids) and torch.equal(plan.dists, e_d), rep
        keep = [0, 1, 2, 3, 4, 5, 7, 8, 9]    # word 6 is the query's device time
        assert torch.equal(plan.qstats[:, keep], e_st[:, keep]), rep
        # eager work between replays
        idx.query(Qd[:7].contiguous(), k=5, beta=0.1, r_min=2.0)
        torch.cuda.synchronize()
    # new queries in the same buffer
    Q2 = torch.from_numpy(w.queries(len(Q) + 50)[50:]).cuda()
    Qbuf.copy_(Q2)
    torch.cuda.synchronize()
    plan.launch()
    torch.cuda.synchronize()
    f_ids, f_d = idx.query(Q2, k=0, beta=0.05, r_min=3.0, k_per_query=ks, c_per_query=cs)
    assert torch.equal(plan.ids, f_ids) and torch.equal(plan.dists, f_d)
    plan.close()


def test_reserved_workspace_gives_the_same_results(env):
    w, X, A, sid, idx, Q, Qd = env
    before = idx.query(Qd, k=w.k, c=w.c, beta=0.05, r_min=3.0)
    idx.reserve(4 * len(Q))
    after = idx.query(Qd, k=w.k, c=w.c, beta=0.05, r_min=3.0)
    assert torch.equal(before[0], after[0]) and torch.equal(before[1], after[1])


def test_plan_low_precision_equals_eager(env):
    w, X, A, sid, idx, Q, Qd = env
    ks, cs = uneven(len(Q), seed=11)
    plan = idx.plan(Qd, k=0, beta=0.05, r_min=3.0, k_per_query=ks, c_per_query=cs,
                    precision="bf16", rescore=4)
    e_ids, e_d = idx.query(Qd, k=0, beta=0.05, r_min=3.0, k_per_query=ks, c_per_query=cs,
                           precision="bf16", rescore=4)
    for rep in range(2):
        plan.ids.fill_(-7)
        plan.launch()
        torch.cuda.synchronize()
        assert torch.equal(plan.ids, e_ids) and torch.equal(plan.dists, e_d), rep
    plan.close()


@pytest.mark.parametrize("precision,list_cap", [("fp32", 0), ("bf16", 0), ("fp8", 0),
                                                ("fp32", 4), ("bf16", 4)])
def test_server_results_same_alone_and_in_the_mix(env, precision, list_cap):
    """list_cap 4: the lanes' slots hold 4 leaves per tree, so most batches answer their
    queries again on full-capacity slots before returning them."""
    w, X, A, sid, idx, Q, Qd = env
    ks, cs = uneven(len(Q), seed=9)
    ks = np.minimum(ks, 50)
    ref_ids, ref_d = idx.query(Qd, k=0, beta=0.05, r_min=3.0, k_per_query=ks, c_per_query=cs,
                               precision=precision, rescore=4)
    ref_ids, ref_d = ref_ids.cpu().numpy(), ref_d.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(ks)])
    idx.set_list_cap(list_cap)
    try:
        sv = idx.server(max_batch=16, lanes=2, k_max=50, precision=precision, beta=0.05,
                        r_min=3.0)
    finally:
        idx.set_list_cap(0)
    # alone: one request in flight at a time
    alone = []
    for qi in range(12):
        rid = sv.submit(Q[qi], int(ks[qi]), float(cs[qi]))
        alone.append(sv.wait(rid, int(ks[qi])))
    # mix: two client threads submit everything at once
    rids = [None] * len(Q)

    def client(sl):
        for qi in sl:
            rids[qi] = sv.submit(Q[qi], int(ks[qi]), float(cs[qi]))

    th = [threading.Thread(target=client, args=(range(j, len(Q), 2),)) for j in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    mix = [sv.wait(rids[qi], int(ks[qi])) for qi in range(len(Q))]
    st = sv.stats()
    print(f"[server {precision}] {st}", flush=True)
    sv.close()
    for qi in range(len(Q)):
        np.testing.assert_array_equal(mix[qi][0], ref_ids[off[qi]:off[qi + 1]])
        np.testing.assert_array_equal(mix[qi][1], ref_d[off[qi]:off[qi + 1]])
        if qi < 12:
            np.testing.assert_array_equal(alone[qi][0], mix[qi][0])
            np.testing.assert_array_equal(alone[qi][1], mix[qi][1])
    assert st["completed"] == 12 + len(Q)
    assert st["mean_batch"] > 1.0          # the mix was batched
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_low_precision_copies_past_one_grid_sweep():
    """The bf16 / fp8 copies are written by a grid that strides over the rows (4M rows per
    sweep); at 5M integer-valued rows of d = 16 the bf16 copy is exact, so bf16
    verification returns the float32 path's ids and distances for every query."""
    w = wl.SIFT_LIKE_1M.scaled(n=5_000_000, d=16, nq=100, k=10)
    X = w.data()
    print(f"\n[lowp-sweep] n={len(X)} d={X.shape[1]}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf,
                     lowp=("bf16", "fp8"))
    Qd = torch.from_numpy(w.queries()).cuda()
    t = idx.autotune(Qd[:64].contiguous(), k=w.k, c=w.c, beta=0.001)
    f_ids, f_d = idx.query(Qd, k=w.k, c=w.c, beta=0.001, r_min=t["r_min"])
    b_ids, b_d = idx.query(Qd, k=w.k, c=w.c, beta=0.001, r_min=t["r_min"], precision="bf16",
                           rescore=4)
    assert torch.equal(f_ids, b_ids)
    np.testing.assert_allclose(b_d.cpu().numpy(), f_d.cpu().numpy(), rtol=1e-6)
    # fp8: every returned distance is the exact distance of the returned id (FP32 rescore)
    e_ids, e_d = idx.query(Qd, k=w.k, c=w.c, beta=0.001, r_min=t["r_min"], precision="fp8",
                           rescore=4)
    ids = e_ids.cpu().numpy()
    exact = np.sqrt(((X[ids].astype(np.float64) - w.queries()[:, None, :]) ** 2).sum(-1))
    np.testing.assert_allclose(e_d.cpu().numpy(), exact, rtol=1e-6)
    rec = np.mean([len(np.intersect1d(a, b)) / w.k for a, b in zip(ids, f_ids.cpu().numpy())])
    print(f"[lowp-sweep] fp8 recall@{w.k} against float32: {rec:.3f}", flush=True)
    idx.close()


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_capped_leaf_lists_answer_overflowed_queries_again(env, precision):
    """Query slots whose leaf lists hold only a few entries per tree (as a large index
    gets to fit more slots): queries that overflow them, in the batched bound kernel or in
    the per-query refinement of later rounds, are answered again with full-capacity slots,
    so ids, distances and statistics equal the uncapped call, eagerly and in a plan."""
    w, X, A, sid, idx, Q, Qd = env
    ks, cs = uneven(len(Q), seed=3)
    kw = dict(k=0, beta=0.05, r_min=3.0, k_per_query=ks, c_per_query=cs, precision=precision,
              rescore=4)
    keep = [0, 1, 2, 3, 4, 5, 7, 8, 9]    # word 6 is the query's device time
    idx.set_tuning(3.0, 1)                # later rounds go through the refinement
    ref_ids, ref_d, ref_st = idx.query(Qd, stats=True, **kw)
    pdet.set_timing(True)
    try:
        for cap in (2, 16, 64):
            idx.set_list_cap(cap)
            ids, d, st = idx.query(Qd, stats=True, **kw)
            retried = pdet.get_timing()["query_retried"]
            print(f"[cap] {precision} cap={cap} retried={retried}/{len(Q)}", flush=True)
            assert torch.equal(ids, ref_ids) and torch.equal(d, ref_d), cap
            assert torch.equal(st[:, keep], ref_st[:, keep]), cap
            if cap == 2:
                assert retried > len(Q) // 2
        idx.set_list_cap(16)
        plan = idx.plan(Qd, stats=True, **kw)
        for rep in range(2):
            plan.ids.fill_(-7)
            plan.launch()
            torch.cuda.synchronize()
            assert torch.equal(plan.ids, ref_ids) and torch.equal(plan.dists, ref_d), rep
            assert torch.equal(plan.qstats[:, keep], ref_st[:, keep]), rep
        plan.close()
    finally:
        pdet.set_timing(False)
        idx.set_list_cap(0)


def test_recycled_device_blocks_give_the_same_index_and_results():
    """Indexes large enough that their buffers, build temporaries and query scratch go
    through the library's block cache: a rebuild on recycled blocks (stale contents) gives
    the same breakpoints, codes, leaves and neighbours, in FP32 and BF16."""
    w = wl.SIFT_LIKE_1M.scaled(n=600_000)
    X, A, sid = w.data(), w.proj(), w.sample()
    Qd = torch.from_numpy(w.queries(500)).cuda()
    print(f"\n[cache] n={w.n} d={w.d}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    kw = dict(k=w.k, c=w.c, beta=0.002, r_min=30.0)
    ref = None
    for rep in range(3):
        idx = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf, lowp=("bf16",))
        got = dict(B=idx.export(pdet.X_BREAKPOINTS), codes=idx.export(pdet.X_CODES),
                   leaves=idx.export(pdet.X_LEAF_COUNT, tree=3),
                   f32=[t.cpu() for t in idx.query(Qd, **kw)],
                   bf16=[t.cpu() for t in idx.query(Qd, precision="bf16", rescore=4, **kw)])
        idx.close()
        if ref is None:
            ref = got
            continue
        for key in ("B", "codes", "leaves"):
            assert np.array_equal(got[key], ref[key]), (rep, key)
        for key in ("f32", "bf16"):
            assert all(torch.equal(a, b) for a, b in zip(got[key], ref[key])), (rep, key)
    pdet.release_cache()


def test_theoretical_beta_mode_equals_explicit_beta(env):
    """beta < 0 takes Lemma 3's beta for each query's c: a mixed-c batch equals the same
    queries run with their theoretical beta passed explicitly (c by c)."""
    w, X, A, sid, idx, Q, Qd = env
    ks, cs = uneven(len(Q), seed=21)
    ks = np.minimum(ks, 10).astype(np.int32)
    ids, dists, st = idx.query(Qd, k=0, beta=-1.0, r_min=2.0, k_per_query=ks, c_per_query=cs,
                               stats=True)
    ids, dists = ids.cpu().numpy(), dists.cpu().numpy()
    off = np.concatenate([[0], np.cumsum(ks)])
    for c in (1.2, 1.5, 2.0):
        sel = np.nonzero(cs == c)[0]
        beta = oracle.theoretical_beta(w.K, w.L, c)
        e_ids, e_d = idx.query(Qd[torch.from_numpy(sel).cuda()].contiguous(), k=0, beta=beta,
                               r_min=2.0, k_per_query=ks[sel], c_per_query=cs[sel])
        e_ids, e_d = e_ids.cpu().numpy(), e_d.cpu().numpy()
        eo = np.concatenate([[0], np.cumsum(ks[sel])])
        for j, q in enumerate(sel):
            np.testing.assert_array_equal(ids[off[q]:off[q + 1]], e_ids[eo[j]:eo[j + 1]])
            np.testing.assert_array_equal(dists[off[q]:off[q + 1]], e_d[eo[j]:eo[j + 1]])


def test_autotuned_radius_equals_the_oracle_counterpart(env):
    """The dataset-level r_min of pdet_autotune against the oracle's reading of the magic
    r_min (first radius from the breakpoint ranges, pilots run from it, one grid step below
    the median terminating radius) on the GPU's breakpoints and codes."""
    w, X, A, sid, idx, Q, Qd = env
    pilots = 64
    t = idx.autotune(Qd[:pilots].contiguous(), k=w.k, c=w.c, beta=0.05)
    B = idx.export(pdet.X_BREAKPOINTS).astype(np.float64)
    codes = np.ascontiguousarray(idx.export(pdet.X_CODES)[:, :, :w.K])
    ref = oracle.build_index(X, A, sid, w.L, w.K, w.Nr, w.max_leaf, B=B, codes=codes)
    eps = oracle.epsilon(w.K, w.L)
    r0 = oracle.autotune_first_radius(B, w.K, w.L)
    r = oracle.autotune_r_min(ref, X, Q[:pilots], w.k, w.c, 0.05, eps, r0)
    print(f"[autotune] library r_min={t['r_min']:.9g} oracle r_min={r:.9g}", flush=True)
    assert abs(t["r_min"] - r) <= 1e-9 * r
