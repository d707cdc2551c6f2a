#!/usr/bin/env python3
"""Benchmark of the DET-LSH hot path on one MI355X.

One step = build the index over the resident data (sample projection, breakpoints,
projection + encoding of every point, the L DE-Trees) + answer the whole query batch
(c^2-k-ANN with FP32 verification). Default workload: the 100M-point batching
configuration (SIFT-like bytes, n = 100,000,000, d = 128, L = 4, K = 16, Nr = 256,
10,000 queries, k = 10, c = 1.5; about 51 GB resident), followed by secondary blocks on
the 1M-point configuration (10,000 queries, k = 50; with the literal query form beside the
optimised one, the (encoding, L, K) study and online insertion of 1k / 10k / 100k points into
an index of the remaining rows) and the 10M-point serving configuration (d = 256, unit-norm rows, FP8 and
FP32 verification under Poisson load).

Per workload, before the timed steps (untimed): ground truth for recall@10 is FP64 brute
force over every point for the first --recall-queries queries; the stop-rule parameter
beta is the smallest value of a ladder whose mean recall@10 reaches 0.9 there, per
verification form, with r_min picked per beta by the library's pilot search.

Prints one JSON line. `value` is queries/s of the FP32 query phase of the primary workload
(inputs resident in HBM); `build_mpts_per_s` is n / build time. `roofline` describes the
search kernel q_main_f32 (timed live with HIP events on the library's stream), `roofline_build`
the whole build; `cpu_baseline` is the FP64 oracle on the host (a bounded sample).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "index build Mpts/s + QPS at recall@10>=0.9 (FP32 vs BF16/FP8 verify), 1 GPU"
HBM_PEAK_GBS = 8000.0
BETA_LADDER = (0.1, 0.05, 0.02, 0.01, 0.005, 0.002, 0.001, 7e-4, 5e-4, 3.5e-4, 2.5e-4, 1.8e-4,
               1.3e-4, 1e-4, 7e-5, 5e-5, 3.5e-5, 2.5e-5, 1.8e-5, 1.3e-5, 1e-5)
GEN_THREADS_N = 4_000_000     # from this size: data drawn in parallel chunks (same values)
MAX_CAL_CANDIDATES = 2e5      # largest beta * n tried by the recall calibration
POOL = 16                     # host worker processes (the GPU machine's CPU share)
LITERAL_MAX_N = 4_000_000     # largest index on which the literal query form is timed
# parameter study on indexes up to this size: (encoding, L, K) per configuration
STUDY_MAX_N = 4_000_000
INSERT_MAX_N = 4_000_000      # largest index grown by online insertion in the benchmark
INSERT_BATCHES = (1_000, 10_000, 100_000)
STUDY = (("dynamic", 4, 16), ("static", 4, 16), ("dynamic", 2, 16), ("dynamic", 8, 16),
         ("dynamic", 4, 8), ("dynamic", 4, 12))
# per workload: low-precision forms measured, and the form of the graph-launched batch
FORMS = {"sift-like-100M-d128": (("bf16",), "bf16"), "sift-like-1M-d128": (("bf16", "fp8"), "fp32"),
         "normed-1M-d960": (("bf16",), "bf16"), "normed-10M-d256": (("fp8",), "fp8"),
         "mixture-10k-d128": (("bf16", "fp8"), "fp32")}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def recall_at(ids, exact, r=10):
    ids, exact = np.asarray(ids)[:, :r], np.asarray(exact)[:, :r]
    return float(np.mean([len(np.intersect1d(a, b)) / r for a, b in zip(ids, exact)]))


def brute_force_knn(Xd, Qd, k, rows=1 << 18):
    """Exact k nearest neighbours by FP64 distances over row chunks of the resident data
    (torch FP64 matrix products on the device; evaluation only, never the library)."""
    import torch
    q = Qd.double()
    qn = (q * q).sum(1, keepdim=True)
    best_d = torch.full((q.shape[0], k), float("inf"), dtype=torch.float64, device=q.device)
    best_i = torch.zeros((q.shape[0], k), dtype=torch.int64, device=q.device)
    for r0 in range(0, Xd.shape[0], rows):
        x = Xd[r0:r0 + rows].double()
        d2 = qn - 2.0 * (q @ x.T) + (x * x).sum(1)[None, :]
        dv, di = torch.topk(d2, min(k, x.shape[0]), dim=1, largest=False)
        cat_d = torch.cat([best_d, dv], 1)
        cat_i = torch.cat([best_i, di + r0], 1)
        o = torch.argsort(cat_d, dim=1, stable=True)[:, :k]
        best_d, best_i = torch.gather(cat_d, 1, o), torch.gather(cat_i, 1, o)
    return best_i.cpu().numpy()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("query.hip", "devutil.h", "internal.h", "common.h"):
        with open(os.path.join(ROOT, "paper_2603_24920_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_traffic(workload_name, nq):
    """HBM traffic of q_main_f32 per launch from committed rocprofv3 counter runs on this
    workload (profiles/q_main_traffic_<workload>.json), or None if absent, taken on another
    batch or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", f"q_main_traffic_{workload_name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        p = json.load(f)
    if p.get("kernel_hash") != kernel_source_hash() or p.get("nq") != nq:
        return None
    return p.get("traffic_bytes_per_launch")


def measure(w, args, primary, helper=None):
    """Everything measured on one workload; returns a dict (the primary one becomes the line)."""
    import torch
    from paper_2603_24920_amd import pdet
    from paper_2603_24920_amd import workloads as wl

    lowp_forms, plan_prec = FORMS.get(w.name, (("bf16",), "fp32"))
    if args.no_lowp:
        lowp_forms = ()
    if args.plan_precision:
        plan_prec = args.plan_precision
    if plan_prec != "fp32" and plan_prec not in lowp_forms:
        lowp_forms = tuple(lowp_forms) + (plan_prec,)
    nq = args.nq or w.nq
    t0 = time.time()
    big = w.n >= GEN_THREADS_N

    def gen_progress(done, total):
        if big and (done % 16 == 0 or done == total):
            log(f"[bench] generating {w.name}: {done}/{total} chunks ({time.time() - t0:.0f}s)")

    X = w.data(threads=POOL if big else 1, progress=gen_progress)
    A, sid, Q = w.proj(), w.sample(), w.queries(nq)
    log(f"[bench] generated {w.name}: n={w.n} d={w.d} nq={nq} ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    torch.cuda.synchronize()
    log(f"[bench] data resident on the device ({time.time() - t0:.1f}s)")
    pdet.set_timing(True)

    # ---- untimed calibration: index, ground truth, beta / r_min per recall target
    idx = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf, lowp=tuple(lowp_forms))
    nrec = min(args.recall_queries, nq)
    Qr = Qd[:nrec].contiguous()
    Qp = Qd[:256].contiguous()
    exact_ids = None
    if not args.no_recall:
        exact_ids = brute_force_knn(Xd, Qr, 10)
        log(f"[bench] FP64 brute-force ground truth for {nrec} queries ({time.time() - t0:.1f}s)")

    def calibrate(precision):
        """(beta, r_min, rounds resolved, recall@10) at the smallest beta reaching 0.9. At
        each beta (descending) the radius schedule autotuned for it and the one accepted at
        the previous beta are both tried; the one with the higher recall is kept."""
        if args.no_recall:
            if args.beta is None or args.r_min is None:
                raise SystemExit("--no-recall needs --beta and --r-min")
            return args.beta, args.r_min, args.rcap, None

        def at(beta, tuning=None):
            if args.r_min is not None:
                tuning = (args.r_min, args.rcap)
            if tuning is None:
                t = idx.autotune(Qp, k=w.k, c=w.c, beta=beta, precision=precision)
                tuning = (t["r_min"], t["rounds_resolved"])
            idx.set_tuning(*tuning)
            ids, _ = idx.query(Qr, k=w.k, c=w.c, beta=beta, r_min=tuning[0],
                               precision=precision, rescore=4)
            rec = recall_at(ids.cpu().numpy(), exact_ids)
            log(f"[bench] {w.name} {precision} beta={beta} r_min={tuning[0]:.4g} "
                f"rounds_resolved={tuning[1]} recall@10={rec:.4f}")
            return beta, tuning[0], tuning[1], rec

        if args.beta is not None:
            return at(args.beta)
        chosen = None
        for beta in BETA_LADDER:
            if beta * w.n > MAX_CAL_CANDIDATES and beta != BETA_LADDER[-1]:
                continue   # a calibration batch at this beta would verify too many rows
            res = at(beta)
            if chosen is not None and args.r_min is None and res[1] != chosen[1]:
                alt = at(beta, (chosen[1], chosen[2]))
                if alt[3] > res[3]:
                    res = alt
            if res[3] >= 0.9:
                chosen = res
            else:
                break
        if chosen is None:
            raise SystemExit("no beta on the ladder reaches recall@10 >= 0.9")
        return chosen

    beta, r_min, rcap, rec = calibrate("fp32")
    lowp_cal = {f: calibrate(f) for f in lowp_forms}
    idx.close()
    del idx
    torch.cuda.synchronize()

    # ---- timed steps: build + query batch (FP32 verification)
    def step(record):
        torch.cuda.synchronize()
        tb = time.perf_counter()
        ix = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf)
        torch.cuda.synchronize()
        tbt = pdet.get_timing()
        ix.set_tuning(r_min, rcap)
        # query scratch sized once for the batch, as a serving process does before traffic;
        # its initialisation (the round table's fill) is queued on the stream, so wait for it
        # here, or it is charged to the query
        tr = time.perf_counter()
        ix.reserve(nq)
        torch.cuda.synchronize()
        tq = time.perf_counter()
        ids, dists, st = ix.query(Qd, k=w.k, c=w.c, beta=beta, r_min=r_min, stats=True)
        torch.cuda.synchronize()
        te = time.perf_counter()
        tqt = pdet.get_timing()
        if record is not None:
            s = st.cpu().numpy()
            record.append(dict(build_s=tr - tb, reserve_s=tq - tr, query_s=te - tq, tb=tbt, tq=tqt,
                               ncand=int(s[:, 1].astype(np.int64).sum()), stops=s[:, 2],
                               qtime=s[:, 6], visits=s[:, 7], band_leaf=s[:, 8], band_b=s[:, 9],
                               khz=ix.info()["wall_clock_khz"]))
        ix.close()

    for _ in range(args.warmup):
        step(None)
    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step(recs)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    log(f"[bench] {w.name}: {args.steps} timed steps in {total:.2f}s")
    bad = sum(int(np.sum(r["stops"] < 0)) for r in recs)
    if bad:
        raise SystemExit(f"{bad} queries ended without a stop rule (stop < 0)")
    build_s = float(np.mean([r["build_s"] for r in recs]))
    query_s = float(np.mean([r["query_s"] for r in recs]))
    qps = nq / query_s

    # roofline of q_main: algorithmic bytes = sum_q |S_q| (4d + 4) + (L-1) 4 |S_q|
    ncand = float(np.mean([r["ncand"] for r in recs]))
    main_ms = float(np.mean([r["tq"]["query_main_ms"] / max(1, r["tq"]["query_main_launches"])
                             for r in recs]))
    launches = int(recs[-1]["tq"]["query_main_launches"])
    bytes_alg = ncand * (4 * w.d + 4 + 4 * (w.L - 1)) / max(1, launches)
    achieved = bytes_alg / (main_ms * 1e-3) / 1e9
    traffic = pmc_traffic(w.name, nq)
    enc_ms = float(np.mean([r["tb"]["build_encode_ms"] for r in recs]))
    enc_bytes = w.n * (4 * w.d + 16 * w.L + 2 * w.L)   # row read; code rows and keys written
    build_bpp = 4 * w.d + 2 * w.L * w.K + 4 * w.L     # read x, write + read codes, write perm
    build_gbs = w.n * build_bpp / build_s / 1e9
    bstage = {k: float(np.mean([r["tb"][k] for r in recs]))
              for k in ("build_sample_ms", "build_sort_ms", "build_encode_ms", "build_tree_ms")}

    # resident index with every low-precision copy for the forms below (query phase only)
    ix = pdet.Index(Xd, A, sid, w.K, w.L, w.Nr, w.max_leaf, lowp=tuple(lowp_forms))

    def timed(fn):
        ts = []
        for it in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if it >= args.warmup:
                ts.append(time.perf_counter() - t1)
        return float(np.mean(ts))

    # precision forms at their own recall-matched beta
    lowp = {}
    for f, (lb, lr, lc, lrec) in lowp_cal.items():
        ix.set_tuning(lr, lc)
        sec = timed(lambda: ix.query(Qd, k=w.k, c=w.c, beta=lb, r_min=lr, precision=f,
                                     rescore=4))
        lowp[f] = dict(beta=lb, r_min=lr, rounds_resolved=lc, recall_at_10=lrec, qps=nq / sec,
                       rescore=4, speedup_vs_fp32=(nq / sec) / qps)
        log(f"[bench] {w.name} {f}: {lowp[f]}")

    # Algorithm 5 as printed (literal range query, every round over every tree) beside the
    # optimised query at the same beta, r_min and eps, on the recall queries
    literal = None
    if not args.no_literal and w.n <= LITERAL_MAX_N and exact_ids is not None:
        ix.set_tuning(r_min, rcap)
        sec_l = timed(lambda: ix.query_literal(Qr, k=w.k, c=w.c, beta=beta, r_min=r_min))
        lids, _, lst = ix.query_literal(Qr, k=w.k, c=w.c, beta=beta, r_min=r_min)
        sec_o = timed(lambda: ix.query(Qr, k=w.k, c=w.c, beta=beta, r_min=r_min))
        oids, _, ost = ix.query(Qr, k=w.k, c=w.c, beta=beta, r_min=r_min, stats=True)
        lst, ost = lst.cpu().numpy(), ost.cpu().numpy()
        literal = dict(queries=nrec, beta=beta, r_min=r_min,
                       qps_literal=nrec / sec_l, qps_optimised=nrec / sec_o,
                       speedup_optimised=sec_l / sec_o,
                       recall_at_10_literal=recall_at(lids.cpu().numpy(), exact_ids),
                       recall_at_10_optimised=recall_at(oids.cpu().numpy(), exact_ids),
                       mean_rounds_literal=float(lst[:, 0].mean()),
                       mean_rounds_optimised=float(ost[:, 0].mean()),
                       mean_candidates_literal=float(lst[:, 1].mean()),
                       mean_candidates_optimised=float(ost[:, 1].mean()),
                       mean_point_visits_literal=float(lst[:, 7].mean()),
                       mean_point_visits_optimised=float(ost[:, 7].mean()))
        log(f"[bench] {w.name} literal vs optimised: {literal}")

    # parameter study (encoding, L, K), FP32 verification at the calibrated beta with the
    # radius schedule autotuned per configuration: recall, QPS and build rate
    study = None
    if not args.no_study and w.n <= STUDY_MAX_N and exact_ids is not None:
        study = []
        for enc, L_s, K_s in STUDY:
            A_s = A if (L_s, K_s) == (w.L, w.K) else wl.projection_matrix(w.d, L_s, K_s,
                                                                          seed=2603 + 16 * L_s + K_s)
            # one untimed build of this shape first: the timed one reuses its device blocks,
            # as the step's builds do (a first build of a new shape allocates, and may first
            # have to release cached blocks of other shapes)
            pdet.Index(Xd, A_s, sid, K_s, L_s, w.Nr, w.max_leaf, encoding=enc).close()
            torch.cuda.synchronize()
            tb0 = time.perf_counter()
            ixs = pdet.Index(Xd, A_s, sid, K_s, L_s, w.Nr, w.max_leaf, encoding=enc)
            torch.cuda.synchronize()
            tbs = time.perf_counter() - tb0
            t = ixs.autotune(Qp, k=w.k, c=w.c, beta=beta)
            sids, _ = ixs.query(Qr, k=w.k, c=w.c, beta=beta, r_min=t["r_min"])
            srec = recall_at(sids.cpu().numpy(), exact_ids)
            ixs.reserve(nq)
            sec_s = timed(lambda: ixs.query(Qd, k=w.k, c=w.c, beta=beta, r_min=t["r_min"]))
            _, _, sst = ixs.query(Qd, k=w.k, c=w.c, beta=beta, r_min=t["r_min"], stats=True)
            sst = sst.cpu().numpy()
            study.append(dict(encoding=enc, L=L_s, K=K_s, beta=beta, r_min=t["r_min"],
                              recall_at_10=srec, qps=nq / sec_s, build_ms=1e3 * tbs,
                              mean_candidates=float(sst[:, 1].mean()),
                              mean_rounds=float(sst[:, 0].mean())))
            log(f"[bench] {w.name} study {study[-1]}")
            ixs.close()
            del ixs

    # online insertion (Algorithm 2's insertion loop into a resident index): an index of the
    # first n - m rows grows by the last m rows in one call; each timed call starts from a
    # fresh index (built untimed). The grown index is then queried at the calibrated beta.
    insertion = None
    if not args.no_insert and w.n <= INSERT_MAX_N:
        insertion = []
        for m in INSERT_BATCHES:
            n0 = w.n - m
            sid0 = sid[sid < n0]
            secs = []
            for it in range(args.warmup + args.steps):
                ixg = pdet.Index(Xd[:n0], A, sid0, w.K, w.L, w.Nr, w.max_leaf)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                ixg.insert(Xd)
                torch.cuda.synchronize()
                if it >= args.warmup:
                    secs.append(time.perf_counter() - t1)
                if it < args.warmup + args.steps - 1:
                    ixg.close()
                    del ixg
            sec = float(np.mean(secs))
            rec = None
            if exact_ids is not None:
                gids, _ = ixg.query(Qr, k=w.k, c=w.c, beta=beta, r_min=r_min)
                rec = recall_at(gids.cpu().numpy(), exact_ids)
            # bytes the grown index's per-point arrays move: every tree's codes (16-byte rows)
            # and permutation copied, and its leaf rows (4L bytes per point) written
            ins_bytes = w.n * w.L * (32 + 8 + 4 * w.L) + m * w.d * 4
            insertion.append(dict(m=m, n_resident=n0, ms_per_call=1e3 * sec,
                                  inserted_pts_per_s=m / sec, recall_at_10_after=rec,
                                  bytes_per_call=ins_bytes,
                                  hbm_frac=ins_bytes / sec / 1e9 / HBM_PEAK_GBS))
            log(f"[bench] {w.name} insertion {insertion[-1]}")
            ixg.close()
            del ixg

    # batching form: one graph-launched batch with k in {1,10,100}, c in {1.2,1.5,2.0}
    batching = None
    if not args.no_plan:
        rng = np.random.default_rng(7)
        ks = rng.choice([1, 10, 100], size=nq).astype(np.int32)
        cs = rng.choice([1.2, 1.5, 2.0], size=nq)
        pb, pr, pc = (beta, r_min, rcap) if plan_prec == "fp32" else lowp_cal[plan_prec][:3]
        ix.set_tuning(pr, pc)
        plan = ix.plan(Qd, k=0, beta=pb, r_min=pr, k_per_query=ks, c_per_query=cs,
                       precision=plan_prec, rescore=4)
        sec_plan = timed(plan.launch)
        pids = plan.ids.cpu().numpy()
        plan.close()
        sec_eager = timed(lambda: ix.query(Qd, k=0, beta=pb, r_min=pr, k_per_query=ks,
                                           c_per_query=cs, precision=plan_prec, rescore=4))
        brec = None
        if exact_ids is not None:
            off = np.concatenate([[0], np.cumsum(ks)])
            sel = [q for q in range(nrec) if ks[q] >= 10]
            brec = recall_at([pids[off[q]:off[q] + 10] for q in sel], exact_ids[sel])
        batching = dict(qps_graph=nq / sec_plan, qps_eager=nq / sec_eager, precision=plan_prec,
                        k_mix=[1, 10, 100], c_mix=[1.2, 1.5, 2.0], beta=pb, r_min=pr,
                        recall_at_10_k_ge_10=brec,
                        search_launches=int(pdet.get_timing()["query_main_launches"]))
        log(f"[bench] {w.name} batching: {batching}")

    # serving form: Poisson arrivals (native client) into the continuous-batching server
    serving = None
    if not args.no_serve:
        serving = {"fp32": serve_measurement(ix, Q, w, beta, r_min, rcap)}
        log(f"[bench] {w.name} serving fp32: {serving['fp32']}")
        for f, (lb, lr, lc, lrec) in lowp_cal.items():
            serving[f] = serve_measurement(ix, Q, w, lb, lr, lc, precision=f)
            serving[f]["recall_at_10"] = lrec
            log(f"[bench] {w.name} serving {f}: {serving[f]}")
    ix.close()
    del Xd
    torch.cuda.empty_cache()

    last = recs[-1]
    out = {
        "workload": w.name, "n": w.n, "d": w.d, "L": w.L, "K": w.K, "Nr": w.Nr,
        "max_leaf": w.max_leaf, "nq": nq, "k": w.k, "c": w.c, "beta": beta, "r_min": r_min,
        "rounds_resolved": rcap, "verify": "fp32 (fp64 accumulate)",
        "qps": qps, "recall_at_10": rec, "recall_queries": nrec,
        "recall_ground_truth": "FP64 brute force over all n points",
        "build_mpts_per_s": w.n / build_s / 1e6, "build_ms": 1e3 * build_s,
        "build_stage_ms": bstage, "query_ms": 1e3 * query_s,
        "reserve_ms": 1e3 * float(np.mean([r["reserve_s"] for r in recs])),
        "step_ms": 1e3 * total / args.steps,
        "mean_candidates_per_query": ncand / nq,
        "queries_answered_again": int(last["tq"].get("query_retried", 0)),
        "stop_rule_A_fraction": float(np.mean([np.mean(r["stops"] == 1) for r in recs])),
        "band": {"leaf_edge_pairs_per_query": float(last["band_leaf"].mean()),
                 "queries_with_leaf_edge_tie": int(np.sum(last["band_leaf"] > 0)),
                 "queries_with_stop_b_tie": int(np.sum(last["band_b"] > 0))},
        "per_query_search_us": {
            "p50": float(np.percentile(last["qtime"], 50) * 1e3 / last["khz"]),
            "p99": float(np.percentile(last["qtime"], 99) * 1e3 / last["khz"]),
            "max": float(last["qtime"].max() * 1e3 / last["khz"])},
        "mean_point_visits_per_query": float(last["visits"].mean()),
        "roofline": {"bound": "hbm", "kernel": "q_main_f32", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": bytes_alg,
                     "ms_per_launch": main_ms, "launches_per_batch": launches},
        "roofline_build": {"bound": "hbm", "achieved": build_gbs, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": build_gbs / HBM_PEAK_GBS,
                           "bytes_per_point": build_bpp,
                           "note": "whole build (host gaps included): read x, write and read "
                                   "codes, write perm"},
        # the encoder reads every row once and writes its codes and keys; its float32 products
        # run as three-way bf16 splits on the matrix cores, whose time at the bf16 peak
        # (six products per float32 one) is below the HBM time
        "roofline_build_encode": {"bound": "hbm", "kernel": "project_kernel(encode)",
                                  "achieved": enc_bytes / (enc_ms * 1e-3) / 1e9,
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": enc_bytes / (enc_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                  "bytes_per_point": 4 * w.d + 16 * w.L + 2 * w.L,
                                  "ms": enc_ms,
                                  "fp32_equivalent_tflops":
                                      2.0 * w.n * w.d * 16 * w.L / (enc_ms * 1e-3) / 1e12},
        "lowp": lowp,
        "literal_vs_optimised": literal,
        "parameter_study": study,
        "insertion": insertion,
        "batching": batching,
        "serving": serving,
    }
    if primary and helper is not None:
        n_cpu = min(w.n, 1 << 20)
        cpu = helper.run(workload=w.name, nq=nq, beta=beta, r_min=r_min)
        if cpu.get("data_sha16") not in (None, hashlib.sha256(X[:n_cpu].tobytes()).hexdigest()[:16]):
            cpu = {"error": "the oracle's sample differs from the benchmark's data"}
        out["cpu_baseline"] = cpu
    del X
    return out


def serve_measurement(ix, Q, w, beta, r_min, rcap, seconds=1.0, max_batch=1024,
                      precision="fp32"):
    """Saturation QPS from a burst, then Poisson arrivals at 25/50/90% of it offered by the
    library's native client: p50 / p99 latency and achieved QPS."""
    ix.set_tuning(r_min, rcap)
    out = {"precision": precision}
    kw = dict(max_batch=max_batch, lanes=2, k_max=w.k, beta=beta, r_min=r_min,
              precision=precision)
    # untimed warm-up server: first-use costs (workspace, code loading) stay out of the burst
    sv = ix.server(**kw)
    sv.offer_poisson(Q[:256], 256, 1e7, w.k, w.c, seed=1)
    sv.close()
    sv = ix.server(**kw)
    n_burst = min(len(Q), 4096)
    t0 = time.perf_counter()
    sv.offer_poisson(Q[:n_burst], n_burst, 1e9, w.k, w.c, seed=2)   # all at once
    sat = n_burst / (time.perf_counter() - t0)
    out["burst"] = dict(sv.stats(), requests=n_burst)
    sv.close()
    for i, frac in enumerate((0.25, 0.5, 0.9)):
        rate = frac * sat
        sv = ix.server(**kw)
        nreq = max(200, int(rate * seconds))
        offered = sv.offer_poisson(Q, nreq, rate, w.k, w.c, seed=11 + i)
        st = sv.stats()
        sv.close()
        out[f"poisson_{int(frac * 100)}pct"] = dict(target_qps=rate, offered_qps=offered,
                                                    achieved_qps=st["qps"], p50_ms=st["p50_ms"],
                                                    p99_ms=st["p99_ms"],
                                                    mean_batch=st["mean_batch"], requests=nreq)
    out["saturation_qps_burst"] = sat
    return out


def _oracle_queries(args):
    """Worker: oracle queries of one share (the index is inherited through fork)."""
    import oracle
    lo, hi = args
    g = _ORACLE_JOB
    out = []
    for q in g["Q"][lo:hi]:
        r = oracle.query(g["idx"], g["X"], q, g["k"], g["c"], g["beta"], g["r_min"], g["eps"])
        out.append((r.ids, r.n_cand, r.stop, r.rounds))
    return out


def _oracle_tree(i):
    import oracle
    g = _ORACLE_JOB
    return oracle.build_tree(g["codes"][i], g["Nr"], g["max_leaf"])


_ORACLE_JOB = {}


def cpu_baseline_job(workload, nq, beta, r_min, n_cpu_max=1 << 20, nq_cpu=200):
    """The FP64 oracle on this host on a bounded sample of the workload: its own index over
    the first n_cpu points (one generator chunk, drawn here from the same seeds; breakpoints
    from its own sample of them) with the GPU's beta and r_min, then nq_cpu queries of the
    batch. Run once on one thread and once on all worker processes (trees, then queries, in
    parallel), with identical outputs asserted. Runs in a process that never touched the GPU."""
    import multiprocessing as mp

    import oracle
    from paper_2603_24920_amd import workloads as wl
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:  # pragma: no cover
        pass
    w = wl.WORKLOADS[workload]
    n_cpu = min(w.n, n_cpu_max)
    Xs = w.data(n=n_cpu)
    Q = w.queries(nq)[:nq_cpu]
    sid = wl.sample_ids(n_cpu, wl.sample_size(n_cpu, w.sample_frac, w.Nr), w.seeds["sample"])
    A = w.proj()
    eps = oracle.epsilon(w.K, w.L)
    # one thread
    t0 = time.perf_counter()
    idx = oracle.build_index(Xs, A, sid, w.L, w.K, w.Nr, w.max_leaf)
    tb1 = time.perf_counter() - t0
    t1 = time.perf_counter()
    res1 = []
    for q in Q:
        r = oracle.query(idx, Xs, q, w.k, w.c, beta, r_min, eps)
        res1.append((r.ids, r.n_cand, r.stop, r.rounds))
    tq1 = time.perf_counter() - t1
    # all worker processes: independent trees, then independent queries
    cores = min(POOL, os.cpu_count() or 1)
    _ORACLE_JOB.update(idx=idx, X=Xs, Q=Q, k=w.k, c=w.c, beta=beta, r_min=r_min, eps=eps,
                       Nr=w.Nr, max_leaf=w.max_leaf)
    ctx = mp.get_context("fork")
    t2 = time.perf_counter()
    H = oracle.project(Xs, A)
    B = oracle.breakpoints(H[sid], w.Nr, H.min(axis=0), H.max(axis=0))
    codes = oracle.encode(H, B, w.L, w.K)
    del H
    _ORACLE_JOB["codes"] = codes
    with ctx.Pool(min(cores, w.L)) as pool:
        trees = pool.map(_oracle_tree, range(w.L))
    tbp = time.perf_counter() - t2
    same_build = np.array_equal(codes, idx.codes) and all(
        np.array_equal(a.perm, b.perm) for a, b in zip(trees, idx.trees))
    shares = [(i * nq_cpu // cores, (i + 1) * nq_cpu // cores) for i in range(cores)]
    t3 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        resp = [r for part in pool.map(_oracle_queries, shares) for r in part]
    tqp = time.perf_counter() - t3
    same_query = all(np.array_equal(a[0], b[0]) and a[1:] == b[1:] for a, b in zip(res1, resp))
    _ORACLE_JOB.clear()
    if not (same_build and same_query):
        return {"error": "the oracle's all-core run differs from its one-thread run"}
    return {"value": nq_cpu / tqp, "unit": "queries/s", "cores": cores, "kind": "oracle",
            "sample": f"{nq_cpu} queries of the {w.name} batch on the oracle's own index over the "
                      f"first {n_cpu} points (beta={beta:g}, r_min={r_min:.4g} as on the GPU; "
                      f"FP64 numpy); value on {cores} worker processes, outputs identical to "
                      f"one thread",
            "data_sha16": hashlib.sha256(Xs.tobytes()).hexdigest()[:16],
            "one_thread": {"queries_per_s": nq_cpu / tq1, "build_mpts_per_s": n_cpu / tb1 / 1e6,
                           "cores": 1},
            "all_cores": {"queries_per_s": nq_cpu / tqp, "build_mpts_per_s": n_cpu / tbp / 1e6,
                          "cores": cores, "build_parallel_over": "trees",
                          "query_parallel_over": "queries"}}


def _helper_main(conn):
    while True:
        job = conn.recv()
        if job is None:
            break
        try:
            conn.send(cpu_baseline_job(**job))
        except Exception as e:  # pragma: no cover
            conn.send({"error": repr(e)})


class OracleHelper:
    """A process forked before this one touches the GPU, which runs the oracle baseline (and
    forks its own workers) without any inherited GPU state."""

    def __init__(self):
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        self.conn, child = ctx.Pipe()
        self.proc = ctx.Process(target=_helper_main, args=(child,))
        self.proc.start()

    def run(self, **job):
        self.conn.send(job)
        return self.conn.recv()

    def close(self):
        try:
            self.conn.send(None)
        except Exception:  # pragma: no cover
            pass
        self.proc.join(timeout=30)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sift-like-100M-d128")
    ap.add_argument("--secondary", default="sift-like-1M-d128,normed-10M-d256",
                    help="comma-separated workloads measured after the primary ('' for none)")
    ap.add_argument("--nq", type=int, default=None)
    ap.add_argument("--beta", type=float, default=None, help="skip the recall calibration")
    ap.add_argument("--r-min", type=float, default=None)
    ap.add_argument("--recall-queries", type=int, default=1000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-lowp", action="store_true", help="skip the low-precision forms")
    ap.add_argument("--rcap", type=int, default=4, help="rounds resolved (with --beta/--r-min)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-plan", action="store_true", help="skip the graph-launched batch")
    ap.add_argument("--no-study", action="store_true",
                    help="skip the (encoding, L, K) parameter study")
    ap.add_argument("--no-insert", action="store_true",
                    help="skip timing online insertion")
    ap.add_argument("--no-literal", action="store_true",
                    help="skip timing the literal query form beside the optimised one")
    ap.add_argument("--no-recall", action="store_true",
                    help="with --beta/--r-min: skip the ground truth (profiling runs)")
    ap.add_argument("--plan-precision", default=None,
                    help="verification form of the graph-launched batch (fp32, bf16, fp8)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 3}))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build measures the DET-LSH path on a single "
              "MI355X (multi-GPU sharding is a design note only). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    from paper_2603_24920_amd import workloads as wl
    t_all = time.time()
    helper = None if args.no_cpu_baseline else OracleHelper()   # before any GPU use
    try:
        prim = measure(wl.WORKLOADS[args.workload], args, primary=True, helper=helper)
        secondary = {}
        for name in [s for s in args.secondary.split(",") if s and s != args.workload]:
            secondary[name] = measure(wl.WORKLOADS[name], args, primary=False)
    finally:
        if helper is not None:
            helper.close()
    cpu = prim.pop("cpu_baseline", None)
    out = {
        "metric": METRIC,
        "value": prim["qps"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": prim["step_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {k: prim[k] for k in ("workload", "n", "d", "L", "K", "Nr", "max_leaf", "nq",
                                        "k", "c", "beta", "r_min", "rounds_resolved", "verify")},
    }
    out.update({k: v for k, v in prim.items() if k not in out["config"] and k != "qps"})
    out["roofline"] = prim["roofline"]
    out["cpu_baseline"] = cpu
    out["secondary"] = secondary
    out["bench_wall_s"] = time.time() - t_all
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
