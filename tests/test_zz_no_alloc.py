"""pdet_query_noalloc (the query without device allocation, over the library's static
scratch array) against pdet_query, through the C ABI: identical ids, distances and
statistics (except the device-time word), on two calls in a row (the second with fewer
queries), on an index whose batch needs several chunks of slots, in FP32 and BF16; the
device's free memory is unchanged by a call; an oversized batch is refused."""
import numpy as np
import pytest

from paper_2603_24920_amd import pdet
from paper_2603_24920_amd import workloads as wl

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KEEP = [0, 1, 2, 3, 4, 5, 7, 8, 9]      # qstats words; word 6 is the query's device time


def _outputs(nq, k):
    return (torch.full((nq * k,), -7, dtype=torch.int64, device="cuda"),
            torch.full((nq * k,), -7.0, dtype=torch.float32, device="cuda"),
            torch.full((nq, pdet.QSTAT_WORDS), -7, dtype=torch.int32, device="cuda"))


def _check(idx, Qd, k, c, beta, r_min, precision, label):
    nq = Qd.shape[0]
    ref_ids, ref_d, ref_st = idx.query(Qd, k=k, c=c, beta=beta, r_min=r_min,
                                       precision=precision, rescore=4, stats=True)
    ids, dists, st = _outputs(nq, k)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    idx.query_noalloc(Qd, ids, dists, st, k=k, c=c, beta=beta, r_min=r_min,
                      precision=precision, rescore=4)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    print(f"[noalloc {label}] nq={nq} k={k} {precision} free memory before/after "
          f"{free0}/{free1}", flush=True)
    assert torch.equal(ids.view(nq, k), ref_ids), label
    assert torch.equal(dists.view(nq, k), ref_d), label
    assert torch.equal(st[:, KEEP], ref_st[:, KEEP]), label
    assert free1 == free0, label


def test_noalloc_equals_query_on_two_calls():
    w = wl.SMALL_MIXTURE
    X = w.data()
    print(f"\n[noalloc] n={len(X)} d={X.shape[1]}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf, lowp=("bf16",))
    Q = torch.from_numpy(w.queries()).cuda()
    for precision in ("fp32", "bf16"):
        _check(idx, Q, 10, 1.5, 0.1, 4.0, precision, "first call")
        # a smaller batch next: the array holds the previous call's contents
        _check(idx, Q[:37].contiguous(), 10, 1.5, 0.05, 1.0, precision, "second call")
    # a query that reaches the dense round table (k = 1000, c = 1.05)
    _check(idx, Q[:9].contiguous(), 1000, 1.05, 1.0, 1.0, "fp32", "dense table")
    idx.close()


def test_noalloc_runs_the_batch_in_chunks_of_slots():
    """600k points: a slot holds ~60k leaves, so the array takes a few dozen slots and a
    batch of 300 queries runs in several chunks."""
    w = wl.SIFT_LIKE_1M.scaled(n=600_000)
    X = w.data()
    print(f"\n[noalloc] n={len(X)} d={X.shape[1]}", flush=True)
    Xd = torch.from_numpy(X).cuda()
    idx = pdet.Index(Xd, w.proj(), w.sample(), w.K, w.L, w.Nr, w.max_leaf)
    leaves = sum(idx.info()["leaves"])
    per_slot = 24 * leaves
    print(f"[noalloc] leaves={leaves} ~{per_slot} bytes per slot", flush=True)
    assert 300 * per_slot > (64 << 20)            # the batch does not fit at once
    Q = torch.from_numpy(w.queries(300)).cuda()
    _check(idx, Q, 10, 1.5, 0.002, 30.0, "fp32", "chunks")
    _check(idx, Q[:50].contiguous(), 10, 1.5, 0.002, 30.0, "fp32", "chunks, smaller")
    idx.close()


def test_noalloc_refuses_oversized_batches_and_per_query_arrays():
    w = wl.SMALL_MIXTURE.scaled(n=2000)
    Xd = torch.from_numpy(w.data()).cuda()
    idx = pdet.Index(Xd, w.proj(), w.sample(), w.K, w.L, w.Nr, 32)
    nq = 300_000                                   # 288 bytes per query of arrays alone
    Q = torch.zeros((nq, w.d), dtype=torch.float32, device="cuda")
    ids, dists, st = _outputs(nq, 1)
    with pytest.raises(pdet.PdetError) as e:
        idx.query_noalloc(Q, ids, dists, st, k=1, c=1.5, beta=0.1, r_min=1.0)
    assert e.value.status == pdet.PDET_EUNSUPPORTED and "scratch" in str(e.value)
    p, keep = idx._params(1, 1.5, 0.1, 1.0, 0.0, "fp32", 4, np.ones(4, np.int32), None)
    import ctypes
    st2 = pdet.lib().pdet_query_noalloc(idx._h, ctypes.c_void_p(Q.data_ptr()), 4,
                                        ctypes.byref(p), ctypes.c_void_p(ids.data_ptr()),
                                        ctypes.c_void_p(dists.data_ptr()), None, None)
    assert st2 == pdet.PDET_EINVAL
    idx.close()
