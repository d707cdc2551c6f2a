"""ctypes binding of libpdet (argument marshalling only; every step runs in HIP kernels).

Device buffers are torch CUDA tensors (HIP on ROCm); torch supplies memory and the
current stream, the library does all the computation. Importing this module does not
touch the GPU; the library is loaded on first use and a missing build is an error.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64,
                    c_void_p)

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpdet.so")

PDET_OK, PDET_EINVAL, PDET_ENOMEM, PDET_EDEVICE, PDET_EUNSUPPORTED = 0, -1, -2, -3, -4
FP32, BF16, FP8_E4M3 = 0, 1, 2
PRECISIONS = {"fp32": FP32, "bf16": BF16, "fp8": FP8_E4M3}
MAX_K, MAX_L, MAX_TOPK, MAX_ROUNDS = 16, 16, 1024, 255
QSTAT_WORDS = 10
QSTAT = dict(rounds=0, ncand=1, stop=2, leaves=3, hsum=4, hmix=5, time=6, visits=7,
             band_leaf=8, band_stop_b=9)
(X_BREAKPOINTS, X_CODES, X_PERM, X_LEAF_START, X_LEAF_COUNT, X_LEAF_HIDX, X_LEAF_OF,
 X_PROJ, X_SAMPLE) = range(9)
EXPORTED = ["pdet_draw_params", "pdet_build", "pdet_insert", "pdet_free", "pdet_query", "pdet_query_literal", "pdet_rc_ann", "pdet_query_candidates", "pdet_query_noalloc", "pdet_reserve", "pdet_info", "pdet_export", "pdet_project",
            "pdet_epsilon", "pdet_theoretical_beta", "pdet_normal_quantile", "pdet_last_error", "pdet_set_timing", "pdet_get_timing",
            "pdet_autotune", "pdet_set_tuning", "pdet_plan_create", "pdet_plan_launch",
            "pdet_plan_free", "pdet_server_create", "pdet_server_submit", "pdet_server_wait",
            "pdet_server_get_stats", "pdet_server_free", "pdet_server_offer_poisson",
            "pdet_set_list_cap",
            "pdet_release_cache"]


class BuildParams(ctypes.Structure):
    _fields_ = [("K", c_int32), ("L", c_int32), ("Nr", c_int32), ("max_leaf", c_int32),
                ("proj", POINTER(c_float)), ("sample_ids", POINTER(c_int64)),
                ("n_sample", c_int64), ("lowp_copies", c_uint32), ("encoding", c_int32),
                ("sample_frac", c_double), ("seed", c_uint64)]


ENCODINGS = {"dynamic": 0, "static": 1}


class QueryParams(ctypes.Structure):
    _fields_ = [("k", c_int32), ("c", c_double), ("k_per_query", POINTER(c_int32)),
                ("c_per_query", POINTER(c_double)), ("beta", c_double), ("r_min", c_double),
                ("eps", c_double), ("precision", c_int32), ("rescore", c_int32)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("n_sample", c_int64), ("d", c_int32), ("K", c_int32),
                ("L", c_int32), ("Nr", c_int32), ("max_leaf", c_int32),
                ("lowp_copies", c_uint32), ("leaves", c_int64 * MAX_L),
                ("device_bytes", c_int64), ("wall_clock_khz", c_int32)]


class Timing(ctypes.Structure):
    _fields_ = [(f, c_double) for f in (
        "build_sample_ms", "build_sort_ms", "build_encode_ms", "build_tree_ms", "build_lowp_ms",
        "query_project_ms", "query_rho_ms", "query_main_ms")] + [("query_main_launches", c_int64),
                                                           ("query_retried", c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("r_min", c_double), ("rounds_resolved", c_int32), ("median_rounds", c_double),
                ("p95_rounds", c_double)]


class ServerParams(ctypes.Structure):
    _fields_ = [("max_batch", c_int32), ("lanes", c_int32), ("k_max", c_int32),
                ("precision", c_int32), ("rescore", c_int32), ("beta", c_double),
                ("r_min", c_double), ("eps", c_double), ("memory_budget", c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed", c_int64), ("batches", c_int64), ("batch_cap", c_int64),
                ("mean_batch", c_double), ("p50_ms", c_double), ("p99_ms", c_double),
                ("qps", c_double)]


class PdetError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"pdet status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libpdet.so (built in-tree by ``build_lib``); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2603_24920_amd.build_lib`")
        L = ctypes.CDLL(LIB_PATH)
        L.pdet_build.argtypes = [c_void_p, c_int64, c_int32, POINTER(BuildParams), c_void_p,
                                 POINTER(c_void_p)]
        L.pdet_draw_params.argtypes = [c_int64, c_int32, c_int32, c_int32, c_int32, c_double,
                                       c_uint64, c_void_p, c_void_p, POINTER(c_int64)]
        L.pdet_insert.argtypes = [c_void_p, c_void_p, c_int64, c_void_p]
        L.pdet_query.argtypes = [c_void_p, c_void_p, c_int64, POINTER(QueryParams), c_void_p,
                                 c_void_p, c_void_p, c_void_p]
        L.pdet_query_candidates.argtypes = [c_void_p, c_void_p, c_int64, POINTER(QueryParams),
                                            c_void_p, c_void_p, c_void_p, c_void_p, c_int64,
                                            c_void_p]
        L.pdet_query_noalloc.argtypes = [c_void_p, c_void_p, c_int64, POINTER(QueryParams),
                                         c_void_p, c_void_p, c_void_p, c_void_p]
        L.pdet_query_literal.argtypes = [c_void_p, c_void_p, c_int64, POINTER(QueryParams),
                                         c_void_p, c_void_p, c_void_p, c_void_p]
        L.pdet_query_literal.restype = c_int32
        L.pdet_rc_ann.argtypes = [c_void_p, c_void_p, c_int64, c_double, c_double, c_double,
                                  c_double, c_void_p, c_void_p, c_void_p, c_void_p]
        L.pdet_rc_ann.restype = c_int32
        L.pdet_reserve.argtypes = [c_void_p, c_int64, c_void_p]
        L.pdet_set_list_cap.argtypes = [c_void_p, c_int64]
        L.pdet_release_cache.argtypes = []
        L.pdet_release_cache.restype = None
        L.pdet_free.argtypes = [c_void_p]
        L.pdet_free.restype = None
        L.pdet_info.argtypes = [c_void_p, POINTER(IndexInfo)]
        L.pdet_export.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_size_t]
        L.pdet_project.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p]
        L.pdet_epsilon.argtypes = [c_int32, c_int32]
        L.pdet_epsilon.restype = c_double
        L.pdet_theoretical_beta.argtypes = [c_int32, c_int32, c_double]
        L.pdet_theoretical_beta.restype = c_double
        L.pdet_normal_quantile.argtypes = [c_double]
        L.pdet_normal_quantile.restype = c_double
        L.pdet_last_error.restype = ctypes.c_char_p
        L.pdet_set_timing.argtypes = [c_int32]
        L.pdet_set_timing.restype = None
        L.pdet_get_timing.argtypes = [POINTER(Timing)]
        L.pdet_get_timing.restype = c_int32
        L.pdet_autotune.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_double, c_double,
                                    c_int32, c_void_p, POINTER(Tuning)]
        L.pdet_set_tuning.argtypes = [c_void_p, c_double, c_int32]
        L.pdet_plan_create.argtypes = [c_void_p, c_void_p, c_int64, POINTER(QueryParams),
                                       c_void_p, c_void_p, c_void_p, POINTER(c_void_p)]
        L.pdet_plan_launch.argtypes = [c_void_p, c_void_p]
        L.pdet_plan_free.argtypes = [c_void_p]
        L.pdet_plan_free.restype = None
        L.pdet_server_create.argtypes = [c_void_p, POINTER(ServerParams), POINTER(c_void_p)]
        L.pdet_server_submit.argtypes = [c_void_p, c_void_p, c_int32, c_double, POINTER(c_int64)]
        L.pdet_server_wait.argtypes = [c_void_p, c_int64, c_void_p, c_void_p, POINTER(c_double)]
        L.pdet_server_get_stats.argtypes = [c_void_p, POINTER(ServerStats)]
        L.pdet_server_offer_poisson.argtypes = [c_void_p, c_void_p, c_int64, c_int64, c_double,
                                                c_int32, c_double, ctypes.c_uint64,
                                                POINTER(c_double)]
        L.pdet_server_offer_poisson.restype = c_int32
        L.pdet_server_free.argtypes = [c_void_p]
        L.pdet_server_free.restype = None
        for f in ("pdet_draw_params", "pdet_build", "pdet_insert", "pdet_query", "pdet_query_candidates", "pdet_query_noalloc",
                  "pdet_reserve", "pdet_info", "pdet_export", "pdet_project",
                  "pdet_autotune", "pdet_set_tuning", "pdet_plan_create", "pdet_plan_launch",
                  "pdet_server_create", "pdet_server_submit", "pdet_server_wait",
                  "pdet_server_get_stats", "pdet_set_list_cap"):
            getattr(L, f).restype = c_int32
        _lib = L
    return _lib


def _check(status):
    if status != PDET_OK:
        raise PdetError(status, lib().pdet_last_error().decode())


def draw_params(n: int, d: int, L: int, K: int, Nr: int = 256, sample_frac: float = 0.1,
                seed: int = 0):
    """The library's seeded projection (float32 [d][L*K]) and sample ids (int64, ascending):
    the ones pdet_build draws when it is given neither (pdet_draw_params)."""
    m = c_int64()
    _check(lib().pdet_draw_params(n, d, L, K, Nr, sample_frac, seed, None, None, ctypes.byref(m)))
    proj = np.empty((d, L * K), dtype=np.float32)
    ids = np.empty((m.value,), dtype=np.int64)
    _check(lib().pdet_draw_params(n, d, L, K, Nr, sample_frac, seed, proj.ctypes.data_as(c_void_p),
                                  ids.ctypes.data_as(c_void_p), ctypes.byref(m)))
    return proj, ids


def epsilon(K: int, L: int) -> float:
    """Projected-radius factor from Eq. 2 / Lemma 3, computed by the library's host code."""
    return lib().pdet_epsilon(K, L)


def normal_quantile(p: float) -> float:
    """Phi^-1(p) as the library's static encoding computes it (host code)."""
    return lib().pdet_normal_quantile(p)


def theoretical_beta(K: int, L: int, c: float) -> float:
    """beta of Lemma 3 for (K, L, c), computed by the library's host code."""
    return lib().pdet_theoretical_beta(K, L, c)


def set_timing(on: bool) -> None:
    """Record per-kernel-family device time (HIP events) for this thread's calls."""
    lib().pdet_set_timing(1 if on else 0)


def release_cache() -> None:
    """Return the library's cached device blocks to the driver (pdet_release_cache)."""
    lib().pdet_release_cache()


def get_timing() -> dict:
    t = Timing()
    _check(lib().pdet_get_timing(ctypes.byref(t)))
    return {f: getattr(t, f) for f, _ in Timing._fields_}


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


class Index:
    """A DE-Tree index resident on the GPU. ``X`` (CUDA float32 [n][d]) is borrowed."""

    def __init__(self, X, proj=None, sample_ids=None, K=16, L=4, Nr=256, max_leaf=128, lowp=(),
                 stream=None, encoding="dynamic", sample_frac=0.1, seed=0):
        """``proj`` (float32 [d][L*K]) and ``sample_ids`` (int64) may be None: the library
        then draws them from ``seed`` (and ``sample_frac``), as draw_params does."""
        import torch
        if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32
                and X.dim() == 2 and X.is_contiguous()):
            raise ValueError("X must be a contiguous CUDA float32 [n][d] tensor")
        self.X = X
        self.n, self.d = X.shape
        pp, sp, ns = None, None, 0
        if proj is not None:
            self._proj = np.ascontiguousarray(proj, dtype=np.float32)
            if self._proj.shape != (self.d, L * K):
                raise ValueError("proj must be [d][L*K]")
            pp = self._proj.ctypes.data_as(POINTER(c_float))
        if sample_ids is not None:
            self._sample = np.ascontiguousarray(sample_ids, dtype=np.int64)
            sp, ns = self._sample.ctypes.data_as(POINTER(c_int64)), len(self._sample)
        mask = 0
        for name in lowp:
            mask |= 1 << PRECISIONS[name]
        p = BuildParams(K, L, Nr, max_leaf, pp, sp, ns, mask, ENCODINGS[encoding],
                        float(sample_frac), int(seed))
        h = c_void_p()
        _check(lib().pdet_build(c_void_p(X.data_ptr()), self.n, self.d, ctypes.byref(p),
                                _stream(stream), ctypes.byref(h)))
        self._h, self._lib = h, lib()
        self.K, self.L, self.Nr, self.max_leaf = K, L, Nr, max_leaf
        self.encoding = encoding

    def close(self):
        # the library handle is held on the object: module globals may already be gone when
        # this runs at interpreter exit
        if getattr(self, "_h", None):
            self._lib.pdet_free(self._h)
            self._h = None

    __del__ = close

    def insert(self, X, stream=None):
        """Online insertion (pdet_insert): X (contiguous CUDA float32 [n_total][d]) holds the
        indexed rows unchanged, then the new ones; the index borrows X from now on."""
        import torch
        if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32
                and X.dim() == 2 and X.is_contiguous() and X.shape[1] == self.d):
            raise ValueError("X must be a contiguous CUDA float32 [n_total][d] tensor")
        _check(lib().pdet_insert(self._h, c_void_p(X.data_ptr()), X.shape[0], _stream(stream)))
        self.X = X
        self.n = X.shape[0]

    def reserve(self, nq: int, stream=None):
        """Size the query workspace for batches of up to nq queries (pdet_reserve)."""
        _check(lib().pdet_reserve(self._h, int(nq), _stream(stream)))

    def set_list_cap(self, cap: int) -> None:
        """Per-tree leaf-list capacity of the query slots (pdet_set_list_cap; 0: automatic)."""
        _check(lib().pdet_set_list_cap(self._h, int(cap)))

    def info(self) -> dict:
        inf = IndexInfo()
        _check(lib().pdet_info(self._h, ctypes.byref(inf)))
        return dict(n=inf.n, n_sample=inf.n_sample, d=inf.d, K=inf.K, L=inf.L, Nr=inf.Nr,
                    max_leaf=inf.max_leaf, lowp_copies=inf.lowp_copies,
                    leaves=list(inf.leaves[:inf.L]), device_bytes=inf.device_bytes,
                    wall_clock_khz=inf.wall_clock_khz)

    def export(self, what: int, tree: int = 0) -> np.ndarray:
        nl = self.info()["leaves"]
        shape, dt = {
            X_BREAKPOINTS: ((self.L * self.K, self.Nr + 1), np.float32),
            X_CODES: ((self.L, self.n, 16), np.uint8),
            X_PERM: ((self.n,), np.int32),
            X_LEAF_START: ((nl[tree],), np.int32),
            X_LEAF_COUNT: ((nl[tree],), np.int32),
            X_LEAF_HIDX: ((nl[tree], 16), np.uint16),
            X_LEAF_OF: ((self.n,), np.int32),
            X_PROJ: ((self.d, self.L * self.K), np.float32),
            X_SAMPLE: ((self.info()["n_sample"],), np.int64),
        }[what]
        out = np.empty(shape, dtype=dt)
        _check(lib().pdet_export(self._h, what, tree, out.ctypes.data_as(c_void_p), out.nbytes))
        return out

    def project(self, x, stream=None):
        import torch
        out = torch.empty((x.shape[0], self.L * self.K), dtype=torch.float32, device=x.device)
        _check(lib().pdet_project(self._h, c_void_p(x.data_ptr()), x.shape[0],
                                  c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def autotune(self, Q_pilot, k=10, c=1.5, beta=0.1, precision="fp32", stream=None) -> dict:
        """Tune the radius schedule from pilot queries (CUDA float32 [m][d]); see pdet.h."""
        t = Tuning()
        _check(lib().pdet_autotune(self._h, c_void_p(Q_pilot.data_ptr()), Q_pilot.shape[0], k, c,
                                   beta, PRECISIONS[precision], _stream(stream), ctypes.byref(t)))
        return dict(r_min=t.r_min, rounds_resolved=t.rounds_resolved,
                    median_rounds=t.median_rounds, p95_rounds=t.p95_rounds)

    def set_tuning(self, r_min: float, rounds_resolved: int = 4) -> None:
        _check(lib().pdet_set_tuning(self._h, r_min, rounds_resolved))

    def _params(self, k, c, beta, r_min, eps, precision, rescore, k_per_query, c_per_query):
        kp = cp = None
        if k_per_query is not None:
            kp = np.ascontiguousarray(k_per_query, dtype=np.int32)
        if c_per_query is not None:
            cp = np.ascontiguousarray(c_per_query, dtype=np.float64)
        p = QueryParams(k, c, kp.ctypes.data_as(POINTER(c_int32)) if kp is not None else None,
                        cp.ctypes.data_as(POINTER(c_double)) if cp is not None else None,
                        beta, r_min, eps, PRECISIONS[precision], rescore)
        return p, (kp, cp)

    def plan(self, Q, k=10, c=1.5, beta=0.1, r_min=1.0, eps=0.0, precision="fp32", rescore=4,
             k_per_query=None, c_per_query=None, stats=False):
        return Plan(self, Q, k, c, beta, r_min, eps, precision, rescore, k_per_query,
                    c_per_query, stats)

    def server(self, max_batch=256, lanes=2, k_max=10, precision="fp32", rescore=4, beta=0.1,
               r_min=0.0, eps=0.0, memory_budget=0):
        return Server(self, max_batch, lanes, k_max, precision, rescore, beta, r_min, eps,
                      memory_budget)

    def query(self, Q, k=10, c=1.5, beta=0.1, r_min=1.0, eps=0.0, precision="fp32",
              rescore=4, k_per_query=None, c_per_query=None, stats=False, stream=None,
              out=None):
        """c^2-k-ANN for every row of Q (CUDA float32 [nq][d]).

        Returns (ids int64, dists float32[, qstats int32 [nq][QSTAT_WORDS]]). With per-query k the
        outputs are flat (CSR in query order); with uniform k they are [nq][k]."""
        import torch
        if not (Q.is_cuda and Q.dtype == torch.float32 and Q.is_contiguous()
                and Q.dim() == 2 and Q.shape[1] == self.d):
            raise ValueError("Q must be a contiguous CUDA float32 [nq][d] tensor")
        nq = Q.shape[0]
        p, keep = self._params(k, c, beta, r_min, eps, precision, rescore, k_per_query,
                               c_per_query)
        total = int(keep[0].sum()) if keep[0] is not None else nq * k
        if out is None:
            ids = torch.empty(total, dtype=torch.int64, device=Q.device)
            dists = torch.empty(total, dtype=torch.float32, device=Q.device)
            st = torch.empty((nq, QSTAT_WORDS), dtype=torch.int32, device=Q.device) if stats else None
        else:
            ids, dists, st = out
        _check(lib().pdet_query(self._h, c_void_p(Q.data_ptr()), nq, ctypes.byref(p),
                                c_void_p(ids.data_ptr()), c_void_p(dists.data_ptr()),
                                c_void_p(st.data_ptr()) if st is not None else None,
                                _stream(stream)))
        if k_per_query is None:
            ids, dists = ids.view(nq, k), dists.view(nq, k)
        return (ids, dists, st) if stats else (ids, dists)


    def query_noalloc(self, Q, ids, dists, qstats=None, k=10, c=1.5, beta=0.1, r_min=1.0,
                      eps=0.0, precision="fp32", rescore=4, stream=None):
        """pdet_query_noalloc into caller-owned outputs (ids int64 [nq*k], dists float32
        [nq*k], qstats int32 [nq][QSTAT_WORDS] or None): uniform k and c, no allocation."""
        p, _ = self._params(k, c, beta, r_min, eps, precision, rescore, None, None)
        _check(lib().pdet_query_noalloc(self._h, c_void_p(Q.data_ptr()), Q.shape[0],
                                        ctypes.byref(p), c_void_p(ids.data_ptr()),
                                        c_void_p(dists.data_ptr()),
                                        c_void_p(qstats.data_ptr()) if qstats is not None else None,
                                        _stream(stream)))

    def query_literal(self, Q, k=10, c=1.5, beta=0.1, r_min=1.0, eps=0.0, stream=None):
        """Algorithm 5 with the literal range query (pdet_query_literal): (ids [nq][k],
        dists [nq][k], qstats [nq][QSTAT_WORDS])."""
        import torch
        nq = Q.shape[0]
        p, _ = self._params(k, c, beta, r_min, eps, "fp32", 1, None, None)
        ids = torch.empty((nq, k), dtype=torch.int64, device=Q.device)
        dists = torch.empty((nq, k), dtype=torch.float32, device=Q.device)
        st = torch.empty((nq, QSTAT_WORDS), dtype=torch.int32, device=Q.device)
        _check(lib().pdet_query_literal(self._h, c_void_p(Q.data_ptr()), nq, ctypes.byref(p),
                                        c_void_p(ids.data_ptr()), c_void_p(dists.data_ptr()),
                                        c_void_p(st.data_ptr()), _stream(stream)))
        return ids, dists, st

    def rc_ann(self, Q, r, c=1.5, beta=0.1, eps=0.0, stream=None):
        """(r,c)-ANN query of Algorithm 4 (pdet_rc_ann): (ids [nq] (-1: none), dists [nq],
        qstats [nq][QSTAT_WORDS])."""
        import torch
        nq = Q.shape[0]
        ids = torch.empty(nq, dtype=torch.int64, device=Q.device)
        dists = torch.empty(nq, dtype=torch.float32, device=Q.device)
        st = torch.empty((nq, QSTAT_WORDS), dtype=torch.int32, device=Q.device)
        _check(lib().pdet_rc_ann(self._h, c_void_p(Q.data_ptr()), nq, float(r), float(c),
                                 float(beta), float(eps), c_void_p(ids.data_ptr()),
                                 c_void_p(dists.data_ptr()), c_void_p(st.data_ptr()),
                                 _stream(stream)))
        return ids, dists, st

    def query_candidates(self, Q, cand_cap, k=10, c=1.5, beta=0.1, r_min=1.0, eps=0.0,
                         precision="fp32", rescore=4, k_per_query=None, c_per_query=None,
                         stream=None):
        """query() with stats, plus each query's candidate set S (pdet_query_candidates).

        Returns (ids, dists, qstats, cands) where cands[q] is the sorted numpy array of the
        first min(|S|, cand_cap) candidate ids of query q (all of S when |S| <= cand_cap)."""
        import torch
        nq = Q.shape[0]
        p, keep = self._params(k, c, beta, r_min, eps, precision, rescore, k_per_query,
                               c_per_query)
        total = int(keep[0].sum()) if keep[0] is not None else nq * k
        ids = torch.empty(total, dtype=torch.int64, device=Q.device)
        dists = torch.empty(total, dtype=torch.float32, device=Q.device)
        st = torch.empty((nq, QSTAT_WORDS), dtype=torch.int32, device=Q.device)
        cand = torch.full((nq, cand_cap), -1, dtype=torch.int32, device=Q.device)
        _check(lib().pdet_query_candidates(self._h, c_void_p(Q.data_ptr()), nq, ctypes.byref(p),
                                           c_void_p(ids.data_ptr()), c_void_p(dists.data_ptr()),
                                           c_void_p(st.data_ptr()), c_void_p(cand.data_ptr()),
                                           int(cand_cap), _stream(stream)))
        if k_per_query is None:
            ids, dists = ids.view(nq, k), dists.view(nq, k)
        cn, sn = cand.cpu().numpy(), st.cpu().numpy()
        cands = [np.sort(cn[q, :min(int(sn[q, QSTAT["ncand"]]), cand_cap)]) for q in range(nq)]
        return ids, dists, st, cands


class Plan:
    """A captured launch sequence for one batch (HIP graph); replay with ``launch()``.
    Outputs live in ``ids`` / ``dists`` (flat CSR in query order) and ``qstats``."""

    def __init__(self, index, Q, k, c, beta, r_min, eps, precision, rescore, k_per_query,
                 c_per_query, stats):
        import torch
        self.index, self.Q = index, Q
        nq = Q.shape[0]
        p, keep = index._params(k, c, beta, r_min, eps, precision, rescore, k_per_query,
                                c_per_query)
        total = int(keep[0].sum()) if keep[0] is not None else nq * k
        self.ids = torch.empty(total, dtype=torch.int64, device=Q.device)
        self.dists = torch.empty(total, dtype=torch.float32, device=Q.device)
        self.qstats = (torch.empty((nq, QSTAT_WORDS), dtype=torch.int32, device=Q.device)
                       if stats else None)
        h = c_void_p()
        torch.cuda.synchronize()
        _check(lib().pdet_plan_create(index._h, c_void_p(Q.data_ptr()), nq, ctypes.byref(p),
                                      c_void_p(self.ids.data_ptr()), c_void_p(self.dists.data_ptr()),
                                      c_void_p(self.qstats.data_ptr()) if stats else None,
                                      ctypes.byref(h)))
        self._h, self._lib = h, lib()

    def launch(self, stream=None):
        _check(lib().pdet_plan_launch(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pdet_plan_free(self._h)
            self._h = None

    __del__ = close


class Server:
    """Continuous-batching request loop over a resident index (see pdet.h)."""

    def __init__(self, index, max_batch, lanes, k_max, precision, rescore, beta, r_min, eps,
                 memory_budget):
        self.index, self.k_max = index, k_max
        p = ServerParams(max_batch, lanes, k_max, PRECISIONS[precision], rescore, beta, r_min,
                         eps, memory_budget)
        h = c_void_p()
        _check(lib().pdet_server_create(index._h, ctypes.byref(p), ctypes.byref(h)))
        self._h, self._lib = h, lib()

    def submit(self, q: np.ndarray, k: int, c: float = 1.5) -> int:
        q = np.ascontiguousarray(q, dtype=np.float32)
        rid = c_int64()
        _check(lib().pdet_server_submit(self._h, q.ctypes.data_as(c_void_p), k, c,
                                        ctypes.byref(rid)))
        return rid.value

    def wait(self, rid: int, k: int):
        ids = np.empty(k, dtype=np.int64)
        dists = np.empty(k, dtype=np.float32)
        lat = c_double()
        _check(lib().pdet_server_wait(self._h, rid, ids.ctypes.data_as(c_void_p),
                                      dists.ctypes.data_as(c_void_p), ctypes.byref(lat)))
        return ids, dists, lat.value

    def offer_poisson(self, Q: np.ndarray, nreq: int, rate_qps: float, k: int, c: float = 1.5,
                      seed: int = 0) -> float:
        """Native Poisson client (pdet_server_offer_poisson); returns the offered rate."""
        Q = np.ascontiguousarray(Q, dtype=np.float32)
        off = c_double()
        _check(lib().pdet_server_offer_poisson(self._h, Q.ctypes.data_as(c_void_p), Q.shape[0],
                                               int(nreq), float(rate_qps), int(k), float(c),
                                               int(seed), ctypes.byref(off)))
        return off.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().pdet_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pdet_server_free(self._h)
            self._h = None

    __del__ = close
