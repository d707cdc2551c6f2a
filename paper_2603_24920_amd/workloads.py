"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke run.

This module only draws random numbers: datasets, queries, the Gaussian
projection matrix and the sample ids. It holds none of the method's
arithmetic (no projection, no breakpoints, no encoding, no search), so both
the GPU path and the CPU oracle can consume its output without sharing code.

The paper measures on public datasets (SIFT, Deep, SPACEV, ...; Table 2 of the
experimental section) that are not available here. The generators below stand
in for them with the same shapes and value structure:

* ``gauss_mixture``: isotropic Gaussian mixture, centres ~ N(0, s^2 I), noise
  sigma, optionally L2-normalised rows (Deep/Turing-like float data).
* ``int_mixture``: integer-valued coordinates in [0, 255] stored as float32,
  clustered around integer centres (SIFT-like byte data).

Every generator is deterministic in its seed. Large sets are drawn in row
chunks from ``SeedSequence.spawn`` children, so a set can be streamed chunk
by chunk and reproduces bit for bit.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CHUNK_ROWS = 1 << 20


def _rng(seed) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _centres(kind: str, n_centres: int, d: int, seed: int, centre_std: float) -> np.ndarray:
    ss = np.random.SeedSequence(seed)
    crng = _rng(ss.spawn(1)[0])
    if kind == "gauss":
        return crng.standard_normal((n_centres, d)) * centre_std
    if kind == "int":
        return crng.integers(0, 256, size=(n_centres, d)).astype(np.float64)
    raise ValueError(kind)


def _draw_rows(kind, centres, rows, rng, sigma, normalize):
    lab = rng.integers(0, centres.shape[0], size=rows)
    x = centres[lab] + rng.standard_normal((rows, centres.shape[1])) * sigma
    if kind == "int":
        x = np.clip(np.rint(x), 0, 255)
    if normalize:
        x = x / np.linalg.norm(x, axis=1, keepdims=True)
    return x.astype(np.float32)


def mixture(kind: str, n: int, d: int, n_centres: int, sigma: float, seed: int,
            centre_seed: int | None = None, centre_std: float = 1.0,
            normalize: bool = False, threads: int = 1, progress=None) -> np.ndarray:
    """Draw ``n`` rows of a clustered mixture (float32, row-major [n][d]).

    ``centre_seed`` fixes the centres (defaults to ``seed``) so that queries can
    be fresh draws from the mixture of a dataset: same centres, other seed.
    Chunks have their own generators, so ``threads`` > 1 draws several chunks at
    once (numpy releases the GIL while filling) with the same result.
    ``progress(done_chunks, total_chunks)`` is called as chunks finish.
    """
    cs = seed if centre_seed is None else centre_seed
    centres = _centres(kind, n_centres, d, cs, centre_std)
    out = np.empty((n, d), dtype=np.float32)
    nchunks = max(1, math.ceil(n / CHUNK_ROWS))
    children = np.random.SeedSequence(seed).spawn(nchunks + 1)[1:]

    def one(c):
        lo, hi = c * CHUNK_ROWS, min(n, (c + 1) * CHUNK_ROWS)
        out[lo:hi] = _draw_rows(kind, centres, hi - lo, _rng(children[c]), sigma, normalize)

    if threads <= 1 or nchunks == 1:
        for c in range(nchunks):
            one(c)
            if progress is not None:
                progress(c + 1, nchunks)
        return out
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=threads) as ex:
        for done, _ in enumerate(ex.map(one, range(nchunks)), 1):
            if progress is not None:
                progress(done, nchunks)
    return out


def projection_matrix(d: int, L: int, K: int, seed: int) -> np.ndarray:
    """Gaussian hash vectors: float32 [d][L*K] row-major, column i*K+j is a_ij ~ N(0, I_d)."""
    return _rng(seed).standard_normal((d, L * K)).astype(np.float32)


def sample_size(n: int, frac: float, Nr: int) -> int:
    """Number of sampled points used for breakpoint selection.

    The paper samples a fraction of the points (0.1 n by default). Its rank
    formula needs at least one sampled point per region, so the sample is
    floored at Nr^2 points (so every region holds >= Nr sampled points) and
    capped at n.
    """
    return int(min(n, max(math.ceil(frac * n), Nr * Nr)))


def sample_ids(n: int, n_s: int, seed: int) -> np.ndarray:
    """``n_s`` distinct point ids drawn uniformly without replacement, ascending, int64."""
    if n_s >= n:
        return np.arange(n, dtype=np.int64)
    return np.sort(_rng(seed).choice(n, size=n_s, replace=False)).astype(np.int64)


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic configuration: data recipe, index parameters and query recipe."""
    name: str
    kind: str           # "gauss" or "int"
    n: int
    d: int
    n_centres: int
    centre_std: float
    sigma: float
    normalize: bool
    L: int
    K: int
    Nr: int
    sample_frac: float
    max_leaf: int
    nq: int
    k: int
    c: float
    beta: float
    seed_base: int

    @property
    def seeds(self):
        b = self.seed_base
        return dict(data=b, queries=b + 1, proj=b + 2, sample=b + 3)

    def data(self, n: int | None = None, threads: int = 1, progress=None) -> np.ndarray:
        return mixture(self.kind, self.n if n is None else n, self.d, self.n_centres, self.sigma,
                       self.seeds["data"], centre_std=self.centre_std, normalize=self.normalize,
                       threads=threads, progress=progress)

    def queries(self, nq: int | None = None) -> np.ndarray:
        return mixture(self.kind, self.nq if nq is None else nq, self.d, self.n_centres, self.sigma,
                       self.seeds["queries"], centre_seed=self.seeds["data"],
                       centre_std=self.centre_std, normalize=self.normalize)

    def proj(self) -> np.ndarray:
        return projection_matrix(self.d, self.L, self.K, self.seeds["proj"])

    def sample(self, n: int | None = None) -> np.ndarray:
        nn = self.n if n is None else n
        return sample_ids(nn, sample_size(nn, self.sample_frac, self.Nr), self.seeds["sample"])

    def scaled(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Gaussian mixture, 16 centres ~ N(0, 10^2 I), unit noise; small enough for the oracle.
SMALL_MIXTURE = Workload("mixture-10k-d128", "gauss", 10_000, 128, 16, 10.0, 1.0, False,
                         4, 16, 256, 0.01, 128, 100, 10, 1.5, 0.1, 0)
# SIFT-like bytes: 1,000 integer centres in [0,255], noise sigma 8, rounded and clipped.
SIFT_LIKE_1M = Workload("sift-like-1M-d128", "int", 1_000_000, 128, 1000, 1.0, 8.0, False,
                        4, 16, 256, 0.1, 128, 10_000, 50, 1.5, 0.1, 1000)
# High-dimensional L2-normalised mixture (precision form).
NORMED_1M_D960 = Workload("normed-1M-d960", "gauss", 1_000_000, 960, 256, 1.0, 0.5, True,
                          4, 16, 256, 0.1, 128, 1000, 10, 1.5, 0.1, 2000)
# SIFT-like bytes at 100M points (batching form).
SIFT_LIKE_100M = Workload("sift-like-100M-d128", "int", 100_000_000, 128, 1000, 1.0, 8.0, False,
                          4, 16, 256, 0.1, 128, 10_000, 10, 1.5, 0.1, 3000)
# Deep-like unit-norm mixture, 4,096 centres (serving form).
NORMED_10M_D256 = Workload("normed-10M-d256", "gauss", 10_000_000, 256, 4096, 1.0, 0.5, True,
                           4, 16, 256, 0.1, 128, 10_000, 10, 1.5, 0.1, 4000)

WORKLOADS = {w.name: w for w in (SMALL_MIXTURE, SIFT_LIKE_1M, NORMED_1M_D960, SIFT_LIKE_100M,
                                 NORMED_10M_D256)}
