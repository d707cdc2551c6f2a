"""CPU oracle for DET-LSH (arxiv 2603.24920). TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 restatement of the method, written from the paper's text.
Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
it; the library never calls it, and it shares no code with the GPU path.

Every function names the passage it follows. Readings of points where the paper
is silent or ambiguous are stated where they are used:

* Encoding ties (Algorithm 1, the binary-search step): a value equal to a
  breakpoint goes to the higher region (upper-bound rule). Region symbols are
  the 0-based region index; the first-layer bit of a dimension is the most
  significant of its log2(Nr) bits.
* Outer breakpoints (encoding phase, breakpoint formula): interior breakpoints
  come from the sample at the paper's 1-based ranks floor(ns/Nr)*(z-1); the two
  outer ones are the min and max over all n points, so every point lies inside
  its node's box.
* Tree creation (Algorithm 2 and the node-split rule of the indexing phase): a
  bulk, insertion-order-free build. A node is split iff its full point set has
  more than max_leaf points and some dimension still has an unrefined bit. The
  split dimension minimises |#bit0 - #bit1|, ties to the smallest dimension.
  Nodes with no points are not leaves. Leaves are numbered in depth-first order
  (first-layer nodes by ascending key, bit-0 child first); inside a leaf,
  points are in ascending id order.
* Node bounds (the bound-distance example of the parallel query section): per
  dimension, the distance from q' to the node's breakpoint interval (zero
  inside), combined as a Euclidean norm; the upper bound takes the far edge.
* Query (Algorithm 5 with the two optimisations of the query-phase
  self-evaluation): a leaf is admitted whole when its lower bound does not
  exceed eps*r; admitted leaves of one tree and round go in ascending
  (lower bound, leaf ordinal) order; stop rule A (|S| >= ceil(beta*n)+k) is
  checked after every admitted leaf; stop rule B (at least k points of S within
  c*r) after all L trees of a round. Leaves admitted in an earlier round are
  not admitted again. Bounds are compared squared: LB^2 <= (eps*r)^2.
* Literal query (Algorithms 3 and 4, and Algorithm 5 as printed): a leaf is pruned
  when its lower bound exceeds r', taken whole when its upper bound is at most r',
  and otherwise only its points at projected distance smaller than r' (strict, as
  Algorithm 3 words it) are taken; stop rule A is checked once per tree.
* Top-k: smallest (distance, id), returned in ascending order.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


# ---------------------------------------------------------------- projection
def project(X: np.ndarray, A: np.ndarray) -> np.ndarray:
    """Hash values h_ij(o) = a_ij . o for every point (Eq. 1, the Euclidean LSH family).

    X: [n][d] (float32 promoted), A: [d][L*K] with column i*K+j = a_ij.
    Returns FP64 [n][L*K].
    """
    return np.asarray(X, dtype=np.float64) @ np.asarray(A, dtype=np.float64)


# --------------------------------------------------------------- breakpoints
def breakpoints(H_sample: np.ndarray, Nr: int, col_min: np.ndarray, col_max: np.ndarray) -> np.ndarray:
    """Dynamic breakpoints (encoding phase, dynamic encoding scheme; Algorithm 1 step 2).

    For each column, sort the sampled hash values ascending (C-up, 1-based) and
    take B(z) = C-up(m*(z-1)) for z = 2..Nr with m = floor(ns/Nr). B(1) and
    B(Nr+1) are the column min and max over all points.

    Returns FP64 [L*K][Nr+1]; entry [col][u] is B(u+1).
    """
    ns, LK = H_sample.shape
    m = ns // Nr
    if m < 1:
        raise ValueError("sample smaller than the number of regions")
    B = np.empty((LK, Nr + 1), dtype=np.float64)
    for col in range(LK):
        srt = np.sort(H_sample[:, col])
        B[col, 0] = col_min[col]
        for z in range(2, Nr + 1):
            B[col, z - 1] = srt[m * (z - 1) - 1]     # 1-based rank m*(z-1)
        B[col, Nr] = col_max[col]
    return B


def encode(H: np.ndarray, B: np.ndarray, L: int, K: int) -> np.ndarray:
    """Region symbols (Algorithm 1, encoding loop): code = #{z in 2..Nr : B(z) <= h}.

    Returns uint8 [L][n][K].
    """
    n = H.shape[0]
    codes = np.empty((L, n, K), dtype=np.uint8)
    for i in range(L):
        for j in range(K):
            col = i * K + j
            interior = B[col, 1:-1]
            codes[i, :, j] = np.searchsorted(interior, H[:, col], side="right")
    return codes


# ---------------------------------------------------------------- DE-Tree
@dataclasses.dataclass
class Tree:
    """One DE-Tree, flattened: leaves in depth-first order over a point permutation."""
    perm: np.ndarray          # int64 [n]: point ids, leaf by leaf
    leaf_start: np.ndarray    # int64 [nl]
    leaf_count: np.ndarray    # int64 [nl]
    leaf_depth: np.ndarray    # int64 [nl][K]: refined bits per dimension (t_j)
    leaf_prefix: np.ndarray   # int64 [nl][K]: the t_j leading bits of the codes

    @property
    def nl(self) -> int:
        return len(self.leaf_start)

    def hidx(self) -> np.ndarray:
        """Node id per dimension: (1 << t_j) | prefix_j."""
        return (np.left_shift(1, self.leaf_depth) | self.leaf_prefix).astype(np.int64)


def first_layer_key(codes_i: np.ndarray, bits: int) -> np.ndarray:
    """First-layer node of each point (Algorithm 2 step 2): the leading code bit of every
    dimension, dimension 0 most significant."""
    n, K = codes_i.shape
    msb = (codes_i.astype(np.int64) >> (bits - 1)) & 1
    key = np.zeros(n, dtype=np.int64)
    for j in range(K):
        key |= msb[:, j] << (K - 1 - j)
    return key


def choose_split(codes_node: np.ndarray, depth: np.ndarray, bits: int) -> int:
    """Node split rule (indexing phase): the dimension whose next bit divides the node's
    points most evenly. Returns -1 when every dimension is fully refined."""
    m, K = codes_node.shape
    best, best_score = -1, None
    for j in range(K):
        t = int(depth[j])
        if t >= bits:
            continue
        cnt1 = int(((codes_node[:, j].astype(np.int64) >> (bits - 1 - t)) & 1).sum())
        score = abs(2 * cnt1 - m)
        if best_score is None or score < best_score:
            best, best_score = j, score
    return best


def build_tree(codes_i: np.ndarray, Nr: int, max_leaf: int) -> Tree:
    """Create one DE-Tree from the codes of one projected space (Algorithm 2, bulk form).

    codes_i: uint8 [n][K]. The root has 2^K first-layer children keyed by the leading
    bits; a node with more than ``max_leaf`` points is split in two on one dimension by
    one more bit (binary refinement).
    """
    n, K = codes_i.shape
    bits = int(round(math.log2(Nr)))
    key = first_layer_key(codes_i, bits)
    order = np.lexsort((np.arange(n), key))            # by key, then id
    keys_sorted = key[order]
    uniq, first = np.unique(keys_sorted, return_index=True)
    bounds = list(first) + [n]

    perm, starts, counts, depths, prefixes = [], [], [], [], []
    pos = 0
    for u in range(len(uniq)):
        ids = order[bounds[u]:bounds[u + 1]]           # ascending id inside the node
        k0 = int(uniq[u])
        depth = np.ones(K, dtype=np.int64)
        prefix = np.array([(k0 >> (K - 1 - j)) & 1 for j in range(K)], dtype=np.int64)
        stack = [(ids, depth, prefix)]
        while stack:
            pts, dep, pre = stack.pop()
            if len(pts) == 0:
                continue
            j = -1 if len(pts) <= max_leaf else choose_split(codes_i[pts], dep, bits)
            if j < 0:
                perm.append(pts)
                starts.append(pos)
                counts.append(len(pts))
                depths.append(dep.copy())
                prefixes.append(pre.copy())
                pos += len(pts)
                continue
            bit = (codes_i[pts, j].astype(np.int64) >> (bits - 1 - dep[j])) & 1
            d1 = dep.copy(); d1[j] += 1
            p0 = pre.copy(); p0[j] = pre[j] * 2
            p1 = pre.copy(); p1[j] = pre[j] * 2 + 1
            stack.append((pts[bit == 1], d1, p1))      # popped second
            stack.append((pts[bit == 0], d1, p0))      # bit-0 child first
    return Tree(np.concatenate(perm).astype(np.int64), np.array(starts, dtype=np.int64),
                np.array(counts, dtype=np.int64), np.array(depths, dtype=np.int64).reshape(-1, K),
                np.array(prefixes, dtype=np.int64).reshape(-1, K))


# ---------------------------------------------------------------- bounds
def leaf_boxes(tree: Tree, B_tree: np.ndarray, Nr: int):
    """Breakpoint interval of every leaf in every dimension (bound-distance example).

    A node fixing the t_j leading bits p_j of dimension j covers regions
    lo = p_j << (b - t_j) .. hi = ((p_j + 1) << (b - t_j)) - 1, i.e. the interval
    [B(lo+1), B(hi+2)]. B_tree: [K][Nr+1] (0-based, entry u is B(u+1)).
    Returns (lo, hi) FP64 [nl][K].
    """
    bits = int(round(math.log2(Nr)))
    sh = bits - tree.leaf_depth
    lo_code = tree.leaf_prefix << sh
    hi_code = ((tree.leaf_prefix + 1) << sh) - 1
    K = B_tree.shape[0]
    cols = np.arange(K)[None, :]
    return B_tree[cols, lo_code], B_tree[cols, hi_code + 1]


def lower_bound_sq(qp: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Squared lower-bound distance from projected query q' to each node box."""
    gap = np.maximum(0.0, np.maximum(lo - qp[None, :], qp[None, :] - hi))
    return (gap * gap).sum(axis=1)


def upper_bound_sq(qp: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Squared upper-bound distance (far edge per dimension)."""
    far = np.maximum(np.abs(qp[None, :] - lo), np.abs(qp[None, :] - hi))
    return (far * far).sum(axis=1)


# ---------------------------------------------------------------- parameters
def epsilon(K: int, L: int) -> float:
    """Projected-radius factor from Eq. 2 and Lemma 3: eps^2 = chi2 upper alpha1 quantile
    with K degrees of freedom, alpha1 = exp(-1/L)."""
    from scipy.stats import chi2
    return float(math.sqrt(chi2.isf(math.exp(-1.0 / L), K)))


def theoretical_beta(K: int, L: int, c: float) -> float:
    """beta = 2 - 2 alpha2^L with c^2 chi2_{alpha2}(K) = eps^2 (Lemma 3, Eq. 2)."""
    from scipy.stats import chi2
    eps2 = chi2.isf(math.exp(-1.0 / L), K)
    alpha2 = float(chi2.sf(eps2 / (c * c), K))
    return 2.0 - 2.0 * alpha2 ** L


# ---------------------------------------------------------------- index
@dataclasses.dataclass
class Index:
    n: int
    d: int
    L: int
    K: int
    Nr: int
    A: np.ndarray             # FP64 [d][L*K]
    B: np.ndarray             # FP64 [L*K][Nr+1]
    codes: np.ndarray         # uint8 [L][n][K]
    trees: list
    boxes: list               # per tree (lo, hi)


def build_index(X, A, sample_ids, L, K, Nr, max_leaf, B=None, codes=None) -> Index:
    """Encoding and indexing phases (Algorithms 1 and 2).

    ``B`` / ``codes`` may be given to rebuild later steps from supplied earlier ones
    (used to check the GPU step by step)."""
    X = np.asarray(X)
    n, d = X.shape
    A64 = np.asarray(A, dtype=np.float64)
    if codes is None or B is None:
        H = project(X, A64)
        if B is None:
            B = breakpoints(H[np.asarray(sample_ids)], Nr, H.min(axis=0), H.max(axis=0))
        if codes is None:
            codes = encode(H, B, L, K)
    trees, boxes = [], []
    for i in range(L):
        t = build_tree(codes[i], Nr, max_leaf)
        trees.append(t)
        boxes.append(leaf_boxes(t, B[i * K:(i + 1) * K], Nr))
    return Index(n, d, L, K, Nr, A64, np.asarray(B, dtype=np.float64), codes, trees, boxes)


# ---------------------------------------------------------------- query
@dataclasses.dataclass
class QueryResult:
    ids: np.ndarray           # int64 [k]
    dists: np.ndarray         # FP64 [k]
    rounds: int               # radius rounds started
    n_cand: int               # |S| at termination
    stop: str                 # "A" (|S| >= T) or "B" (k points within c*r)
    leaves: int               # admitted leaves
    cand: np.ndarray          # int64 [|S|]: S in insertion order
    radius: float             # r of the last round
    trace: list = dataclasses.field(default_factory=list)
    # one (round, tree, leaf ordinal, LB^2, new points) record per admitted leaf, in
    # admission order (the optimised query); the literal query records one
    # (round, tree, -1, eps*r, new points) per range query instead


def radius_ladder(r_min: float, c: float, rounds: int):
    """r = r_min, r_min*c, r_min*c^2, ... (preliminaries, c^2-ANN by growing radius)."""
    r = r_min
    for _ in range(rounds):
        yield r
        r = c * r


def _dist(X, ids, q64):
    return np.sqrt(((np.asarray(X)[ids].astype(np.float64) - q64) ** 2).sum(axis=1))


def query(index: Index, X, q, k: int, c: float, beta: float, r_min: float, eps: float,
          max_rounds: int = 255) -> QueryResult:
    """c^2-k-ANN query (Algorithm 5 with relaxed leaf admission and lower-bound order)."""
    X = np.asarray(X)
    n = index.n
    T = math.ceil(beta * n) + k
    q64 = np.asarray(q, dtype=np.float64)
    qp = q64 @ index.A
    inS = np.zeros(n, dtype=bool)
    cand, cdist, trace = [], [], []
    n_s = 0
    leaves = 0
    prev_t2 = -1.0
    rho = 0
    for rho, r in enumerate(radius_ladder(r_min, c, max_rounds)):
        t = eps * r
        t2 = t * t
        for i in range(index.L):
            tr = index.trees[i]
            lo, hi = index.boxes[i]
            lb2 = lower_bound_sq(qp[i * index.K:(i + 1) * index.K], lo, hi)
            adm = np.nonzero((lb2 <= t2) & (lb2 > prev_t2))[0]
            adm = adm[np.lexsort((adm, lb2[adm]))]
            for leaf in adm:
                leaves += 1
                ids = tr.perm[tr.leaf_start[leaf]:tr.leaf_start[leaf] + tr.leaf_count[leaf]]
                new = ids[~inS[ids]]
                trace.append((rho, i, int(leaf), float(lb2[leaf]), len(new)))
                if len(new):
                    inS[new] = True
                    n_s += len(new)
                    cand.append(new)
                    cdist.append(_dist(X, new, q64))
                if n_s >= T:
                    return _finish(cand, cdist, k, rho + 1, "A", leaves, r, trace)
        if n_s >= k:
            alld = np.concatenate(cdist)
            if np.partition(alld, k - 1)[k - 1] <= c * r:
                return _finish(cand, cdist, k, rho + 1, "B", leaves, r, trace)
        prev_t2 = t2
    raise RuntimeError("radius ladder exhausted")


def _finish(cand, cdist, k, rounds, stop, leaves, r, trace=()) -> QueryResult:
    allc, alld = np.concatenate(cand), np.concatenate(cdist)
    o = np.lexsort((allc, alld))[:k]
    return QueryResult(allc[o], alld[o], rounds, len(allc), stop, leaves, allc, r, list(trace))


# ------------------------------------------------ literal query (Algorithms 3 and 4)
def range_query_literal(index: Index, X, i: int, qp_i: np.ndarray, r_prime: float):
    """DET Range Query on tree i (Algorithm 3, as the query phase describes it).

    Leaves whose lower bound exceeds r' are pruned (a pruned inner node prunes every
    leaf below it, and bounds only tighten towards the leaves, so testing the leaves
    gives the same set). A leaf whose upper bound is at most r' contributes all of its
    points; a leaf with LB <= r' < UB contributes the points whose projected distance
    to q' is smaller than r'. Projections are recomputed from X in FP64 (Eq. 1).
    Returns (ids ascending, leaves examined, leaves taken whole)."""
    tr = index.trees[i]
    lo, hi = index.boxes[i]
    K = index.K
    qp_i = np.asarray(qp_i, dtype=np.float64)
    lb2 = lower_bound_sq(qp_i, lo, hi)
    ub2 = upper_bound_sq(qp_i, lo, hi)
    r2 = r_prime * r_prime
    out, examined, whole = [], 0, 0
    A_i = index.A[:, i * K:(i + 1) * K]
    for leaf in range(tr.nl):
        if lb2[leaf] > r2:
            continue
        examined += 1
        ids = tr.perm[tr.leaf_start[leaf]:tr.leaf_start[leaf] + tr.leaf_count[leaf]]
        if ub2[leaf] <= r2:
            whole += 1
            out.append(ids)
            continue
        h = np.asarray(X)[ids].astype(np.float64) @ A_i
        dist2 = ((h - qp_i[None, :]) ** 2).sum(axis=1)
        out.append(ids[dist2 < r2])
    ids = np.sort(np.concatenate(out)) if out else np.empty(0, dtype=np.int64)
    return ids.astype(np.int64), examined, whole


def rc_ann_query(index: Index, X, q, c: float, r: float, beta: float, eps: float):
    """(r,c)-ANN query (Algorithm 4): range queries at eps*r tree by tree; once
    |S| >= beta*n + 1 the point of S closest to q is returned; after all L trees the
    closest point of S is returned if some point of S lies within c*r, else None.
    Returns (id or None, distance or None, |S|, trees queried)."""
    n = index.n
    T1 = math.ceil(beta * n) + 1
    q64 = np.asarray(q, dtype=np.float64)
    qp = q64 @ index.A
    S = np.empty(0, dtype=np.int64)

    def closest(ids):
        d = _dist(X, ids, q64)
        o = np.lexsort((ids, d))[0]
        return int(ids[o]), float(d[o])

    for i in range(index.L):
        Si, _, _ = range_query_literal(index, X, i, qp[i * index.K:(i + 1) * index.K], eps * r)
        S = np.union1d(S, Si)
        if len(S) >= T1:
            return (*closest(S), len(S), i + 1)
    if len(S) and np.any(_dist(X, S, q64) <= c * r):
        return (*closest(S), len(S), index.L)
    return None, None, len(S), index.L


def query_literal(index: Index, X, q, k: int, c: float, beta: float, r_min: float, eps: float,
                  max_rounds: int = 255) -> QueryResult:
    """c^2-k-ANN query with the literal range query (Algorithm 5 as printed, without the
    optimisations of the query-phase self-evaluation): every round re-runs Algorithm 3 on
    each tree at eps*r, S is their union, stop rule A (|S| >= beta*n + k) is checked
    after each tree, stop rule B (k points of S within c*r) after all L trees."""
    X = np.asarray(X)
    n = index.n
    T = math.ceil(beta * n) + k
    q64 = np.asarray(q, dtype=np.float64)
    qp = q64 @ index.A
    inS = np.zeros(n, dtype=bool)
    cand, cdist, trace = [], [], []
    n_s = 0
    examined = 0
    for rho, r in enumerate(radius_ladder(r_min, c, max_rounds)):
        for i in range(index.L):
            Si, ex, _ = range_query_literal(index, X, i, qp[i * index.K:(i + 1) * index.K],
                                            eps * r)
            examined += ex
            new = Si[~inS[Si]]
            trace.append((rho, i, -1, eps * r, len(new)))
            if len(new):
                inS[new] = True
                n_s += len(new)
                cand.append(new)
                cdist.append(_dist(X, new, q64))
            if n_s >= T:
                return _finish(cand, cdist, k, rho + 1, "A", examined, r, trace)
        if n_s >= k:
            alld = np.concatenate(cdist)
            if np.partition(alld, k - 1)[k - 1] <= c * r:
                return _finish(cand, cdist, k, rho + 1, "B", examined, r, trace)
    raise RuntimeError("radius ladder exhausted")


# ---------------------------------------------------------------- brute force
def knn_exact(X, Q, k: int, block: int = 4096):
    """Exact k nearest neighbours by FP64 brute force (difference form), ties by id."""
    X64 = np.asarray(X, dtype=np.float64)
    ids_out = np.empty((len(Q), k), dtype=np.int64)
    d_out = np.empty((len(Q), k), dtype=np.float64)
    for qi, q in enumerate(np.asarray(Q, dtype=np.float64)):
        dist = np.empty(len(X64))
        for s in range(0, len(X64), block):
            dist[s:s + block] = np.sqrt(((X64[s:s + block] - q) ** 2).sum(axis=1))
        o = np.lexsort((np.arange(len(X64)), dist))[:k]
        ids_out[qi], d_out[qi] = o, dist[o]
    return ids_out, d_out


def recall(ids, exact_ids) -> float:
    """|R intersect R*| / k averaged over queries (evaluation measures)."""
    ids, exact_ids = np.asarray(ids), np.asarray(exact_ids)
    k = exact_ids.shape[1]
    return float(np.mean([len(np.intersect1d(a[:k], b)) / k for a, b in zip(ids, exact_ids)]))


def overall_ratio(dists, exact_dists) -> float:
    """(1/k) sum_i ||q,o_i|| / ||q,o*_i||, averaged over queries (evaluation measures)."""
    d, e = np.asarray(dists, dtype=np.float64), np.asarray(exact_dists, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(e > 0, d / e, 1.0)
    return float(r.mean())


# ------------------------------------------- parameters and radius schedule (Section 5.2)
def candidate_count(index: Index, q, r: float, eps: float) -> int:
    """|S| after one full round at radius r with no stop rule: the points whose leaf lower
    bound in some tree is within eps*r (relaxed admission, Section 6.2.2)."""
    qp = np.asarray(q, dtype=np.float64) @ index.A
    t2 = (eps * r) ** 2
    inS = np.zeros(index.n, dtype=bool)
    for i in range(index.L):
        tr = index.trees[i]
        lo, hi = index.boxes[i]
        lb2 = lower_bound_sq(qp[i * index.K:(i + 1) * index.K], lo, hi)
        for leaf in np.nonzero(lb2 <= t2)[0]:
            inS[tr.perm[tr.leaf_start[leaf]:tr.leaf_start[leaf] + tr.leaf_count[leaf]]] = True
    return int(inS.sum())


def magic_r_min(index: Index, q, k: int, beta: float, c: float, eps: float, r0: float,
                max_steps: int = 254):
    """The "magic" r_min of the parameter settings (Section 5.2.1) on the grid r0 * c^j:
    the smallest grid radius at which |S| >= beta*n + k, so that at one grid step below it
    |S| < beta*n + k. Returns (j, r) or None if the grid runs out."""
    T = math.ceil(beta * index.n) + k
    r = r0
    for j in range(max_steps + 1):
        if candidate_count(index, q, r, eps) >= T:
            return j, r
        r = c * r
    return None


def autotune_first_radius(B: np.ndarray, K: int, L: int) -> float:
    """First pilot radius of the dataset-level schedule: its projected threshold eps*r0 is
    1e-4 of the median breakpoint range (B(Nr+1) - B(1)) over the L*K columns (the upper
    median for an even count)."""
    rng = np.sort(np.asarray(B, dtype=np.float64)[:, -1] - np.asarray(B, dtype=np.float64)[:, 0])
    return max(1e-30, 1e-4 * rng[len(rng) // 2] / epsilon(K, L))


def autotune_r_min(index: Index, X, pilots, k: int, c: float, beta: float, eps: float,
                   r0: float) -> float:
    """Dataset-level r_min from pilot queries (a reading of Section 5.2.1, which defines the
    magic r_min per query): run Algorithm 5 from r0 for every pilot, take the median number
    of rounds started over the pilots (the upper median) and return the radius one grid
    step below the median terminating radius, r0 * c^max(0, median - 2). For a pilot that
    stops by rule A the terminating radius is its magic r_min on the r0 grid."""
    rounds = sorted(query(index, X, q, k, c, beta, r0, eps).rounds for q in pilots)
    med = rounds[len(rounds) // 2]
    r = r0
    for _ in range(max(0, med - 2)):
        r = c * r
    return r


def theoretical_beta_for(K: int, L: int, c) -> np.ndarray:
    """beta of Lemma 3 for each c (the library's theoretical mode takes it per query)."""
    return np.array([theoretical_beta(K, L, float(x)) for x in np.atleast_1d(c)])


# ------------------------------------------------ static encoding (Section 3.1, contrast)
def static_breakpoints(H_sample: np.ndarray, Nr: int, col_min: np.ndarray,
                       col_max: np.ndarray) -> np.ndarray:
    """Static iSAX breakpoints (the scheme the encoding phase contrasts with its dynamic
    one): interior breakpoints at the equal-mass quantiles of N(0,1), b_z = Phi^-1(z/Nr),
    applied to each projected coordinate after normalising it by its sampled mean and
    standard deviation (iSAX assumes normalised values): B(z) = mu + sigma * Phi^-1((z-1)/Nr)
    for z = 2..Nr. B(1) and B(Nr+1) are the column min and max over all points, as for the
    dynamic scheme. Returns FP64 [L*K][Nr+1]."""
    from scipy.stats import norm
    H = np.asarray(H_sample, dtype=np.float64)
    mu = H.mean(axis=0)
    sd = H.std(axis=0)
    z = norm.ppf(np.arange(1, Nr) / Nr)
    B = np.empty((H.shape[1], Nr + 1), dtype=np.float64)
    B[:, 0] = col_min
    B[:, 1:Nr] = mu[:, None] + sd[:, None] * z[None, :]
    B[:, Nr] = col_max
    return B
