"""Seeded synthetic KKT sequences shaped like the interior-point systems of the paper.

The paper solves sequences K_k dx_k = r_k (eq. (kktlinear), Section 1.2) whose matrices
share one sparsity pattern ("Summary" paragraph of Section 1.2).  Its own matrices
(ACTIVSg series, Table 1) are not available here, so this module draws stand-ins with
the same block structure and density (about 3 lower-triangle nonzeros per row):

    K = [[H + D, J^T],
         [J,     -delta I]]          delta = 1e-8 (dual regularisation)

* H (n x n): symmetric; pattern = a planar-like graph of average degree 3 (a Euclidean
  k-nearest-neighbour spanning forest plus the shortest remaining candidate edges),
  N(0,1) off-diagonals, diagonal shifted to 1 + sum |h_ij| (so H is SPD).
* D: diagonal, log-uniform over a configurable range (the X^{-1} Z term of Section 1.2,
  which is what makes K_k ill-conditioned as the barrier parameter goes to zero).
* J (m x n): three nonzeros per row at graph-neighbouring columns, N(0,1).
* Later steps redraw D, perturb H/J off-diagonal values by 1 % N(0,1) and draw a fresh
  right-hand side; the pattern never changes.

This module only draws inputs.  It holds none of the solver's arithmetic and is shared,
unchanged, by the CPU oracle and by the GPU library's tests and benchmark.

Random streams: numpy PCG64 seeded by SeedSequence([2401, config, pattern, step]); the
structure and the base values use step 0, the values of system k use step k.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
from scipy.spatial import cKDTree

BASE_SEED = 2401
DUAL_REG = 1e-8

#: Workload shapes: (n, m, log10 D range, number of systems in the sequence).
WORKLOAD_SHAPES = {
    1: dict(n=4_000, m=3_000, dlog=(-8.0, 8.0), steps=1),
    2: dict(n=35_000, m=25_000, dlog=(-10.0, 10.0), steps=20),
    3: dict(n=290_000, m=210_000, dlog=(-12.0, 12.0), steps=10),
    5: dict(n=1_150_000, m=850_000, dlog=(-12.0, 12.0), steps=5),
}
#: Serving workload: 8 pattern dimensions spread over 7,000 .. 500,000, n = round(0.58 N).
SERVING_DIMS = [7_000, 77_429, 147_857, 218_286, 288_714, 359_143, 429_571, 500_000]
SERVING_DLOG = (-10.0, 10.0)


def _rng(config: int, pattern: int, step: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, config, pattern, step])))


def _graph_edges(points: np.ndarray, n_edges: int):
    """Planar-like edge set: kNN(4) candidates, Kruskal forest first, then shortest extras.

    Returns (ei, ej) with ei < ej, in (length, min, max) order.
    """
    n = points.shape[0]
    k = min(4, n - 1)
    tree = cKDTree(points)
    _, nbr = tree.query(points, k=k + 1)
    src = np.repeat(np.arange(n, dtype=np.int64), k)
    dst = nbr[:, 1:].reshape(-1).astype(np.int64)
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    length = np.sqrt(((points[lo] - points[hi]) ** 2).sum(axis=1))
    order = np.lexsort((hi, lo, length))
    lo, hi, length = lo[order], hi[order], length[order]
    # Kruskal forest over the candidates.  Candidate lengths are distinct with probability
    # one, so the minimum spanning forest is unique and equals Kruskal's in sorted order.
    g = sp.coo_matrix((length, (lo, hi)), shape=(n, n)).tocsr()
    mst = csgraph.minimum_spanning_tree(g).tocoo()
    fkey = np.minimum(mst.row, mst.col).astype(np.int64) * n + np.maximum(mst.row, mst.col)
    forest_mask = np.isin(lo * n + hi, fkey)
    extra_needed = max(0, n_edges - int(forest_mask.sum()))
    extra_idx = np.flatnonzero(~forest_mask)[:extra_needed]
    keep = forest_mask.copy()
    keep[extra_idx] = True
    return lo[keep], hi[keep]


def _j_columns(n: int, ei: np.ndarray, ej: np.ndarray, anchors: np.ndarray) -> np.ndarray:
    """Three columns per J row: the anchor plus the first two vertices of a BFS from it
    (neighbours visited in ascending index).  Returns an (m, 3) array sorted per row."""
    adj = sp.coo_matrix((np.ones(2 * ei.size), (np.r_[ei, ej], np.r_[ej, ei])), shape=(n, n)).tocsr()
    adj.sum_duplicates()
    adj.sort_indices()
    ptr, ind = adj.indptr, adj.indices
    deg = np.diff(ptr)
    m = anchors.size
    cols = np.empty((m, 3), dtype=np.int64)
    cols[:, 0] = anchors
    d = deg[anchors]
    two = d >= 2
    cols[two, 1] = ind[ptr[anchors[two]]]
    cols[two, 2] = ind[ptr[anchors[two]] + 1]
    for r in np.flatnonzero(~two):
        c = anchors[r]
        if deg[c] == 0:
            raise ValueError("isolated vertex in the synthetic graph")
        u = ind[ptr[c]]
        nb = [v for v in ind[ptr[u]:ptr[u + 1]] if v != c]
        if not nb:
            raise ValueError("graph component too small for a 3-column J row")
        cols[r, 1] = u
        cols[r, 2] = nb[0]
    cols.sort(axis=1)
    return cols


@dataclasses.dataclass
class KKTPattern:
    """One sparsity pattern of the sequence plus everything needed to fill values."""
    config: int
    pattern: int
    n: int
    m: int
    dlog: tuple
    rowptr: np.ndarray        # int64, N+1
    colidx: np.ndarray        # int32, nnz (full matrix, sorted per row)
    # value sources, in CSR order, as indices into the per-step source vector
    _src: np.ndarray
    _edge_i: np.ndarray
    _edge_j: np.ndarray
    _h_base: np.ndarray
    _j_base: np.ndarray       # (m, 3)
    delta: float = DUAL_REG   # the (2,2) block is -delta I

    @property
    def N(self) -> int:
        return self.n + self.m

    @property
    def nnz(self) -> int:
        return int(self.colidx.size)

    @property
    def nnz_lower(self) -> int:
        return (self.nnz + self.N) // 2

    def system(self, step: int):
        """Values (float64, CSR order) and right-hand side of system `step` (1-based)."""
        if step < 1:
            raise ValueError("steps are numbered from 1")
        rng = _rng(self.config, self.pattern, step)
        n, m = self.n, self.m
        dvals = 10.0 ** rng.uniform(self.dlog[0], self.dlog[1], size=n)
        h = self._h_base
        jv = self._j_base
        if step >= 2:
            h = h * (1.0 + 0.01 * rng.standard_normal(h.size))
            jv = jv * (1.0 + 0.01 * rng.standard_normal(jv.shape))
        b = rng.standard_normal(n + m)
        hdiag = np.ones(n)
        np.add.at(hdiag, self._edge_i, np.abs(h))
        np.add.at(hdiag, self._edge_j, np.abs(h))
        # source vector layout: [h (E), h again for the mirror (E), H diag + D (n),
        #                        J (3m), J^T (3m), -delta (m)]
        src = np.concatenate([h, h, hdiag + dvals, jv.reshape(-1), jv.reshape(-1),
                              np.full(m, -self.delta)])
        return src[self._src], b


@functools.lru_cache(maxsize=16)
def make_pattern(config: int, pattern: int = 0, n: int | None = None, m: int | None = None,
                 dlog: tuple | None = None, delta: float = DUAL_REG) -> KKTPattern:
    """Build the pattern (and base values) for a workload; see the module docstring.
    `delta` sets the dual regularisation (the moderate family uses 1)."""
    if n is None:
        if config == 4:
            dim = SERVING_DIMS[pattern]
            n = int(round(0.58 * dim))
            m = dim - n
            dlog = SERVING_DLOG
        else:
            c = WORKLOAD_SHAPES[config]
            n, m, dlog = c["n"], c["m"], c["dlog"]
    if dlog is None:
        dlog = (-8.0, 8.0)
    if not (0 < m < n) or n < 6:
        raise ValueError("need 0 < m < n and n >= 6")
    rng = _rng(config, pattern, 0)
    points = rng.random((n, 2))
    ei, ej = _graph_edges(points, int(round(1.5 * n)))
    h_base = rng.standard_normal(ei.size)
    anchors = rng.permutation(n)[:m]
    jcols = _j_columns(n, ei, ej, anchors)
    j_base = rng.standard_normal((m, 3))

    N = n + m
    E = ei.size
    rows = np.concatenate([ei, ej, np.arange(n), n + np.repeat(np.arange(m), 3),
                           jcols.reshape(-1), n + np.arange(m)])
    cols = np.concatenate([ej, ei, np.arange(n), jcols.reshape(-1),
                           n + np.repeat(np.arange(m), 3), n + np.arange(m)])
    src = np.arange(rows.size, dtype=np.int64)
    order = np.lexsort((cols, rows))
    rows, cols, src = rows[order], cols[order], src[order]
    if np.any((rows[1:] == rows[:-1]) & (cols[1:] == cols[:-1])):
        raise ValueError("duplicate entry in the synthetic pattern")
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    assert rowptr[-1] == 2 * E + n + 6 * m + m
    return KKTPattern(config=config, pattern=pattern, n=n, m=m, dlog=tuple(dlog), rowptr=rowptr,
                      colidx=cols.astype(np.int32), _src=src, _edge_i=ei, _edge_j=ej,
                      _h_base=h_base, _j_base=j_base, delta=float(delta))


def small_kkt(n: int, m: int, seed: int, dlog=(-8.0, 8.0), delta: float = DUAL_REG) -> KKTPattern:
    """A tiny pattern of the same family, for brute-force checks (config id 0)."""
    return make_pattern(0, seed, n=n, m=m, dlog=tuple(dlog), delta=float(delta))


#: The moderately conditioned family: D log-uniform in [1e-2, 1e2], delta = 1.  With these
#: values the condition number is small enough that a forward-error bound of the form
#: 1e-8 * cond-estimate is informative (on the workload configs it is vacuous).
MODERATE_DLOG = (-2.0, 2.0)
MODERATE_DELTA = 1.0


def moderate_kkt(n: int, m: int, seed: int = 0) -> KKTPattern:
    """A pattern of the moderate family (config id 6) with the generator's structure."""
    return make_pattern(6, seed, n=n, m=m, dlog=MODERATE_DLOG, delta=MODERATE_DELTA)


def to_dense(rowptr: np.ndarray, colidx: np.ndarray, values: np.ndarray, N: int) -> np.ndarray:
    """Dense copy of a CSR matrix (tiny inputs only)."""
    a = np.zeros((N, N))
    for i in range(N):
        a[i, colidx[rowptr[i]:rowptr[i + 1]]] = values[rowptr[i]:rowptr[i + 1]]
    return a


class ArrowKKT:
    """A KKT matrix of the same block form with one dense constraint row ("arrow head"):
    H on a path graph (h_i,i+1 ~ N(0,1), diagonal 1 + sum |h_ij|), constraint 0 couples
    `dense` primal variables (every n/dense-th), constraints 1..m-1 three consecutive ones.
    A minimum-degree ordering eliminates the dense constraint last, so its factor column
    and its row of L hold about `dense` entries: long columns and rows of the kind the
    generator's planar-like graphs never produce.  Steps redraw D, perturb H/J by 1 % and
    draw a fresh right-hand side, as the generator does."""

    def __init__(self, n: int, m: int, dense: int, seed: int = 0, dlog=(-8.0, 8.0), delta: float = DUAL_REG):
        if not (2 <= m <= n - 3) or not (3 <= dense <= n):
            raise ValueError("need 2 <= m <= n - 3 and 3 <= dense <= n")
        self.n, self.m, self.dlog, self.delta, self.seed = n, m, tuple(dlog), float(delta), seed
        rng = np.random.default_rng([BASE_SEED, 7, seed, 0])
        self._h = rng.standard_normal(n - 1)
        cols = [np.unique(np.linspace(0, n - 1, dense).round().astype(np.int64))]
        starts = rng.integers(0, n - 2, size=m - 1)
        cols += [np.arange(s, s + 3) for s in starts]
        self._jcols = cols
        self._jbase = [rng.standard_normal(c.size) for c in cols]
        N = n + m
        rows, colsl, kind, idx = [], [], [], []
        # kind 0: h edge (idx = edge), 1: H diagonal (idx = i), 2: J entry (idx = flat), 3: -delta
        e = np.arange(n - 1)
        rows += [e, e + 1]; colsl += [e + 1, e]; kind += [np.zeros(n - 1, int)] * 2; idx += [e, e]
        rows.append(np.arange(n)); colsl.append(np.arange(n)); kind.append(np.ones(n, int)); idx.append(np.arange(n))
        flat = 0
        for r, c in enumerate(cols):
            fi = np.arange(flat, flat + c.size)
            rows += [np.full(c.size, n + r), c]; colsl += [c, np.full(c.size, n + r)]
            kind += [np.full(c.size, 2)] * 2; idx += [fi, fi]
            flat += c.size
        rows.append(n + np.arange(m)); colsl.append(n + np.arange(m)); kind.append(np.full(m, 3)); idx.append(np.arange(m))
        rows, colsl = np.concatenate(rows), np.concatenate(colsl)
        kind, idx = np.concatenate(kind), np.concatenate(idx)
        order = np.lexsort((colsl, rows))
        rows, colsl, self._kind, self._idx = rows[order], colsl[order], kind[order], idx[order]
        if np.any((rows[1:] == rows[:-1]) & (colsl[1:] == colsl[:-1])):
            raise ValueError("duplicate entry in the arrow pattern")
        rowptr = np.zeros(N + 1, dtype=np.int64)
        np.add.at(rowptr, rows + 1, 1)
        self.rowptr = np.cumsum(rowptr)
        self.colidx = colsl.astype(np.int32)

    @property
    def N(self) -> int:
        return self.n + self.m

    def system(self, step: int):
        if step < 1:
            raise ValueError("steps are numbered from 1")
        rng = np.random.default_rng([BASE_SEED, 7, self.seed, step])
        n = self.n
        d = 10.0 ** rng.uniform(self.dlog[0], self.dlog[1], size=n)
        h = self._h
        jv = np.concatenate(self._jbase)
        if step >= 2:
            h = h * (1.0 + 0.01 * rng.standard_normal(h.size))
            jv = jv * (1.0 + 0.01 * rng.standard_normal(jv.size))
        b = rng.standard_normal(self.N)
        hd = np.ones(n)
        np.add.at(hd, np.arange(n - 1), np.abs(h))
        np.add.at(hd, np.arange(1, n), np.abs(h))
        vals = np.empty(self._kind.size)
        k = self._kind
        vals[k == 0] = h[self._idx[k == 0]]
        vals[k == 1] = (hd + d)[self._idx[k == 1]]
        vals[k == 2] = jv[self._idx[k == 2]]
        vals[k == 3] = -self.delta
        return vals, b
