"""Dense brute force for pinning the sparse oracle on tiny matrices (N <= ~200).

TEST INFRASTRUCTURE ONLY.  Independent of oracle.c: works on a dense array and knows
nothing about patterns, closures or sparse storage.

dense_lu: left-looking LU of A(:,Q) with threshold partial pivoting, the elimination of
Section 1.3's "numerical factorization with pivoting" done the textbook dense way.  For
column j it applies every earlier step k in ascending order (structurally absent
updates multiply by an exact zero and leave values unchanged), chooses the pivot among
all not-yet-pivoted rows with the same rule as the sparse code (diagonal row if
|x_c| >= tau * max, else the largest magnitude, ties to the smaller row), and divides.
Products and differences are separate numpy ufuncs, so each is rounded once, as in the
C code.
"""
from __future__ import annotations

import numpy as np


def dense_lu(A: np.ndarray, Q: np.ndarray, tau: float):
    """Returns (prow, Lfull, Ufull): Lfull[i, j] is L(row i, step j) for original row i;
    Ufull[k, j] is U(step k, step j).  Raises ZeroDivisionError for a singular column."""
    n = A.shape[0]
    Lfull = np.zeros((n, n))
    Ufull = np.zeros((n, n))
    prow = np.full(n, -1, dtype=np.int64)
    pivoted = np.zeros(n, dtype=bool)
    for j in range(n):
        c = int(Q[j])
        x = A[:, c].astype(np.float64).copy()
        for k in range(j):
            u = x[prow[k]]
            Ufull[k, j] = u
            x = x - Lfull[:, k] * u
        cand = np.flatnonzero(~pivoted)
        mags = np.abs(x[cand])
        amax = mags.max() if cand.size else 0.0
        if not amax > 0.0:
            raise ZeroDivisionError("singular column %d" % j)
        piv = int(cand[int(np.argmax(mags))])  # first maximum = smallest row
        if not pivoted[c] and abs(x[c]) >= tau * amax:
            piv = c
        ujj = x[piv]
        Ufull[j, j] = ujj
        prow[j] = piv
        pivoted[piv] = True
        others = cand[cand != piv]
        Lfull[others, j] = x[others] / ujj
    return prow, Lfull, Ufull


def dense_solve(prow, Lfull, Ufull, Q, b, dtype=np.float64):
    """x = Q U^-1 L^-1 P b, scalar loops over the dense factors, every operation in `dtype`
    (b rounded to it first; float32 factors with dtype=np.float32 give a binary32 solve).
    Returns float64."""
    n = b.size
    Lfull = np.asarray(Lfull).astype(dtype)
    Ufull = np.asarray(Ufull).astype(dtype)
    w = b.astype(dtype).copy()
    z = np.zeros(n, dtype=dtype)
    for k in range(n):
        z[k] = w[prow[k]]
        w = w - Lfull[:, k] * z[k]
    for j in range(n - 1, -1, -1):
        z[j] = z[j] / Ufull[j, j]
        z[:j] = z[:j] - Ufull[:j, j] * z[j]
    x = np.zeros(n)
    x[np.asarray(Q)] = z.astype(np.float64)
    return x


def dense_lu_static(A: np.ndarray, Q: np.ndarray, prow: np.ndarray, dtype=np.float64):
    """Left-looking LU of A(:,Q) with the row of each step fixed to prow (static pivots),
    computed entirely in `dtype` (float64 or float32).  No guard: the caller picks inputs
    whose pivots stay well away from zero.  Returns (Lfull, Ufull) like dense_lu."""
    n = A.shape[0]
    A = A.astype(dtype)
    Lfull = np.zeros((n, n), dtype=dtype)
    Ufull = np.zeros((n, n), dtype=dtype)
    done = np.zeros(n, dtype=bool)
    for j in range(n):
        x = A[:, int(Q[j])].copy()
        for k in range(j):
            u = x[prow[k]]
            Ufull[k, j] = u
            x = x - Lfull[:, k] * u
        piv = int(prow[j])
        Ufull[j, j] = x[piv]
        done[piv] = True
        rest = np.flatnonzero(~done)
        Lfull[rest, j] = x[rest] / x[piv]
    return Lfull, Ufull


def dense_symbolic(Apat: np.ndarray, Q: np.ndarray, prow: np.ndarray):
    """Boolean elimination with a given pivot sequence: the structural patterns of L and U
    (structure only, no values), for comparing with the sparse code's reach closure."""
    n = Apat.shape[0]
    Lpat = np.zeros((n, n), dtype=bool)
    Upat = np.zeros((n, n), dtype=bool)
    pivoted = np.zeros(n, dtype=bool)
    for j in range(n):
        x = Apat[:, int(Q[j])].astype(bool).copy()
        for k in range(j):
            if x[prow[k]]:
                Upat[k, j] = True
                x |= Lpat[:, k]
        Upat[j, j] = True
        pivoted[prow[j]] = True
        Lpat[:, j] = x & ~pivoted
    return Lpat, Upat


def md_order_bruteforce(n: int, edges) -> list:
    """Exact minimum degree by explicit elimination-graph sets: repeatedly take the live
    vertex of least degree (ties: smallest index), join its neighbours into a clique and
    drop it.  Pure Python, tiny graphs only."""
    adj = [set() for _ in range(n)]
    for a, b in edges:
        if a != b:
            adj[a].add(b)
            adj[b].add(a)
    alive = set(range(n))
    order = []
    while alive:
        v = min(alive, key=lambda u: (len(adj[u]), u))
        order.append(v)
        alive.discard(v)
        nb = adj[v]
        for u in nb:
            adj[u] |= nb
            adj[u].discard(u)
            adj[u].discard(v)
        adj[v] = set()
    return order
