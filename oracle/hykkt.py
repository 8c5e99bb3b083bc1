"""HyKKT oracle (Section 5, eq. (kktlineargamma)): plain CPU reference for the GPU HyKKT path.

TEST INFRASTRUCTURE ONLY (tests/, the smoke check and the benchmark's CPU leg): it shares no
code with the GPU library.

The KKT system of eq. (kktlinear) has a zero (2,2) block:
    [[H + D, J^T], [J, 0]] [dx; dl] = [r_x; r_l].
Adding gamma J^T times the second block row to the first (which leaves the solution unchanged)
gives H_gamma = H + D + gamma J^T J, symmetric positive definite when H + D is (always for the
synthetic systems; for full-rank J and large enough gamma in general).  Then
    S dl = J H_gamma^-1 (r_x + gamma J^T r_l) - r_l,   S = J H_gamma^-1 J^T   (SPD),
solved by conjugate gradients with S applied as products (never formed), and
    dx = H_gamma^-1 (r_x + gamma J^T r_l - J^T dl).
H_gamma^-1 is applied with a factorization of H_gamma whose pattern is analysed once and
refactored per system without pivoting (here the oracle's LU with diagonal pivots, which for an
SPD matrix is the Cholesky factorization up to the diagonal scaling: U = diag(U) L^T).

Readings where the paper is silent:
  * gamma (the paper says "large enough"): gamma = gamma_scale * max_i (H + D)_ii /
    max_i (J^T J)_ii with gamma_scale = 1e4, from the first system, fixed for the sequence.
  * entries of H_gamma: (H + D)(i, j) + gamma * s(i, j), s(i, j) = sum over constraint rows r in
    ascending order of J(r, i) * J(r, j) (each product and sum rounded; the gamma product
    rounded, then added).  Pattern: that of H + D joined with the structural pattern of J^T J.
  * CG: x0 = 0, stop when ||r_k|| <= tol * ||r_0|| (tol 1e-12) or after max_iter iterations;
    the textbook recurrences (Hestenes and Stiefel): alpha = r.r / p.Sp, beta = r'.r' / r.r.
"""
from __future__ import annotations

import numpy as np

from . import LU, _csr

GAMMA_SCALE = 1e4


def split_kkt(rowptr, colidx, values, n):
    """Blocks of a full KKT CSR with n primal rows: (A = H + D as dict-of-rows, J rows), and the
    check that the (2,2) block holds only zeros.  Returns (A_rows, J_rows) where A_rows[i] maps
    column -> value for i < n and J_rows[r] maps column (< n) -> value for constraint r."""
    rp, ci, v = _csr(rowptr, colidx, values)
    N = rp.size - 1
    A_rows = [dict() for _ in range(n)]
    J_rows = [dict() for _ in range(N - n)]
    for i in range(N):
        for p in range(rp[i], rp[i + 1]):
            c = int(ci[p])
            if i < n and c < n:
                A_rows[i][c] = float(v[p])
            elif i >= n and c < n:
                J_rows[i - n][c] = float(v[p])
            elif i >= n and c >= n and v[p] != 0.0:
                raise ValueError("HyKKT needs a zero (2,2) block (eq. (kktlinear))")
    return A_rows, J_rows


def gamma_rule(A_rows, J_rows, n, scale=GAMMA_SCALE):
    """gamma = scale * max_i A_ii / max_i (J^T J)_ii (the (J^T J)_ii summed over rows in order)."""
    amax = max(A_rows[i].get(i, 0.0) for i in range(n))
    jtj = [0.0] * n
    for row in J_rows:
        for c, x in row.items():
            prod = x * x
            jtj[c] = jtj[c] + prod
    return scale * amax / max(jtj)


def h_gamma(rowptr, colidx, values, n, gamma):
    """H_gamma in CSR (int64 row pointers, int32 sorted columns, float64 values), entries as
    described in the module docstring."""
    A_rows, J_rows = split_kkt(rowptr, colidx, values, n)
    # for every primal column, the constraint rows that touch it, ascending
    col_rows = [[] for _ in range(n)]
    for r, row in enumerate(J_rows):
        for c in row:
            col_rows[c].append(r)
    rows_out = []
    for i in range(n):
        cols = set(A_rows[i])
        for r in col_rows[i]:
            cols.update(J_rows[r].keys())
        entries = []
        for j in sorted(cols):
            s = 0.0
            for r in col_rows[i]:  # ascending r
                if j in J_rows[r]:
                    prod = J_rows[r][i] * J_rows[r][j]
                    s = s + prod
            t = gamma * s
            entries.append((j, A_rows[i].get(j, 0.0) + t))
        rows_out.append(entries)
    rp = np.zeros(n + 1, np.int64)
    for i, e in enumerate(rows_out):
        rp[i + 1] = rp[i] + len(e)
    ci = np.array([j for e in rows_out for j, _ in e], np.int32)
    hv = np.array([x for e in rows_out for _, x in e], np.float64)
    return rp, ci, hv


class HyKKT:
    """Analysis of one KKT pattern for the HyKKT method: gamma from the first system, the
    pattern of H_gamma and its factorization (the ordering and pivots reused for later
    systems), then per system `solve`."""

    def __init__(self, rowptr, colidx, values_first, n, gamma=None, gamma_scale=GAMMA_SCALE):
        self.n = int(n)
        self.N = int(np.asarray(rowptr).size - 1)
        self.m = self.N - self.n
        A_rows, J_rows = split_kkt(rowptr, colidx, values_first, self.n)
        self.gamma = float(gamma) if gamma else gamma_rule(A_rows, J_rows, self.n, gamma_scale)
        self.hrp, self.hci, hv = h_gamma(rowptr, colidx, values_first, self.n, self.gamma)
        self.lu = LU(self.hrp, self.hci, hv)

    def refactor(self, rowptr, colidx, values):
        """(H_gamma values, L values, U values) of a later system with the fixed pivots."""
        _, _, hv = h_gamma(rowptr, colidx, values, self.n, self.gamma)
        lx, ux, _ = self.lu.refactor64(self.hrp, self.hci, hv)
        return hv, lx, ux

    def solve(self, rowptr, colidx, values, b, tol=1e-12, max_iter=1000):
        """HyKKT solution of K x = b; returns (x, info) with the CG iteration count and the CG
        relative residual."""
        rp, ci, v = _csr(rowptr, colidx, values)
        n, m = self.n, self.m
        _, lx, ux = self.refactor(rp, ci, v)
        K = _to_scipy(rp, ci, v, self.N)
        A = K[:n, :n]
        J = K[n:, :n].tocsr()
        JT = J.T.tocsr()
        del A
        b = np.asarray(b, np.float64)
        rx, rl = b[:n], b[n:]

        def hinv(y):
            return self.lu.solve(y, lx, ux)

        rhat = rx + self.gamma * (JT @ rl)
        c = J @ hinv(rhat) - rl
        lam = np.zeros(m)
        r = c.copy()
        p = r.copy()
        rr = float(r @ r)
        r0 = np.sqrt(rr)
        it = 0
        hist = [r0]
        while np.sqrt(rr) > tol * r0 and it < max_iter:
            q = J @ hinv(JT @ p)
            alpha = rr / float(p @ q)
            lam = lam + alpha * p
            r = r - alpha * q
            rr_new = float(r @ r)
            beta = rr_new / rr
            p = r + beta * p
            rr = rr_new
            it += 1
            hist.append(np.sqrt(rr))
        dx = hinv(rhat - JT @ lam)
        x = np.concatenate([dx, lam])
        return x, dict(cg_iterations=it, cg_rel_resid=np.sqrt(rr) / r0 if r0 > 0 else 0.0,
                       converged=bool(np.sqrt(rr) <= tol * r0), gamma=self.gamma, hist=np.array(hist))


def _to_scipy(rp, ci, v, N):
    import scipy.sparse as sp
    return sp.csr_matrix((v, ci, rp), shape=(N, N))
