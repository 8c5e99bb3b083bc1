"""Pins of the HyKKT oracle (Section 5, eq. (kktlineargamma)) against what the mathematics fixes:
the entries of H_gamma against a dense product, the solution against a dense solve of the
original system (the transformation leaves it unchanged), a decoupled KKT whose Schur
complement is diagonal (closed-form solution, CG converging in as many iterations as it has
distinct eigenvalues) and the gamma rule on a hand-computed case."""
import numpy as np
import pytest

import kkt_synth as ks
import oracle
from oracle import hykkt as hy


def dense(rp, ci, v, N):
    return ks.to_dense(rp, ci, v, N)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_h_gamma_matches_dense_product(seed):
    p = ks.small_kkt(40, 25, 500 + seed, dlog=(-3.0, 3.0), delta=0.0)
    v, _ = p.system(2)
    K = dense(p.rowptr, p.colidx, v, p.N)
    n = p.n
    A, J = K[:n, :n], K[n:, :n]
    gamma = 123.25
    rp, ci, hv = hy.h_gamma(p.rowptr, p.colidx, v, n, gamma)
    Hd = A + gamma * (J.T @ J)
    H = dense(rp, ci, hv, n)
    # every nonzero of the dense product is in the pattern, and the values agree to rounding
    assert np.all((Hd != 0) <= (dense(rp, ci, np.ones_like(hv), n) != 0))
    assert np.abs(H - Hd).max() <= 1e-14 * np.abs(Hd).max()
    # symmetric positive definite
    assert np.array_equal(rp, np.asarray(rp)) and np.allclose(H, H.T, rtol=0, atol=1e-14 * np.abs(H).max())
    np.linalg.cholesky(H)


def test_gamma_rule_hand_case():
    # K = [[3, 0, 1], [0, 5, 2], [1, 2, 0]]: max A_ii = 5, (J^T J)_ii = (1, 4) -> gamma = s * 5 / 4
    rp = np.array([0, 2, 4, 7], np.int64)
    ci = np.array([0, 2, 1, 2, 0, 1, 2], np.int32)
    v = np.array([3.0, 1.0, 5.0, 2.0, 1.0, 2.0, 0.0])
    f = hy.HyKKT(rp, ci, v, n=2, gamma_scale=8.0)
    assert f.gamma == 8.0 * 5.0 / 4.0
    with pytest.raises(ValueError):
        hy.split_kkt(rp, ci, np.array([3.0, 1.0, 5.0, 2.0, 1.0, 2.0, -1e-8]), 2)


@pytest.mark.parametrize("seed", [1, 2])
@pytest.mark.parametrize("dlog", [(-2.0, 2.0), (-6.0, 6.0)])
def test_solution_equals_dense_solve_of_original(seed, dlog):
    p = ks.small_kkt(60, 35, 700 + seed, dlog=dlog, delta=0.0)
    v1, _ = p.system(1)
    f = hy.HyKKT(p.rowptr, p.colidx, v1, n=p.n)
    for step in (1, 2, 3):
        v, b = p.system(step)
        K = dense(p.rowptr, p.colidx, v, p.N)
        xd = np.linalg.solve(K, b)
        x, info = f.solve(p.rowptr, p.colidx, v, b)
        assert info["converged"]
        kappa = np.linalg.cond(K, 1)
        assert np.abs(x - xd).max() <= 1e-8 * kappa * np.abs(xd).max()
        m = oracle.metrics(p.rowptr, p.colidx, v, x, b)
        # the CG tolerance (1e-12 on the Schur residual) bounds the backward error
        assert m["nrbe"] <= 1e-12


def decoupled_kkt(a, m):
    """n = len(a) primal variables with H + D = diag(a), m <= n constraints J = [I_m 0]."""
    n = len(a)
    rows = []
    for i in range(n):
        e = [(i, a[i])]
        if i < m:
            e.append((n + i, 1.0))
        rows.append(e)
    for r in range(m):
        rows.append([(r, 1.0), (n + r, 0.0)])
    rp = np.zeros(n + m + 1, np.int64)
    for i, e in enumerate(rows):
        rp[i + 1] = rp[i] + len(e)
    ci = np.array([c for e in rows for c, _ in e], np.int32)
    v = np.array([x for e in rows for _, x in e])
    return rp, ci, v


@pytest.mark.parametrize("distinct", [1, 2, 3])
def test_decoupled_schur_complement_closed_form(distinct):
    # S = J H_gamma^-1 J^T = diag(1 / (a_i + gamma)) for i < m: CG needs exactly as many
    # iterations as S has distinct eigenvalues; [[a, 1], [1, 0]] [dx; dl] = [rx; rl] gives
    # dx = rl, dl = rx - a rl
    m, n = 9, 12
    vals = [2.0, 7.0, 31.0][:distinct]
    a = np.array([vals[i % distinct] for i in range(n)])
    rp, ci, v = decoupled_kkt(a, m)
    rng = np.random.default_rng(distinct)
    b = rng.standard_normal(n + m)
    f = hy.HyKKT(rp, ci, v, n=n, gamma=10.0)
    x, info = f.solve(rp, ci, v, b)
    assert info["converged"] and info["cg_iterations"] == distinct
    rx, rl = b[:n], b[n:]
    dx = np.concatenate([rl, rx[m:] / a[m:]])
    dl = rx[:m] - a[:m] * rl
    assert np.allclose(x[:n], dx, rtol=1e-12, atol=1e-12)
    assert np.allclose(x[n:], dl, rtol=1e-12, atol=1e-12)


def test_cg_iteration_cap_reports_not_converged():
    p = ks.small_kkt(60, 35, 901, dlog=(-2.0, 2.0), delta=0.0)
    v, b = p.system(1)
    f = hy.HyKKT(p.rowptr, p.colidx, v, n=p.n, gamma=1.0)
    _, info = f.solve(p.rowptr, p.colidx, v, b, max_iter=2)
    assert not info["converged"] and info["cg_iterations"] == 2


def test_refactor_first_system_reproduces_analysis_factors():
    p = ks.small_kkt(80, 45, 333, delta=0.0)
    v1, _ = p.system(1)
    f = hy.HyKKT(p.rowptr, p.colidx, v1, n=p.n)
    _, lx, ux = f.refactor(p.rowptr, p.colidx, v1)
    assert np.array_equal(lx, f.lu.Lx) and np.array_equal(ux, f.lu.Ux)
    # diagonal pivots on the SPD H_gamma: P = Q
    assert np.array_equal(f.lu.prow, f.lu.Q)
