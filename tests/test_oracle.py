"""Pins for the CPU oracle, against things other than itself.

Every check here compares the oracle with an independent statement of the mathematics:
dense brute force (oracle/dense.py), LAPACK getrf via scipy, closed-form inverses,
textbook GMRES (scipy), exact condition numbers (numpy), hand-derived orderings, and
backward-error bounds.  A dropped term, a wrong sign or index, or a transposed operand
anywhere in oracle.c breaks at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import kkt_synth as ks
import oracle
from oracle import dense


def csr_of(A):
    M = sp.csr_matrix(A)
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data.astype(np.float64)


def csr_pattern_of_edges(n, edges, diag=True):
    rows, cols = [], []
    for a, b in edges:
        rows += [a, b]
        cols += [b, a]
    if diag:
        rows += list(range(n))
        cols += list(range(n))
    M = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    M.sum_duplicates()
    M.sort_indices()
    return M.indptr.astype(np.int64), M.indices.astype(np.int32)


def random_sparse(n, density, seed, sym_pattern=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    if sym_pattern:
        mask = (A != 0) | (A.T != 0)
        A = np.where(mask, rng.standard_normal((n, n)), 0.0)
    A[np.arange(n), np.arange(n)] += rng.standard_normal(n)
    return A


def lu_to_dense(f):
    n = f.n
    Ls = np.zeros((n, n))
    Us = np.zeros((n, n))
    for j in range(n):
        Ls[f.Li[f.Lp[j]:f.Lp[j + 1]], j] = f.Lx[f.Lp[j]:f.Lp[j + 1]]
        Us[f.Ui[f.Up[j]:f.Up[j + 1]], j] = f.Ux[f.Up[j]:f.Up[j + 1]]
    return Ls, Us


# ----------------------------------------------------------------------------------------
# generator
# ----------------------------------------------------------------------------------------

def test_generator_deterministic_and_shaped():
    p1 = ks.make_pattern(1)
    ks.make_pattern.cache_clear()
    p2 = ks.make_pattern(1)
    assert p1.N == 7000 and p1.n == 4000 and p1.m == 3000
    assert np.array_equal(p1.rowptr, p2.rowptr) and np.array_equal(p1.colidx, p2.colidx)
    v1, b1 = p1.system(1)
    v2, b2 = p2.system(1)
    assert np.array_equal(v1, v2) and np.array_equal(b1, b2)
    # a = 4n + 7m full nonzeros: 1.5n edges twice, n + m diagonal, 3m J and 3m J^T
    assert p1.nnz == 4 * p1.n + 7 * p1.m
    K = sp.csr_matrix((v1, p1.colidx, p1.rowptr), shape=(p1.N, p1.N))
    assert abs(K - K.T).max() == 0.0
    assert oracle.check_csr(p1.rowptr, p1.colidx)
    d = K.diagonal()
    assert np.all(d[p1.n:] == -ks.DUAL_REG)
    # later steps keep the pattern, change the values
    v3, b3 = p1.system(3)
    assert v3.shape == v1.shape and not np.array_equal(v3, v1) and not np.array_equal(b3, b1)


def test_moderate_and_arrow_generators():
    # the moderate family: D in [1e-2, 1e2] and delta = 1 on the (2,2) block
    p = ks.moderate_kkt(300, 200)
    v, b = p.system(2)
    K = sp.csr_matrix((v, p.colidx, p.rowptr), shape=(p.N, p.N))
    assert abs(K - K.T).max() == 0.0 and np.all(K.diagonal()[p.n:] == -1.0)
    h = K.diagonal()[:p.n] - (1.0 + np.asarray(abs(K[:p.n, :p.n]).sum(axis=1)).ravel() - np.abs(K.diagonal()[:p.n]))
    assert np.all((h > 10 ** -2.0 * (1 - 1e-12)) & (h < 10 ** 2.0 * (1 + 1e-12)))
    # the arrow-head KKT: symmetric, one constraint row with `dense` entries, pattern fixed
    a = ks.ArrowKKT(400, 150, 250, seed=3)
    v1, b1 = a.system(1)
    v2, b2 = a.system(2)
    A = sp.csr_matrix((v1, a.colidx, a.rowptr), shape=(a.N, a.N))
    assert abs(A - A.T).max() == 0.0 and oracle.check_csr(a.rowptr, a.colidx)
    assert np.diff(a.rowptr)[a.n] == 250 + 1 and np.all(A.diagonal()[a.n:] == -ks.DUAL_REG)
    assert not np.array_equal(v1, v2) and not np.array_equal(b1, b2)
    assert np.array_equal(a.system(2)[0], v2)


# ----------------------------------------------------------------------------------------
# ordering (hand-derived cases follow the nested-dissection rules step by step)
# ----------------------------------------------------------------------------------------

def test_order_path7():
    rp, ci = csr_pattern_of_edges(7, [(i, i + 1) for i in range(6)])
    # root 0 (min degree, smallest); levels {0}..{6}; separator level 3; halves {0,1,2}
    # -> [0, 2, 1] and {4,5,6} -> [4, 6, 5]
    assert oracle.order(rp, ci, method="nd", leaf=1).tolist() == [0, 2, 1, 4, 6, 5, 3]
    assert oracle.order(rp, ci, method="nd").tolist() == list(range(7))  # a leaf at the default size


def test_order_star():
    rp, ci = csr_pattern_of_edges(7, [(0, i) for i in range(1, 7)])
    # root 1; levels {1},{0},{2..6}; s clamped to 1 -> separator {0}; {2..6} splits into
    # five single-vertex components
    assert oracle.order(rp, ci, method="nd", leaf=1).tolist() == [1, 2, 3, 4, 5, 6, 0]


def test_order_grid3x3():
    edges = []
    for r in range(3):
        for c in range(3):
            v = 3 * r + c
            if c < 2:
                edges.append((v, v + 1))
            if r < 2:
                edges.append((v, v + 3))
    rp, ci = csr_pattern_of_edges(9, edges)
    # root 0; levels {0},{1,3},{2,4,6},{5,7},{8}; separator {2,4,6}; {0,1,3} -> [1,3,0];
    # {5,7,8} -> [5,7,8]
    assert oracle.order(rp, ci, method="nd", leaf=1).tolist() == [1, 3, 0, 5, 7, 8, 2, 4, 6]


def test_order_two_components():
    # component A = path 3-4-5 (smallest vertex 3), component B = path 0-6-7-1... wait:
    # B = path 0-1-2 (smallest vertex 0) -> B first
    edges = [(3, 4), (4, 5), (0, 1), (1, 2)]
    rp, ci = csr_pattern_of_edges(6, edges)
    assert oracle.order(rp, ci, method="nd", leaf=1).tolist() == [0, 2, 1, 3, 5, 4]


def test_order_is_permutation_and_reduces_fill():
    p = ks.make_pattern(1)
    v, _ = p.system(1)
    Q = oracle.order(p.rowptr, p.colidx)
    assert sorted(Q.tolist()) == list(range(p.N))
    f_nd = oracle.LU(p.rowptr, p.colidx, v, Q=Q)
    f_nat = oracle.LU(p.rowptr, p.colidx, v, Q=np.arange(p.N, dtype=np.int32))
    assert f_nd.lnz + f_nd.unz < 0.5 * (f_nat.lnz + f_nat.unz)


# ----------------------------------------------------------------------------------------
# pivoted LU
# ----------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("tau", [1e-10, 0.1, 1.0])
def test_factor_matches_dense_bruteforce_kkt(seed, tau):
    p = ks.small_kkt(30 + 3 * seed, 20 + 2 * seed, seed)
    v, _ = p.system(1 + seed % 3)
    Q = oracle.order(p.rowptr, p.colidx, leaf=4)
    f = oracle.LU(p.rowptr, p.colidx, v, Q=Q, tau=tau)
    A = ks.to_dense(p.rowptr, p.colidx, v, p.N)
    prow, Lf, Uf = dense.dense_lu(A, Q, tau)
    assert np.array_equal(prow, f.prow)
    Ls, Us = lu_to_dense(f)
    assert np.array_equal(Ls, Lf) and np.array_equal(Us, Uf)   # bit-identical values
    # the structural pattern contains every numeric nonzero (symmetric KKT values can
    # cancel exactly, so it may hold a few more)
    assert f.lnz >= np.count_nonzero(Lf) and f.unz >= np.count_nonzero(Uf)


@pytest.mark.parametrize("seed", range(6))
def test_factor_matches_dense_bruteforce_general(seed):
    n = 40
    A = random_sparse(n, 0.08, 100 + seed)
    rp, ci, v = csr_of(A)
    Q = np.random.default_rng(seed).permutation(n).astype(np.int32)
    f = oracle.LU(rp, ci, v, Q=Q, tau=0.5)
    prow, Lf, Uf = dense.dense_lu(A, Q, 0.5)
    Ls, Us = lu_to_dense(f)
    assert np.array_equal(prow, f.prow)
    assert np.array_equal(Ls, Lf) and np.array_equal(Us, Uf)
    # the structural patterns equal a boolean elimination with the same pivot sequence
    Lpat, Upat = dense.dense_symbolic(A != 0, Q, prow)
    Lsp = np.zeros((n, n), bool)
    Usp = np.zeros((n, n), bool)
    for j in range(n):
        Lsp[f.Li[f.Lp[j]:f.Lp[j + 1]], j] = True
        Usp[f.Ui[f.Up[j]:f.Up[j + 1]], j] = True
    assert np.array_equal(Lsp, Lpat) and np.array_equal(Usp, Upat)


@pytest.mark.parametrize("seed", range(5))
def test_partial_pivoting_matches_lapack(seed):
    n = 60
    A = random_sparse(n, 0.1, 200 + seed)
    rp, ci, v = csr_of(A)
    f = oracle.LU(rp, ci, v, Q=np.arange(n, dtype=np.int32), tau=1.0)
    lu, piv = sla.lu_factor(A)
    perm = np.arange(n)
    for k in range(n):
        perm[[k, piv[k]]] = perm[[piv[k], k]]
    assert np.array_equal(perm, f.prow)
    Ls, Us = lu_to_dense(f)
    Lst = Ls[f.prow] + np.eye(n)   # rows in step order, unit diagonal
    assert np.allclose(Lst, np.tril(lu, -1) + np.eye(n), rtol=1e-12, atol=1e-13)
    assert np.allclose(Us, np.triu(lu), rtol=1e-12, atol=1e-12 * np.abs(lu).max())


@pytest.mark.parametrize("cfg_seed", range(4))
def test_factor_backward_error_bound(cfg_seed):
    p = ks.small_kkt(120, 80, 10 + cfg_seed)
    v, _ = p.system(2)
    f = oracle.LU(p.rowptr, p.colidx, v, Q=oracle.order(p.rowptr, p.colidx, leaf=8))
    A = ks.to_dense(p.rowptr, p.colidx, v, p.N)
    Ls, Us = lu_to_dense(f)
    Lst = Ls[f.prow] + np.eye(p.N)
    PAQ = A[f.prow][:, f.Q]
    err = np.abs(PAQ - Lst @ Us).max()
    bound = p.N * np.finfo(float).eps * (np.abs(Lst) @ np.abs(Us)).max()
    assert err <= bound


def test_closed_form_decoupled_kkt():
    # m = n, J = I, H diagonal: independent blocks [[a, 1], [1, -delta]], a = h + d
    nb = 50
    rng = np.random.default_rng(7)
    a = 10.0 ** rng.uniform(-6, 6, nb)
    delta = 1e-8
    N = 2 * nb
    A = np.zeros((N, N))
    A[np.arange(nb), np.arange(nb)] = a
    A[np.arange(nb), nb + np.arange(nb)] = 1.0
    A[nb + np.arange(nb), np.arange(nb)] = 1.0
    A[nb + np.arange(nb), nb + np.arange(nb)] = -delta
    rp, ci, v = csr_of(A)
    Q = np.arange(N, dtype=np.int32)
    f = oracle.LU(rp, ci, v, Q=Q, tau=0.1)
    # pivot rule: first column of block i has candidates {i: a_i, nb+i: 1}
    for i in range(nb):
        expect = i if a[i] >= 0.1 else nb + i
        assert f.prow[i] == expect
    b = rng.standard_normal(N)
    x = f.solve(b)
    det = -a * delta - 1.0
    x1 = (-delta * b[:nb] - b[nb:]) / det
    x2 = (-b[:nb] + a * b[nb:]) / det
    xt = np.r_[x1, x2]
    assert np.abs(x - xt).max() <= 1e-13 * np.abs(xt).max()


@pytest.mark.parametrize("seed", range(4))
def test_solve_matches_numpy_and_manufactured(seed):
    p = ks.small_kkt(80, 50, 30 + seed, dlog=(-2.0, 2.0))
    v, b = p.system(1)
    A = ks.to_dense(p.rowptr, p.colidx, v, p.N)
    # threshold partial pivoting: the forward error of a backward-stable solve
    xs, f = oracle.direct_solve(p.rowptr, p.colidx, v, b, Q=oracle.order(p.rowptr, p.colidx, leaf=8), tau=0.1)
    xn = np.linalg.solve(A, b)
    kappa = np.linalg.cond(A, 1)
    assert np.linalg.norm(xs - xn) / np.linalg.norm(xn) <= 100 * np.finfo(float).eps * kappa
    xt = np.random.default_rng(seed).standard_normal(p.N)
    bt = A @ xt
    xm = f.solve(bt)
    assert np.linalg.norm(xm - xt) / np.linalg.norm(xt) <= 100 * np.finfo(float).eps * kappa
    # dense brute-force solves with the same factors are bit-identical, for threshold
    # pivoting and for the default diagonal-preferring threshold
    prow, Lf, Uf = dense.dense_lu(A, f.Q, 0.1)
    assert np.array_equal(prow, f.prow)
    assert np.array_equal(dense.dense_solve(prow, Lf, Uf, f.Q, b), xs)
    xd, g = oracle.direct_solve(p.rowptr, p.colidx, v, b, Q=f.Q)
    prow, Lf, Uf = dense.dense_lu(A, f.Q, 1e-10)
    assert np.array_equal(prow, g.prow) and np.array_equal(prow, g.Q)   # diagonal pivots: P = Q
    assert np.array_equal(dense.dense_solve(prow, Lf, Uf, f.Q, b), xd)


def test_metrics_definitions_on_known_residual():
    A = np.array([[4.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 4.0]])
    rp, ci, v = csr_of(A)
    x = np.array([1.0, 2.0, -3.0])
    b = np.array([0.5, 10.0, -12.0])
    r = b - A @ x
    m = oracle.metrics(rp, ci, v, x, b)
    knorm = 6.0
    assert m["knorm"] == knorm
    assert m["nrbe"] == pytest.approx(np.linalg.norm(r) / (knorm * np.linalg.norm(x) + np.linalg.norm(b)), rel=1e-15)
    assert m["nsr"] == pytest.approx(np.abs(r).max() / (knorm * np.abs(x).max()), rel=1e-15)
    assert m["rel_resid"] == pytest.approx(np.linalg.norm(r) / np.linalg.norm(b), rel=1e-15)


@pytest.mark.parametrize("cfg", [1, 2])
def test_direct_solve_nrbe_near_machine_eps(cfg):
    p = ks.make_pattern(cfg)
    v, b = p.system(1)
    x, f = oracle.direct_solve(p.rowptr, p.colidx, v, b, Q=oracle.order(p.rowptr, p.colidx))
    assert oracle.metrics(p.rowptr, p.colidx, v, x, b)["nrbe"] <= 1e-14


@pytest.mark.parametrize("seed", range(4))
def test_condest_bounds(seed):
    p = ks.small_kkt(60, 40, 50 + seed, dlog=(-3.0, 3.0))
    v, _ = p.system(1)
    f = oracle.LU(p.rowptr, p.colidx, v, Q=oracle.order(p.rowptr, p.colidx, leaf=8))
    A = ks.to_dense(p.rowptr, p.colidx, v, p.N)
    k1 = np.linalg.cond(A, 1)
    ke = f.condest(p.rowptr, v)
    assert ke <= k1 * (1 + 1e-8)
    assert ke >= k1 / 10


# ----------------------------------------------------------------------------------------
# static-pivot refactorization
# ----------------------------------------------------------------------------------------

def test_refactor_first_system_bit_identical():
    p = ks.make_pattern(1)
    v, _ = p.system(1)
    f = oracle.LU(p.rowptr, p.colidx, v)
    Lx, Ux, ng = f.refactor64(p.rowptr, p.colidx, v)
    assert ng == 0
    assert np.array_equal(Lx, f.Lx) and np.array_equal(Ux, f.Ux)


@pytest.mark.parametrize("seed", range(5))
def test_refactor_matches_dense_static(seed):
    p = ks.small_kkt(40, 25, 60 + seed, dlog=(-1.0, 1.0))
    v1, _ = p.system(1)
    v2, _ = p.system(2)
    # threshold pivoting keeps every FP32 static pivot clear of the guard
    f = oracle.LU(p.rowptr, p.colidx, v1, Q=oracle.order(p.rowptr, p.colidx, leaf=4), tau=0.1)
    A2 = ks.to_dense(p.rowptr, p.colidx, v2, p.N)
    Lx, Ux, ng = f.refactor64(p.rowptr, p.colidx, v2)
    Lf, Uf = dense.dense_lu_static(A2, f.Q, f.prow, np.float64)
    g = oracle.LU.__new__(oracle.LU)
    g.__dict__.update({k: getattr(f, k) for k in ("n", "Lp", "Li", "Up", "Ui")})
    g.Lx, g.Ux = Lx, Ux
    Ls, Us = lu_to_dense(g)
    assert ng == 0
    assert np.array_equal(Ls, Lf) and np.array_equal(Us, Uf)
    Lx32, Ux32, ng32 = f.refactor32(p.rowptr, p.colidx, v2)
    Lf32, Uf32 = dense.dense_lu_static(A2, f.Q, f.prow, np.float32)
    g.Lx, g.Ux = Lx32.astype(np.float64), Ux32.astype(np.float64)
    Ls32, Us32 = lu_to_dense(g)
    assert ng32 == 0
    assert np.array_equal(Ls32, Lf32.astype(np.float64)) and np.array_equal(Us32, Uf32.astype(np.float64))
    # the FP32 solve is the binary32 substitution with these factors, bit for bit
    b = np.random.default_rng(seed).standard_normal(p.N)
    x32 = f.solve32(b, Lx32, Ux32)
    assert np.array_equal(x32, dense.dense_solve(f.prow, Lf32, Uf32, f.Q, b, dtype=np.float32))


def test_refactor_pivot_guard():
    # K_1 = [[4, 2], [2, 3]]: both diagonal pivots.  K_2 = [[4, 2], [2, 1]] makes the second
    # static pivot 1 - 2*2/4 = 0 exactly: guarded to +u * colmax = 2^-53 * 2.
    A1 = np.array([[4.0, 2.0], [2.0, 3.0]])
    A2 = np.array([[4.0, 2.0], [2.0, 1.0]])
    rp, ci, v1 = csr_of(A1)
    _, _, v2 = csr_of(A2)
    f = oracle.LU(rp, ci, v1, Q=np.arange(2, dtype=np.int32), tau=0.1)
    assert f.prow.tolist() == [0, 1]
    Lx, Ux, ng = f.refactor64(rp, ci, v2)
    assert ng == 1
    assert Ux[-1] == 2.0 * 2.0 ** -53
    with pytest.raises(oracle.OracleError) as e:
        f.refactor64(rp, ci, v2, guard_policy=1)
    assert e.value.code == oracle.ESINGULAR
    Lx32, Ux32, ng32 = f.refactor32(rp, ci, v2)
    assert ng32 == 1 and Ux32[-1] == np.float32(2.0 * 2.0 ** -24)


def test_singular_column_reported():
    A = np.array([[1.0, 1.0, 0.0], [1.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    rp, ci, v = csr_of(A)
    with pytest.raises(oracle.OracleError) as e:
        oracle.LU(rp, ci, v, Q=np.arange(3, dtype=np.int32))
    assert e.value.code == oracle.ESINGULAR


def test_bad_csr_rejected():
    rp = np.array([0, 2, 3], np.int64)
    ci = np.array([1, 0, 1], np.int32)   # unsorted row 0
    assert not oracle.check_csr(rp, ci)
    ci2 = np.array([0, 5, 1], np.int32)  # out of range
    assert not oracle.check_csr(rp, ci2)


# ----------------------------------------------------------------------------------------
# FGMRES-IR
# ----------------------------------------------------------------------------------------

def identity_lu(n):
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    return oracle.LU(rp, ci, np.ones(n), Q=np.arange(n, dtype=np.int32))


@pytest.mark.parametrize("gs", ["cgs2", "dcgs2"])
def test_fgmres_identity_preconditioner_is_gmres(gs):
    n = 120
    rng = np.random.default_rng(3)
    A = sp.random(n, n, density=0.05, random_state=4, format="csr") + sp.eye(n) * 4.0
    A = sp.csr_matrix(A)
    A.sort_indices()
    rp, ci, v = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    b = rng.standard_normal(n)
    fI = identity_lu(n)
    R = 8
    x, info = fI.fgmres_ir(rp, ci, v, b, restart=R, max_restarts=0, eta=1e-30, mode=1, gs=gs)
    # scipy GMRES from the same initial guess x0 = M^-1 b = b, one cycle of R steps
    hist = []
    r0 = np.linalg.norm(b - A @ b)
    spla.gmres(A, b, x0=b.copy(), restart=R, maxiter=1, rtol=1e-30, atol=0.0,
               callback=lambda pr: hist.append(pr), callback_type="pr_norm")
    ours = info["hist"][:R] / np.linalg.norm(b)   # scipy reports ||r_i|| / ||b||
    assert len(hist) >= R - 1 and r0 > 0
    k = min(len(hist), R)
    assert np.allclose(ours[:k], np.array(hist[:k]), rtol=1e-8)
    # one full cycle of GMRES minimises the residual over the Krylov space
    xs, _ = spla.gmres(A, b, x0=b.copy(), restart=R, maxiter=1, rtol=1e-30, atol=0.0)
    assert np.linalg.norm(b - A @ x) == pytest.approx(np.linalg.norm(b - A @ xs), rel=1e-8)


@pytest.mark.parametrize("gs", ["cgs2", "dcgs2"])
def test_fgmres_distinct_eigenvalues(gs):
    n = 90
    d = np.repeat([2.0, 3.0, 7.0], n // 3)   # x0 = b, so rho0 = (1 - d) b keeps all three
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    b = np.random.default_rng(5).standard_normal(n)
    fI = identity_lu(n)
    x, info = fI.fgmres_ir(rp, ci, d, b, restart=10, max_restarts=0, eta=1e-13, mode=1, gs=gs)
    assert info["converged"] and info["iters"] == 3
    assert np.abs(d * x - b).max() < 1e-12


@pytest.mark.parametrize("gs", ["cgs2", "dcgs2"])
def test_fgmres_estimate_equals_true_residual_at_restart(gs):
    n = 150
    A = sp.random(n, n, density=0.04, random_state=8, format="csr") + sp.eye(n) * 3.0
    A = sp.csr_matrix(A)
    A.sort_indices()
    rp, ci, v = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    b = np.random.default_rng(9).standard_normal(n)
    fI = identity_lu(n)
    x, info = fI.fgmres_ir(rp, ci, v, b, restart=5, max_restarts=0, eta=1e-30, mode=1, gs=gs)
    assert info["est"] == pytest.approx(info["true_resid"], rel=1e-6)
    assert np.all(np.diff(info["hist"]) <= 1e-12 * info["hist"][0])   # non-increasing


def test_fgmres_ir_exact_preconditioner_and_sequence():
    p = ks.make_pattern(1)
    v1, b1 = p.system(1)
    f = oracle.LU(p.rowptr, p.colidx, v1)
    # exact factors: x0 already meets the NRBE target, so refinement is skipped
    x, info = f.fgmres_ir(p.rowptr, p.colidx, v1, b1, mode=0, eta=1e-12)
    assert info["iters"] == 0 and info["converged"]
    # paper's relative-residual control on a static-pivot system of a longer sequence
    p2 = ks.make_pattern(2)
    w1, _ = p2.system(1)
    g = oracle.LU(p2.rowptr, p2.colidx, w1)
    w3, b3 = p2.system(3)
    Lx, Ux, _ = g.refactor64(p2.rowptr, p2.colidx, w3)
    x0 = g.solve(b3, Lx, Ux)
    m0 = oracle.metrics(p2.rowptr, p2.colidx, w3, x0, b3)
    x, info = g.fgmres_ir(p2.rowptr, p2.colidx, w3, b3, Lx=Lx, Ux=Ux, restart=10, mode=1, eta=1e-14)
    m = oracle.metrics(p2.rowptr, p2.colidx, w3, x, b3)
    assert info["converged"] and 1 <= info["iters"] <= 30
    assert m["nrbe"] <= 1e-12 and m["resid"] < 0.1 * m0["resid"]
    # down to the rounding floor of a backward-stable solve (threshold-pivoted, fresh)
    xs, _ = oracle.direct_solve(p2.rowptr, p2.colidx, w3, b3, Q=g.Q, tau=0.1)
    assert m["resid"] <= 10 * oracle.metrics(p2.rowptr, p2.colidx, w3, xs, b3)["resid"]


# ----------------------------------------------------------------------------------------
# minimum degree ordering (default): hand-derived orders and an elimination-graph brute force
# ----------------------------------------------------------------------------------------

def test_md_path_star_grid():
    rp, ci = csr_pattern_of_edges(7, [(i, i + 1) for i in range(6)])
    # ends have degree 1; eliminating 0 leaves 1 with degree 1, and so on
    assert oracle.order(rp, ci).tolist() == [0, 1, 2, 3, 4, 5, 6]
    rp, ci = csr_pattern_of_edges(7, [(0, i) for i in range(1, 7)])
    # leaves 1..5 (degree 1) go first; then 0 and 6 both have degree 1 -> 0 first
    assert oracle.order(rp, ci).tolist() == [1, 2, 3, 4, 5, 0, 6]
    edges = []
    for r in range(3):
        for c in range(3):
            v = 3 * r + c
            if c < 2:
                edges.append((v, v + 1))
            if r < 2:
                edges.append((v, v + 3))
    rp, ci = csr_pattern_of_edges(9, edges)
    # corners (degree 2) 0, 2, 6, 8; then 1 (degree 3, smallest), 3, then 4, 5, 7
    assert oracle.order(rp, ci).tolist() == [0, 2, 6, 8, 1, 3, 4, 5, 7]


@pytest.mark.parametrize("seed", range(8))
def test_md_matches_elimination_graph_bruteforce(seed):
    if seed % 2:
        p = ks.small_kkt(50 + 3 * seed, 30 + 2 * seed, 900 + seed)
        rp, ci = p.rowptr, p.colidx
        n = p.N
    else:
        n = 80
        A = random_sparse(n, 0.04, 950 + seed)
        rp, ci, _ = csr_of(A)
    rows = np.repeat(np.arange(n), np.diff(rp))
    edges = [(int(a), int(b)) for a, b in zip(rows, ci) if a != b]
    assert oracle.order(rp, ci).tolist() == dense.md_order_bruteforce(n, edges)


@pytest.mark.parametrize("cfg", [1, 2])
def test_md_fill_below_nested_dissection(cfg):
    p = ks.make_pattern(cfg)
    v, _ = p.system(1)
    f_md = oracle.LU(p.rowptr, p.colidx, v, Q=oracle.order(p.rowptr, p.colidx))
    f_nd = oracle.LU(p.rowptr, p.colidx, v, Q=oracle.order(p.rowptr, p.colidx, method="nd"))
    assert f_md.lnz + f_md.unz < 0.5 * (f_nd.lnz + f_nd.unz)


# ---------------------------------------------------------------------------------------
# extended-precision (double-double) residual
# ---------------------------------------------------------------------------------------

def test_residual_dd_hand_cancellation():
    # 3 * fl(1/3) = 1 - 2^-54 exactly; in binary64 it rounds to 1 (tie to even), so the
    # working-precision residual of b = 0 against x = (fl(1/3), -1) is 0 while the exact
    # residual is 2^-54.
    rp = np.array([0, 2], np.int64)
    ci = np.array([0, 1], np.int32)
    v = np.array([3.0, 1.0])
    x = np.array([1.0 / 3.0, -1.0])
    b = np.array([0.0])
    assert oracle.residual(rp, ci, v, x, b)[0] == 0.0
    assert oracle.residual(rp, ci, v, x, b, "dd")[0] == 2.0 ** -54


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_residual_dd_matches_exact_rounding(seed):
    from fractions import Fraction
    from exact import exact_residual
    p = ks.small_kkt(30, 20, seed)
    v, b = p.system(1)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(p.N) * 10.0 ** rng.uniform(-6, 6, p.N)
    ex = exact_residual(p.rowptr, p.colidx, v, x, b)
    r = oracle.residual(p.rowptr, p.colidx, v, x, b, "dd")
    for i in range(p.N):
        mag = abs(b[i]) + sum(abs(v[q] * x[p.colidx[q]]) for q in range(p.rowptr[i], p.rowptr[i + 1]))
        rounded = float(ex[i])  # correctly rounded exact value
        bound = 0.5 * np.spacing(abs(rounded)) + 2.0 ** -103 * mag
        assert abs(Fraction(float(r[i])) - ex[i]) <= Fraction(bound), i
    # the double-double rows are the correctly rounded exact residual far more often than
    # the working-precision ones
    r64 = oracle.residual(p.rowptr, p.colidx, v, x, b)
    exact_dd = sum(float(r[i]) == float(ex[i]) for i in range(p.N))
    exact_64 = sum(float(r64[i]) == float(ex[i]) for i in range(p.N))
    assert exact_dd >= p.N - 1 and exact_dd > exact_64


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fgmres_dd_residual_reaches_working_accuracy(seed):
    # With residuals in double-double, refinement converges to the exact solution of the
    # stored system to about the unit roundoff componentwise (three-precision IR), where the
    # working-precision residual stalls near cond * u; exact solution by rational elimination.
    from exact import exact_solve, max_componentwise_error
    p = ks.small_kkt(24, 16, seed)
    v, b = p.system(1)
    xe = exact_solve(ks.to_dense(p.rowptr, p.colidx, v, p.N), b)
    f = oracle.LU(p.rowptr, p.colidx, v)
    x, info = f.fgmres_ir(p.rowptr, p.colidx, v, b, mode=1, eta=1e-14, residual="dd")
    assert info["converged"]
    assert max_componentwise_error(x, xe) <= 2.0 ** -52


def _spread_diag_system(n, lo, hi, seed):
    """Diagonal-plus-upper-band matrix with eigenvalues spread over [10^lo, 10^hi]: the Krylov
    vectors align fast, so one Gram-Schmidt pass leaves visible components along the basis."""
    rng = np.random.default_rng(seed)
    d = np.logspace(lo, hi, n)
    A = sp.diags([d, 0.3 * d[:-1]], [0, 1], format="csr")
    A.sort_indices()
    return A, rng.standard_normal(n)


@pytest.mark.parametrize("R, eta, restarts", [(30, 1e-30, 1), (40, 1e-10, 3)])
def test_dcgs2_equals_cgs2_on_a_fast_aligning_krylov_basis(R, eta, restarts):
    # delayed CGS2 builds the same basis and Hessenberg matrix as CGS2 in exact arithmetic
    # (Bielich et al. 2022); on a basis where one pass loses orthogonality the deferred
    # corrections (second pass, Hessenberg and z_j updates) are what keeps them equal
    A, b = _spread_diag_system(400, 0.0, 7.0, 17)
    rp, ci, v = A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data
    fI = identity_lu(A.shape[0])
    x2, i2 = fI.fgmres_ir(rp, ci, v, b, restart=R, max_restarts=restarts, eta=eta, mode=1, gs="cgs2")
    xd, id_ = fI.fgmres_ir(rp, ci, v, b, restart=R, max_restarts=restarts, eta=eta, mode=1, gs="dcgs2")
    assert id_["iters"] == i2["iters"] and id_["cycles"] == i2["cycles"]
    assert np.allclose(id_["hist"], i2["hist"], rtol=1e-7, atol=0.0)
    assert np.linalg.norm(xd - x2) <= 1e-8 * np.linalg.norm(x2)
    # one extra preconditioner application per cycle that ends before its restart length
    early = int(i2["iters"] < i2["cycles"] * R)
    assert id_["applications"] == i2["applications"] + early


def test_dcgs2_inexact_lu_preconditioner():
    # right preconditioning by LU factors of a nearby matrix (the refactorization setting)
    p = ks.small_kkt(300, 200, 5, (-4.0, 4.0))
    v1, b2 = p.system(1)
    v2 = v1 * (1.0 + 0.02 * np.random.default_rng(11).standard_normal(v1.size))
    f = oracle.LU(p.rowptr, p.colidx, v1)
    x2, i2 = f.fgmres_ir(p.rowptr, p.colidx, v2, b2, restart=10, max_restarts=5, eta=1e-12, mode=1,
                         gs="cgs2")
    xd, id_ = f.fgmres_ir(p.rowptr, p.colidx, v2, b2, restart=10, max_restarts=5, eta=1e-12, mode=1,
                          gs="dcgs2")
    assert i2["converged"] and id_["converged"]
    assert id_["iters"] == i2["iters"]
    # equal to rounding: relative to each estimate, or to the initial residual once tiny
    assert np.allclose(id_["hist"], i2["hist"], rtol=1e-6, atol=1e-13 * i2["hist"][0])
    assert np.linalg.norm(xd - x2) <= 1e-9 * np.linalg.norm(x2)


def test_dcgs2_breakdown_and_application_count():
    # three distinct eigenvalues: the fourth vector vanishes (breakdown found when its delayed
    # second pass gives beta = 0), after one preconditioner application more than CGS2
    n = 90
    d = np.repeat([2.0, 3.0, 7.0], n // 3)
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    b = np.random.default_rng(5).standard_normal(n)
    fI = identity_lu(n)
    _, ic = fI.fgmres_ir(rp, ci, d, b, restart=10, max_restarts=0, eta=1e-30, mode=1, gs="cgs2")
    _, idl = fI.fgmres_ir(rp, ci, d, b, restart=10, max_restarts=0, eta=1e-30, mode=1, gs="dcgs2")
    assert ic["iters"] == idl["iters"] == 3
    assert ic["applications"] == 1 + 3 and idl["applications"] == 1 + 4


def _arnoldi_invariants(A, M, V, Z, H, k):
    """Relative error of the Arnoldi relation A Z = V Hbar, loss of orthonormality of V and
    error of Z = M^-1 V over the first k - 1 columns."""
    m = k - 1
    AZ = A @ Z[:, :m]
    rel = np.linalg.norm(AZ - V[:, :m + 1] @ H[:m + 1, :m]) / np.linalg.norm(AZ)
    orth = np.linalg.norm(V[:, :m + 1].T @ V[:, :m + 1] - np.eye(m + 1))
    zr = np.linalg.norm(M @ Z[:, :m] - V[:, :m]) / np.sqrt(m)
    return rel, orth, zr


@pytest.mark.parametrize("gs", ["cgs2", "dcgs2"])
def test_arnoldi_relation_and_orthonormal_basis(gs):
    # Eight eigenvalue clusters of width 1e-9: Arnoldi nearly breaks down after eight steps,
    # where one Gram-Schmidt pass leaves components of relative size ~1e-8 along the basis.
    # The delayed corrections divided by the small norm (Hbar s / beta in the Hessenberg
    # column, Z s / beta in z_j, V s in v_j) are what keeps K Z = V Hbar, Z = M^-1 V and
    # V^T V = I at rounding level; dropping any one leaves errors >= 1e-9 here.
    rng = np.random.default_rng(3)
    n = 400
    d = np.concatenate([c + 1e-9 * rng.standard_normal(n // 8) for c in np.arange(1, 9)])
    A = sp.diags([d], [0], format="csr")
    A.sort_indices()
    b = rng.standard_normal(n)
    fI = identity_lu(n)
    V, Z, H, k = fI.arnoldi(A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, b, 20, gs)
    assert k == 20
    rel, orth, zr = _arnoldi_invariants(A, sp.eye(n), V, Z, H, k)
    assert rel <= 1e-13 and orth <= 1e-13 and zr <= 1e-14
    # right preconditioning by LU factors of a nearby KKT matrix
    p = ks.small_kkt(300, 200, 5, (-4.0, 4.0))
    v1, bk = p.system(1)
    v2 = v1 * (1.0 + 1e-6 * np.random.default_rng(11).standard_normal(v1.size))
    f = oracle.LU(p.rowptr, p.colidx, v1, tau=0.1)   # threshold pivoting: small |L||U|
    nk = p.rowptr.size - 1
    K2 = sp.csr_matrix((v2, p.colidx, p.rowptr), shape=(nk, nk))
    K1 = sp.csr_matrix((v1, p.colidx, p.rowptr), shape=(nk, nk))
    V, Z, H, k = f.arnoldi(p.rowptr, p.colidx, v2, bk, 10, gs)
    assert k == 10
    rel, orth, zr = _arnoldi_invariants(K2, K1, V, Z, H, k)
    assert rel <= 1e-12 and orth <= 1e-13 and zr <= 1e-11


# ----------------------------------------------------------------------------------------
# binary32 triangular solves and the FP32-preconditioned FGMRES cycle
# ----------------------------------------------------------------------------------------

def _fp32_static_factors(seed, n=50, perturb=0.0):
    """A well-conditioned sparse matrix, its pivoted FP64 analysis, FP32 static-pivot
    factors from the oracle and the same factors from the dense brute force; with perturb > 0
    the factors are those of a matrix whose entries differ by that relative amount (an
    inexact preconditioner)."""
    A = random_sparse(n, 0.08, 700 + seed)
    A[np.arange(n), np.arange(n)] += 6.0 * np.sign(A[np.arange(n), np.arange(n)] + 1e-300)
    rp, ci, v = csr_of(A)
    Q = np.random.default_rng(seed).permutation(n).astype(np.int32)
    f = oracle.LU(rp, ci, v, Q=Q, tau=0.1)
    v1 = v * (1.0 + perturb * np.random.default_rng(seed + 1).standard_normal(v.size))
    Lx32, Ux32, ng = f.refactor32(rp, ci, v1)
    assert ng == 0
    A1 = sp.csr_matrix((v1, ci, rp), shape=(n, n)).toarray()
    Lf32, Uf32 = dense.dense_lu_static(A1, f.Q, f.prow, np.float32)
    return A, rp, ci, v, f, Lx32, Ux32, Lf32, Uf32


@pytest.mark.parametrize("seed", range(4))
def test_solve32_is_a_binary32_substitution(seed):
    # or_solve_with32 rounds b to binary32 and substitutes in binary32: bit-identical to the
    # dense float32 substitution with the same factors (and not to a binary64 one)
    A, rp, ci, v, f, Lx32, Ux32, Lf32, Uf32 = _fp32_static_factors(seed)
    b = np.random.default_rng(40 + seed).standard_normal(A.shape[0])
    x = f.solve32(b, Lx32, Ux32)
    x_d32 = dense.dense_solve(f.prow, Lf32, Uf32, f.Q, b, dtype=np.float32)
    x_d64 = dense.dense_solve(f.prow, Lf32, Uf32, f.Q, b, dtype=np.float64)
    assert np.array_equal(x, x_d32)
    assert not np.array_equal(x, x_d64)


@pytest.mark.parametrize("gs", ["cgs2", "dcgs2"])
def test_fgmres_with_fp32_preconditioner(gs):
    # precision 1: x0 and every z_j = M^-1 v_j are binary32 solves with the FP32 factors
    # (bit-identical to the dense float32 substitution), and the cycle's update minimises
    # the residual over x0 + span(Z) (flexible GMRES, Saad 1993)
    A, rp, ci, v, f, Lx32, Ux32, Lf32, Uf32 = _fp32_static_factors(9, perturb=0.05)
    n = A.shape[0]
    K = sp.csr_matrix((v, ci, rp), shape=(n, n))
    b = np.random.default_rng(19).standard_normal(n)
    x0 = dense.dense_solve(f.prow, Lf32, Uf32, f.Q, b, dtype=np.float32)
    R = 3
    x, info = f.fgmres_ir(rp, ci, v, b, Lx32=Lx32, Ux32=Ux32, restart=R, max_restarts=0, eta=1e-30, mode=1,
                          gs=gs)
    assert info["nrbe0"] == oracle.metrics(rp, ci, v, x0, b)["nrbe"]
    r0 = oracle.residual(rp, ci, v, x0, b)
    V, Z, H, k = f.arnoldi(rp, ci, v, r0, R, gs, Lx32=Lx32, Ux32=Ux32)
    assert k == info["iters"] == R
    m = k if gs == "cgs2" else k - 1   # DCGS2 leaves its last vector after one pass
    for j in range(m):
        zd = dense.dense_solve(f.prow, Lf32, Uf32, f.Q, V[:, j], dtype=np.float32)
        if gs == "cgs2" or j == 0:
            assert np.array_equal(Z[:, j], zd)
        else:
            # DCGS2 forms z_j = (M^-1 u_j - Z s) / beta from the linearity of M^-1, which the
            # binary32 solve has only to its rounding
            assert np.linalg.norm(Z[:, j] - zd) <= 1e-5 * np.linalg.norm(zd)
    beta = np.linalg.norm(r0)
    e1 = np.zeros(k + 1)
    e1[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
    # the update x - x0 = Z y is small next to x: compare at x's rounding level
    assert np.linalg.norm(x - (x0 + Z[:, :k] @ y)) <= 1e-8 * np.linalg.norm(x - x0) + 4e-16 * np.linalg.norm(x)
    yls = np.linalg.lstsq((K @ Z[:, :k]), r0, rcond=None)[0]
    best = np.linalg.norm(r0 - K @ (Z[:, :k] @ yls))
    assert np.linalg.norm(b - K @ x) <= best * (1 + 1e-6) + 1e-14 * beta


# ----------------------------------------------------------------------------------------
# Richardson iterative refinement: closed forms with M = c K
# ----------------------------------------------------------------------------------------

def _scaled_factors(c, n=60, seed=3):
    """K well conditioned; factors of c K, so M^-1 = K^-1 / c and every Richardson
    correction multiplies the error by q = 1 - 1/c exactly (up to rounding)."""
    A = random_sparse(n, 0.06, 900 + seed)
    A[np.arange(n), np.arange(n)] = 8.0 + np.abs(A[np.arange(n), np.arange(n)])
    rp, ci, v = csr_of(A)
    f = oracle.LU(rp, ci, c * v, Q=np.arange(n, dtype=np.int32), tau=0.1)
    b = np.random.default_rng(seed).standard_normal(n)
    return A, rp, ci, v, f, b


def test_richardson_contraction_closed_form():
    # q = 1/4: x_k = x*(1 - q^(k+1)), rho_k = q^(k+1) b, ||rho_k|| / ||rho_0|| = q^k; the first k
    # with q^k < 1e-6 is 10 (q^9 = 3.8e-6, q^10 = 9.5e-7); NSR_k / NSR_(k-1) =
    # q (1 - q^k) / (1 - q^(k+1)) < 1/2, so MA57's ratio test never stops it earlier
    c = 4.0 / 3.0
    q = 1.0 - 1.0 / c
    A, rp, ci, v, f, b = _scaled_factors(c)
    xs = np.linalg.solve(A, b)
    x, info = oracle.richardson(f, rp, ci, v, b, max_it=50, tol=1e-6, ratio=0.5)
    assert info["converged"] and info["corrections"] == 10 and info["applications"] == 11
    assert info["rr"] == pytest.approx(q ** 10, rel=1e-8)
    assert np.linalg.norm(x - xs * (1 - q ** 11)) <= 1e-12 * np.linalg.norm(xs)
    h = info["hist"]
    for k in range(1, len(h)):
        assert h[k] / h[k - 1] == pytest.approx(q * (1 - q ** (k + 1)) / (1 - q ** (k + 2)), rel=1e-8)


def test_richardson_ratio_stop_closed_form():
    # q = 0.8: the NSR ratio is q/(1+q) = 0.444 after the first correction and
    # 0.8 * 0.36 / 0.488 = 0.590 > 1/2 after the second, so the ratio test stops at 2
    c = 5.0
    A, rp, ci, v, f, b = _scaled_factors(c)
    x, info = oracle.richardson(f, rp, ci, v, b, max_it=50, tol=1e-12, ratio=0.5)
    assert info["corrections"] == 2 and not info["converged"]
    assert info["rr"] == pytest.approx(0.8 ** 2, rel=1e-8)
    # with a laxer ratio (0.9 > every step's 0.8 (1 - 0.8^k) / (1 - 0.8^(k+1))) it runs to max_it
    x, info = oracle.richardson(f, rp, ci, v, b, max_it=7, tol=1e-12, ratio=0.9)
    assert info["corrections"] == 7 and not info["converged"]
    assert info["rr"] == pytest.approx(0.8 ** 7, rel=1e-8)


def test_richardson_error_system_fgmres_is_exact_in_one_step():
    # with M = c K the preconditioned operator K M^-1 is I / c: the inner FGMRES solves
    # K d = rho exactly in one Arnoldi step (x0 and z_0: two applications), so one
    # correction reaches the solution: 1 + 2 applications
    c = 4.0 / 3.0
    A, rp, ci, v, f, b = _scaled_factors(c)
    xs = np.linalg.solve(A, b)
    x, info = oracle.richardson(f, rp, ci, v, b, max_it=50, tol=1e-10, ratio=0.5, inner_restart=5,
                                inner_tol=1e-2)
    assert info["converged"] and info["corrections"] == 1 and info["applications"] == 3
    assert np.linalg.norm(x - xs) <= 1e-13 * np.linalg.norm(xs)


def test_richardson_divergence_returns_best_iterate():
    # c = 1/4: q = 1 - 1/c = -3, so x0 = 4 x*, rho0 = -3 b and the first correction gives
    # x1 = -8 x*, rho1 = 9 b.  NSR goes from 3/4 to 9/8 of ||b||inf / (||K||inf ||x*||inf), a
    # ratio of 1.5 > 1/2, so MA57's test stops after one correction; x1's residual is three
    # times x0's, so the refinement returns x0 itself (the direct solve), with rr = 1
    c = 0.25
    A, rp, ci, v, f, b = _scaled_factors(c)
    xs = np.linalg.solve(A, b)
    x0 = f.solve(b)
    x, info = oracle.richardson(f, rp, ci, v, b, max_it=50, tol=1e-12, ratio=0.5)
    assert info["corrections"] == 1 and not info["converged"]
    assert np.array_equal(x, x0)
    assert np.linalg.norm(x - 4.0 * xs) <= 1e-12 * np.linalg.norm(xs)
    assert info["rr"] == 1.0
    # with a ratio that lets it run, every correction triples the residual: x0 again
    x, info = oracle.richardson(f, rp, ci, v, b, max_it=4, tol=1e-12, ratio=10.0)
    assert info["corrections"] == 4 and not info["converged"]
    assert np.array_equal(x, x0) and info["rr"] == 1.0
