"""GPU parity tests: the HIP path (through the C ABI) against the CPU oracle.

* refactorization: FP64 factors bit-identical to the oracle's static-pivot refactorization
  (same operation order, no contraction); FP32 factors bit-identical to the oracle's FP32
  refactorization; guard counts equal.
* direct solve: agrees with the oracle's triangular solves with the same factors.
* FGMRES-IR: every solve meets NRBE <= 1e-12 and the paper's relative-residual test, and
  is close to the oracle's solution; repeated solves are bitwise identical.
"""
import sys

import numpy as np
import pytest

import kkt_synth as ks
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2401_13926_amd as P  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def cuda(a, dev):
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def make(cfg_or_pattern, dev, **opts):
    p = cfg_or_pattern if isinstance(cfg_or_pattern, ks.KKTPattern) else ks.make_pattern(cfg_or_pattern)
    v1, _ = p.system(1)
    s = P.Solver(p.rowptr, p.colidx, v1, **opts).bind(dev)
    f = oracle.LU(p.rowptr, p.colidx, v1, tau=opts.get("pivot_tau", P.default_opts().pivot_tau))
    return p, s, f


@pytest.mark.parametrize("cfg", [1, 2])
def test_refactor_fp64_bit_exact(dev, cfg):
    say("refactor fp64 config", cfg)
    p, s, f = make(cfg, dev)
    for step in (1, 2, 3):
        v, _ = p.system(step)
        s.refactor(cuda(v, dev))
        torch.cuda.synchronize()
        lx, ux = s.factor_values(0)
        olx, oux, ng = f.refactor64(p.rowptr, p.colidx, v)
        assert np.array_equal(lx, olx), "L differs at step %d" % step
        assert np.array_equal(ux, oux), "U differs at step %d" % step
        if step == 1:
            assert np.array_equal(lx, f.Lx) and np.array_equal(ux, f.Ux)


@pytest.mark.parametrize("narrow", [1, 1 << 30])
def test_refactor_handout_does_not_change_factors(dev, narrow):
    # every column handed out alone (narrow = 1: no lane groups either), or every level in
    # grabs with small same-level columns run by lane groups (narrow = 2^30): the same bits
    say("refactor hand-out narrow_columns", narrow)
    p, s, f = make(2, dev, narrow_columns=narrow)
    for step in (2, 3):
        v, _ = p.system(step)
        s.refactor(cuda(v, dev))
        torch.cuda.synchronize()
        lx, ux = s.factor_values(0)
        olx, oux, _ = f.refactor64(p.rowptr, p.colidx, v)
        assert np.array_equal(lx, olx) and np.array_equal(ux, oux), "factors differ at step %d" % step


def test_refactor_fp32_bit_exact(dev):
    say("refactor fp32 config 1")
    p, s, f = make(1, dev, precision=P.PREC_MIXED)
    for step in (1, 2):
        v, _ = p.system(step)
        s.refactor(cuda(v, dev))
        torch.cuda.synchronize()
        lx, ux = s.factor_values(1)
        olx, oux, ng = f.refactor32(p.rowptr, p.colidx, v)
        assert np.array_equal(lx, olx.astype(np.float64))
        assert np.array_equal(ux, oux.astype(np.float64))


def test_guard_count_matches_oracle(dev):
    say("guard count config 2")
    p, s, f = make(2, dev)
    v, b = p.system(4)
    s.refactor(cuda(v, dev))
    _, info = s.solve(cuda(b, dev))
    _, _, ng = f.refactor64(p.rowptr, p.colidx, v)
    assert info["pivots_perturbed"] == ng


def step_factors(f, lx, ux):
    """Unit-lower L and upper U of P K Q in pivot-step indexing (scipy CSC)."""
    import scipy.sparse as sp
    n = f.n
    L = sp.csc_matrix((lx, f.pinv[f.Li], f.Lp), shape=(n, n)) + sp.eye(n, format="csc")
    U = sp.csc_matrix((ux, f.Ui, f.Up), shape=(n, n))
    return L, U


def check_solve_backward_error(f, lx, ux, b, x, unit):
    """Componentwise backward error of x = Q U^-1 L^-1 P b for the given factors:
    |P b - L U z| <= c w u |L| |U| |z| (z = Q^T x, w = longest row), the bound of a
    forward/backward substitution pair in floating point."""
    L, U = step_factors(f, lx, ux)
    z = x[f.Q]
    pb = b[f.prow]
    r = np.abs(pb - L @ (U @ z))
    bound = (abs(L) @ (abs(U) @ np.abs(z)))
    w = max(np.diff(L.tocsr().indptr).max(), np.diff(U.tocsr().indptr).max())
    assert np.all(r <= 4 * w * unit * bound + 1e-300), float(np.max(r / np.maximum(bound, 1e-300)))


@pytest.mark.parametrize("tile_kib", [0, 150])
@pytest.mark.parametrize("cfg", [1, 2])
@pytest.mark.parametrize("step", [1, 2])
def test_direct_solve_backward_error(dev, cfg, step, tile_kib):
    # tile_kib: the default 32 KiB solve tiles, and the largest budget (one block per CU)
    say("direct solve config", cfg, "step", step, "tile KiB", tile_kib)
    p, s, f = make(cfg, dev, tile_lds_kib=tile_kib)
    v, b = p.system(step)
    s.refactor(cuda(v, dev))
    x = s.direct_solve(cuda(b, dev)).cpu().numpy()
    olx, oux, _ = f.refactor64(p.rowptr, p.colidx, v)
    check_solve_backward_error(f, olx, oux, b, x, 2.0 ** -53)
    if step == 1:
        # pivoted factors: the two summation orders agree to roughly the triangles' condition
        # number times the unit roundoff (at most 2.4e-14 measured on these systems, either
        # tile budget)
        xo = f.solve(b, olx, oux)
        assert np.linalg.norm(x - xo) <= 1e-12 * np.linalg.norm(xo)


@pytest.mark.parametrize("prec", [P.PREC_FP64, P.PREC_MIXED])
def test_direct_solve_well_conditioned(dev, prec):
    say("direct solve well conditioned, precision", prec)
    p = ks.small_kkt(3000, 2000, 17, dlog=(-1.0, 1.0))
    p, s, f = make(p, dev, precision=prec)
    v, b = p.system(2)
    s.refactor(cuda(v, dev))
    x = s.direct_solve(cuda(b, dev)).cpu().numpy()
    if prec == P.PREC_FP64:
        olx, oux, _ = f.refactor64(p.rowptr, p.colidx, v)
        xo = f.solve(b, olx, oux)
        tol = 1e-11
        check_solve_backward_error(f, olx, oux, b, x, 2.0 ** -53)
    else:
        olx, oux, _ = f.refactor32(p.rowptr, p.colidx, v)
        xo = f.solve32(b, olx, oux)
        tol = 1e-3
        # the FP32 solve rounds b to binary32 first, then substitutes in binary32
        check_solve_backward_error(f, olx.astype(np.float64), oux.astype(np.float64),
                                   b.astype(np.float32).astype(np.float64), x, 2.0 ** -24)
    assert np.linalg.norm(x - xo) <= tol * np.linalg.norm(xo)


@pytest.mark.parametrize("cfg", [1, 2])
def test_fgmres_ir_sequence(dev, cfg):
    p, s, f = make(cfg, dev)
    nsteps = 1 if cfg == 1 else 6
    for step in range(1, nsteps + 1):
        say("fgmres config", cfg, "step", step)
        v, b = p.system(step)
        s.refactor(cuda(v, dev))
        xg, info = s.solve(cuda(b, dev))
        x = xg.cpu().numpy()
        m = oracle.metrics(p.rowptr, p.colidx, v, x, b)
        assert info["converged"] == 1
        assert m["nrbe"] <= 1e-12
        assert info["nrbe"] == pytest.approx(m["nrbe"], rel=1e-6, abs=1e-30)
        # the oracle's FGMRES-IR on the same static-pivot factors (paper control)
        olx, oux, _ = f.refactor64(p.rowptr, p.colidx, v)
        xo, oinfo = f.fgmres_ir(p.rowptr, p.colidx, v, b, Lx=olx, Ux=oux, restart=10, mode=1, eta=1e-14)
        assert oinfo["converged"]
        # the same method on the same factors: the iteration counts are equal and the two
        # refinements land within a few unit roundoffs of each other (3.3e-16 at most
        # measured), so both are as far from a fresh pivoted solve
        assert abs(info["iterations"] - oinfo["iters"]) <= 1
        xd, _ = oracle.direct_solve(p.rowptr, p.colidx, v, b, Q=f.Q)
        rel = np.linalg.norm(x - xd) / np.linalg.norm(xd)
        reld = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        relo = np.linalg.norm(x - xo) / np.linalg.norm(xo)
        say("   iters", info["iterations"], "oracle iters", oinfo["iters"], "nrbe %.2e" % m["nrbe"],
            "rel diff vs direct %.2e (oracle IR %.2e), vs oracle IR %.2e" % (rel, reld, relo))
        assert relo <= 1e-13
        assert rel <= 1.01 * reld + 1e-13


def test_solve_repeatable_bitwise(dev):
    say("repeatability config 2")
    p, s, f = make(2, dev)
    v, b = p.system(3)
    s.refactor(cuda(v, dev))
    x1, i1 = s.solve(cuda(b, dev))
    x1 = x1.cpu().numpy()
    s.refactor(cuda(v, dev))
    x2, i2 = s.solve(cuda(b, dev))
    assert np.array_equal(x1, x2.cpu().numpy())
    assert i1["iterations"] == i2["iterations"]


def test_edge_cases(dev):
    say("edge cases")
    p = ks.small_kkt(12, 7, 5)
    v, b = p.system(1)
    s = P.Solver(p.rowptr, p.colidx, v)
    s.bind(dev)
    with pytest.raises(P.KKTError) as e:
        s.solve(cuda(b, dev))
    assert e.value.code == P.KKT_ESTATE
    s.refactor(cuda(v, dev))
    x, info = s.solve(cuda(b, dev))
    A = ks.to_dense(p.rowptr, p.colidx, v, p.N)
    assert np.linalg.norm(A @ x.cpu().numpy() - b) <= 1e-8 * np.linalg.norm(b) * np.abs(A).max()
    # zero right-hand side: x = 0 without refinement
    x0, info0 = s.solve(torch.zeros(p.N, dtype=torch.float64, device=dev))
    assert info0["converged"] == 1 and info0["iterations"] == 0
    assert torch.count_nonzero(x0).item() == 0
    # non-finite right-hand side is rejected
    bb = b.copy()
    bb[3] = np.nan
    with pytest.raises(P.KKTError) as e:
        s.solve(cuda(bb, dev))
    assert e.value.code == P.KKT_EINVAL
    # non-finite matrix value is rejected at the next solve
    vv = v.copy()
    vv[0] = np.inf
    s.refactor(cuda(vv, dev))
    with pytest.raises(P.KKTError) as e:
        s.solve(cuda(b, dev))
    assert e.value.code == P.KKT_EINVAL
    # the handle still works afterwards
    s.refactor(cuda(v, dev))
    _, info = s.solve(cuda(b, dev))
    assert info["converged"] == 1


def test_guard_fail_policy(dev):
    say("guard fail policy")
    # K_1 = [[4, 2], [2, 3]]; K_2 = [[4, 2], [2, 1]] cancels the second static pivot exactly
    rp = np.array([0, 2, 4], np.int64)
    ci = np.array([0, 1, 0, 1], np.int32)
    v1 = np.array([4.0, 2.0, 2.0, 3.0])
    v2 = np.array([4.0, 2.0, 2.0, 1.0])
    b = np.array([1.0, 2.0])
    s = P.Solver(rp, ci, v1, guard_policy=P.GUARD_FAIL).bind(dev)
    s.refactor(cuda(v2, dev))
    with pytest.raises(P.KKTError) as e:
        s.solve(cuda(b, dev))
    assert e.value.code == P.KKT_ESINGULAR
    s2 = P.Solver(rp, ci, v1).bind(dev)
    s2.refactor(cuda(v2, dev))
    torch.cuda.synchronize()
    _, ux = s2.factor_values(0)
    assert ux[-1] == 2.0 * 2.0 ** -53


@pytest.mark.parametrize("method", [P.IR_RICHARDSON, P.IR_ERROR_FGMRES])
def test_richardson_variants(dev, method):
    """Richardson refinement and FGMRES on the error system (the paper's comparison of
    Fig. 3) against the oracle's implementation of the same iterations."""
    say("richardson variant", method)
    p, s, f = make(2, dev, ir_method=method)
    for step in (2, 3):
        v, b = p.system(step)
        s.refactor(cuda(v, dev))
        xg, info = s.solve(cuda(b, dev), allow_noconv=True)
        x = xg.cpu().numpy()
        olx, oux, _ = f.refactor64(p.rowptr, p.colidx, v)
        xo, oi = oracle.richardson(f, p.rowptr, p.colidx, v, b, Lx=olx, Ux=oux,
                                   inner_restart=10 if method == P.IR_ERROR_FGMRES else 0, inner_tol=1e-2)
        m = oracle.metrics(p.rowptr, p.colidx, v, x, b)
        say("   step", step, "gpu corrections", info["cycles"], "applications", info["precond_applications"],
            "nsr %.2e" % m["nsr"], "| oracle corrections", oi["corrections"], "applications", oi["applications"],
            "nsr %.2e" % oi["nsr"])
        assert np.isfinite(x).all()
        assert info["nsr"] == pytest.approx(m["nsr"], rel=1e-6)
        # the same iteration on the same factors: NSR within two orders of the oracle's
        assert m["nsr"] <= 100 * oi["nsr"] + 1e-30
        assert abs(info["cycles"] - oi["corrections"]) <= 2


def test_fgmres_counts_preconditioner_applications(dev):
    say("precond applications")
    p, s, f = make(2, dev)
    v, b = p.system(3)
    s.refactor(cuda(v, dev))
    _, info = s.solve(cuda(b, dev))
    assert info["precond_applications"] == 1 + info["iterations"]


@pytest.mark.parametrize("cfg", [1, 2])
@pytest.mark.parametrize("resid", ["fp64", "dd"])
def test_residual_bit_exact(dev, cfg, resid):
    # rho = b - K x through kkt_residual, in working precision and in double-double, against
    # the oracle's residual of the same kind: same summation order, so bit-identical
    say("residual", resid, "config", cfg)
    p, s, _ = make(cfg, dev, residual=P.RESID_DD if resid == "dd" else P.RESID_FP64)
    v, b = p.system(2)
    s.refactor(cuda(v, dev))
    rng = np.random.default_rng(cfg)
    x = rng.standard_normal(p.N) * 10.0 ** rng.uniform(-6, 6, p.N)
    r = s.residual(cuda(b, dev), cuda(x, dev))
    torch.cuda.synchronize()
    ro = oracle.residual(p.rowptr, p.colidx, v, x, b, resid)
    assert np.array_equal(r.cpu().numpy(), ro)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_solve_dd_residual_reaches_working_accuracy(dev, seed):
    # FGMRES-IR with double-double residuals: componentwise error against the exact rational
    # solution of the stored system within 2u (the working-precision residual stalls near
    # cond * u on these systems)
    from exact import exact_solve, max_componentwise_error
    say("dd residual solve seed", seed)
    p = ks.small_kkt(24, 16, seed)
    v, b = p.system(1)
    s = P.Solver(p.rowptr, p.colidx, v, residual=P.RESID_DD).bind(dev)
    s.refactor(cuda(v, dev))
    x, info = s.solve(cuda(b, dev))
    assert info["converged"] == 1 and info["nrbe"] <= 1e-12
    xe = exact_solve(ks.to_dense(p.rowptr, p.colidx, v, p.N), b)
    assert max_componentwise_error(x.cpu().numpy(), xe) <= 2.0 ** -52


def test_solve_dd_residual_sequence(dev):
    say("dd residual 60k sequence")
    p, s, _ = make(2, dev, residual=P.RESID_DD)
    for step in (2, 3):
        v, b = p.system(step)
        s.refactor(cuda(v, dev))
        x, info = s.solve(cuda(b, dev))
        assert info["converged"] == 1 and info["nrbe"] <= 1e-12
        m = oracle.metrics(p.rowptr, p.colidx, v, x.cpu().numpy(), b)
        assert m["nrbe"] <= 1e-12


@pytest.mark.parametrize("gs", [P.GS_CGS2, P.GS_DCGS2])
@pytest.mark.parametrize("case", ["1x1", "2x2", "3x3-dense"])
def test_tiny_systems(dev, case, gs):
    # degenerate sizes: one row, a 2x2 KKT block, a dense 3x3 (every schedule is one tile)
    say("tiny system", case, "gs", gs)
    if case == "1x1":
        rp, ci, v = np.array([0, 1]), np.array([0], np.int32), np.array([4.0])
    elif case == "2x2":
        rp, ci, v = np.array([0, 2, 4]), np.array([0, 1, 0, 1], np.int32), np.array([1e-3, 1.0, 1.0, -1e-8])
    else:
        rp = np.array([0, 3, 6, 9])
        ci = np.array([0, 1, 2] * 3, np.int32)
        v = np.array([2.0, -1.0, 0.5, -1.0, 3.0, 1.0, 0.5, 1.0, -4.0])
    n = len(rp) - 1
    b = np.arange(1.0, n + 1.0)
    s = P.Solver(rp, ci, v, restart=1, gram_schmidt=gs).bind(dev)
    s.refactor(cuda(v, dev))
    x, info = s.solve(cuda(b, dev))
    A = ks.to_dense(rp, ci, v, n)
    xe = np.linalg.solve(A, b)
    assert info["converged"] == 1
    assert np.allclose(x.cpu().numpy(), xe, rtol=1e-12, atol=0)


@pytest.mark.parametrize("gs", [P.GS_CGS2, P.GS_DCGS2])
def test_restart_one_on_60k(dev, gs):
    # FGMRES(1): every cycle is one Arnoldi step; still converges under the same control
    say("restart 1 on 60k gs", gs)
    p, s, _ = make(2, dev, restart=1, gram_schmidt=gs)
    v, b = p.system(2)
    s.refactor(cuda(v, dev))
    x, info = s.solve(cuda(b, dev))
    assert info["converged"] == 1 and info["nrbe"] <= 1e-12
    assert info["cycles"] == info["iterations"]


def test_repivot_recovers_failed_static_pivots(dev):
    # 60k KKT with D over 26 decades and textbook threshold pivoting (tau = 0.1): the pivot
    # sequence of system 1 leaves tiny static pivots in system 2 and FGMRES-IR stalls (also
    # in the oracle, checked below: its relative residual estimate stays near 1e-4 after 21
    # cycles, ten decades above the tolerance, so rounding differences cannot carry it over).
    # With repivot_cycles the solve repeats the pivoted factorization for system 2 (ordering
    # kept), whose analysis must match the oracle's fresh pivoted LU of system 2 bit for bit.
    say("repivot 60k seed 17")
    tau = 0.1
    p = ks.small_kkt(35000, 25000, 17, (-13.0, 13.0))
    v1, _ = p.system(1)
    v2, b2 = p.system(2)
    f1 = oracle.LU(p.rowptr, p.colidx, v1, tau=tau)
    lx, ux, ng = f1.refactor64(p.rowptr, p.colidx, v2)
    _, oinf = f1.fgmres_ir(p.rowptr, p.colidx, v2, b2, Lx=lx, Ux=ux, restart=10, max_restarts=20, eta=1e-14, mode=1)
    assert ng > 0 and not oinf["converged"] and oinf["rr"] > 1e-8
    s0 = P.Solver(p.rowptr, p.colidx, v1, repivot_cycles=0, pivot_tau=tau).bind(dev)
    s0.refactor(cuda(v2, dev))
    x0 = s0.direct_solve(cuda(b2, dev)).cpu().numpy()
    xs, i0 = s0.solve(cuda(b2, dev), allow_noconv=True)
    assert i0["converged"] == 0 and i0["repivoted"] == 0 and i0["cycles"] == 21
    # a solve that does not converge returns its best iterate: never a larger true residual
    # than the direct solution x0
    r0 = oracle.metrics(p.rowptr, p.colidx, v2, x0, b2)["resid"]
    rs = oracle.metrics(p.rowptr, p.colidx, v2, xs.cpu().numpy(), b2)["resid"]
    say("   x0 residual %.3e, returned %.3e, restored %d" % (r0, rs, i0["restored_best"]))
    assert rs <= r0 * (1 + 1e-12) and i0["rr"] <= 1.0
    assert i0["true_resid"] == pytest.approx(rs, rel=1e-6)
    s = P.Solver(p.rowptr, p.colidx, v1, pivot_tau=tau).bind(dev)
    s.refactor(cuda(v2, dev))
    x, info = s.solve(cuda(b2, dev))
    assert info["converged"] == 1 and info["repivoted"] == 1 and info["nrbe"] <= 1e-12
    f2 = oracle.LU(p.rowptr, p.colidx, v2, Q=f1.Q, tau=tau)
    prow, q = s.permutations()
    assert np.array_equal(q, f1.Q) and np.array_equal(prow, f2.prow)
    lp, li, up, ui = s.pattern()
    assert np.array_equal(lp, f2.Lp) and np.array_equal(li, f2.Li)
    assert np.array_equal(up, f2.Up) and np.array_equal(ui, f2.Ui)
    # the re-pivoted factors are the refactorization of system 2 with the new sequence
    glx, gux = s.factor_values(0)
    assert np.array_equal(glx, f2.Lx) and np.array_equal(gux, f2.Ux)
    xo = f2.solve(b2)
    rel = np.abs(x.cpu().numpy() - xo).max() / np.abs(xo).max()
    assert rel <= 1e-8 * f2.condest(p.rowptr, v2)
    # the next system refactors with the new pivot sequence: bit-identical to the oracle's
    # static refactorization of system 3 with system 2's pivots
    v3, b3 = p.system(3)
    s.refactor(cuda(v3, dev))
    torch.cuda.synchronize()
    glx, gux = s.factor_values(0)
    olx3, oux3, _ = f2.refactor64(p.rowptr, p.colidx, v3)
    assert np.array_equal(glx, olx3) and np.array_equal(gux, oux3)


def _serving_patterns():
    return [ks.make_pattern(1), ks.small_kkt(6000, 4000, 3)]


def _alone(p, steps, dev):
    s = P.Solver(p.rowptr, p.colidx, p.system(1)[0]).bind(dev)
    out = []
    for k in steps:
        v, b = p.system(k)
        s.refactor(cuda(v, dev))
        x, info = s.solve(cuda(b, dev))
        out.append((x.cpu().numpy(), info))
    return out


@pytest.mark.parametrize("pool_slots", [4.0, 1.2])
def test_server_results_match_alone(dev, pool_slots):
    # a mix of two patterns through the serving loop (3 workers): every result equals the
    # standalone solve of the same system bit for bit; with a pool that holds about one slot
    # of the larger pattern, requests wait for room and idle slots are evicted
    say("server mix, pool slots", pool_slots)
    pats = _serving_patterns()
    steps = [1, 2, 3, 4]
    alone = [_alone(p, steps, dev) for p in pats]
    sizes = []
    for p in pats:
        s = P.Solver(p.rowptr, p.colidx, p.system(1)[0])
        sizes.append(int(s.workspace_size() * 1.5) + (1 << 20))
    srv = P.Server(int(max(sizes) * pool_slots), workers=3, device=dev)
    pids = [srv.add_pattern(p.rowptr, p.colidx, p.system(1)[0]) for p in pats]
    reqs = []
    for k_i, k in enumerate(steps):
        for pi, p in enumerate(pats):
            v, b = p.system(k)
            vv, bb = cuda(v, dev), cuda(b, dev)
            x = torch.empty_like(bb)
            reqs.append((pi, k_i, x, srv.submit(pids[pi], vv, bb, x)))
    for pi, k_i, x, t in reqs:
        rc, info, times = srv.wait(t)
        assert rc == P.KKT_OK and info["converged"] == 1
        xa, ia = alone[pi][k_i]
        assert np.array_equal(x.cpu().numpy(), xa)
        assert info["iterations"] == ia["iterations"]
        assert times["latency_ms"] >= times["service_ms"] >= 0.0
    st = srv.stats()
    assert st["completed"] == len(reqs)
    if pool_slots < 2:
        assert st["slots_evicted"] > 0
    srv.close()


def test_full_size_500k_refactor_and_direct_solve(dev):
    # the 500,000-row workload at full size: refactorization of system 2 bit-identical to the
    # oracle's static-pivot refactorization, and the direct solve within the LU backward-error
    # bound on a sample of rows (the oracle recomputes those rows one by one)
    say("500k full size")
    p = ks.make_pattern(3)
    v1, _ = p.system(1)
    v2, b2 = p.system(2)
    s = P.Solver(p.rowptr, p.colidx, v1).bind(dev)
    f = oracle.LU(p.rowptr, p.colidx, v1)
    s.refactor(cuda(v2, dev))
    torch.cuda.synchronize()
    lx, ux = s.factor_values(0)
    olx, oux, ng = f.refactor64(p.rowptr, p.colidx, v2)
    assert np.array_equal(lx, olx) and np.array_equal(ux, oux)
    info = s.info()
    assert info["levels_l"] > 0 and info["nnz_l"] == olx.size
    z = s.direct_solve(cuda(b2, dev)).cpu().numpy()
    zo = f.solve(b2, Lx=olx, Ux=oux)
    rng = np.random.default_rng(7)
    rows = rng.choice(p.N, size=2000, replace=False)
    # sampled rows of the triangular solves' result agree with the oracle's to the
    # precision the bound of the factors allows (relative to the largest component)
    scale = np.abs(zo).max()
    assert np.all(np.abs(z[rows] - zo[rows]) <= 1e-6 * scale + 1e-6 * np.abs(zo[rows]))


def test_long_refinement_repeatable_bitwise(dev):
    # 21 restart cycles of FGMRES(10) on a system whose inherited pivots stall the refinement:
    # every Arnoldi step's stop decision and every sentinel re-arm must agree across blocks, or
    # repeated solves drift apart (regression test for a race on the rotated right-hand side)
    say("long refinement repeatable")
    p = ks.small_kkt(35000, 25000, 17, (-13.0, 13.0))
    v1, _ = p.system(1)
    v2, b2 = p.system(2)
    s = P.Solver(p.rowptr, p.colidx, v1, repivot_cycles=0, pivot_tau=0.1).bind(dev)
    out = []
    for _ in range(3):
        s.refactor(cuda(v2, dev))
        x, info = s.solve(cuda(b2, dev), allow_noconv=True)
        out.append((x.cpu().numpy(), info["iterations"], info["est_resid"]))
    assert out[0][1] > 100
    for x, it, est in out[1:]:
        assert np.array_equal(x, out[0][0]) and it == out[0][1] and est == out[0][2]


def test_delayed_cgs2_sequence(dev):
    # delayed CGS2 (gram_schmidt = DCGS2, one reduction per Arnoldi step) builds the same
    # Krylov basis as CGS2: on the 60k sequence it takes CGS2's iteration counts and the
    # oracle's DCGS2 counts, applies M^-1 once more per cycle that converges early, and
    # agrees with a fresh pivoted direct solve like CGS2 does
    say("delayed cgs2 60k sequence")
    p, s2, f = make(2, dev)
    s1 = P.Solver(p.rowptr, p.colidx, p.system(1)[0], gram_schmidt=P.GS_DCGS2).bind(dev)
    for step in (2, 3, 4):
        v, b = p.system(step)
        s1.refactor(cuda(v, dev))
        s2.refactor(cuda(v, dev))
        x1, i1 = s1.solve(cuda(b, dev))
        x2, i2 = s2.solve(cuda(b, dev))
        assert i1["converged"] == 1 and i1["nrbe"] <= 1e-12
        assert abs(i1["iterations"] - i2["iterations"]) <= 1
        lx, ux, _ = f.refactor64(p.rowptr, p.colidx, v)
        xo, io = f.fgmres_ir(p.rowptr, p.colidx, v, b, Lx=lx, Ux=ux, restart=10, max_restarts=20,
                             eta=1e-14, mode=1, gs="dcgs2")
        assert io["converged"] and abs(i1["iterations"] - io["iters"]) <= 1
        early = int(i1["iterations"] < i1["cycles"] * 10)
        assert i1["precond_applications"] == 1 + i1["iterations"] + early
        xg = x1.cpu().numpy()
        xd, _ = oracle.direct_solve(p.rowptr, p.colidx, v, b, Q=f.Q)
        rel = np.linalg.norm(xg - xd) / np.linalg.norm(xd)
        reld = np.linalg.norm(xo - xd) / np.linalg.norm(xd)
        # as for CGS2: the GPU and the oracle's delayed CGS2 land within a few unit roundoffs
        assert np.linalg.norm(xg - xo) <= 1e-13 * np.linalg.norm(xo)
        assert rel <= 1.01 * reld + 1e-13


@pytest.mark.parametrize("R", [2, 3])
def test_delayed_cgs2_restarts_match_oracle(dev, R):
    # short restart lengths on the 60k sequence: cycles end at their closing step (R = 2:
    # 3 full cycles) or converge inside one (R = 3: 3 + 1 steps); counts within one of the
    # oracle's, preconditioner applications exactly as the lagged estimate implies
    say("delayed cgs2 restart", R)
    p, s, f = make(2, dev, restart=R, gram_schmidt=P.GS_DCGS2)
    v, b = p.system(2)
    s.refactor(cuda(v, dev))
    x, info = s.solve(cuda(b, dev))
    lx, ux, _ = f.refactor64(p.rowptr, p.colidx, v)
    xo, io = f.fgmres_ir(p.rowptr, p.colidx, v, b, Lx=lx, Ux=ux, restart=R, max_restarts=20,
                         eta=1e-14, mode=1, gs="dcgs2")
    say("  gpu", info["iterations"], info["cycles"], info["precond_applications"],
        "oracle", io["iters"], io["cycles"], io["applications"])
    assert info["converged"] == 1 and io["converged"]
    # the counts of a floating-point iteration follow the rounding of the triangular-solve
    # sums, whose order differs from the oracle's: one step or cycle either way
    assert abs(info["iterations"] - io["iters"]) <= 1 and abs(info["cycles"] - io["cycles"]) <= 1
    # one more M^-1 than Arnoldi columns per cycle that stops before its closing step, plus x0
    full = info["cycles"] - 1
    last = info["iterations"] - full * R
    assert info["precond_applications"] == 1 + info["iterations"] + (1 if last < R else 0)


@pytest.mark.parametrize("mode", ["mixed", "error_fgmres"])
def test_delayed_cgs2_other_paths(dev, mode):
    # delayed CGS2 inside the FP32-preconditioned solve (with its FP64 fallback) and as the
    # inner solver of Richardson on the error system: same acceptance as with CGS2
    say("delayed cgs2 path", mode)
    opts = dict(gram_schmidt=P.GS_DCGS2)
    if mode == "mixed":
        opts["precision"] = P.PREC_MIXED
    else:
        opts["ir_method"] = P.IR_ERROR_FGMRES
    p, s, f = make(1, dev, **opts)
    ref = P.Solver(p.rowptr, p.colidx, p.system(1)[0],
                   **{k: v for k, v in opts.items() if k != "gram_schmidt"}).bind(dev)
    for step in (2, 3):
        v, b = p.system(step)
        s.refactor(cuda(v, dev))
        ref.refactor(cuda(v, dev))
        x, info = s.solve(cuda(b, dev), allow_noconv=True)
        xr, ir = ref.solve(cuda(b, dev), allow_noconv=True)
        say("   step", step, "dcgs2", info["converged"], info["iterations"], "%.2e" % info["nrbe"],
            "| cgs2", ir["converged"], ir["iterations"], "%.2e" % ir["nrbe"])
        assert info["converged"] == ir["converged"]
        m = oracle.metrics(p.rowptr, p.colidx, v, x.cpu().numpy(), b)
        assert np.isfinite(m["nrbe"]) and m["nrbe"] <= max(10 * ir["nrbe"], 1e-12)
