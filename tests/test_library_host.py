"""Host-side checks of the GPU library: the C ABI loads and exports every declared symbol,
and its host analysis (an independent implementation of the ordering and pivot rules)
reproduces the oracle's permutations, patterns and FP64 factor values bit for bit.
No GPU needed: kkt_analyze and the getters make no device calls."""
import pathlib
import re

import numpy as np
import pytest

import kkt_synth as ks
import oracle
import paper_2401_13926_amd as P
from paper_2401_13926_amd import kkt as K

ROOT = pathlib.Path(__file__).resolve().parents[1]


def test_exports_every_declared_symbol():
    header = (ROOT / "include" / "kkt.h").read_text()
    declared = sorted(set(re.findall(r"\b(kkt_[a-z_]+)\s*\(", header)))
    assert declared, "no declarations found"
    assert sorted(K.EXPORTS) == declared
    lib = P.lib()
    for name in declared:
        assert hasattr(lib, name), name
    # every entry point that takes arguments has its ctypes argument types declared (a float
    # argument without them cannot be passed)
    for name in declared:
        if "(void)" not in header.split(name + "(")[1][:8]:
            assert getattr(lib, name).argtypes is not None, name


def check_parity(rowptr, colidx, values, leaf=64, tau=0.1, method="md"):
    s = P.Solver(rowptr, colidx, values, nd_leaf=leaf, pivot_tau=tau,
                 ordering=P.ORDER_MD if method == "md" else P.ORDER_ND)
    Q = oracle.order(rowptr, colidx, method=method, leaf=leaf)
    f = oracle.LU(rowptr, colidx, values, Q=Q, tau=tau)
    prow, q = s.permutations()
    assert np.array_equal(q, f.Q)
    assert np.array_equal(prow, f.prow)
    lp, li, up, ui = s.pattern()
    assert np.array_equal(lp, f.Lp) and np.array_equal(li, f.Li)
    assert np.array_equal(up, f.Up) and np.array_equal(ui, f.Ui)
    lx, ux = s.analysis_values()
    assert np.array_equal(lx, f.Lx) and np.array_equal(ux, f.Ux)
    inf = s.info()
    assert inf["nnz_l"] == f.lnz and inf["nnz_u"] == f.unz
    assert inf["offdiag_pivots"] == int(np.sum(f.prow != f.Q))
    return s, f


@pytest.mark.parametrize("cfg", [1, 2])
def test_analysis_bit_exact_configs(cfg):
    p = ks.make_pattern(cfg)
    v, _ = p.system(1)
    check_parity(p.rowptr, p.colidx, v)


@pytest.mark.parametrize("cfg", [1, 2])
def test_analysis_bit_exact_configs_default_tau(cfg):
    # the default threshold 1e-10 keeps every diagonal pivot of the quasi-definite K: P = Q
    p = ks.make_pattern(cfg)
    v, _ = p.system(1)
    s, f = check_parity(p.rowptr, p.colidx, v, tau=1e-10)
    assert s.info()["offdiag_pivots"] == 0 and np.array_equal(f.prow, f.Q)


def test_analysis_arrow_long_column_and_unstaged_row():
    # a dense constraint row: one factor column beyond the refactorization's 1,024-entry LDS
    # stage and an L row too long for a staged solve tile; the analysis still matches the
    # oracle bit for bit and reports both
    a = ks.ArrowKKT(4000, 1500, 2500, seed=1)
    v, _ = a.system(1)
    s, f = check_parity(a.rowptr, a.colidx, v, tau=1e-10)
    inf = s.info()
    assert inf["max_column"] == int((np.diff(f.Up) + np.diff(f.Lp)).max()) > 1024
    assert inf["unstaged_l"] >= 1 and inf["tiles_l"] > inf["unstaged_l"]
    s16 = P.Solver(a.rowptr, a.colidx, v, tile_lds_kib=16)
    assert s16.info()["unstaged_l"] >= 1 and s16.info()["tiles_l"] > inf["tiles_l"]


@pytest.mark.parametrize("seed", range(12))
def test_analysis_bit_exact_small(seed):
    p = ks.small_kkt(40 + 7 * seed, 25 + 4 * seed, 300 + seed, dlog=(-8.0, 8.0))
    v, _ = p.system(1 + seed % 4)
    check_parity(p.rowptr, p.colidx, v, leaf=[1, 4, 16, 64][seed % 4], tau=[0.1, 0.5, 1.0, 1e-10][seed % 4])


def test_analysis_general_unsymmetric():
    rng = np.random.default_rng(11)
    n = 300
    import scipy.sparse as sp
    A = sp.random(n, n, density=0.01, random_state=12, format="csr") + sp.diags(rng.standard_normal(n))
    A = sp.csr_matrix(A)
    A.sort_indices()
    check_parity(A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data, leaf=8, tau=0.3)


def test_errors():
    rp = np.array([0, 2, 3], np.int64)
    ci = np.array([1, 0, 1], np.int32)
    with pytest.raises(P.KKTError) as e:
        P.Solver(rp, ci, np.ones(3))
    assert e.value.code == P.KKT_EINVAL
    rp = np.array([0, 2, 4, 5], np.int64)
    ci = np.array([0, 1, 0, 1, 2], np.int32)
    with pytest.raises(P.KKTError) as e:
        P.Solver(rp, ci, np.array([1.0, 1.0, 1.0, 1.0, 1.0]))
    assert e.value.code == P.KKT_ESINGULAR
    with pytest.raises(P.KKTError) as e:
        P.Solver(rp, ci, np.array([1.0, np.nan, 1.0, 1.0, 1.0]))
    assert e.value.code == P.KKT_EINVAL
    p = ks.small_kkt(20, 10, 1)
    v, _ = p.system(1)
    with pytest.raises(P.KKTError) as e:
        P.Solver(p.rowptr, p.colidx, v, restart=0)
    assert e.value.code == P.KKT_EINVAL
    s = P.Solver(p.rowptr, p.colidx, v)
    assert s.workspace_size() > 0


@pytest.mark.parametrize("opt", [dict(tile_lds_kib=8), dict(tile_lds_kib=151), dict(gram_schmidt=2),
                                 dict(restart=65), dict(residual=3), dict(narrow_columns=-1),
                                 dict(deterministic=0)])
def test_option_validation(opt):
    p = ks.small_kkt(20, 10, 1)
    v, _ = p.system(1)
    with pytest.raises(P.KKTError) as e:
        P.Solver(p.rowptr, p.colidx, v, **opt)
    assert e.value.code == P.KKT_EINVAL


def test_tile_budget_changes_the_schedule_not_the_factors():
    # a larger LDS budget per solve tile packs more levels per tile (fewer windows); the
    # factor patterns, pivots and refactorization levels do not depend on it
    p = ks.make_pattern(1)
    v, _ = p.system(1)
    a = P.Solver(p.rowptr, p.colidx, v)
    b = P.Solver(p.rowptr, p.colidx, v, tile_lds_kib=150)
    ia, ib = a.info(), b.info()
    for k in ("nnz_l", "nnz_u", "offdiag_pivots", "levels_refactor", "levels_l", "levels_u", "updates"):
        assert ia[k] == ib[k], k
    assert [np.array_equal(x, y) for x, y in zip(a.pattern(), b.pattern())] == [True] * 4
    assert b.workspace_size() > 0 and a.workspace_size() > 0


def test_narrow_level_threshold_keeps_the_factors():
    # the hand-out threshold of the refactorization changes only which levels go a column at a
    # time; patterns, pivots and the level structure are the same
    p = ks.make_pattern(1)
    v, _ = p.system(1)
    a = P.Solver(p.rowptr, p.colidx, v)
    b = P.Solver(p.rowptr, p.colidx, v, narrow_columns=1)
    c = P.Solver(p.rowptr, p.colidx, v, narrow_columns=1 << 30)
    for s in (b, c):
        assert s.info()["levels_refactor"] == a.info()["levels_refactor"]
        assert all(np.array_equal(x, y) for x, y in zip(a.pattern(), s.pattern()))


def test_profiling_mask_rejects_unknown_classes():
    p = ks.small_kkt(20, 10, 1)
    v, _ = p.system(1)
    s = P.Solver(p.rowptr, p.colidx, v)
    s.set_profiling(True, classes=["trsv_u"])
    s.set_profiling(False)
    from paper_2401_13926_amd import kkt as K
    assert K.lib().kkt_set_profiling_mask(s._h, 1 << len(K.KERNEL_CLASSES)) == P.KKT_EINVAL


@pytest.mark.parametrize("cfg", [1, 2])
def test_analysis_bit_exact_nested_dissection(cfg):
    p = ks.make_pattern(cfg)
    v, _ = p.system(1)
    check_parity(p.rowptr, p.colidx, v, method="nd")


@pytest.mark.parametrize("seed", range(4))
def test_analysis_bit_exact_small_nd(seed):
    p = ks.small_kkt(60 + 7 * seed, 35 + 4 * seed, 700 + seed)
    v, _ = p.system(2)
    check_parity(p.rowptr, p.colidx, v, leaf=[1, 4, 16, 64][seed], method="nd")


def test_abi_struct_sizes_match_header(tmp_path):
    import ctypes as C
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "sz.c"
    src.write_text('#include "kkt.h"\n#include <stdio.h>\nint main(void){printf("%zu %zu %zu %zu %zu\\n",'
                   'sizeof(kkt_opts_t), sizeof(kkt_solve_info_t), sizeof(kkt_analysis_info_t),'
                   'sizeof(kkt_kernel_times_t), sizeof(kkt_request_times_t)); return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run([cc, "-I", str(ROOT / "include"), "-o", str(exe), str(src)], check=True)
    sizes = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert sizes == [C.sizeof(K.Opts), C.sizeof(K.SolveInfo), C.sizeof(K.AnalysisInfo), C.sizeof(K.KernelTimes),
                     C.sizeof(K.RequestTimes)]


def test_noalloc_direct_solve_rejects_oversize_before_device_calls():
    # the allocation-free direct solve has a static scratch of 2^21 rows: a larger handle is
    # refused with KKT_EINVAL before any device call (so this runs without a GPU)
    import ctypes as C
    n = (1 << 21) + 1
    s = P.Solver(np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32), np.full(n, 2.0))
    rc = K.lib().kkt_direct_solve_noalloc(s._h, C.c_void_p(8), C.c_void_p(16), None)
    assert rc == K.KKT_EINVAL
    assert b"static scratch" in K.lib().kkt_last_error(s._h)


@pytest.mark.parametrize("size", [(60, 35, 41), (3500, 2500, 42)])
def test_hykkt_analysis_matches_oracle(size):
    # HyKKT (zero (2,2) block): gamma, the pattern of H_gamma and the factorization of system 1's
    # H_gamma match the oracle's (the factors depend on every entry of H_gamma, so the entries
    # match too)
    from oracle import hykkt as hy
    n, m, seed = size
    p = ks.small_kkt(n, m, seed, dlog=(-8.0, 8.0), delta=0.0)
    v, _ = p.system(1)
    g = P.HyKKT(p.rowptr, p.colidx, v, n_primal=p.n)
    f = hy.HyKKT(p.rowptr, p.colidx, v, n=p.n)
    rp, ci, _, gamma = g.hgamma(with_values=False)
    assert gamma == f.gamma
    assert np.array_equal(rp, f.hrp) and np.array_equal(ci, f.hci)
    h = K.C.c_void_p()
    assert K.lib().kkt_hykkt_factor_handle(g._h, K.C.byref(h)) == 0
    inner = P.Solver.__new__(P.Solver)
    inner._h, inner.n = h, p.n
    try:
        lx, ux = inner.analysis_values()
        prow, q = inner.permutations()
    finally:
        inner._h = None
    assert np.array_equal(lx, f.lu.Lx) and np.array_equal(ux, f.lu.Ux)
    assert np.array_equal(q, f.lu.Q) and np.array_equal(prow, f.lu.prow)


def test_hykkt_rejects_nonzero_22_block_and_bad_sizes():
    p = ks.small_kkt(40, 25, 9)  # delta = 1e-8 on the (2,2) block
    v, _ = p.system(1)
    with pytest.raises(P.KKTError) as e:
        P.HyKKT(p.rowptr, p.colidx, v, n_primal=p.n)
    assert e.value.code == P.KKT_EINVAL and "(2,2)" in str(e.value)
    q = ks.small_kkt(40, 25, 9, delta=0.0)
    w, _ = q.system(1)
    for bad in (0, q.N):
        with pytest.raises(P.KKTError):
            P.HyKKT(q.rowptr, q.colidx, w, n_primal=bad)
