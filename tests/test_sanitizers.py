"""The host analysis (analysis.cpp) built with AddressSanitizer and UndefinedBehaviorSanitizer
(g++, host code only) and run on the workload's small systems, the arrow-head KKT, the
moderate family, nested dissection, a tile budget of 16 KiB and rejected inputs: no sanitizer
report, and the same sizes and schedule statistics as the library's own build.  The driver also
replays both triangular-solve schedules on the CPU as the solve kernel reads them (LDS slots,
externals, unstaged rows, dense blocks) with random factors: the result must match plain
substitution to rounding; and it replays the refactorization of a second system from the
hand-out metadata: bit-identical to the oracle's static-pivot refactorization."""
import os
import pathlib
import shutil
import subprocess

import numpy as np
import pytest

import kkt_synth as ks
import oracle
import paper_2401_13926_amd as P

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2401_13926_amd" / "csrc"


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no g++")
    out = tmp_path_factory.mktemp("asan") / "analysis_driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-I", str(CSRC), "-o", str(out),
           str(ROOT / "tests" / "sanitize" / "analysis_driver.cpp"), str(CSRC / "analysis.cpp")]
    subprocess.run(cmd, check=True)
    return out


def run(driver, tmp_path, rowptr, colidx, values, tau=1e-10, ordering=0, tile_kib=0, values2=None):
    f = tmp_path / "in.bin"
    rp = np.ascontiguousarray(rowptr, np.int64)
    ci = np.ascontiguousarray(colidx, np.int32)
    v = np.ascontiguousarray(values, np.float64)
    with open(f, "wb") as fh:
        fh.write(np.array([rp.size - 1, ci.size], np.int64).tobytes())
        fh.write(np.array([tau], np.float64).tobytes())
        fh.write(np.array([ordering, tile_kib], np.int32).tobytes())
        fh.write(rp.tobytes() + ci.tobytes() + v.tobytes())
        if values2 is not None:
            fh.write(np.ascontiguousarray(values2, np.float64).tobytes())
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    cmd = [str(driver), str(f)] + ([str(tmp_path / "factors.bin")] if values2 is not None else [])
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return dict(kv.split("=", 1) for kv in r.stdout.split() if "=" in kv)


CASES = {
    "7k": lambda: (ks.make_pattern(1), {}),
    "small-tau0.1": lambda: (ks.small_kkt(300, 200, 4), dict(tau=0.1)),
    "nd": lambda: (ks.small_kkt(400, 250, 6), dict(ordering=1)),
    "tile16": lambda: (ks.small_kkt(2000, 1500, 8), dict(tile_kib=16)),
    "moderate": lambda: (ks.moderate_kkt(2000, 1500), {}),
}


def assert_schedules_replay(out):
    # "ok:<relative difference from plain substitution>", or the first violated property
    for k in ("sched_l", "sched_u"):
        assert out[k].startswith("ok:") and float(out[k][3:]) <= 1e-12, (k, out[k])


@pytest.mark.parametrize("case", sorted(CASES))
def test_analysis_under_sanitizers_matches_library(driver, tmp_path, case):
    p, kw = CASES[case]()
    v, _ = p.system(1)
    out = run(driver, tmp_path, p.rowptr, p.colidx, v, **kw)
    assert out["status"] == "0"
    assert_schedules_replay(out)
    assert int(out["dense_l"]) > 0  # the replay covers dense segments
    opts = dict(pivot_tau=kw.get("tau", 1e-10), ordering=kw.get("ordering", 0), tile_lds_kib=kw.get("tile_kib", 0),
                narrow_columns=1024)
    info = P.Solver(p.rowptr, p.colidx, v, **opts).info()
    for k in ("nnz_l", "nnz_u", "levels_refactor", "levels_l", "levels_u", "updates", "offdiag_pivots",
              "tiles_l", "tiles_u"):
        assert int(out[k]) == info[k], k


def test_arrow_head_under_sanitizers(driver, tmp_path):
    a = ks.ArrowKKT(4000, 1500, 2500, seed=1)
    v, _ = a.system(1)
    out = run(driver, tmp_path, a.rowptr, a.colidx, v)
    assert out["status"] == "0" and int(out["nnz_u"]) > 0
    assert_schedules_replay(out)


def test_rejected_inputs_under_sanitizers(driver, tmp_path):
    # unsorted columns, an out-of-range column, a non-finite value and a structurally singular
    # matrix: each is reported, none trips a sanitizer
    rp = np.array([0, 2, 4], np.int64)
    out = run(driver, tmp_path, rp, np.array([1, 0, 0, 1], np.int32), np.ones(4))
    assert out["status"] != "0"
    out = run(driver, tmp_path, rp, np.array([0, 5, 0, 1], np.int32), np.ones(4))
    assert out["status"] != "0"
    out = run(driver, tmp_path, rp, np.array([0, 1, 0, 1], np.int32), np.array([1.0, np.nan, 1.0, 1.0]))
    assert out["status"] != "0"
    out = run(driver, tmp_path, np.array([0, 1, 2], np.int64), np.array([0, 0], np.int32), np.ones(2))
    assert out["status"] != "0"


REFACTOR_CASES = {
    "7k": lambda: (ks.make_pattern(1), 1e-10),
    "arrow": lambda: (ks.ArrowKKT(4000, 1500, 2500, seed=1), 1e-10),
    # inherited threshold pivots that leave tiny static pivots in system 2: the guard fires
    "60k-guarded": lambda: (ks.small_kkt(35000, 25000, 17, (-13.0, 13.0)), 0.1),
}


@pytest.mark.parametrize("case", sorted(REFACTOR_CASES))
def test_refactor_metadata_replay_matches_oracle(driver, tmp_path, case):
    # the refactorization of system 2 replayed on the CPU from the hand-out metadata (items
    # in hand-out order, staging map into the vector-order copy of K, flat update lists, the
    # scatter into the solve layout) equals the oracle's static-pivot refactorization bit for
    # bit, and no item reads a source that a later item produces
    p, tau = REFACTOR_CASES[case]()
    v1, _ = p.system(1)
    v2, _ = p.system(2)
    out = run(driver, tmp_path, p.rowptr, p.colidx, v1, tau=tau, values2=v2)
    assert out["status"] == "0" and out["refactor"] == "ok", out.get("refactor")
    fac = np.fromfile(tmp_path / "factors.bin", np.float64)
    nl = int(out["nnz_l"])
    f = oracle.LU(p.rowptr, p.colidx, v1, tau=tau)
    olx, oux, guarded = f.refactor64(p.rowptr, p.colidx, v2)
    assert np.array_equal(fac[:nl], olx) and np.array_equal(fac[nl:], oux)
    if case == "60k-guarded":
        assert guarded > 0
