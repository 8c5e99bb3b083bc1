"""GPU tests of batched refactorization and of the serving loop through the C ABI.

* kkt_refactor_batch / kkt_refactor_batch_graph: several systems of one pattern in one
  launch (slots are clones of one handle), each slot's factors bit-identical to the oracle's
  static-pivot refactorization of its own system and to a single kkt_refactor; graph
  replays with other values and eager work in between give the same bits every time.
* The serving loop on eight patterns of the serving workload's shape (dimensions spread over
  a range, n = 0.58 N, D log-uniform in [1e-10, 1e10]), with same-pattern batching and graphs
  on and off: every result equals the standalone solve of the same system bit for bit.
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


@pytest.mark.parametrize("precision", [P.PREC_FP64, P.PREC_MIXED])
@pytest.mark.parametrize("graph", [False, True])
def test_refactor_batch_matches_single_and_oracle(dev, precision, graph):
    say("batch refactor precision", precision, "graph", graph)
    p = ks.make_pattern(2)
    v1, _ = p.system(1)
    base = P.Solver(p.rowptr, p.colidx, v1, precision=precision)
    slots = [base.clone().bind(dev) for _ in range(3)]
    single = P.Solver(p.rowptr, p.colidx, v1, precision=precision).bind(dev)
    f = oracle.LU(p.rowptr, p.colidx, v1)
    prec = 1 if precision == P.PREC_MIXED else 0
    for rnd, steps in enumerate([(2, 3, 4), (5, 6, 7), (2, 8, 3)]):
        vals = [cuda(p.system(k)[0], dev) for k in steps]
        P.refactor_batch(slots, vals, graph=graph)
        torch.cuda.synchronize()
        for s, k, vv in zip(slots, steps, vals):
            lx, ux = s.factor_values(prec)
            v = p.system(k)[0]
            if prec:
                olx, oux, _ = f.refactor32(p.rowptr, p.colidx, v)
                olx, oux = olx.astype(np.float64), oux.astype(np.float64)
            else:
                olx, oux, _ = f.refactor64(p.rowptr, p.colidx, v)
            assert np.array_equal(lx, olx) and np.array_equal(ux, oux), "round %d system %d" % (rnd, k)
            single.refactor(vv)
            torch.cuda.synchronize()
            slx, sux = single.factor_values(prec)
            assert np.array_equal(lx, slx) and np.array_equal(ux, sux)
        # eager work on the slots between replays: a solve each
        for s, k in zip(slots, steps):
            _, info = s.solve(cuda(p.system(k)[1], dev), allow_noconv=True)
            assert info["nrbe"] <= 1e-12
    if graph:
        assert [s.graph_launches() for s in slots] == [3, 3, 3]


def test_refactor_batch_rejects_mixed_analyses(dev):
    p = ks.make_pattern(1)
    v1, _ = p.system(1)
    a = P.Solver(p.rowptr, p.colidx, v1).bind(dev)
    b = P.Solver(p.rowptr, p.colidx, v1).bind(dev)  # same pattern, another analysis
    vv = cuda(v1, dev)
    with pytest.raises(P.KKTError) as e:
        P.refactor_batch([a, b], [vv, vv])
    assert e.value.code == P.KKT_EINVAL
    with pytest.raises(P.KKTError) as e:
        P.refactor_batch([a, a], [vv, vv])
    assert e.value.code == P.KKT_EINVAL
    c = a.clone()  # not bound
    with pytest.raises(P.KKTError) as e:
        P.refactor_batch([a, c], [vv, vv])
    assert e.value.code == P.KKT_ESTATE


SERVE_DIMS = [7_000, 12_000, 17_000, 22_000, 27_000, 32_000, 37_000, 42_000]


def _serving_patterns():
    out = []
    for k, dim in enumerate(SERVE_DIMS):
        n = int(round(0.58 * dim))
        out.append(ks.make_pattern(4, k, n=n, m=dim - n, dlog=ks.SERVING_DLOG))
    return out


@pytest.mark.parametrize("max_batch,graphs", [(4, True), (8, False), (1, False)])
def test_server_eight_patterns_match_alone(dev, max_batch, graphs):
    # 8 patterns x 4 systems submitted in one burst to 3 workers: same-pattern requests that
    # wait together are batched; every result equals the standalone refactor + solve bit for bit
    say("server 8 patterns, max_batch", max_batch, "graphs", graphs)
    pats = _serving_patterns()
    steps = [1, 2, 3, 4]
    alone = {}
    for pi, p in enumerate(pats):
        s = P.Solver(p.rowptr, p.colidx, p.system(1)[0]).bind(dev)
        for k in steps:
            v, b = p.system(k)
            s.refactor(cuda(v, dev))
            x, info = s.solve(cuda(b, dev))
            alone[pi, k] = (x.cpu().numpy(), info["iterations"])
    sizes = [P.Solver(p.rowptr, p.colidx, p.system(1)[0]).workspace_size() for p in pats]
    srv = P.Server(int(sum(sizes) * 1.6 * 3), workers=3, device=dev, max_batch=max_batch, graphs=graphs)
    pids = [srv.add_pattern(p.rowptr, p.colidx, p.system(1)[0]) for p in pats]
    # inputs prepared first, then submitted in one burst, the systems of a pattern together
    # (as an optimizer instance's requests would queue up), so workers find same-pattern
    # requests waiting and batch them
    inputs = []
    for pi, p in enumerate(pats):
        for k in steps:
            v, b = p.system(k)
            inputs.append((pi, k, cuda(v, dev), cuda(b, dev)))
    torch.cuda.synchronize()
    reqs = []
    for pi, k, vv, bb in inputs:
        x = torch.empty_like(bb)
        reqs.append((pi, k, x, srv.submit(pids[pi], vv, bb, x)))
    for pi, k, x, t in reqs:
        rc, info, times = srv.wait(t)
        assert rc == P.KKT_OK and info["converged"] == 1 and info["nrbe"] <= 1e-12
        xa, ita = alone[pi, k]
        assert np.array_equal(x.cpu().numpy(), xa), "pattern %d system %d" % (pi, k)
        assert info["iterations"] == ita
    st = srv.stats()
    say("   stats", st)
    assert st["completed"] == len(reqs)
    if max_batch > 1:
        assert st["batches"] >= 1 and st["batched_requests"] >= 2
    else:
        assert st["batches"] == 0
    if graphs:
        assert st["graph_launches"] >= 1
    srv.close()


def test_server_repivot_retires_slot(dev):
    # A pattern whose inherited pivots fail on system 2 (D over 26 decades, tau = 0.1): the
    # request re-pivots inside its slot, which the server then retires, so the next request of
    # the pattern runs on a slot with the pattern's own analysis.  Every result equals the
    # standalone refactor + solve of a fresh handle on that analysis, bit for bit, whatever the
    # slot served before.
    say("server re-pivoting pattern")
    tau = 0.1
    p = ks.small_kkt(35000, 25000, 17, (-13.0, 13.0))
    v1, _ = p.system(1)
    order = [2, 3, 2]
    alone = {}
    for k in set(order):
        s = P.Solver(p.rowptr, p.colidx, v1, pivot_tau=tau).bind(dev)
        v, b = p.system(k)
        s.refactor(cuda(v, dev))
        x, info = s.solve(cuda(b, dev))
        assert info["converged"] == 1
        alone[k] = (x.cpu().numpy(), info["repivoted"], info["iterations"])
    assert alone[2][1] == 1
    size = P.Solver(p.rowptr, p.colidx, v1, pivot_tau=tau).workspace_size()
    srv = P.Server(int(size * 1.6 * 3), workers=1, device=dev, max_batch=1, graphs=False)
    pid = srv.add_pattern(p.rowptr, p.colidx, v1, pivot_tau=tau)
    for k in order:
        v, b = p.system(k)
        vv, bb = cuda(v, dev), cuda(b, dev)
        x = torch.empty_like(bb)
        rc, info, _ = srv.wait(srv.submit(pid, vv, bb, x))
        say("   system %d: repivoted %d, iterations %d" % (k, info["repivoted"], info["iterations"]))
        assert rc == P.KKT_OK and info["converged"] == 1 and info["nrbe"] <= 1e-12
        xa, rpa, ita = alone[k]
        assert np.array_equal(x.cpu().numpy(), xa), "system %d" % k
        assert info["repivoted"] == rpa and info["iterations"] == ita
    st = srv.stats()
    say("   stats", st)
    assert st["completed"] == len(order)
    # a new slot for the first request and after every request that re-pivoted
    assert st["slots_created"] == 1 + sum(alone[k][1] for k in order[:-1])
    srv.close()
