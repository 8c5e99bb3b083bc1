"""kkt_direct_solve_noalloc (the direct solve for callers that cannot allocate) against
kkt_direct_solve through the C ABI: the same kernels on the same factors, so the same bits.
Two handles in a row, the second smaller, then FP32 factors: the static scratch keeps the
previous call's contents, and each call must re-arm what it reads."""
import sys

import numpy as np
import pytest

import kkt_synth as ks

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2401_13926_amd as P  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def test_direct_solve_noalloc_matches_direct_solve(dev):
    cases = [(ks.make_pattern(2), P.PREC_FP64), (ks.make_pattern(1), P.PREC_FP64),
             (ks.small_kkt(600, 400, 7), P.PREC_MIXED)]
    for p, prec in cases:
        print("no-alloc direct solve N =", p.N, "precision", prec, flush=True)
        sys.stdout.flush()
        v1, _ = p.system(1)
        v, b = p.system(2)
        s = P.Solver(p.rowptr, p.colidx, v1, precision=prec).bind(dev)
        s.refactor(torch.as_tensor(v, device=dev))
        bb = torch.as_tensor(b, device=dev)
        xr = s.direct_solve(bb)
        for _ in range(2):
            xn = torch.full_like(bb, float("nan"))
            s.direct_solve_noalloc(bb, xn)
            torch.cuda.synchronize()
            assert torch.equal(xr, xn)
        assert np.isfinite(xr.cpu().numpy()).all()
