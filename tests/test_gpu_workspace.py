"""Single-signal calls on a caller-provided workspace (cs_set_workspace):
the same results as on library memory, and a block that is too small is
rejected before anything is enqueued."""
import numpy as np
import pytest

import workloads
from oracle import dense, problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("no GPU", allow_module_level=True)

import paper_1707_02244_amd as cs  # noqa: E402

DEV = torch.device("cuda:0")


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def h(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_solves_on_caller_workspace_match_library_memory():
    pr = problem.build(workloads.parity_signal())
    big = problem.build(workloads.signal(1 << 16, 4, 64, 5))
    need = max(cs.workspace_bytes(pr.n, pr.d, 1), cs.workspace_bytes(big.n, big.d, 2))
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    ref = {}
    for p in (pr, big):
        c, y = g(p.c), g(p.y)
        ref[p.n] = (h(cs.ista_solve(c, p.d, y, p.lam, p.tau, 40)),
                    [h(v) for v in cs.admm_solve(c, p.d, y, p.lam, 1.0, 30)],
                    h(cs.circ_apply(c, p.d, g(p.x_true))))
    cs.set_workspace(ws)
    try:
        # alternate sizes so the block's twiddle tables are rewritten
        for p in (pr, big, pr):
            c, y = g(p.c), g(p.y)
            xi = h(cs.ista_solve(c, p.d, y, p.lam, p.tau, 40))
            xa = [h(v) for v in cs.admm_solve(c, p.d, y, p.lam, 1.0, 30)]
            ya = h(cs.circ_apply(c, p.d, g(p.x_true)))
            ri, ra, ry = ref[p.n]
            assert rel(xi, ri) <= 1e-6 and all(rel(a, b) <= 1e-6 for a, b in zip(xa, ra))
            assert rel(ya, ry) <= 1e-6
        cs.check_device()
        # the oracle on the small case
        xo = dense.ista(pr.A(), pr.y.astype(np.float64), float(pr.lam), float(pr.tau), 40)
        assert rel(h(cs.ista_solve(g(pr.c), pr.d, g(pr.y), pr.lam, pr.tau, 40)), xo) <= 1e-4
        # a block too small for n = 2^17 is rejected, nothing enqueued
        x = torch.zeros(1 << 17, device=DEV)
        with pytest.raises(cs.CsError, match="too small"):
            cs.ista_solve(g(np.ones(1 << 17)), 4, g(np.ones(1 << 15)), 0.1, 0.1, 5, x=x)
        assert float(x.abs().max()) == 0.0
    finally:
        cs.set_workspace(None)
    torch.cuda.synchronize()
