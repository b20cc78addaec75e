"""PCG results do not depend on how iterations are queued between host
checks.  The solve's scalars and stopping test live on the device; the x
update of an iteration is applied by its direction kernel, so the
iteration that stops a solve must still apply it, and iterations queued
after the stop must change nothing.  One iteration per host check, the
default batching and 256 iterations per check (most of them queued after
the stop) must give bitwise identical iterates and equal iteration counts;
the first is also checked against the oracle (Sec. 3.1 BE + PCG)."""
import numpy as np
import pytest

from paper_2403_01004_amd import inputs

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01004_amd import paradv
    paradv.load()
    return paradv


CASES = [
    ("conduction", "jacobi", "fp64"),
    ("viscosity", "jacobi", "fp64"),
    ("viscosity", "bilu0", "fp64"),
    ("viscosity", "jacobi", "fp32"),
    ("conduction", "jacobi", "fp32"),
]


@pytest.mark.parametrize("kind,pc,prec", CASES)
def test_batching_invariant(dev, oracle_mod, kind, pc, prec):
    _log("pcg batching", kind, pc, prec)
    if kind == "conduction":
        prob = inputs.conduction(17, 24, 40, seed=31)
    else:
        prob = inputs.viscosity(17, 24, 40, seed=32)
    runs = []
    for batch in (1, 16, 256):
        # a fresh context each time: the first batch of a solve follows the
        # previous solve's count on the context, and a fresh one queues the
        # full batch (mostly after the stop at 256)
        g = dev.Operator.from_problem(prob, prec=prec)
        dt = 50.0 * g.dt_explicit()
        g.set_options(pc=dev.PCS[pc], pcg_batch=batch)
        u = g.bind(prob.u)
        st = g.advance_be(dt, 1e-10, 2)
        runs.append((batch, u.cpu().numpy().copy(), st))
        _log("  batch", batch, "iterations", st["iters_total"], "per cycle", list(st["per_cycle"]))
    u1, s1 = runs[0][1], runs[0][2]
    for batch, ub, sb in runs[1:]:
        assert list(sb["per_cycle"]) == list(s1["per_cycle"]), batch
        assert np.array_equal(ub, u1), (batch, np.abs(ub - u1).max())
    if prec == "fp64":
        o = oracle_mod.Oracle.from_problem(prob)
        if pc == "bilu0":
            o.set_pc("bilu0", (8, 4, 16))
        uo, so = o.advance_be(prob.u, dt, 1e-10, 2)
        rel = np.linalg.norm(u1 - uo) / np.linalg.norm(uo)
        _log("  oracle rel", rel, "iterations", list(so["per_cycle"]))
        # two equal cycles on both sides; the stopping test may fall either
        # side of the tolerance within rounding in a cycle (one iteration
        # more or less), and both iterates then meet it
        if list(so["per_cycle"]) == list(s1["per_cycle"]):
            assert rel <= 1e-12
        else:
            assert rel <= 1e-7
