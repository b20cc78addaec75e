"""Per-class kernel timing (the `timing` option) observes and changes
nothing: RKL2 and Backward Euler advances give bitwise identical fields and
statistics with it on and off, and with it on every queued launch of a
class is counted (the PCG classes once per queued iteration, the direction
class also once per group x update)."""
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


@pytest.mark.parametrize("kind", ["conduction", "viscosity"])
def test_timing_changes_nothing(dev, kind):
    _log("timing on/off", kind)
    if kind == "conduction":
        prob = inputs.conduction(17, 24, 40, seed=41)
    else:
        prob = inputs.viscosity(17, 24, 40, seed=42)
    out = {}
    for timing in (0, 1):
        g = dev.Operator.from_problem(prob)
        dt = 50.0 * g.dt_explicit()
        g.set_options(timing=timing)
        u = g.bind(prob.u)
        sr = g.advance_rkl2(dt, 0)
        ur = u.cpu().numpy().copy()
        u = g.bind(prob.u)
        sb = g.advance_be(dt, 1e-10, 0)
        out[timing] = (ur, u.cpu().numpy().copy(), sr, sb)
    (ur0, ub0, sr0, sb0), (ur1, ub1, sr1, sb1) = out[0], out[1]
    assert np.array_equal(ur0, ur1) and np.array_equal(ub0, ub1)
    for a, b in ((sr0, sr1), (sb0, sb1)):
        for key in ("cycles", "s_total", "iters_total"):
            assert a[key] == b[key], key
        assert list(a["per_cycle"]) == list(b["per_cycle"])
        assert all(v == 0 for v in a["kernel_ms"].values())
    # timed: the classes that ran were counted and took time
    assert sr1["kernel_calls"]["stage"] > 0 and sr1["kernel_ms"]["stage"] > 0
    assert sr1["kernel_calls"]["first"] >= sr1["cycles"]
    mv = sb1["kernel_calls"]["matvec"]
    assert mv >= sb1["iters_total"] > 0
    assert sb1["kernel_calls"]["update"] == mv
    # the direction class: one launch per queued iteration, plus the x update
    # of every group of PA_PCG_XGROUP queued iterations and of each solve's
    # last, incomplete group
    assert mv <= sb1["kernel_calls"]["dir"] <= mv + mv // dev.PA_PCG_XGROUP + sb1["cycles"]
    assert all(sb1["kernel_ms"][c] > 0 for c in ("matvec", "update", "dir", "reduce"))
    _log("  iterations", sb1["iters_total"], "queued", mv)
