"""The four PTL-cycled advances of the 151 x 301 x 400 benchmark step, run
exactly as the benchmark runs them (default options, dt = 50 dt_E of each
operator, tol 1e-10; the viscosity in its vector form), against the oracle
on the same inputs; the same advances with FP32 stages / FP32 matvecs
against the oracle's FP64 result; and the benchmark's unfloored RKL2 leg.

Bars:
* STS (Sec. 3.1, App. A): identical cycle schedules (every cycle length to
  1e-12, stages per cycle equal) and relative L2 error <= 1e-12.
* Backward Euler + Jacobi PCG (Sec. 3.1): identical cycle schedules and
  PCG iterations per cycle; the FP64 true residual of the GPU result,
  evaluated with the oracle's operator, meets the tolerance; and the two
  fields agree to BE_DRIFT = 1e-12.  With equal decisions both sides
  execute the same iterations, so the difference is the rounding drift of
  the dot products over the 104 (conduction) and 184 (viscosity)
  iterations: measured on the MI355X 2.3e-16 and 4.4e-16.
* Where the schedules part, every differing decision must be a genuine
  near-tie: the first differing cycle count's argument t_rem / max(dt_PTL,
  dt_E), evaluated by the oracle on its field at that cycle's start, within
  1e-12 of an integer; a differing stage count's argument (sqrt(9 + 16
  dt_c/dt_E) - 1)/2 within 1e-12 of an integer; a differing iteration count
  with the oracle's residual at the earlier count within 1e-12 of tol.  (At
  dt = 50 dt_E with the limit floored to dt_E the arguments are 50, and 13
  for a last cycle of 45 dt_E, up to the last bits of each side's own dt_E.)
  The oracle then follows the GPU's decisions cycle by cycle and the bars
  above apply to that run.
* FP32 stages / FP32-matvec BE (mixed precision): per component
  relative L2 error against the oracle's FP64 result <= 1e-5.

The oracle's results are computed once per module and shared by the FP64
and FP32 tests.
"""
import math

import numpy as np
import pytest

from paper_2403_01004_amd import inputs

# the oracle's full-size advances take one to two minutes each on the host
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL = 1e-10
BE_DRIFT = 1e-12
FP32_REL = 1e-5


def _log(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01004_amd import paradv
    paradv.load()
    return paradv


@pytest.fixture(scope="module")
def probs():
    _log("building 151x301x400 conduction and viscosity inputs")
    return {"conduction": inputs.conduction(), "viscosity": inputs.viscosity(vector=True)}


class OracleRuns:
    """The oracle's advances of the benchmark step, computed on first use."""

    def __init__(self, oracle_mod, probs):
        self.om = oracle_mod
        self.probs = probs
        self.ops = {}
        self.res = {}

    def oracle(self, name):
        if name not in self.ops:
            self.ops[name] = self.om.Oracle.from_problem(self.probs[name])
        return self.ops[name]

    def run(self, name, kind, dt):
        key = (name, kind)
        if key not in self.res:
            o = self.oracle(name)
            u = self.probs[name].u
            _log(f"oracle: {kind} {name}")
            if kind in ("rkl2", "rkg2"):
                self.res[key] = o.advance_sts(u, dt, 0, kind)
            else:
                self.res[key] = o.advance_be(u, dt, TOL, 0)
        return self.res[key]


@pytest.fixture(scope="module")
def oruns(oracle_mod, probs):
    return OracleRuns(oracle_mod, probs)


def first_split(st, so):
    dg, do = np.asarray(st["dt_cycle"]), np.asarray(so["dt_cycle"])
    for c in range(min(len(dg), len(do))):
        if abs(dg[c] - do[c]) > 1e-12 * do[c]:
            return c
    return min(len(dg), len(do))


def parted_on_near_tie(o, kind, u0, st, so, dt):
    """The cycle-count decision where the schedules part, on the oracle's
    field at that cycle's start: (argument of the ceiling, is near-tie)."""
    c0 = first_split(st, so)
    dg = np.asarray(st["dt_cycle"])
    u = u0
    if c0:
        pre = dg[:c0]
        u, _ = (o.advance_sts(u0, pre.sum(), 0, kind, replay=pre) if kind != "be"
                else o.advance_be(u0, pre.sum(), TOL, 0, replay=pre))
    t_rem = dt - dg[:c0].sum()
    x = t_rem / max(o.ptl(u)[0], o.dt_explicit())
    return x, abs(x - round(x)) <= 1e-12 * x


def follow_gpu(om, o, kind, u0, st):
    """The oracle taking the GPU's decisions cycle by cycle (its cycle
    lengths, and its stage or iteration count per cycle).  Each count that
    differs from the oracle's own must be a genuine near-tie: the stage
    formula giving the GPU's count for dt_c/dt_E moved by 1e-12 relative
    (for RKL2 its ceiling argument (sqrt(9 + 16 dt_c/dt_E) - 1)/2 within
    1e-12 of an integer), or the oracle's residual at the earlier stopping
    count within 1e-12 of tol (both sides' residuals agree to ~1e-15 of
    ||b||)."""
    dtE = o.dt_explicit()
    u, flips = u0, 0
    for dtc, n in zip(np.asarray(st["dt_cycle"]), np.asarray(st["per_cycle"])):
        n = int(n)
        if kind != "be":
            own = om.sts_stages(kind, dtc / dtE)
            if own != n:
                near = {om.sts_stages(kind, dtc / dtE * (1.0 + e)) for e in (-1e-12, 1e-12)}
                _log(f"  stage count {n} against the oracle's {own} (counts within 1e-12: {near})")
                assert n in near, (n, own, dtc / dtE)
                flips += 1
            u, _ = o.advance_sts(u, dtc, 1, kind, s_override=n)
        else:
            uf, sf = o.advance_be(u, dtc, TOL, 1)
            if sf["iters_total"] == n:
                u = uf
                continue
            ug, sg = o.advance_be(u, dtc, TOL, 1, force_iters=n)
            early = sg["rel_residual"] if n < sf["iters_total"] else sf["rel_residual"]
            _log(f"  iterations {n} against the oracle's {sf['iters_total']}: residual {early!r}")
            assert abs(sf["iters_total"] - n) == 1 and abs(early - TOL) <= 1e-12, early
            u, flips = ug, flips + 1
    return u, flips


def oracle_for(oruns, name, kind, st, so, dt):
    """The oracle's advance to compare with: its own when the schedules
    agree; else, after the near-tie checks, the oracle following the GPU's
    decisions."""
    if same_schedule(st, so):
        return oruns.run(name, kind, dt)
    o, u0 = oruns.oracle(name), oruns.probs[name].u
    if first_split(st, so) < max(len(st["dt_cycle"]), len(so["dt_cycle"])):
        x, tie = parted_on_near_tie(o, kind, u0, st, so, dt)
        _log(f"{kind} {name}: schedules part at a cycle-count decision with argument {x!r}")
        assert tie, (x, list(st["dt_cycle"]), list(so["dt_cycle"]))
    u, flips = follow_gpu(oruns.om, o, kind, u0, st)
    assert flips <= 3
    return u, st


def same_schedule(st, so):
    dg, do = np.asarray(st["dt_cycle"]), np.asarray(so["dt_cycle"])
    return (st["cycles"] == so["cycles"] and len(dg) == len(do)
            and np.all(np.abs(dg - do) <= 1e-12 * do)
            and list(st["per_cycle"]) == list(so["per_cycle"]))


def be_true_residual(o, u0, x, dt):
    """||b - M x|| / ||b|| with the oracle's operator (M = V + dt L,
    b = V u^n + dt V F(0))."""
    V = o.volumes()[None]
    b = V * u0 + dt * V * o.apply(np.zeros_like(u0))
    Mx = V * x - dt * V * o.apply(x, affine=False)
    return np.linalg.norm(b - Mx) / np.linalg.norm(b)


def gpu_advance(dev, prob, kind, prec="fp64"):
    g = dev.Operator.from_problem(prob, prec=prec)
    dt = 50.0 * g.dt_explicit()
    u = g.bind(prob.u)
    st = g.advance_sts(dt, 0, sts=kind) if kind != "be" else g.advance_be(dt, TOL, 0)
    out = u.cpu().numpy()
    del g, u
    return out, st, dt


@pytest.mark.parametrize("kind", ["rkl2", "rkg2"])
@pytest.mark.parametrize("name", ["conduction", "viscosity"])
def test_sts_ptl_cycled(dev, probs, oruns, name, kind):
    """RKL2 (the timed step) and RKG2 (the benchmark's RKG2-against-BE leg)."""
    prob = probs[name]
    ug, st, dt = gpu_advance(dev, prob, kind)
    uo, so = oruns.run(name, kind, dt)
    _log(f"{kind} {name}: cycles {st['cycles']}/{so['cycles']}, stages {st['s_total']}/{so['s_total']}")
    uo, so = oracle_for(oruns, name, kind, st, so, dt)
    err = rel_l2(ug, uo)
    _log(f"{kind} {name}: rel L2 {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("name", ["conduction", "viscosity"])
def test_rkl2_unfloored(dev, oracle_mod, probs, oruns, name):
    """The benchmark's unfloored leg: RKL2 cycled at the paper's limit
    without the floor of dt_E (ptl_floor = 0), as bench.py runs it, against
    the oracle replaying the GPU's schedule (every cycle length the oracle's
    own decision to 1e-12, except where the limit is ill-conditioned: a
    flattened limiting pair), no cycle floored, fields to 1e-12."""
    from ptl_follow import replay_unfloored
    prob = probs[name]
    g = dev.Operator.from_problem(prob)
    dt = 50.0 * g.dt_explicit()
    g.set_options(ptl_floor=0.0, max_cycles=20000)
    u = g.bind(prob.u)
    st = g.advance_rkl2(dt, 0)
    ug = u.cpu().numpy()
    del g, u
    _log(f"unfloored rkl2 {name}: cycles {st['cycles']}, stages {st['s_total']}")
    assert st["floored"] == 0
    uo, ill = replay_unfloored(oracle_mod, oruns.oracle(name), prob.u, dt, st, log=_log)
    _log(f"unfloored rkl2 {name}: ill-conditioned cycles {ill}")
    err = rel_l2(ug, uo)
    _log(f"unfloored rkl2 {name}: rel L2 {err:.3e}")
    assert err <= 1e-12


@pytest.mark.parametrize("name", ["conduction", "viscosity"])
def test_be_ptl_cycled(dev, probs, oruns, name):
    prob = probs[name]
    ug, st, dt = gpu_advance(dev, prob, "be")
    uo, so = oruns.run(name, "be", dt)
    _log(f"be {name}: cycles {st['cycles']}/{so['cycles']}, "
         f"iterations {st['iters_total']}/{so['iters_total']}")
    assert st["status"] == 0 and so["status"] == 0
    uo, so = oracle_for(oruns, name, "be", st, so, dt)
    err = rel_l2(ug, uo)
    _log(f"be {name}: rel L2 {err:.3e}")
    assert err <= BE_DRIFT
    # the last cycle's system, with the oracle's operator: its right-hand
    # side is the GPU's field before that cycle, which the GPU reproduces
    # by replaying its own schedule without the last cycle
    dts = np.asarray(st["dt_cycle"])
    if len(dts) > 1:
        g = dev.Operator.from_problem(prob)
        g.set_options(replay=dts[:-1])
        u = g.bind(prob.u)
        s2 = g.advance_be(float(dts[:-1].sum()), TOL, 0)
        assert list(s2["per_cycle"]) == list(st["per_cycle"][:-1])
        un = u.cpu().numpy()
        del g, u
    else:
        un = prob.u
    res = be_true_residual(oruns.oracle(name), un, ug, dts[-1])
    _log(f"be {name}: true residual of the last cycle {res:.3e}")
    assert res <= 1.001 * TOL


def follow_fp32(o, kind, u0, st):
    """The oracle (FP64) taking the FP32 path's cycle lengths and per-cycle
    stage counts (RKL2) or cycle lengths (BE, solved to the same tolerance):
    the FP32 path takes its decisions from its own FP32 F."""
    u = u0
    for dtc, n in zip(np.asarray(st["dt_cycle"]), np.asarray(st["per_cycle"])):
        u, _ = (o.advance_sts(u, dtc, 1, "rkl2", s_override=int(n)) if kind == "rkl2"
                else o.advance_be(u, dtc, TOL, 1))
    return u


@pytest.mark.parametrize("name", ["conduction", "viscosity"])
@pytest.mark.parametrize("kind", ["rkl2", "be"])
def test_fp32_against_oracle(dev, probs, oruns, name, kind):
    """FP32 stencil and stages (RKL2) or FP32 matvecs inside the FP64 defect
    correction (BE) against the oracle's FP64 advance.  The FP32 path takes
    its own cycle decisions from its FP32 F; where they part from the
    oracle's, the oracle follows them."""
    prob = probs[name]
    ug, st, dt = gpu_advance(dev, prob, kind, prec="fp32")
    uo, so = oruns.run(name, kind, dt)
    if not same_schedule(st, so):
        _log(f"fp32 {kind} {name}: decisions part from the oracle's; following them")
        uo = follow_fp32(oruns.oracle(name), kind, prob.u, st)
    errs = [rel_l2(ug[c], uo[c]) for c in range(prob.ncomp)]
    _log(f"fp32 {kind} {name}: cycles {st['cycles']}, rel L2 per component "
         + ", ".join(f"{e:.2e}" for e in errs))
    assert max(errs) <= FP32_REL
