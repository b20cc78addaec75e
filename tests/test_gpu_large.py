"""The largest workload, 256 x 512 x 1024 (134 M cells, 1.07 GB per FP64
field): transition-region conduction (T jump at i_tr = 20 + 4 S(501)) and
three-component viscosity as on the 151 x 301 x 400 grid.

Whole-field comparisons with the oracle: the operator (element-wise),
Dt_E, the practical time step limit, one RKL2 cycle (1e-12), and the FP64
true residual of a Backward Euler solve evaluated with the oracle's
operator.  Launch shapes are the ones the advances use at this size
(several radial chunks, 33 x 64 tile planes, more than 2^31 bytes per
array), the block ILU(0) preconditioner's apply and BE solve on the
three-component field (262144 boxes, fields of 3.2 GB), and twenty
consecutive advances with the diffusivity re-lagged before each one (FP32
stages against FP64 on the same schedules)."""
import numpy as np
import pytest

from paper_2403_01004_amd import inputs

# building the 134 M-cell inputs and the oracle's passes take minutes on the host
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SHAPE = (256, 512, 1024)


def _log(*a):
    print(*a, flush=True)


def rel_l2(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01004_amd import paradv
    paradv.load()
    return paradv


@pytest.fixture(scope="module")
def cond5():
    _log("building 256x512x1024 transition-region conduction")
    return inputs.transition_region(*SHAPE, seed=501, i_tr0=20.0, i_amp=4.0)


def test_large_conduction(dev, oracle_mod, cond5):
    prob = cond5
    g = dev.Operator.from_problem(prob)
    o = oracle_mod.Oracle.from_problem(prob)
    _log("large conduction: apply")
    Fg = g.apply(prob.u).cpu().numpy()
    Fo = o.apply(prob.u)
    assert np.abs(Fg - Fo).max() <= 1e-13 * np.abs(Fo).max()
    del Fg, Fo
    dtE = o.dt_explicit()
    assert abs(g.dt_explicit() - dtE) <= 1e-13 * dtE
    g.bind(prob.u)
    pg, po = g.ptl(), o.ptl(prob.u)
    assert pg[1] == po[1] and abs(pg[0] - po[0]) <= 1e-12 * abs(po[0])
    _log("large conduction: one RKL2 cycle, s = 5")
    dt = 6.0 * dtE
    u = g.bind(prob.u)
    st = g.advance_rkl2(dt, 1)
    uo, so = o.advance_sts(prob.u, dt, 1, "rkl2")
    assert st["s_total"] == so["s_total"] == 5
    assert rel_l2(u.cpu().numpy(), uo) <= 1e-12


def test_large_conduction_be_true_residual(dev, oracle_mod, cond5):
    prob = cond5
    g = dev.Operator.from_problem(prob)
    o = oracle_mod.Oracle.from_problem(prob)
    dt = 50.0 * g.dt_explicit()
    _log("large conduction: BE solve")
    u = g.bind(prob.u)
    st = g.advance_be(dt, 1e-10, 1)
    x = u.cpu().numpy()
    _log("  iterations", st["iters_total"])
    V = o.volumes()[None]
    b = V * prob.u + dt * V * o.apply(np.zeros_like(prob.u))
    Mx = V * x - dt * V * o.apply(x, affine=False)
    res = np.linalg.norm(b - Mx) / np.linalg.norm(b)
    _log("  true residual", res)
    assert res <= 1.001e-10


def test_large_viscosity_apply(dev, oracle_mod):
    """Three-component constant-coefficient operator on an N(0,1) field (a
    stricter operand than the smooth recipe, and cheap to build at this size)."""
    _log("building 256x512x1024 x 3 random field")
    mesh = inputs.shell_mesh(*SHAPE)
    rng = np.random.default_rng(505)
    u = rng.standard_normal((3,) + SHAPE)
    ub = rng.standard_normal((3, SHAPE[1], SHAPE[2]))
    prob = inputs.Problem(mesh, "iso7", 3, u, ub, -ub, None, 1e-3, 0.0, None, name="visc_large")
    g = dev.Operator.from_problem(prob)
    o = oracle_mod.Oracle.from_problem(prob)
    for affine in (True, False):
        Fg = g.apply(prob.u, affine).cpu().numpy()
        Fo = o.apply(prob.u, affine)
        assert np.abs(Fg - Fo).max() <= 1e-13 * np.abs(Fo).max()
    assert abs(g.dt_explicit() - o.dt_explicit()) <= 1e-13 * o.dt_explicit()


def test_large_bilu0(dev, oracle_mod):
    """Block ILU(0) (PC2) on the three-component 7-point operator at this size:
    the preconditioner element-wise against the oracle's, and a BE solve
    whose FP64 true residual, evaluated with the oracle's operator, meets
    the tolerance."""
    _log("building 256x512x1024 x 3 random field")
    mesh = inputs.shell_mesh(*SHAPE)
    rng = np.random.default_rng(506)
    u = rng.standard_normal((3,) + SHAPE)
    ub = rng.standard_normal((3, SHAPE[1], SHAPE[2]))
    prob = inputs.Problem(mesh, "iso7", 3, u, ub, -ub, None, 1e-3, 0.0, None, name="visc_large")
    g = dev.Operator.from_problem(prob)
    g.set_options(pc=dev.PCS["bilu0"])
    o = oracle_mod.Oracle.from_problem(prob)
    o.set_pc("bilu0", (8, 4, 16))
    dt = 5.0 * o.dt_explicit()
    _log("large bilu0: apply")
    zg = g.bilu0_apply(u, dt).cpu().numpy()
    zo = o.precondition(u, dt)
    assert np.abs(zg - zo).max() <= 1e-13 * np.abs(zo).max()
    del zg, zo
    _log("large bilu0: BE solve")
    x = g.bind(u)
    st = g.advance_be(dt, 1e-10, 1)
    _log("  iterations", st["iters_total"])
    V = o.volumes()[None]
    b = V * u + dt * V * o.apply(np.zeros_like(u))
    xh = x.cpu().numpy()
    Mx = V * xh - dt * V * o.apply(xh, affine=False)
    res = np.linalg.norm(b - Mx) / np.linalg.norm(b)
    _log("  true residual", res)
    assert res <= 1.001e-10


def test_large_sequence_fp32_stages(dev, oracle_mod, cond5):
    """Twenty PTL-cycled RKL2 advances of the 256x512x1024 transition-region
    conduction with the diffusivity re-lagged from the current field before
    each advance and the time step fixed from the first (50 dt_E): FP32
    stages against the FP64 path (which matches the oracle at this size) on
    the same cycle schedules, then one Backward Euler advance of the FP64
    field whose FP64 true residual, with the oracle's operator, meets the
    tolerance."""
    torch = pytest.importorskip("torch")
    prob = cond5
    g64 = dev.Operator.from_problem(prob)
    g32 = dev.Operator.from_problem(prob, prec="fp32")
    dt = 50.0 * g64.dt_explicit()
    u64 = g64.bind(prob.u)
    u32 = g32.bind(prob.u)
    for adv in range(20):
        if adv > 0:
            g64.set_coefficients(u64[0], prob.scale, prob.expo, prob.B)
            g32.set_coefficients(u32[0], prob.scale, prob.expo, prob.B)
        st = g64.advance_rkl2(dt, 0)
        g32.set_options(replay=np.asarray(st["dt_cycle"]))
        s32 = g32.advance_rkl2(dt, 0)
        g32.set_options()
        assert s32["cycles"] == st["cycles"] and s32["s_total"] == st["s_total"]
        assert bool(torch.isfinite(u64).all()) and bool(torch.isfinite(u32).all())
        if adv % 5 == 4:
            _log("large sequence: advance", adv + 1, "cycles", st["cycles"],
                 "fp32 rel err", float(torch.linalg.vector_norm(u32 - u64) /
                                       torch.linalg.vector_norm(u64)))
    err = float(torch.linalg.vector_norm(u32 - u64) / torch.linalg.vector_norm(u64))
    assert err <= 1e-5, err
    del g32, u32
    _log("large sequence: BE advance of the relaxed field")
    g64.set_coefficients(u64[0], prob.scale, prob.expo, prob.B)
    un = u64.cpu().numpy()
    st = g64.advance_be(dt, 1e-10, 1)
    x = u64.cpu().numpy()
    o = oracle_mod.Oracle.from_problem(prob)
    o.set_coefficients(un[0], prob.scale, prob.expo, prob.B)
    V = o.volumes()[None]
    b = V * un + dt * V * o.apply(np.zeros_like(un))
    Mx = V * x - dt * V * o.apply(x, affine=False)
    res = np.linalg.norm(b - Mx) / np.linalg.norm(b)
    _log("  iterations", st["iters_total"], "true residual", res)
    assert res <= 1.001e-10


def test_large_first_two_advances(dev, oracle_mod, cond5):
    """The first two advances of the 256x512x1024 sequence against the
    oracle, bounded to one RKL2 cycle each (s = 5 at dt = 6 dt_E) so that the
    oracle finishes in about a minute: conduction with the diffusivity
    re-lagged from the advanced temperature before the second advance, FP64
    (1e-12) and FP32 stages (1e-5) after each advance."""
    torch = pytest.importorskip("torch")
    prob = cond5
    o = oracle_mod.Oracle.from_problem(prob)
    g64 = dev.Operator.from_problem(prob)
    g32 = dev.Operator.from_problem(prob, prec="fp32")
    dt = 6.0 * o.dt_explicit()
    u64, u32 = g64.bind(prob.u), g32.bind(prob.u)
    uo = prob.u
    Bd = torch.as_tensor(prob.B, device=u64.device)
    for adv in range(2):
        if adv:
            _log("large first advances: re-lag the diffusivity")
            # each side from its own advanced temperature
            o.set_coefficients(uo[0], prob.scale, prob.expo, prob.B)
            g64.set_coefficients(u64[0].clone(), prob.scale, prob.expo, Bd)
            g32.set_coefficients(u32[0].clone(), prob.scale, prob.expo, Bd)
        _log("large first advances: advance", adv + 1)
        s64 = g64.advance_rkl2(dt, 1)
        g32.advance_rkl2(dt, 1)
        uo, so = o.advance_sts(uo, dt, 1, "rkl2")
        assert s64["s_total"] == so["s_total"] == 5
        e64 = rel_l2(u64.cpu().numpy(), uo)
        e32 = rel_l2(u32.cpu().numpy(), uo)
        _log("  rel L2 fp64", e64, "fp32", e32)
        assert e64 <= 1e-12 and e32 <= 1e-5


def test_large_vector_viscosity_first_two_advances(dev, oracle_mod):
    """The vector viscosity at 256x512x1024 (fields built on the GPU with the
    recipe's waves): two one-cycle RKL2 advances (s = 5) against the oracle,
    FP64 (1e-12) and FP32 stages (1e-5)."""
    torch = pytest.importorskip("torch")
    _log("building 256x512x1024 vector viscosity")
    pd = inputs.viscosity_device(*SHAPE, torch, "cuda")
    prob = inputs.Problem(pd.mesh, "viscv", 3, pd.u.cpu().numpy(), pd.ub_in.cpu().numpy(),
                          pd.ub_out.cpu().numpy(), None, pd.scale, 0.0, None, name=pd.name)
    del pd
    o = oracle_mod.Oracle.from_problem(prob)
    g64 = dev.Operator.from_problem(prob)
    g32 = dev.Operator.from_problem(prob, prec="fp32")
    dt = 6.0 * o.dt_explicit()
    u64, u32 = g64.bind(prob.u), g32.bind(prob.u)
    uo = prob.u
    for adv in range(2):
        _log("large vector viscosity: advance", adv + 1)
        s64 = g64.advance_rkl2(dt, 1)
        g32.advance_rkl2(dt, 1)
        uo, so = o.advance_sts(uo, dt, 1, "rkl2")
        assert s64["s_total"] == so["s_total"] == 5
        e64 = rel_l2(u64.cpu().numpy(), uo)
        e32 = max(rel_l2(u32[c].cpu().numpy(), uo[c]) for c in range(3))
        _log("  rel L2 fp64", e64, "fp32 (worst component)", e32)
        assert e64 <= 1e-12 and e32 <= 1e-5
