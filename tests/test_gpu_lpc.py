"""Learned preconditioner on the GPU against the oracle (oracle/lpc.py) and
against the method without it.

* input channels: equal to the oracle's (brute-force face couplings,
  rounded to BF16) except for rare one-ulp rounding flips;
* network output and the energy-norm loss gradient: the oracle emulating
  the BF16 roundings, forward <= 1e-3 relative, gradient <= 5e-3 relative
  L2, with two pairs in one batched launch;
* FCG(1) with a zero network reproduces Jacobi PCG;
* training is deterministic and lowers the loss; on a held-out problem the
  trained network's step estimates the error far better than the Jacobi
  step, and the solve that uses it reaches the same true residual;
  corrupted weights still converge through the fallbacks.
"""
import numpy as np
import pytest

from oracle import lpc
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


def rel_l2(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300)


def setup(dev, oracle_mod, op, shape, seed, bc="dirichlet"):
    nr, nt, np_ = shape
    if op == "aligned":
        prob = inputs.conduction(nr, nt, np_, seed=seed, noise_amp=0.02)
    else:
        prob = inputs.heat_iso(nr, nt, np_, seed=seed)
    prob.bc_in = prob.bc_out = bc
    g = dev.Operator.from_problem(prob)
    o = oracle_mod.Oracle.from_problem(prob)
    V = o.volumes()
    dt = 40.0 * o.dt_explicit()
    D = V + dt * o.diag()
    cpl = lpc.face_couplings(lambda x: o.apply(x[None], affine=False)[0], V)
    return prob, g, o, V, dt, D, cpl


def true_residual(o, prob, x, dt):
    V = o.volumes()[None]
    b = V * prob.u + dt * V * o.apply(np.zeros_like(prob.u))
    Mx = V * x - dt * V * o.apply(x, affine=False)
    return np.linalg.norm(b - Mx) / np.linalg.norm(b)


@pytest.mark.parametrize("op,shape", [("iso7", (5, 6, 9)), ("aligned", (6, 8, 13))])
def test_features_match_oracle(dev, oracle_mod, op, shape):
    _log("features", op, shape)
    prob, g, o, V, dt, D, cpl = setup(dev, oracle_mod, op, shape, 31)
    r = inputs.random_field(shape, 5)
    fg = g.lpc_features(dt, r).cpu().numpy().astype(np.float64)
    fo = lpc.bf16(lpc.features(r, D, V, cpl, dt))
    diff = np.abs(fg - fo)
    flips = diff > 0
    # a flip is one BF16 ulp (relative 2^-8) of a value on a rounding boundary
    assert (diff <= 2.0 ** -7 * np.abs(fo) + 1e-30).all()
    assert flips.mean() < 2e-3, flips.mean()
    assert np.abs(fo[2:]).max() > 0


def _theta(seed, bias=0.05):
    th = lpc.he_init(np.random.default_rng(seed))
    rng = np.random.default_rng(seed + 1)
    th[3456:3472] = bias * rng.standard_normal(16)
    th[10384:10400] = bias * rng.standard_normal(16)
    return th.astype(np.float32)


@pytest.mark.parametrize("op,shape", [("iso7", (5, 6, 9)), ("aligned", (6, 8, 13)),
                                      ("aligned", (3, 17, 40))])
def test_apply_matches_oracle(dev, oracle_mod, op, shape):
    _log("lpc apply", op, shape)
    prob, g, o, V, dt, D, cpl = setup(dev, oracle_mod, op, shape, 37)
    th = _theta(41)
    g.lpc_set_weights(th)
    assert np.array_equal(g.lpc_get_weights(), th)
    r = inputs.random_field(shape, 6)
    z = g.lpc_apply(dt, r).cpu().numpy()
    static = lpc.features(r, D, V, cpl, dt)[1:]
    zo = lpc.precondition(th.astype(np.float64), r, D, static, bf16_mode=True)
    zj = r / D
    sigma = np.sqrt(np.mean(zj * zj))
    # compare the network part sigma N(c), whose scale is that of r/D
    assert rel_l2(z - zj, zo - zj) <= 1e-3
    # positive homogeneity
    z2 = g.lpc_apply(dt, 4.0 * r).cpu().numpy()
    assert rel_l2(z2, 4.0 * z) <= 1e-12
    _ = sigma


@pytest.mark.parametrize("op,shape", [("iso7", (5, 6, 9)), ("aligned", (4, 9, 20)),
                                      ("aligned", (3, 17, 40))])
def test_loss_grad_matches_oracle(dev, oracle_mod, op, shape):
    """Energy-norm loss and gradient over two pairs in one batched launch."""
    _log("lpc grad", op, shape)
    prob, g, o, V, dt, D, cpl = setup(dev, oracle_mod, op, shape, 43)
    th = _theta(47)
    g.lpc_set_weights(th)
    pairs = [(inputs.random_field(shape, 50 + i), inputs.random_field(shape, 60 + i))
             for i in range(2)]
    r = np.stack([p[0] for p in pairs])
    e = np.stack([p[1] for p in pairs])
    loss, grad = g.lpc_loss_grad(dt, r, e)
    static = lpc.features(pairs[0][0], D, V, cpl, dt)[1:]

    def matvec(v):
        return V * v - dt * V * o.apply(v[None], affine=False)[0]

    lo, go = lpc.loss_and_grad(th.astype(np.float64), pairs, D, static, matvec, bf16_mode=True)
    _log("  loss", loss, lo, "grad rel", rel_l2(grad, go))
    assert abs(loss - lo) <= 1e-3 * abs(lo)
    assert rel_l2(grad, go) <= 5e-3
    for name, sl in (("W1", slice(0, 3456)), ("b1", slice(3456, 3472)),
                     ("W2", slice(3472, 10384)), ("b2", slice(10384, 10400)),
                     ("W3", slice(10400, 10832))):
        assert rel_l2(grad[sl], go[sl]) <= 2e-2, name


@pytest.mark.parametrize("op,shape", [("iso7", (9, 10, 13)), ("aligned", (10, 16, 24))])
def test_fcg_zero_network_is_pcg(dev, oracle_mod, op, shape):
    """With N == 0 the preconditioner is Jacobi and FCG(1) is PCG: the first
    10 iterates agree (the hand-over rule first looks at iteration 10), and
    the full solve reaches the tolerance in about as many iterations."""
    _log("fcg zero", op, shape)
    prob, g, o, V, dt, D, cpl = setup(dev, oracle_mod, op, shape, 53)
    u0 = prob.u.copy()
    g.set_options(force_iters=10)
    g.bind(u0)
    g.advance_be(dt, 1e-10, 1)
    x10j = g.field.cpu().numpy()
    g.lpc_set_weights(np.zeros(dev.PA_LPC_NPARAM, np.float32))
    g.set_options(pc=dev.PCS["learned"], force_iters=10)
    g.bind(u0)
    s10 = g.advance_be(dt, 1e-10, 1)
    x10l = g.field.cpu().numpy()
    assert s10["iters_total"] == 10 and s10["fallbacks"] == 0
    assert rel_l2(x10l, x10j) <= 1e-12
    g.set_options()
    g.bind(u0)
    sj = g.advance_be(dt, 1e-10, 1)
    g.set_options(pc=dev.PCS["learned"])
    g.bind(u0)
    sl = g.advance_be(dt, 1e-10, 1)
    xl = g.field.cpu().numpy()
    _log("  iters", sj["iters_total"], sl["iters_total"], "fallbacks", sl["fallbacks"])
    assert sl["iters_total"] <= 1.15 * sj["iters_total"] + 2
    assert true_residual(o, prob, xl, dt) <= 1.001e-10


def test_learned_requires_weights_and_one_component(dev):
    prob = inputs.viscosity(4, 6, 8, seed=3)
    g = dev.Operator.from_problem(prob)
    with pytest.raises(dev.PaError):
        g.set_options(pc=dev.PCS["learned"])
    prob = inputs.heat_iso(4, 6, 8, seed=3)
    g = dev.Operator.from_problem(prob)
    with pytest.raises(dev.PaError):
        g.set_options(pc=dev.PCS["learned"])
    bad = np.zeros(dev.PA_LPC_NPARAM, np.float32)
    bad[7] = np.nan
    with pytest.raises(dev.PaError):
        g.lpc_set_weights(bad)


def _tr(seed, shape=(24, 48, 64)):
    nr, nt, np_ = shape
    return inputs.transition_region(nr, nt, np_, seed=seed, i_tr0=7.0, i_amp=2.0, width=3.0)


TRAIN = dict(nsnap=16, batch=2, epochs=30, seed=4300, lr=1e-3, tol_star=1e-12)


def _train(dev, prob, init_seed=4300, **kw):
    g = dev.Operator.from_problem(prob)
    g.bind(prob.u)
    dt = 50.0 * g.dt_explicit()
    g.lpc_set_weights(dev.he_init(init_seed))
    opts = dict(TRAIN)
    opts.update(kw)
    rep = g.lpc_train(dt, **opts)
    return g, dt, rep


def test_training_deterministic_and_leaves_field(dev):
    prob = _tr(401, (12, 24, 32))
    g1, dt, rep1 = _train(dev, prob, nsnap=6, epochs=2)
    assert np.array_equal(g1.field.cpu().numpy(), prob.u)
    g2, _, rep2 = _train(dev, prob, nsnap=6, epochs=2)
    assert np.array_equal(g1.lpc_get_weights(), g2.lpc_get_weights())
    assert rep1["loss_last"] == rep2["loss_last"] and rep1["snapshots"] >= 2


def _solve(dev, o_prob, theta, pc, tol=1e-10):
    g = dev.Operator.from_problem(o_prob)
    dt = 50.0 * g.dt_explicit()
    if theta is not None:
        g.lpc_set_weights(theta)
    g.set_options(pc=dev.PCS[pc])
    g.bind(o_prob.u)
    s = g.advance_be(dt, tol, 1)
    return g.field.cpu().numpy(), s, dt


def _pairs(dev, o, prob, ks):
    """(r_k, e_k) from Jacobi-PCG iterates x_k of the held-out system."""
    g = dev.Operator.from_problem(prob)
    dt = 50.0 * g.dt_explicit()
    u = g.bind(prob.u)
    g.advance_be(dt, 1e-13, 1)
    xs = u.cpu().numpy()[0]
    V = o.volumes()
    b = V * prob.u[0] + dt * V * o.apply(np.zeros_like(prob.u))[0]
    rs, es = [], []
    for k in ks:
        g.set_options(force_iters=k)
        u = g.bind(prob.u)
        g.advance_be(dt, 1e-10, 1)
        x = u.cpu().numpy()[0]
        rs.append(b - (V * x - dt * V * o.apply(x[None], affine=False)[0]))
        es.append(xs - x)
    return np.stack(rs), np.stack(es), dt


def test_training_gain_on_held_out_problem(dev, oracle_mod):
    """The trained network's step P(r) is a far better estimate of the error
    than the Jacobi step r/D on a held-out problem (energy norm); in the
    solve it is used while it beats Jacobi PCG's pace, and the solve reaches
    the same true residual."""
    g, dt, rep = _train(dev, _tr(401))
    _log("  train", rep)
    assert rep["loss_last"] < 0.5 * rep["loss_first"]
    theta = g.lpc_get_weights()
    held = _tr(402)
    o = oracle_mod.Oracle.from_problem(held)
    r, e, dth = _pairs(dev, o, held, (1, 3, 9, 27))
    gh = dev.Operator.from_problem(held)
    gh.lpc_set_weights(theta)
    loss_l, _ = gh.lpc_loss_grad(dth, r, e)
    gh.lpc_set_weights(np.zeros_like(theta))
    loss_j, _ = gh.lpc_loss_grad(dth, r, e)
    _log("  held-out energy loss learned", loss_l, "jacobi step", loss_j)
    assert loss_l <= 0.3 * loss_j
    xj, sj, dt = _solve(dev, held, None, "jacobi")
    xl, sl, _ = _solve(dev, held, theta, "learned")
    _log("  held-out iters jacobi", sj["iters_total"], "learned", sl["iters_total"],
         "fallbacks", sl["fallbacks"], "ms", sj["ms_total"], sl["ms_total"])
    assert true_residual(o, held, xl, dt) <= 1.001e-10
    assert true_residual(o, held, xj, dt) <= 1.001e-10


def test_corrupted_weights_still_converge(dev, oracle_mod):
    held = _tr(403, (12, 24, 32))
    o = oracle_mod.Oracle.from_problem(held)
    theta = (dev.he_init(7) * 300.0).astype(np.float32)
    theta[10400:] *= -1.0
    xl, sl, dt = _solve(dev, held, theta, "learned")
    _log("  corrupted: iters", sl["iters_total"], "fallbacks", sl["fallbacks"])
    assert true_residual(o, held, xl, dt) <= 1.001e-10


@pytest.mark.timeout(600)
def test_learned_solve_full_size(dev, oracle_mod):
    """The transition-region conduction problem at the benchmark's size
    (151 x 301 x 400): trained on seed 401 with the default recipe, the
    learned FCG(1) solve of the held-out seed 402 (one BE step of 50 dt_E)
    reaches the same FP64 true residual as Jacobi PCG, evaluated with the
    oracle's operator.  The iteration counts are reported, not asserted:
    the network does not lower them (the measured negative result)."""
    prob = inputs.transition_region(151, 301, 400, seed=401)
    g, dt, rep = _train(dev, prob)
    _log("  full-size training", rep)
    theta = g.lpc_get_weights()
    assert np.all(np.isfinite(theta)) and rep["loss_last"] < rep["loss_first"]
    del g
    held = inputs.transition_region(151, 301, 400, seed=402)
    o = oracle_mod.Oracle.from_problem(held)
    xj, sj, dt = _solve(dev, held, None, "jacobi")
    xl, sl, _ = _solve(dev, held, theta, "learned")
    rj, rl = true_residual(o, held, xj, dt), true_residual(o, held, xl, dt)
    _log("  full-size held-out: iterations jacobi", sj["iters_total"], "learned", sl["iters_total"],
         "fallbacks", sl["fallbacks"], "true residual", rj, rl)
    assert sl["status"] == dev.PA_OK and sj["status"] == dev.PA_OK
    assert rl <= 1.001e-10 and rj <= 1.001e-10
