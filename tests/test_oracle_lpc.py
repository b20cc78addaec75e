"""Pins of the learned-preconditioner oracle (oracle/lpc.py) against library
routines and mathematical identities: torch's round-to-nearest-even BF16
conversion, torch's conv3d (with periodic phi / zero r, theta padding built
by hand), adjointness of the transposed convolution, central finite
differences of the loss, torch.optim.Adam, positive homogeneity of the
preconditioner, and flexible CG reducing to PCG for the Jacobi
preconditioner."""
import numpy as np
import pytest
import torch

from oracle import lpc
from paper_2403_01004_amd import inputs


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-8, 8, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.001953125, 3.0e38]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(lpc.bf16(x), ref)


def torch_conv(W, x):
    t = torch.tensor(x)[None]                       # [1, ci, nr, nt, np]
    t = torch.cat([t[..., -1:], t, t[..., :1]], -1)  # periodic phi
    t = torch.nn.functional.pad(t, (0, 0, 1, 1, 1, 1))  # zero theta, r
    return torch.nn.functional.conv3d(t, torch.tensor(W)).numpy()[0]


def test_conv_matches_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((8, 5, 6, 7))
    W = rng.standard_normal((16, 8, 3, 3, 3))
    assert np.allclose(lpc.conv(W, x), torch_conv(W, x), rtol=1e-12, atol=1e-12)


def test_conv_transpose_is_adjoint_and_wgrad():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((16, 4, 5, 6))
    W = rng.standard_normal((3, 16, 3, 3, 3))
    g = rng.standard_normal((3, 4, 5, 6))
    lhs = np.vdot(lpc.conv(W, x), g)
    assert abs(lhs - np.vdot(x, lpc.conv_t(W, g))) < 1e-10 * abs(lhs)
    assert abs(lhs - np.vdot(W, lpc.conv_wgrad(x, g))) < 1e-10 * abs(lhs)


def small_problem(seed=3):
    rng = np.random.default_rng(seed)
    shape = (5, 6, 8)
    D = 1.0 + rng.random(shape)
    static = rng.random((7,) + shape)
    pairs = [(rng.standard_normal(shape), rng.standard_normal(shape)) for _ in range(2)]
    theta = lpc.he_init(np.random.default_rng(seed + 10))
    theta[3456:3472] = 0.1 * rng.standard_normal(16)       # nonzero biases
    theta[10384:10400] = 0.1 * rng.standard_normal(16)
    n = D.size
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    Mdense = A @ A.T + np.diag(D.ravel())                   # SPD
    return theta, pairs, D, static, lambda v: (Mdense @ v.ravel()).reshape(v.shape)


def test_gradient_matches_finite_differences():
    theta, pairs, D, static, mv = small_problem()
    L, g = lpc.loss_and_grad(theta, pairs, D, static, mv)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(3456, 6, replace=False), [3456, 3465],
                          3472 + rng.choice(6912, 6, replace=False), [10384, 10390],
                          10400 + rng.choice(432, 6, replace=False)])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (lpc.loss_and_grad(tp, pairs, D, static, mv)[0]
              - lpc.loss_and_grad(tm, pairs, D, static, mv)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-7, (i, fd, g[i])


def test_energy_loss_of_exact_inverse_is_zero_and_jacobi_value():
    """With N == 0, P(r) = r/D: the loss is |r/D - e|_M^2/|e|_M^2, computed
    here from the dense matrix directly; and it vanishes when r/D = e."""
    theta, pairs, D, static, mv = small_problem(19)
    zero = np.zeros_like(theta)
    L, g = lpc.loss_and_grad(zero, pairs, D, static, mv)
    ref = np.mean([np.vdot(r / D - e, mv(r / D - e)) / np.vdot(e, mv(e)) for r, e in pairs])
    assert abs(L - ref) <= 1e-13 * ref
    r = pairs[0][0]
    L0, _ = lpc.loss_and_grad(zero, [(r, r / D)], D, static, mv)
    assert L0 == 0.0


def test_adam_matches_torch():
    rng = np.random.default_rng(6)
    theta = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.tensor(theta.copy()))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for t in range(1, 6):
        grad = rng.standard_normal(50)
        theta, m, v = lpc.adam_step(theta, grad, m, v, t)
        opt.zero_grad()
        p.grad = torch.tensor(grad)
        opt.step()
    assert np.allclose(theta, p.detach().numpy(), rtol=0, atol=1e-14)


def test_preconditioner_positively_homogeneous():
    theta, pairs, D, static, _ = small_problem(7)
    r = pairs[0][0]
    z1 = lpc.precondition(theta, r, D, static)
    z2 = lpc.precondition(theta, 3.5 * r, D, static)
    assert np.allclose(z2, 3.5 * z1, rtol=1e-13, atol=1e-13)
    assert not np.allclose(lpc.precondition(theta, -r, D, static), -z1)   # not odd


def test_fcg_with_jacobi_is_pcg(oracle_mod):
    """FCG(1) with P = D^-1 reproduces the oracle's PCG iterates."""
    prob = inputs.conduction(6, 8, 10, seed=9)
    o = oracle_mod.Oracle.from_problem(prob)
    V = o.volumes()
    dt = 30 * o.dt_explicit()
    u = prob.u[0]
    D = V + dt * o.diag()

    def matvec(x):
        return V * x - dt * V * o.apply(x[None], affine=False)[0]

    b = V * u + dt * V * o.apply(np.zeros_like(prob.u))[0]
    for n in (1, 4, 9):
        x, its = lpc.fcg(matvec, b, u.copy(), D, lambda r: r / D, tol=0.0, max_iter=n)
        xo, st = o.advance_be(prob.u, dt, cycles=1, force_iters=n)
        assert its == n
        assert np.linalg.norm(x - xo[0]) <= 1e-12 * np.linalg.norm(xo[0])


def test_conv_zero_phi_padding_matches_torch():
    rng = np.random.default_rng(11)
    x = rng.standard_normal((16, 4, 5, 6))
    W = rng.standard_normal((3, 16, 3, 3, 3))
    ref = torch.nn.functional.conv3d(torch.tensor(x)[None], torch.tensor(W), padding=1).numpy()[0]
    assert np.allclose(lpc.conv(W, x, periodic=False), ref, rtol=1e-12, atol=1e-12)
    g = rng.standard_normal((3, 4, 5, 6))
    lhs = np.vdot(lpc.conv(W, x, periodic=False), g)
    assert abs(lhs - np.vdot(x, lpc.conv_t(W, g, periodic=False))) < 1e-10 * abs(lhs)
    assert abs(lhs - np.vdot(W, lpc.conv_wgrad(x, g, periodic=False))) < 1e-10 * abs(lhs)


def test_bf16_gradient_close_to_exact():
    """The BF16-rounding emulation changes the gradient by about the BF16
    unit roundoff, not more."""
    theta, pairs, D, static, mv = small_problem(17)
    L, g = lpc.loss_and_grad(theta, pairs, D, static, mv)
    Lb, gb = lpc.loss_and_grad(theta, pairs, D, static, mv, bf16_mode=True)
    assert abs(Lb - L) <= 2e-2 * L
    assert np.linalg.norm(gb - g) <= 3e-2 * np.linalg.norm(g)


def _coupling_setup(oracle_mod, op, seed):
    prob = (inputs.conduction(4, 5, 7, seed=seed) if op == "aligned"
            else inputs.heat_iso(4, 5, 7, seed=seed))
    o = oracle_mod.Oracle(prob.mesh, prob.op, 1, "noflux", "noflux")
    o.set_coefficients(prob.T0, prob.scale, prob.expo, prob.B)
    V = o.volumes()
    cpl = lpc.face_couplings(lambda x: o.apply(x[None], affine=False)[0], V)
    return o, V, cpl


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_face_couplings_symmetric(oracle_mod, op):
    """L is symmetric: the coupling of m to its r+ neighbour equals that
    neighbour's coupling to its r- neighbour (same for theta, phi)."""
    o, V, cpl = _coupling_setup(oracle_mod, op, 23)
    assert np.allclose(cpl[1][:-1], cpl[0][1:], rtol=1e-12, atol=1e-15)
    assert np.allclose(cpl[3][:, :-1], cpl[2][:, 1:], rtol=1e-12, atol=1e-15)
    assert np.allclose(cpl[5], np.roll(cpl[4], -1, axis=2), rtol=1e-12, atol=1e-15)
    assert not cpl[0][0].any() and not cpl[1][-1].any()
    assert not cpl[2][:, 0].any() and not cpl[3][:, -1].any()
    assert (cpl[0][1:] != 0).any()


def test_face_couplings_iso7_closed_form(oracle_mod):
    """7-point operator with no-flux faces: zero row sums (diag + the six
    couplings), and the radial coupling is -c_face * A_face / d_face."""
    o, V, cpl = _coupling_setup(oracle_mod, "iso7", 29)
    assert np.allclose(cpl.sum(axis=0), -o.diag(), rtol=1e-12, atol=1e-15)
    assert (cpl <= 0).all()
    # constant-coefficient check on a uniform shell: L(m, r+) = -A_f / d
    mesh = inputs.shell_mesh(3, 4, 6, stretch=1.0)
    oc = oracle_mod.Oracle(mesh, "iso7", 1, "noflux", "noflux")
    oc.set_coefficients(None, 1.0, 0.0, None)
    Vc = oc.volumes()
    cc = lpc.face_couplings(lambda x: oc.apply(x[None], affine=False)[0], Vc)
    R, T, P = mesh.r_faces, mesh.t_faces, mesh.p_faces
    rc = 0.5 * (R[1:] + R[:-1])
    j, k = 1, 2
    area = R[1] ** 2 * (np.cos(T[j]) - np.cos(T[j + 1])) * (P[k + 1] - P[k])
    assert np.isclose(cc[1][0, j, k], -area / (rc[1] - rc[0]), rtol=1e-12)
