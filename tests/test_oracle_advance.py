"""Pins of the oracle's advances (STS and BE+PCG), the practical time step
limit and the cycle controller: dense spectral solutions on tiny grids,
closed-form decay of eigenmodes, hand-worked PTL values (Eqs. ptl-ptl3),
the forward-Euler sign identity behind Eq. (ptl2), energy decay and
conservation with no-flux boundaries."""
import math

import numpy as np
import pytest
from scipy.special import eval_gegenbauer, eval_legendre

from paper_2403_01004_amd import inputs


def poly(kind, s, z):
    if kind == "rkl2":
        b = (s * s + s - 2) / (2 * s * (s + 1))
        return 1 - b + b * eval_legendre(s, 1 + 4 / (s * s + s - 2) * z)
    b = 4 * (s - 1) * (s + 4) / (3 * s * (s + 1) * (s + 2) * (s + 3))
    return 1 - b * eval_gegenbauer(s, 1.5, 1.0) + b * eval_gegenbauer(s, 1.5, 1 + 6 / ((s + 4) * (s - 1)) * z)


def tiny(oracle_mod, op, bc="dirichlet", seed=5):
    mesh = inputs.shell_mesh(4, 6, 8, stretch=1.1)
    rng = np.random.default_rng(seed)
    o = oracle_mod.Oracle(mesh, op, 1, bc, bc)
    o.set_coefficients(1.0 + 0.5 * rng.random(mesh.shape), 1.0, 2.5, inputs.dipole_corners(mesh))
    return o, mesh, rng


def spectral(o, mesh):
    V = o.volumes().ravel()
    N = V.size
    L = np.zeros((N, N))
    for n in range(N):
        e = np.zeros(N)
        e[n] = 1
        L[:, n] = -V * o.apply(e, affine=False).ravel()
    S = L / np.sqrt(V)[:, None] / np.sqrt(V)[None, :]
    lam, Q = np.linalg.eigh(0.5 * (S + S.T))
    return V, L, lam, Q


@pytest.mark.parametrize("op", ["iso7", "aligned"])
@pytest.mark.parametrize("kind", ["rkl2", "rkg2"])
def test_sts_advance_matches_dense_spectral(oracle_mod, op, kind):
    """One STS cycle on the homogeneous problem equals
    V^-1/2 Q R_s(-dt Lambda) Q^T V^1/2 u with the closed-form polynomial."""
    o, mesh, rng = tiny(oracle_mod, op)
    V, L, lam, Q = spectral(o, mesh)
    u = rng.standard_normal(V.size)
    dtE = o.dt_explicit()
    for ratio, s_ovr in ((7.3, 0), (20.0, 9)):
        dt = ratio * dtE
        out, st = o.advance_sts(u, dt, cycles=1, sts=kind, s_override=s_ovr)
        s = st["s_max"]
        if s_ovr:
            assert s == s_ovr
        else:
            assert s == oracle_mod.sts_stages(kind, ratio, True)
        Rs = np.array([poly(kind, s, -dt * l) for l in lam])
        ref = (Q @ (Rs * (Q.T @ (np.sqrt(V) * u)))) / np.sqrt(V)
        assert np.linalg.norm(out.ravel() - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_be_matches_dense_solve(oracle_mod, op):
    o, mesh, rng = tiny(oracle_mod, op)
    nr, nt, np_ = mesh.shape
    o.set_bc(rng.standard_normal((1, nt, np_)), rng.standard_normal((1, nt, np_)))
    V, L, lam, Q = spectral(o, mesh)
    h = V * o.apply(np.zeros(V.size)).ravel()
    u = rng.standard_normal(V.size)
    dt = 40 * o.dt_explicit()
    out, st = o.advance_be(u, dt, tol=1e-14, cycles=1)
    M = np.diag(V) + dt * L
    x = np.linalg.solve(M, V * u + dt * h)
    cond = np.linalg.cond(M)
    assert st["status"] == 0
    assert np.linalg.norm(out.ravel() - x) <= 10 * cond * 1e-14 * np.linalg.norm(x)
    assert st["rel_residual"] <= 1e-14


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_eigenmode_closed_form_decay(oracle_mod, op):
    """cos(m phi) with constant coefficient and no-flux radial boundaries:
    STS multiplies each column by R_s(dt lambda_ij), BE by 1/(1 - dt lambda_ij).
    7-point: one radial shell and two rows mirror-symmetric about the equator,
    so the columns never couple and lambda has the finite-volume closed form
    -c A_phi/(V d_phi) 4 sin^2(m dphi/2).  Field-aligned with bhat = phihat:
    only longitude differences enter, so every column is independent on any
    mesh; lambda_ij is read from one application of F."""
    m = 2
    if op == "iso7":
        mesh = inputs.shell_mesh(1, 2, 24)
        o = oracle_mod.Oracle(mesh, "iso7", 1, "noflux", "noflux")
        o.set_coefficients(None, 0.9, 0.0, None)
        rc, tc, pc = inputs.cell_centres(mesh)
        R, TH = mesh.r_faces, mesh.t_faces
        dphi = 2 * math.pi / mesh.shape[2]
        Aphi = 0.5 * (R[1:] ** 2 - R[:-1] ** 2)[:, None] * np.diff(TH)[None, :]
        V = ((R[1:] ** 3 - R[:-1] ** 3) / 3)[:, None] * (np.cos(TH[:-1]) - np.cos(TH[1:]))[None, :] * dphi
        lam = -0.9 * Aphi / (V * rc[:, None] * np.sin(tc)[None, :] * dphi) * 4 * math.sin(m * dphi / 2) ** 2
    else:
        mesh = inputs.shell_mesh(1, 2, 24)
        o = oracle_mod.Oracle(mesh, "aligned", 1, "noflux", "noflux")
        o.set_coefficients(None, 0.9, 0.0, inputs.uniform_direction_corners(mesh, 2))
        rc, tc, pc = inputs.cell_centres(mesh)
    u = np.broadcast_to(np.cos(m * pc), mesh.shape)[None].copy()
    if op == "aligned":
        lam = (o.apply(u)[0] / u[0])[:, :, 0]
    dt = 30 * o.dt_explicit()
    for kind in ("rkl2", "rkg2"):
        out, st = o.advance_sts(u, dt, cycles=1, sts=kind)
        s = st["s_max"]
        assert s > 5
        ref = np.vectorize(lambda z: poly(kind, s, z))(dt * lam)[:, :, None] * u[0]
        assert np.abs(out[0] - ref).max() < 1e-12
    out, st = o.advance_be(u, dt, tol=1e-14, cycles=1)
    ref = u[0] / (1 - dt * lam)[:, :, None]
    assert np.abs(out[0] - ref).max() < 1e-11


# ------------------------------------------------------------------ PTL

def test_ptl_hand_values(oracle_mod):
    """Eq. (ptl3) on hand-worked spikes: 1-D [0,0,1,0,0] with the unit
    three-point Laplacian gives F_k = -2, F_nb = 1, so -(1-0)/(-2-1) = 1/3;
    the 3-D seven-point spike gives -(1)/(-6-1) = 1/7."""
    u = np.zeros((1, 1, 1, 5))
    u[0, 0, 0, 2] = 1
    F = np.zeros_like(u)
    F[0, 0, 0, 1:4] = [1, -2, 1]
    dt, k = oracle_mod.ptl_from(u, F)
    assert k == 2 and abs(dt - 1 / 3) < 1e-16
    u = np.zeros((1, 3, 3, 4))
    u[0, 1, 1, 1] = 1
    F = np.zeros_like(u)
    F[0, 1, 1, 1] = -6
    for nb in [(0, 1, 1), (2, 1, 1), (1, 0, 1), (1, 2, 1), (1, 1, 0), (1, 1, 2)]:
        F[(0,) + nb] = 1
    dt, k = oracle_mod.ptl_from(u, F)
    assert k == 1 * 12 + 1 * 4 + 1 and abs(dt - 1 / 7) < 1e-16


def test_ptl_edge_cases(oracle_mod):
    # no admissible neighbour (same signs) -> +inf
    u = np.zeros((1, 2, 2, 3))
    F = np.zeros_like(u)
    F[0, 0, 0, 0] = 1.0
    dt, _ = oracle_mod.ptl_from(u, F)
    assert dt == math.inf
    # ties: lowest linear index wins
    F = np.zeros((2, 2, 2, 3))
    F[0, 1, 1, 2] = -3
    F[1, 0, 0, 0] = 3
    _, k = oracle_mod.ptl_from(np.zeros_like(F), F)
    assert k == 1 * 6 + 1 * 3 + 2
    # phi wraps: spike at k=0 sees k=np-1
    u = np.zeros((1, 1, 1, 4))
    u[0, 0, 0, 0] = 1
    F = np.zeros_like(u)
    F[0, 0, 0, :] = [-2, 0, 0, 1.5]
    dt, k = oracle_mod.ptl_from(u, F)
    assert k == 0 and abs(dt - 1 / 3.5) < 1e-16


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_ptl_sign_identity_and_fullgrid(oracle_mod, op):
    """A forward-Euler step of length dt_PTL zeroes the limiting difference
    (Eq. ptl2 at equality), and the full-grid minimum never exceeds it."""
    mesh = inputs.shell_mesh(6, 8, 10)
    o = oracle_mod.Oracle(mesh, op)
    rng = np.random.default_rng(11)
    o.set_coefficients(1 + 0.3 * rng.random(mesh.shape), 1.0, 2.5, inputs.dipole_corners(mesh))
    nr, nt, np_ = mesh.shape
    o.set_bc(rng.random((1, nt, np_)), rng.random((1, nt, np_)))
    u = rng.random((1,) + mesh.shape)
    F = o.apply(u)
    dt, k = o.ptl(u)
    assert (dt, k) == oracle_mod.ptl_from(u, F)
    assert np.argmax(np.abs(F).ravel()) == k
    u1 = (u + dt * F).ravel()
    uf, Ff = u.ravel(), F.ravel()
    i, j, kk = np.unravel_index(k, mesh.shape)
    nbs = []
    if i > 0: nbs.append(k - nt * np_)
    if i < nr - 1: nbs.append(k + nt * np_)
    if j > 0: nbs.append(k - np_)
    if j < nt - 1: nbs.append(k + np_)
    nbs += [k - kk + (kk - 1) % np_, k - kk + (kk + 1) % np_]
    gaps = [abs(u1[k] - u1[n]) / abs(uf[k] - uf[n]) for n in nbs
            if (uf[k] - uf[n]) * (Ff[k] - Ff[n]) < 0]
    assert min(gaps) < 1e-12
    assert oracle_mod.ptl_fullgrid(u, F) <= dt


# -------------------------------------------------------------- cycling

@pytest.mark.parametrize("scheme", ["sts", "be"])
def test_controller(oracle_mod, scheme):
    prob = inputs.conduction(8, 12, 16, seed=3, noise_amp=0.05)
    o = oracle_mod.Oracle.from_problem(prob)
    dt = 60 * o.dt_explicit()
    run = (lambda **kw: o.advance_sts(prob.u, dt, **kw)) if scheme == "sts" else \
        (lambda **kw: o.advance_be(prob.u, dt, **kw))
    out, st = run(cycles=0)
    assert st["status"] == 0 and st["cycles"] >= 2
    assert abs(st["dt_cycle"].sum() - dt) <= 1e-14 * dt
    # equal split of the remaining time: lengths never shrink below the PTL
    # of the cycle; first cycle is (t / ceil(t / ptl))
    n0 = math.ceil(dt / st["dt_ptl_first"])
    assert abs(st["dt_cycle"][0] - dt / n0) <= 1e-15 * dt
    # replaying the schedule reproduces the field bit for bit
    out2, st2 = run(replay=st["dt_cycle"])
    assert np.array_equal(out, out2)
    # fixed cycles
    _, st3 = run(cycles=3)
    assert st3["cycles"] == 3 and np.allclose(st3["dt_cycle"], dt / 3, rtol=1e-15)
    # a limit larger than dt gives one cycle
    _, st4 = (o.advance_sts if scheme == "sts" else o.advance_be)(prob.u, 1e-3 * st["dt_ptl_first"])
    assert st4["cycles"] == 1
    # too many cycles needed -> error 8
    _, st5 = run(cycles=0, max_cycles=1)
    assert st5["status"] == 8
    # with the limit floored at dt_E, an equal split t/ceil(t/lim) with t >= lim
    # never gives a cycle shorter than dt_E/2 (the final cycle aside)
    assert np.all(st["dt_cycle"][:-1] >= 0.5 * o.dt_explicit() * (1 - 1e-12))


def test_unfloored_ptl_collapses_for_be(oracle_mod):
    """Without a floor, stepping at the limit flattens the limiting pair and
    the next limit collapses; a BE cycle too short to move the iterate then
    repeats forever (reported as too many cycles)."""
    prob = inputs.conduction(8, 12, 16, seed=3, noise_amp=0.05)
    o = oracle_mod.Oracle.from_problem(prob)
    dtE = o.dt_explicit()
    _, st = o.advance_be(prob.u, 60 * dtE, cycles=0, ptl_floor=0.0, max_cycles=60)
    assert st["status"] == 8 and st["dt_ptl_min"] < 1e-6 * dtE
    _, st = o.advance_be(prob.u, 60 * dtE, cycles=0, ptl_floor=1.0, max_cycles=60)
    assert st["status"] == 0 and st["floored"] >= 1


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_energy_and_conservation_noflux(oracle_mod, op):
    mesh = inputs.shell_mesh(6, 8, 12)
    o = oracle_mod.Oracle(mesh, op, 1, "noflux", "noflux")
    rng = np.random.default_rng(2)
    o.set_coefficients(1 + 0.5 * rng.random(mesh.shape), 1.0, 2.5, inputs.dipole_corners(mesh))
    V = o.volumes()
    u = rng.standard_normal((1,) + mesh.shape)
    dt = 40 * o.dt_explicit()
    E0, M0 = (V * u[0] ** 2).sum(), (V * u[0]).sum()
    for kind in ("rkl2", "rkg2"):
        out, _ = o.advance_sts(u, dt, cycles=1, sts=kind)
        assert (V * out[0] ** 2).sum() <= E0
        assert abs((V * out[0]).sum() - M0) <= 1e-12 * np.abs(V * u[0]).sum()
    out, st = o.advance_be(u, dt, tol=1e-12, cycles=1)
    assert (V * out[0] ** 2).sum() <= E0
    assert abs((V * out[0]).sum() - M0) <= 1e-9 * np.abs(V * u[0]).sum()
    # dynamic PTL cycling decays energy monotonically too
    out, st = o.advance_sts(u, dt, cycles=0)
    assert (V * out[0] ** 2).sum() <= E0


def test_pcg_errors(oracle_mod):
    prob = inputs.conduction(6, 8, 10, seed=4)
    o = oracle_mod.Oracle.from_problem(prob)
    dt = 50 * o.dt_explicit()
    _, st = o.advance_be(prob.u, dt, cycles=1, max_iter=1)
    assert st["status"] == 4
    _, st = o.advance_be(prob.u, dt, cycles=1, force_iters=3)
    assert st["status"] == 0 and st["iters_total"] == 3


def test_ptl_fullgrid_hand_example(oracle_mod):
    """Periodic ring of 4 cells, u = (0, 1, 0, 0.5), F = (1, -2, 1.5, -1).
    Argmax |F| is cell 1: its pairs give 1/3 (cell 0) and 1/3.5 (cell 2), so
    Eq. (ptl3) gives 1/3.5.  Over every pair the pair (2, 3) has du = -0.5,
    dF = 2.5 -> 0.2, and (3, 0) gives 0.5/2 = 0.25: the full-grid minimum is
    0.2."""
    u = np.array([0.0, 1.0, 0.0, 0.5]).reshape(1, 1, 1, 4)
    F = np.array([1.0, -2.0, 1.5, -1.0]).reshape(1, 1, 1, 4)
    dt, k = oracle_mod.ptl_from(u, F)
    assert k == 1 and abs(dt - 1 / 3.5) < 1e-16
    assert abs(oracle_mod.ptl_fullgrid(u, F) - 0.2) < 1e-16
    # no constraining pair at all
    assert oracle_mod.ptl_fullgrid(np.ones_like(u), F) == np.inf
