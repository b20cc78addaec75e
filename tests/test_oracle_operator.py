"""Pins of the oracle's operator, geometry and explicit limit against facts
that do not come from the oracle itself: exact volumes, invariants of a
symmetric conservative diffusion operator, closed-form eigenpairs and
second-order convergence to the continuous operators of Eq. (visc)/(tc)."""
import math

import numpy as np
import pytest

from paper_2403_01004_amd import inputs


def dense_L(o, V):
    """Dense L = -V F_lin by unit-vector probing (brute force, tiny grids)."""
    N = V.size * o.nc
    L = np.zeros((N, N))
    Vf = np.tile(V.ravel(), o.nc)
    for n in range(N):
        e = np.zeros(N)
        e[n] = 1.0
        L[:, n] = -Vf * o.apply(e, affine=False).ravel()
    return L, Vf


@pytest.fixture(scope="module", params=["iso7", "aligned"])
def small(request, oracle_mod):
    mesh = inputs.shell_mesh(5, 6, 8)
    rng = np.random.default_rng(7)
    T0 = 1.0 + 0.4 * rng.random(mesh.shape)
    return request.param, mesh, T0


def make(oracle_mod, op, mesh, T0, bc="dirichlet", nc=1, B=None):
    o = oracle_mod.Oracle(mesh, op, nc, bc, bc)
    o.set_coefficients(T0, 1.3, 2.5, inputs.dipole_corners(mesh) if B is None else B)
    return o


def test_volumes_sum_to_shell(oracle_mod):
    mesh = inputs.shell_mesh(9, 7, 11, r_in=1.0, r_out=2.5, stretch=1.05)
    o = oracle_mod.Oracle(mesh, "iso7")
    exact = 4.0 * math.pi / 3.0 * (2.5 ** 3 - 1.0)
    assert abs(o.volumes().sum() - exact) / exact < 1e-14


def test_mesh_stretch():
    mesh = inputs.shell_mesh(151, 4, 4)
    dr = np.diff(mesh.r_faces)
    assert np.allclose(dr[1:] / dr[:-1], 1.02, rtol=1e-10)
    assert abs(mesh.r_faces[-1] - 2.5) < 1e-15 and abs(dr[0] - 1.588e-3) < 1e-6


def test_symmetric_psd(oracle_mod, small):
    op, mesh, T0 = small
    for bc in ("dirichlet", "noflux"):
        o = make(oracle_mod, op, mesh, T0, bc)
        V = o.volumes()
        L, _ = dense_L(o, V)
        scale = np.abs(L).max()
        assert np.abs(L - L.T).max() <= 1e-14 * scale
        assert np.linalg.eigvalsh(0.5 * (L + L.T)).min() >= -1e-13 * scale


def test_constant_is_steady(oracle_mod, small):
    op, mesh, T0 = small
    nr, nt, np_ = mesh.shape
    for bc in ("dirichlet", "noflux"):
        o = make(oracle_mod, op, mesh, T0, bc)
        o.set_bc(np.full((1, nt, np_), 2.5), np.full((1, nt, np_), 2.5))
        F = o.apply(np.full((1, nr, nt, np_), 2.5))
        assert np.abs(F).max() < 1e-12


def test_conservation_noflux(oracle_mod, small):
    op, mesh, T0 = small
    o = make(oracle_mod, op, mesh, T0, "noflux")
    V = o.volumes()
    u = np.random.default_rng(3).standard_normal((1,) + mesh.shape)
    F = o.apply(u)
    assert abs((V * F[0]).sum()) < 1e-12 * np.abs(V * F[0]).sum()


def test_gershgorin_and_diag(oracle_mod, small):
    op, mesh, T0 = small
    o = make(oracle_mod, op, mesh, T0)
    V = o.volumes()
    L, Vf = dense_L(o, V)
    A = L / Vf[:, None]
    lam_max = np.linalg.eigvals(A).real.max()
    gersh = np.abs(A).sum(axis=1).max()
    rho = 2.0 / o.dt_explicit()
    assert rho >= gersh * (1 - 1e-12) and rho >= lam_max
    if op == "iso7":                 # the 7-point bound is the exact Gershgorin bound
        assert abs(rho - gersh) <= 1e-12 * gersh
    assert np.allclose(o.diag().ravel(), np.diag(L), rtol=1e-13, atol=0)


def test_gershgorin_1d_limit(oracle_mod):
    """A 1-D-like column (one longitude wave dominating): on a uniform thin shell
    with constant coefficient the bound approaches 4 c / h^2 in phi."""
    nr, nt, np_ = 1, 2, 64
    mesh = inputs.Mesh(np.array([1.0, 1.0 + 1e-3]), np.array([0.0, math.pi / 2, math.pi]),
                       np.linspace(0, 2 * math.pi, np_ + 1))
    o = oracle_mod.Oracle(mesh, "iso7", 1, "noflux", "noflux")
    o.set_coefficients(None, 1.0, 0.0, None)
    # Equator-adjacent cells: phi spacing r sin(theta_c) dphi; theta couplings
    # across the equator are much weaker (large theta spacing).
    rho = 2.0 / o.dt_explicit()
    rc = 1.0 + 0.5e-3
    hphi = rc * math.sin(math.pi / 4) * 2 * math.pi / np_
    Vt = (math.cos(0) - math.cos(math.pi / 2))
    Aphi = 0.5 * ((1 + 1e-3) ** 2 - 1) * (math.pi / 2)
    V = ((1 + 1e-3) ** 3 - 1) / 3 * Vt * (2 * math.pi / np_)
    At = math.sin(math.pi / 2) * 0.5 * ((1 + 1e-3) ** 2 - 1) * (2 * math.pi / np_)
    expect = (4 * Aphi / hphi + 2 * At / (rc * math.pi / 2)) / V
    assert abs(rho - expect) <= 1e-12 * expect


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_longitude_eigenmode(oracle_mod, op):
    """u = cos(m phi) is an exact eigenvector of each (r, theta) column when
    the coefficient is constant, the radial boundaries are no-flux and (for the
    aligned operator) bhat = phihat.  Eigenvalue for the 7-point operator:
    -c A_phi/(V d_phi) 4 sin^2(m dphi/2) (finite-volume flux through the two
    longitude faces)."""
    mesh = inputs.shell_mesh(6, 8, 16)
    nr, nt, np_ = mesh.shape
    o = oracle_mod.Oracle(mesh, op, 1, "noflux", "noflux")
    o.set_coefficients(None, 0.7, 0.0, inputs.uniform_direction_corners(mesh, 2))
    rc, tc, pc = inputs.cell_centres(mesh)
    m = 3
    u = np.broadcast_to(np.cos(m * pc), mesh.shape)[None].copy()
    F = o.apply(u)[0]
    lam = F / u[0]
    ok = np.abs(u[0]) > 0.3
    # eigenvector: the ratio is constant along phi in each column
    col = np.where(ok, lam, np.nan)
    spread = np.nanmax(col, axis=2) - np.nanmin(col, axis=2)
    assert np.nanmax(np.abs(spread)) < 1e-9 * np.nanmax(np.abs(col))
    if op == "iso7":
        R, TH = mesh.r_faces, mesh.t_faces
        dphi = 2 * math.pi / np_
        Aphi = 0.5 * (R[1:] ** 2 - R[:-1] ** 2)[:, None] * np.diff(TH)[None, :]
        V = ((R[1:] ** 3 - R[:-1] ** 3) / 3)[:, None] * (np.cos(TH[:-1]) - np.cos(TH[1:]))[None, :] * dphi
        d = rc[:, None] * np.sin(tc)[None, :] * dphi
        expect = -0.7 * Aphi / (V * d) * 4 * math.sin(m * dphi / 2) ** 2
        assert np.allclose(np.nanmean(col, axis=2), expect, rtol=1e-12)


def _mms_error(oracle_mod, op, n):
    sp = pytest.importorskip("sympy")
    r, t, p = sp.symbols("r t p")
    u = sp.sin(2 * r) * sp.cos(t) ** 2 * sp.cos(p) + 0.3 * r * sp.sin(t) * sp.sin(2 * p) + 0.2 * r ** 2
    kap = 1 + 0.3 * sp.sin(r) * sp.cos(t) + 0.2 * sp.sin(t) ** 2 * sp.cos(p)
    if op == "iso7":
        ex = (sp.diff(r ** 2 * kap * sp.diff(u, r), r) / r ** 2
              + sp.diff(sp.sin(t) * kap * sp.diff(u, t), t) / (r ** 2 * sp.sin(t))
              + sp.diff(kap * sp.diff(u, p), p) / (r ** 2 * sp.sin(t) ** 2))
    else:
        a = sp.rad(10)
        mx, mz = sp.sin(a), sp.cos(a)
        mr = mx * sp.sin(t) * sp.cos(p) + mz * sp.cos(t)
        Br = 2 * mr / r ** 3
        Bt = -(mx * sp.cos(t) * sp.cos(p) - mz * sp.sin(t)) / r ** 3
        Bp = -(-mx * sp.sin(p)) / r ** 3
        Bm = sp.sqrt(Br ** 2 + Bt ** 2 + Bp ** 2)
        br, bt, bp = Br / Bm, Bt / Bm, Bp / Bm
        G = br * sp.diff(u, r) + bt * sp.diff(u, t) / r + bp * sp.diff(u, p) / (r * sp.sin(t))
        ex = (sp.diff(r ** 2 * kap * G * br, r) / r ** 2
              + sp.diff(sp.sin(t) * kap * G * bt, t) / (r * sp.sin(t))
              + sp.diff(kap * G * bp, p) / (r * sp.sin(t)))
    fu, fk, fe = (sp.lambdify((r, t, p), e, "numpy") for e in (u, kap, ex))
    mesh = inputs.shell_mesh(8 * n, 12 * n, 24 * n, stretch=1.0)
    rc, tc, pc = inputs.cell_centres(mesh)
    R, T, P = np.meshgrid(rc, tc, pc, indexing="ij")
    o = oracle_mod.Oracle(mesh, op, 1)
    o.set_coefficients(fk(R, T, P), 1.0, 1.0, inputs.dipole_corners(mesh))
    o.set_bc(fu(mesh.r_faces[0] + 0 * T[0], T[0], P[0])[None],
             fu(mesh.r_faces[-1] + 0 * T[0], T[0], P[0])[None])
    F = o.apply(fu(R, T, P)[None])[0]
    ir = np.arange(mesh.shape[0])[:, None, None]
    jt = np.arange(mesh.shape[1])[None, :, None]
    # away from the radial boundary cells (half-cell Dirichlet closure) and
    # from the poles, where the 1/sin(theta) metric makes the truncation error
    # non-uniform on any spherical mesh
    del jt
    mask = (ir > 0) & (ir < mesh.shape[0] - 1) & (T > 0.5) & (T < math.pi - 0.5)
    return np.abs(F - fe(R, T, P))[mask].max()


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_second_order_convergence(oracle_mod, op):
    """F converges at second order to div(c grad u) (7-point) and to
    div(kappa bhat bhat . grad u) (field-aligned, tilted dipole) -- pins every
    metric factor (areas, distances, sin theta, corner weights)."""
    e1, e2, e4 = (_mms_error(oracle_mod, op, n) for n in (1, 2, 4))
    assert e2 / e4 > 3.2 and e1 / e2 > 2.5, (e1, e2, e4)


def test_checkerboard_nullspace(oracle_mod):
    """Known property of the symmetric corner scheme: the 3-D checkerboard
    has zero corner gradient (no-flux radial boundaries)."""
    mesh = inputs.shell_mesh(4, 6, 8)
    o = oracle_mod.Oracle(mesh, "aligned", 1, "noflux", "noflux")
    o.set_coefficients(None, 1.0, 0.0, inputs.dipole_corners(mesh))
    i, j, k = np.meshgrid(*[np.arange(n) for n in mesh.shape], indexing="ij")
    u = ((-1.0) ** (i + j + k))[None]
    assert np.abs(o.apply(u)).max() < 1e-10
