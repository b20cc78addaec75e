"""Pins of the oracle's full operator forms (Eqs. visc and tc): the weight w
of F = (1/w) div(...), the radial profile f_c(r) and the low-temperature
modification f_m(T0) (conductivity held at its Tc value below Tc).

Each pin ties the weighted / profiled operator to the unweighted one or to
a dense solve, by identities that hold exactly (up to rounding)."""
import numpy as np
import pytest

from paper_2403_01004_amd import inputs


def _oracle(oracle_mod, op, shape, bc="dirichlet", seed=0):
    mesh = inputs.shell_mesh(*shape)
    rng = np.random.default_rng(seed)
    o = oracle_mod.Oracle(mesh, op, 1, bc, bc)
    T0 = 0.5 + rng.random(mesh.shape)
    B = inputs.dipole_corners(mesh)
    o.set_bc(rng.random((1,) + mesh.shape[1:]), rng.random((1,) + mesh.shape[1:]))
    u = rng.random((1,) + mesh.shape)
    return mesh, o, T0, B, u, rng


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_constant_weight_scales_operator(oracle_mod, op):
    mesh, o, T0, B, u, rng = _oracle(oracle_mod, op, (5, 6, 8))
    o.set_coefficients(T0, 1.0, 2.5, B)
    F, dtE = o.apply(u), o.dt_explicit()
    o.set_profile(np.full(mesh.shape, 2.5))
    o.set_coefficients(T0, 1.0, 2.5, B)
    assert np.allclose(o.apply(u), F / 2.5, rtol=1e-14, atol=0)
    assert abs(o.dt_explicit() - 2.5 * dtE) <= 1e-14 * dtE
    assert np.allclose(o.volumes(weighted=True), 2.5 * o.volumes(), rtol=1e-15, atol=0)


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_weighted_conservation_noflux(oracle_mod, op):
    """With no-flux boundaries the weighted volume integral of F vanishes:
    sum_m w_m V_m F_m = -sum_m (L u)_m = 0 (L has zero row sums)."""
    mesh, o, T0, B, u, rng = _oracle(oracle_mod, op, (5, 6, 8), bc="noflux", seed=1)
    w = 0.3 + rng.random(mesh.shape)
    o.set_profile(w)
    o.set_coefficients(T0, 1.0, 2.5, B)
    wV = o.volumes(weighted=True)
    F = o.apply(u)[0]
    assert abs(np.sum(wV * F)) <= 1e-12 * np.sum(np.abs(wV * F))
    # and the unweighted sum does not vanish (the weight matters)
    assert abs(np.sum(o.volumes() * F)) > 1e-6 * np.sum(np.abs(wV * F))


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_weighted_backward_euler_dense(oracle_mod, op):
    """(w V + dt L) x = w V u + dt h solved densely equals the PCG result."""
    mesh, o, T0, B, u, rng = _oracle(oracle_mod, op, (3, 4, 6), seed=2)
    w = 0.5 + rng.random(mesh.shape)
    o.set_profile(w)
    o.set_coefficients(T0, 1.0, 2.5, B)
    wV = o.volumes(weighted=True).ravel()
    n = wV.size
    L = np.empty((n, n))
    e = np.zeros((1,) + mesh.shape)
    for q in range(n):
        e.ravel()[q] = 1.0
        L[:, q] = -wV * o.apply(e, affine=False).ravel()
        e.ravel()[q] = 0.0
    assert np.allclose(L, L.T, rtol=1e-12, atol=1e-14 * np.abs(L).max())
    dt = 20.0 * o.dt_explicit()
    h = wV * o.apply(np.zeros_like(u)).ravel()
    x = np.linalg.solve(np.diag(wV) + dt * L, wV * u.ravel() + dt * h)
    xo, st = o.advance_be(u, dt, tol=1e-14, cycles=1)
    assert np.linalg.norm(xo.ravel() - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_fm_holds_conductivity_below_threshold(oracle_mod, op):
    """f_m(T0) T0^expo = Tc^expo below Tc: the operator equals the one with
    T0 clamped from below at Tc."""
    mesh, o, T0, B, u, rng = _oracle(oracle_mod, op, (5, 6, 8), seed=3)
    Tc = 0.9                                 # about 40% of the cells lie below
    o.set_profile(Tc=Tc)
    o.set_coefficients(T0, 1.0, 2.5, B)
    F = o.apply(u)
    o.set_profile()
    o.set_coefficients(np.maximum(T0, Tc), 1.0, 2.5, B)
    assert np.array_equal(o.apply(u), F)
    assert 0.2 < np.mean(T0 < Tc) < 0.8


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_fc_profile_folds_into_coefficient(oracle_mod, op):
    """c = scale f_c(r_i) T0 (expo 1) equals the plain operator on
    T0' = f_c(r_i) T0, and without T0 the constant scale f_c(r_i)."""
    mesh, o, T0, B, u, rng = _oracle(oracle_mod, op, (5, 6, 8), seed=4)
    fc = 0.2 + rng.random(mesh.shape[0])
    o.set_profile(fc=fc)
    o.set_coefficients(T0, 2.0, 1.0, B)
    F1 = o.apply(u)
    o.set_coefficients(None, 2.0, 0.0, B)
    F2 = o.apply(u)
    o.set_profile()
    o.set_coefficients(fc[:, None, None] * T0, 2.0, 1.0, B)
    assert np.allclose(F1, o.apply(u), rtol=1e-13, atol=1e-13 * np.abs(F1).max())
    o.set_coefficients(np.broadcast_to(fc[:, None, None], mesh.shape).copy(), 2.0, 1.0, B)
    assert np.allclose(F2, o.apply(u), rtol=1e-14, atol=0)


def test_profile_rejects_bad_values(oracle_mod):
    mesh, o, T0, B, u, rng = _oracle(oracle_mod, "iso7", (3, 4, 6))
    w = np.ones(mesh.shape)
    w[1, 1, 1] = 0.0
    with pytest.raises(ValueError):
        o.set_profile(w)
    with pytest.raises(ValueError):
        o.set_profile(fc=-np.ones(mesh.shape[0]))
