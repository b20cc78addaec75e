"""Pins of the oracle's block ILU(0) preconditioner (PC2 of Sec. 3.1,
non-overlapping ILU(0)) for the 7-point and the field-aligned operators
(the latter couples each cell's 3 x 3 x 3 neighbourhood).

The factors are tied to the operator and to the definition of ILU(0) by
checks that do not run the oracle's elimination again:
  - the block-diagonal matrix equals M = wV + dt L read column by column
    from the operator apply, with every coupling between boxes (and the
    periodic phi wrap) removed;
  - (L U)_ij = M_ij on the sparsity pattern of M, with L unit lower and U
    upper in that pattern: the property that defines ILU(0);
  - boxes that are lines (radial or longitudinal) make each block
    tridiagonal, where ILU(0) is the exact LU: P^{-1} r equals a dense solve;
  - boxes of one cell reduce PC2 to point Jacobi (PC1), bit for bit;
  - PCG with PC2 reaches the dense Backward Euler solution."""
import numpy as np
import pytest

from paper_2403_01004_amd import inputs


def _problem(oracle_mod, shape=(5, 6, 8), seed=0, weighted=False, bc="dirichlet", op="iso7"):
    mesh = inputs.shell_mesh(*shape)
    rng = np.random.default_rng(seed)
    if op == "aligned":
        prob = inputs.conduction(*shape, seed=300 + seed, noise_amp=0.05)
        prob.bc_in = prob.bc_out = bc
        o = oracle_mod.Oracle.from_problem(prob)
        u = prob.u
    else:
        o = oracle_mod.Oracle(mesh, "iso7", 2, bc, bc)
        o.set_coefficients(0.5 + rng.random(mesh.shape), 1.0, 2.5)
        o.set_bc(rng.random((2,) + mesh.shape[1:]), rng.random((2,) + mesh.shape[1:]))
        u = rng.random((2,) + mesh.shape)
    if weighted:
        o.set_profile(0.5 + rng.random(mesh.shape))
    return mesh, o, u, rng


def _dense_M(o, dt):
    """M = wV + dt L column by column from the linear part of the operator
    (L x = -wV F_lin(x))."""
    wV = o.volumes(weighted=True).ravel()
    n = wV.size
    M = np.empty((n, n))
    e = np.zeros((o.nc, o.nr, o.nt, o.np))
    for q in range(n):
        e[0].ravel()[q] = 1.0
        M[:, q] = -dt * wV * o.apply(e, affine=False)[0].ravel()
        M[q, q] += wV[q]
        e[0].ravel()[q] = 0.0
    return M


def _box_mask(shape, block):
    nr, nt, npp = shape
    I, J, K = np.unravel_index(np.arange(nr * nt * npp), shape)
    box = (I // block[0]) * 1000000 + (J // block[1]) * 1000 + K // block[2]
    same = box[:, None] == box[None, :]
    # couplings across the periodic phi wrap (k = np-1 <-> 0) never enter the blocks
    wrap = np.abs(K[:, None] - K[None, :]) == npp - 1
    return same & ~wrap


def _dense_csr(rowp, col, val, n):
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rowp[i]:rowp[i + 1]]] = val[rowp[i]:rowp[i + 1]]
    return A


OPS = ["iso7", "aligned"]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("block,weighted", [((2, 4, 3), False), ((3, 2, 5), True)])
def test_block_matrix_is_the_operator(oracle_mod, block, weighted, op):
    mesh, o, u, rng = _problem(oracle_mod, seed=1, weighted=weighted, op=op)
    dt = 7.0 * o.dt_explicit()
    o.set_pc("bilu0", block)
    rowp, col, m0, lu = o.bilu0_csr(dt)
    n = o.nr * o.nt * o.np
    M = _dense_M(o, dt)
    Mb = np.where(_box_mask(mesh.shape, block), M, 0.0)
    A = _dense_csr(rowp, col, m0, n)
    assert np.abs(A - Mb).max() <= 1e-13 * np.abs(M).max()
    # pattern: exactly the nonzeros of the block-diagonal part, columns ascending
    assert np.array_equal(A != 0, Mb != 0)
    for i in range(n):
        c = col[rowp[i]:rowp[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    # boxes are proper: couplings between boxes exist in M and are dropped
    assert np.count_nonzero(M) > np.count_nonzero(Mb)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("block", [(2, 4, 3), (5, 6, 8), (3, 2, 5)])
def test_ilu0_defining_property(oracle_mod, block, op):
    """L unit lower and U upper with the sparsity of M, and L U = M on that
    sparsity (the fill outside it is what ILU(0) drops)."""
    mesh, o, u, rng = _problem(oracle_mod, seed=2, op=op)
    dt = 20.0 * o.dt_explicit()
    o.set_pc("bilu0", block)
    rowp, col, m0, lu = o.bilu0_csr(dt)
    n = o.nr * o.nt * o.np
    A = _dense_csr(rowp, col, m0, n)
    F = _dense_csr(rowp, col, lu, n)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    pat = A != 0
    LU = L @ U
    assert np.abs(LU[pat] - A[pat]).max() <= 1e-13 * np.abs(A).max()
    assert np.all(F[~pat] == 0.0)
    assert np.all(np.diag(U) > 0.0)
    # the whole-box case has fill: L U differs from M off the pattern
    if block == (5, 6, 8):
        assert np.abs(LU[~pat]).max() > 1e-6 * np.abs(A).max()
    # symmetric M: U = diag(U) L^T (ILU(0) is incomplete Cholesky here)
    assert np.allclose(U, np.diag(np.diag(U)) @ L.T, rtol=1e-12, atol=1e-14 * np.abs(A).max())


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("line", ["radial", "longitude"])
def test_line_boxes_are_exact(oracle_mod, line, op):
    """Tridiagonal blocks have no fill: P^{-1} r is the exact solve with
    the block-diagonal matrix."""
    mesh, o, u, rng = _problem(oracle_mod, seed=3, op=op)
    block = (o.nr, 1, 1) if line == "radial" else (1, 1, o.np)
    dt = 30.0 * o.dt_explicit()
    o.set_pc("bilu0", block)
    n = o.nr * o.nt * o.np
    Mb = np.where(_box_mask(mesh.shape, block), _dense_M(o, dt), 0.0)
    r = rng.standard_normal((o.nc, o.nr, o.nt, o.np))
    z = o.precondition(r, dt)
    for c in range(o.nc):
        zd = np.linalg.solve(Mb, r[c].ravel())
        assert np.linalg.norm(z[c].ravel() - zd) <= 1e-13 * np.linalg.norm(zd)
    assert n == Mb.shape[0]


@pytest.mark.parametrize("op", OPS)
def test_unit_boxes_are_jacobi(oracle_mod, op):
    mesh, o, u, rng = _problem(oracle_mod, seed=4, weighted=True, op=op)
    dt = 25.0 * o.dt_explicit()
    r = rng.standard_normal((o.nc, o.nr, o.nt, o.np))
    zj = o.precondition(r, dt)
    xj, sj = o.advance_be(u, dt, tol=1e-10, cycles=2)
    o.set_pc("bilu0", (1, 1, 1))
    assert np.array_equal(o.precondition(r, dt), zj)
    xb, sb = o.advance_be(u, dt, tol=1e-10, cycles=2)
    assert np.array_equal(xb, xj) and sb["iters_total"] == sj["iters_total"]
    # and the Jacobi preconditioner is r / (wV + dt diag L)
    D = o.volumes(weighted=True) + dt * o.diag()
    assert np.allclose(zj, r / D[None], rtol=1e-15, atol=0)


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("bc", ["dirichlet", "noflux"])
def test_bilu0_pcg_reaches_dense_solve(oracle_mod, bc, op):
    mesh, o, u, rng = _problem(oracle_mod, shape=(4, 5, 6), seed=5, weighted=True, bc=bc, op=op)
    dt = 40.0 * o.dt_explicit()
    o.set_pc("bilu0", (2, 3, 4))
    M = _dense_M(o, dt)
    wV = o.volumes(weighted=True).ravel()
    h = wV[None] * o.apply(np.zeros_like(u)).reshape(o.nc, -1)
    xo, st = o.advance_be(u, dt, tol=1e-14, cycles=1)
    assert st["status"] == 0
    for c in range(o.nc):
        x = np.linalg.solve(M, wV * u[c].ravel() + dt * h[c])
        assert np.linalg.norm(xo[c].ravel() - x) <= 1e-11 * np.linalg.norm(x)


def test_bilu0_fewer_iterations(oracle_mod):
    """PC2 needs fewer PCG iterations than PC1 (Sec. 3.1) on the isotropic
    workloads' recipes at dt = 50 dt_E."""
    for prob in (inputs.viscosity(16, 24, 32), inputs.heat_iso(16, 24, 32)):
        o = oracle_mod.Oracle.from_problem(prob)
        dt = 50.0 * o.dt_explicit()
        _, sj = o.advance_be(prob.u, dt, tol=1e-10, cycles=1)
        o.set_pc("bilu0", (8, 4, 16))
        _, sb = o.advance_be(prob.u, dt, tol=1e-10, cycles=1)
        assert sb["status"] == 0 and sb["rel_residual"] <= 1e-10
        assert sb["iters_total"] <= 0.6 * sj["iters_total"], (sb["iters_total"], sj["iters_total"])


def test_bilu0_fewer_iterations_field_aligned(oracle_mod):
    """PC2 on the field-aligned operator (its 27-point sparsity fills within
    itself, so the factors differ from M off the diagonal too): fewer PCG
    iterations than PC1 on the conduction and transition-region recipes at
    dt = 50 dt_E (measured 43 against 79 and 57 against 82 at 24 x 48 x 64),
    at the same true residual."""
    for prob, bound in ((inputs.conduction(24, 48, 64), 0.65),
                        (inputs.transition_region(24, 48, 64, i_tr0=7.0, i_amp=2.0, width=3.0), 0.8)):
        o = oracle_mod.Oracle.from_problem(prob)
        dt = 50.0 * o.dt_explicit()
        _, sj = o.advance_be(prob.u, dt, tol=1e-10, cycles=1)
        o.set_pc("bilu0", (8, 4, 16))
        _, sb = o.advance_be(prob.u, dt, tol=1e-10, cycles=1)
        assert sb["status"] == 0 and sb["rel_residual"] <= 1e-10
        assert sb["iters_total"] <= bound * sj["iters_total"], (sb["iters_total"], sj["iters_total"])


def test_bilu0_rejects(oracle_mod):
    mesh = inputs.shell_mesh(3, 4, 6)
    o = oracle_mod.Oracle(mesh, "viscv", 3)
    with pytest.raises(ValueError):
        o.set_pc("bilu0", (2, 2, 2))
    o = oracle_mod.Oracle(mesh, "iso7", 1)
    with pytest.raises(ValueError):
        o.set_pc("bilu0", (0, 2, 2))


MUTANTS = {
    "longitude colours that repeat across the wrap":
        ("return np % 3 == 0 ? 3 : np % 4 == 0 ? 4 : np % 5 == 0 ? 5 : np;", "return 3;"),
    "offsets with dj and dk swapped":
        ("const int i2 = i + t / 9 - 1, j2 = j + (t / 3) % 3 - 1, k2 = k + t % 3 - 1;",
         "const int i2 = i + t / 9 - 1, j2 = j + t % 3 - 1, k2 = k + (t / 3) % 3 - 1;"),
    "probe not scaled by the volume":
        ("const double Lm = -F[m] * wvol(o, i, j, k);", "const double Lm = -F[m];"),
    "coupling with the wrong sign":
        (": dt * Lc[27 * (size_t)m + t];", ": -dt * Lc[27 * (size_t)m + t];"),
}


def test_planted_mistakes_fail(tmp_path):
    """Each planted mistake in the field-aligned block assembly (in a copy of
    the oracle, on the CPU) fails at least two of the pins above."""
    import os
    import shutil
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    src = open(os.path.join(root, "oracle", "oracle.c")).read()
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        d = tmp_path / name.replace(" ", "_")
        shutil.copytree(os.path.join(root, "oracle"), d / "oracle",
                        ignore=shutil.ignore_patterns("*.so*", "__pycache__"))
        (d / "oracle" / "oracle.c").write_text(src.replace(old, new))
        # run from the copy's folder, so that its `oracle` is the one imported
        env = dict(os.environ, PYTHONPATH=f"{d}{os.pathsep}{root}")
        out = subprocess.run([sys.executable, "-m", "pytest", __file__, "-q", "-p",
                              "no:cacheprovider", "-k", "aligned and not planted"], cwd=d,
                             env=env, capture_output=True, text=True, timeout=600).stdout
        m = [ln for ln in out.splitlines() if " failed" in ln]
        nfail = int(m[-1].split(" failed")[0].split()[-1]) if m else 0
        assert nfail >= 2, (name, out[-400:])
