"""Pins of the oracle's Dirichlet radial closure (Sec. 2, Eqs. visc and tc, with
Dirichlet data at the shell's radial boundaries) against the mathematics, not
against the oracle itself.

The closure under test: the 7-point operator couples a boundary cell to its
Dirichlet value over the half-cell distance between the cell centre and the
boundary face; the field-aligned operator sees a mirror ghost 2 u_b - u at
the boundary corners, whose dual volume is half a radial extent.  Invariants
(symmetry, PSD, steady constants, conservation) hold whatever that distance
or weight is, so these pins use closed forms instead:

* a profile linear in r has an exact finite-volume flux through every radial
  face, the boundary faces included, so F equals the cell average of
  div(c grad u) = 2 c b / r exactly in every cell (7-point operator);
* with bhat = rhat the field-aligned operator acts on a radial profile as the
  radial Laplacian times a per-column factor, so F / F_exact is the same in
  every cell of a column, the two boundary cells included;
* the steady shell solution u = a + b / r (harmonic) with its Dirichlet data:
  the discrete steady state converges at second order in every cell, the
  boundary cells included, and the local truncation error of F in a
  boundary cell stays bounded under refinement (a wrong boundary distance
  or weight gives first order and a 1/h growth).

`test_planted_closure_mistakes_fail` builds copies of the oracle with the
boundary distance or the boundary corner weight doubled and checks that these
pins reject every one of them.
"""
from __future__ import annotations

import json
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2403_01004_amd import inputs  # noqa: E402

A_COEF, B_COEF = 0.3, 1.7          # u = a + b r (linear) or a + b / r (harmonic)


def _radial_oracle(oracle_mod, op, mesh, scale=1.0):
    o = oracle_mod.Oracle(mesh, op, 1, "dirichlet", "dirichlet")
    o.set_coefficients(None, scale, 0.0, inputs.uniform_direction_corners(mesh, 0))
    return o


def _dirichlet_data(o, mesh, prof):
    nt, np_ = mesh.shape[1], mesh.shape[2]
    o.set_bc(np.full((1, nt, np_), prof(mesh.r_faces[0])),
             np.full((1, nt, np_), prof(mesh.r_faces[-1])))


def _column(mesh, prof):
    rc = inputs.cell_centres(mesh)[0]
    return np.broadcast_to(prof(rc)[:, None, None], mesh.shape).copy()


def linear_profile_F(oracle_mod, op, mesh, scale=1.3):
    """(F, F_exact) for u = a + b r with exact Dirichlet data; F_exact is the
    cell average of div(c grad u) = 2 c b / r over the cell's volume:
    3 c b (R+^2 - R-^2) / (R+^3 - R-^3)."""
    o = _radial_oracle(oracle_mod, op, mesh, scale)
    prof = lambda r: A_COEF + B_COEF * r  # noqa: E731
    _dirichlet_data(o, mesh, prof)
    F = o.apply(_column(mesh, prof)[None])[0]
    R = mesh.r_faces
    fe = 3.0 * scale * B_COEF * (R[1:] ** 2 - R[:-1] ** 2) / (R[1:] ** 3 - R[:-1] ** 3)
    return F, np.broadcast_to(fe[:, None, None], mesh.shape)


def steady_shell(oracle_mod, op, nr, nt=4, np_=4):
    """Discrete steady state of F(u) = 0 with the Dirichlet data of the
    harmonic shell solution u = a + b / r, by a dense least-squares solve of
    the operator probed column by column (minimum norm: the corner operator's
    null space, patterns with zero 2 x 2 transverse sums, is orthogonal to the
    column-constant solution for even nt).  Returns (max error over all cells,
    max |F(u_exact)| in the inner and outer boundary cells)."""
    mesh = inputs.shell_mesh(nr, nt, np_, stretch=1.0)
    o = _radial_oracle(oracle_mod, op, mesh)
    prof = lambda r: A_COEF + B_COEF / r  # noqa: E731
    _dirichlet_data(o, mesh, prof)
    N = nr * nt * np_
    A = np.zeros((N, N))
    for n in range(N):
        e = np.zeros(N)
        e[n] = 1.0
        A[:, n] = o.apply(e, affine=False).ravel()
    f0 = o.apply(np.zeros(N)).ravel()          # F(0): the boundary-data part
    u, *_ = np.linalg.lstsq(A, -f0, rcond=None)
    ex = _column(mesh, prof)
    Fe = o.apply(ex[None])[0]
    return float(np.abs(u - ex.ravel()).max()), float(np.abs(Fe[0]).max()), float(np.abs(Fe[-1]).max())


# ------------------------------------------------------------------ checks

def check_linear_iso7(oracle_mod):
    mesh = inputs.shell_mesh(7, 6, 8, stretch=1.05)
    F, fe = linear_profile_F(oracle_mod, "iso7", mesh)
    return float(np.abs(F - fe).max() / np.abs(fe).max())


def check_linear_aligned(oracle_mod):
    """Spread of F / F_exact along r in each column, relative."""
    mesh = inputs.shell_mesh(7, 6, 8, stretch=1.05)
    F, fe = linear_profile_F(oracle_mod, "aligned", mesh)
    ratio = F / fe
    return float((ratio.max(axis=0) - ratio.min(axis=0)).max() / np.abs(ratio).max())


def check_steady(oracle_mod, op):
    """(convergence order of the last two refinements, growth of the
    boundary-cell truncation error over the last refinement)."""
    res = [steady_shell(oracle_mod, op, nr) for nr in (16, 32, 64)]
    order = float(np.log2(res[1][0] / res[2][0]))
    growth = max(res[2][1] / res[1][1], res[2][2] / res[1][2])
    return order, float(growth)


def run_checks(oracle_mod):
    out = {"linear_iso7": check_linear_iso7(oracle_mod),
           "linear_aligned": check_linear_aligned(oracle_mod)}
    for op in ("iso7", "aligned"):
        out[f"steady_{op}"] = check_steady(oracle_mod, op)
    return out


def outcomes(res):
    """Which pins a result set passes (the bars of the tests below)."""
    return {
        "linear_iso7": res["linear_iso7"] <= 1e-12,
        "linear_aligned": res["linear_aligned"] <= 1e-12,
        **{f"steady_{op}": res[f"steady_{op}"][0] >= 1.8 and res[f"steady_{op}"][1] <= 1.1
           for op in ("iso7", "aligned")},
    }


# ------------------------------------------------------------------ tests

def test_linear_profile_exact_iso7(oracle_mod):
    """u linear in r: every radial face flux is exact, so F equals the cell
    average of 2 c b / r in all cells, boundary cells included."""
    assert check_linear_iso7(oracle_mod) <= 1e-12


def test_linear_profile_aligned_radial_field(oracle_mod):
    """bhat = rhat, u linear in r: F / F_exact does not depend on the radial
    index in any column (the boundary cells' ghost and half dual volume give
    the interior flux exactly), and it tends to 1 away from the poles."""
    assert check_linear_aligned(oracle_mod) <= 1e-12
    mesh = inputs.shell_mesh(7, 24, 8, stretch=1.05)
    F, fe = linear_profile_F(oracle_mod, "aligned", mesh)
    tc = inputs.cell_centres(mesh)[1]
    eq = (tc > 1.0) & (tc < np.pi - 1.0)
    assert np.abs(F / fe - 1.0)[:, eq].max() < 5e-3


@pytest.mark.parametrize("op", ["iso7", "aligned"])
def test_steady_shell_second_order_with_boundary_cells(oracle_mod, op):
    """The harmonic shell solution a + b / r: the discrete steady state
    converges at second order in the max norm over all cells, and the
    boundary cells' truncation error of F stays O(1) under refinement."""
    order, growth = check_steady(oracle_mod, op)
    assert order >= 1.8, order
    assert growth <= 1.1, growth


MUTANTS = {
    "7-point inner boundary distance doubled":
        ("if (ir == 0) d = o->rc[0] - o->R[0];", "if (ir == 0) d = 2.0 * (o->rc[0] - o->R[0]);"),
    "7-point outer boundary distance doubled":
        ("else if (ir == o->nr) d = o->R[o->nr] - o->rc[o->nr - 1];",
         "else if (ir == o->nr) d = 2.0 * (o->R[o->nr] - o->rc[o->nr - 1]);"),
    "corner inner boundary dual volume doubled":
        ("*hr = 2.0 * (o->rc[0] - o->R[0]);\n        wr = 0.5 * *hr;",
         "*hr = 2.0 * (o->rc[0] - o->R[0]);\n        wr = *hr;"),
    "corner outer boundary dual volume doubled":
        ("*hr = 2.0 * (o->R[o->nr] - o->rc[o->nr - 1]);\n        wr = 0.5 * *hr;",
         "*hr = 2.0 * (o->R[o->nr] - o->rc[o->nr - 1]);\n        wr = *hr;"),
}


def test_planted_closure_mistakes_fail(tmp_path):
    """Each planted closure mistake (in a copy of the oracle, on the CPU) is
    rejected by at least two of the pins above."""
    src = open(os.path.join(ROOT, "oracle", "oracle.c")).read()
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, name
        d = tmp_path / name.replace(" ", "_")
        shutil.copytree(os.path.join(ROOT, "oracle"), d / "oracle",
                        ignore=shutil.ignore_patterns("*.so*", "__pycache__"))
        (d / "oracle" / "oracle.c").write_text(src.replace(old, new))
        out = subprocess.run([sys.executable, __file__, str(d)], capture_output=True, text=True,
                             timeout=600, check=True).stdout
        ok = outcomes(json.loads(out.strip().splitlines()[-1]))
        assert sum(not v for v in ok.values()) >= 2, (name, ok)


if __name__ == "__main__":
    # run the checks against the oracle copy in sys.argv[1]
    sys.path.insert(0, sys.argv[1])
    import oracle as mutant  # noqa: E402
    assert os.path.dirname(mutant.__file__).startswith(sys.argv[1])
    mutant.build(force=True)
    print(json.dumps(run_checks(mutant)))
