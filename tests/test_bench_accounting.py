"""The algorithmic-byte accounting behind bench.py's roofline figures (CPU):
per-cell bytes of each kernel class equal the read/write lists of the
kernels (every array the kernel needs read once, every output written once,
FP64, three coefficients per corner of the field-aligned operator)."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

N, NCO = 1000, 1010


@pytest.mark.parametrize("cls,op,nc,per_cell", [
    ("first", "aligned", 1, 16 + 24 * 1.01),          # u, y0 + e
    ("matvec", "aligned", 1, 16 + 24 * 1.01),         # p, q + e
    ("update", "aligned", 1, 24 + 8),                 # r, q, D; r
    ("dir", "aligned", 1, 24 + 8),                    # r, p, D; the next p
    ("first", "iso7", 3, 3 * 16),
    ("matvec", "iso7", 3, 3 * 16),
    ("update", "iso7", 3, 3 * 24 + 8),                # 80 B per cell
    ("dir", "iso7", 3, 3 * 24 + 8),                   # 80 B per cell
    ("update", "viscv", 3, 3 * 24 + 8),
    ("dir", "viscv", 3, 3 * 24 + 8),
    ("init", "iso7", 3, 3 * 32 + 16),                 # u, y0, diag L; r, p, D
    ("xgroup", "iso7", 3, 3 * 16),                    # x read and written once per group
])
def test_bytes_per_cell(cls, op, nc, per_cell):
    got = bench.bytes_per_launch(op, nc, cls, N, NCO, False) / N
    assert got == pytest.approx(per_cell, rel=1e-12)


def test_stage_bytes_per_cycle():
    """Stage k reads u_{k-1}, u_{k-2}, u0, y0 (k >= 4); stage 2 forms u1 on
    the fly (reads u0, y0), stage 3 reads u2, u0, y0; stage 1 is never
    materialised."""
    f = 8 * N
    coef = 24 * NCO
    s = 5
    want = (3 * f + coef) + (4 * f + coef) + 2 * (5 * f + coef)
    assert bench.stage_bytes("aligned", 1, N, NCO, False, [s]) == want
    assert bench.stage_bytes("iso7", 3, N, NCO, False, [3, 2]) == \
        (3 * 3 * f + 4 * 3 * f) + 3 * 3 * f
    # a variable 7-point coefficient adds one read per launch
    assert bench.bytes_per_launch("iso7", 1, "matvec", N, NCO, True) == 2 * f + 8 * N


def test_dir_class_bytes():
    """Per solve of n iterations: n - 1 direction launches (the stopping
    iteration writes no direction), every iteration's direction read once by
    its group's x update, x read and written once per group of 8."""
    f = 8 * N * 3
    d = bench.bytes_per_launch("iso7", 3, "dir", N, NCO, False)
    assert d == 3 * f + 8 * N
    want = (11 * d + 12 * f + 2 * 2 * f) + (6 * d + 7 * f + 1 * 2 * f) + (0 * d + 1 * f + 2 * f)
    assert bench.dir_class_bytes("iso7", 3, N, NCO, [12, 0, 7, 1], 8) == want
    import paper_2403_01004_amd.paradv as paradv
    assert bench.XGROUP == paradv.PA_PCG_XGROUP


def test_fp32_bytes():
    """The FP32 stencil kernels move 4-byte values, corner coefficients
    included (12 B per corner)."""
    assert bench.bytes_per_launch("aligned", 1, "first", N, NCO, False, word=4) == 8 * N + 12 * NCO
    assert bench.bytes_per_launch("viscv", 3, "stage", N, NCO, False, stage_k=5, word=4) == 5 * 12 * N
    assert bench.stage_bytes("viscv", 3, N, NCO, False, [3], word=4) == 3 * 12 * N + 4 * 12 * N


@pytest.mark.parametrize("cls,per_cell", [
    ("update", 3 * 24),        # r, q; r (D from the row terms)
    ("dir", 3 * 24),           # r, p; the next p
    ("init", 3 * 32 + 8),      # u, y0; r, p, D
])
def test_bytes_with_row_diagonal(cls, per_cell):
    """With the point-Jacobi diagonal formed from per-(r, theta) row terms
    (7-point operator, constant coefficient, no weight) the PCG kernels read
    no per-cell D, and the start of a solve reads no diag(L)."""
    got = bench.bytes_per_launch("viscv", 3, cls, N, NCO, False, rows=True) / N
    assert got == pytest.approx(per_cell, rel=1e-12)
    f = 8 * N * 3
    assert bench.dir_class_bytes("viscv", 3, N, NCO, [9], 8, rows=True) == \
        8 * 3 * f + 9 * f + 2 * 2 * f


def test_kernel_accounting_follows_the_flag():
    """kernel_accounting charges the row form only when the advance reports it."""
    s = {"kernel_ms": {"update": 1.0, "dir": 1.0, "init": 1.0},
         "kernel_calls": {"update": 10, "dir": 10, "init": 1},
         "iters_total": 9, "per_cycle": [9]}
    plain = bench.kernel_accounting(dict(s, jacobi_rows=False), "viscv", 3, N, NCO)
    rows = bench.kernel_accounting(dict(s, jacobi_rows=True), "viscv", 3, N, NCO)
    assert plain["update"][2] - rows["update"][2] == 9 * 8 * N
    assert plain["dir"][2] - rows["dir"][2] == 8 * 8 * N
    assert plain["init"][2] - rows["init"][2] == 8 * N
