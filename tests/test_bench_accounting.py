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
    ("dir", "aligned", 1, 40 + 8),                    # r, p, x, D; p, x
    ("first", "iso7", 3, 3 * 16),
    ("matvec", "iso7", 3, 3 * 16),
    ("update", "iso7", 3, 3 * 24 + 8),                # 80 B per cell
    ("dir", "iso7", 3, 3 * 40 + 8),                   # 128 B per cell
    ("update", "viscv", 3, 3 * 24 + 8),
    ("dir", "viscv", 3, 3 * 40 + 8),
    ("init", "iso7", 3, 3 * 32 + 16),                 # u, y0, diag L; r, p, D
    ("dir_last", "iso7", 3, 3 * 24),                  # x, p; x
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


def test_dir_saving():
    """One short direction launch per solve that took iterations."""
    f = 8 * N
    per = bench.bytes_per_launch("iso7", 3, "dir", N, NCO, False) - 9 * f
    assert per == 6 * f + 8 * N
    assert bench.dir_saving("iso7", 3, N, NCO, [12, 0, 7, 1]) == 3 * per


def test_fp32_bytes():
    """The FP32 stencil kernels move 4-byte values, corner coefficients
    included (12 B per corner)."""
    assert bench.bytes_per_launch("aligned", 1, "first", N, NCO, False, word=4) == 8 * N + 12 * NCO
    assert bench.bytes_per_launch("viscv", 3, "stage", N, NCO, False, stage_k=5, word=4) == 5 * 12 * N
    assert bench.stage_bytes("viscv", 3, N, NCO, False, [3], word=4) == 3 * 12 * N + 4 * 12 * N
