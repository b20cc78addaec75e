"""Oracle thread control and the host-bandwidth reference used by the CPU
timings (not part of the method): the operator application is computed cell
by cell, so one thread and all threads give bitwise equal results."""
import numpy as np

from paper_2403_01004_amd import inputs


def test_apply_independent_of_threads(oracle_mod):
    oracle = oracle_mod
    prob = inputs.conduction(6, 10, 16, seed=7)
    o = oracle.Oracle.from_problem(prob)
    n0 = oracle.num_threads()
    try:
        F_all = o.apply(prob.u)
        oracle.set_num_threads(1)
        assert oracle.num_threads() == 1
        F_one = o.apply(prob.u)
    finally:
        oracle.set_num_threads(n0)
    assert oracle.num_threads() == n0
    assert np.array_equal(F_all, F_one)


def test_stream_triad_positive(oracle_mod):
    assert oracle_mod.stream_triad(1 << 20, 2) > 0.0
