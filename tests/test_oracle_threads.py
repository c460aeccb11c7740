"""The oracle's thread count (used only to time it on all host cores) changes
no bit: red-black half sweeps update cells that do not read each other, and
every sum over cells stays sequential in cell order."""
import ctypes as C

import numpy as np

import oracle
from paper_1608_06721_amd import workloads as W


def test_threads_change_no_bit():
    L = oracle.lib()
    L.orc_get_threads.restype = C.c_int
    prob = W.channel(64, 32, n_levels=3, gamma=2, max_newton=3, eps_p=0.2)
    out = []
    try:
        for th in (1, 4):
            L.orc_set_threads(th)
            assert L.orc_get_threads() == th
            U, st = oracle.newton_solve(prob, tol=0.0)
            A, b, tot = oracle.assemble(prob, U)
            out.append((U, st["res_hist"], st["init_sweeps"], A, b, tot))
    finally:
        L.orc_set_threads(1)
    (U1, h1, s1, A1, b1, t1), (U4, h4, s4, A4, b4, t4) = out
    assert s1 == s4 and s1 > 0
    np.testing.assert_array_equal(U1, U4)
    np.testing.assert_array_equal(h1, h4)
    np.testing.assert_array_equal(A1, A4)
    np.testing.assert_array_equal(b1, b4)
    assert t1 == t4
