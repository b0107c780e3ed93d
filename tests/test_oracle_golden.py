"""Regression pin: the oracle's kernel table and correction equal the stored values written
by tests/golden/make_golden.py (which calls only oracle/)."""
import os

import numpy as np

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_kernel_table_golden(orc):
    ref = np.loadtxt(os.path.join(GOLD, "kernel_table_w7_o8.txt"))
    np.testing.assert_allclose(orc.kernel_table(7, 8), ref, rtol=1e-14, atol=0)


def test_correction_golden(orc):
    ref = np.loadtxt(os.path.join(GOLD, "correction_n16_w7.txt"))
    np.testing.assert_allclose(orc.correction(16, 7), ref, rtol=1e-14, atol=0)
