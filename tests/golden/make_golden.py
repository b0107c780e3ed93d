"""Write the stored oracle values under tests/golden/ (calls only oracle/).

The paper prints no worked example or intermediate value (its only numbers are the Table 1
task timings), so every stored value here comes from the oracle and serves as a regression
pin: a later change to the oracle's kernel arithmetic must name the passage that justifies it.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    t = oracle.kernel_table(7, 8)
    np.savetxt(os.path.join(HERE, "kernel_table_w7_o8.txt"), t, fmt="%.17e",
               header="oracle.kernel_table(7, 8): rows = phase -4..3, columns = taps -3..3")
    c = oracle.correction(16, 7)
    np.savetxt(os.path.join(HERE, "correction_n16_w7.txt"), c, fmt="%.17e",
               header="oracle.correction(16, 7): pixels 0..15, x = (p - 8)/16")


if __name__ == "__main__":
    main()
