"""Hand-derived kernel values (tests/golden/kernel_values.txt) against the
oracle's evaluation with the leaf size at least N, where K~ is the kernel
matrix itself (Section 2.1: one node, one near block).  Pins the kernel
definitions the compression and the blocks are built from: the 2h^2 of the
Gaussian (Section 1) and the unsquared distance of the Laplace kernel."""
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle.oracle import OracleH2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kernel_values.txt")
CORNERS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [1.0, 1.0, 0.0], [1.0, 1.0, 1.0]])
KERNELS = {"gaussian": wl.KERNEL_GAUSSIAN, "laplace": wl.KERNEL_LAPLACE}


def rows():
    out = []
    for line in open(GOLDEN):
        line = line.split("#", 1)[0].split()
        if line:
            k, h, i, j, num, den, sq = line
            x = math.sqrt(int(num)) if sq == "1" else float(num)
            out.append((k, float(h), int(i), int(j), math.exp(-x / int(den))))
    return out


@pytest.mark.parametrize("kernel,h", sorted({(r[0], r[1]) for r in rows()}))
def test_kernel_matrix_matches_closed_forms(kernel, h):
    w = wl.small("corners", N=4, d=3, m=4, kernel=KERNELS[kernel], h=h, Q=4)
    H = OracleH2.from_workload(w, CORNERS)
    assert H.n_nodes == 1 and H.n_near == 1 and H.n_far == 0
    K = H.eval(np.eye(4))
    checked = 0
    for k, hh, i, j, v in rows():
        if (k, hh) != (kernel, h):
            continue
        assert abs(K[i, j] - v) <= 1e-15 * v, (i, j, K[i, j], v)
        assert K[j, i] == K[i, j]  # symmetric kernel evaluation, bitwise
        checked += 1
    assert checked >= 3
    np.testing.assert_array_equal(np.diag(K), np.ones(4))  # r = 0
