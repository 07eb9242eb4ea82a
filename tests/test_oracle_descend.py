"""The oracle's coefficient descent (gradient descent with Armijo
backtracking on the k-cycle loss) against calculus: at the point where it
stops, central finite differences of the loss vanish, and descent from the
four +-10% sign patterns around M7 reaches the same point."""
import numpy as np

import oracle as O
from paper_2206_05543_amd import M7
from paper_2206_05543_amd.workloads import random_errors


def test_descend_stops_at_a_stationary_point():
    d, N, K = 3, 8, 2
    e0 = random_errors(d, N, 5, 3)["e0"]
    b = np.zeros((N - 1,) * d)
    c0 = np.array(M7) * np.array([1.1, 0.9])
    g0 = O.grad_kcycles(d, N, c0, e0, b, K)[1]
    c, L, steps = O.descend(d, N, c0, e0, b, K)
    assert 0 < steps <= 200
    assert L < O.loss_kcycles(d, N, c0, e0, b, K)
    # central differences of the loss at the result, step 1e-5 relative
    for j in range(2):
        h = 1e-5 * abs(c[j])
        cp, cm = c.copy(), c.copy()
        cp[j] += h
        cm[j] -= h
        fd = (O.loss_kcycles(d, N, cp, e0, b, K) - O.loss_kcycles(d, N, cm, e0, b, K)) / (2 * h)
        assert abs(fd) <= 1e-4 * np.abs(g0).max()


def test_descend_patterns_agree():
    d, N, K = 3, 8, 2
    e0 = random_errors(d, N, 5, 3)["e0"]
    b = np.zeros((N - 1,) * d)
    res = []
    for sx in (1, -1):
        for sy in (1, -1):
            c0 = np.array(M7) * np.array([1 + 0.1 * sx, 1 + 0.1 * sy])
            res.append(O.descend(d, N, c0, e0, b, K)[0])
    for c in res[1:]:
        assert np.max(np.abs(c - res[0]) / np.abs(res[0])) <= 1e-4
