"""Exact earth mover's distance on tiny inputs, independent of the oracle.

Used only to pin the oracle: the entropic distance at convergence lies in
[EMD, EMD + min(H(r), H(c)) / lambda].
"""
import itertools

import numpy as np
from scipy.optimize import linear_sum_assignment, linprog


def emd_bruteforce_uniform(M: np.ndarray) -> float:
    """n x n cost, both sides uniform 1/n: by Birkhoff-von Neumann an optimal
    plan is a permutation matrix / n, so EMD = min_sigma mean M[k, sigma(k)]."""
    n = M.shape[0]
    assert M.shape == (n, n) and n <= 8
    best = np.inf
    for perm in itertools.permutations(range(n)):
        best = min(best, sum(M[k, perm[k]] for k in range(n)) / n)
    return float(best)


def emd_assignment_uniform(M: np.ndarray) -> float:
    rows, cols = linear_sum_assignment(M)
    return float(M[rows, cols].sum() / M.shape[0])


def emd_lp(M: np.ndarray, r: np.ndarray, c: np.ndarray) -> float:
    """Transportation LP: min <P, M>, P 1 = r, P^T 1 = c, P >= 0 (HiGHS)."""
    m, n = M.shape
    A_eq = np.zeros((m + n, m * n))
    for k in range(m):
        A_eq[k, k * n:(k + 1) * n] = 1.0
    for i in range(n):
        A_eq[m + i, i::n] = 1.0
    b_eq = np.concatenate([r, c])
    res = linprog(M.ravel(), A_eq=A_eq, b_eq=b_eq, bounds=(0, None), method="highs")
    assert res.status == 0
    return float(res.fun)


def entropy(p: np.ndarray) -> float:
    p = p[p > 0]
    return float(-(p * np.log(p)).sum())
