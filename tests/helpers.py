"""Small helpers shared by the tests (metrics only, no method arithmetic)."""

import numpy as np
from scipy.optimize import linear_sum_assignment


def factor_match_score(A_est, A_true):
    """Mean over matched components of prod_k |cos(a_r^(k), a_hat^(k))|,
    components matched by the best permutation (Hungarian assignment)."""
    R = A_true[0].shape[1]
    Re = A_est[0].shape[1]
    score = np.ones((R, Re))
    for At, Ae in zip(A_true, A_est):
        nt = At / np.linalg.norm(At, axis=0, keepdims=True)
        ne = Ae / np.maximum(np.linalg.norm(Ae, axis=0, keepdims=True), 1e-300)
        score *= np.abs(nt.T @ ne)
    rows, cols = linear_sum_assignment(-score)
    return float(np.mean(score[rows, cols]))


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
