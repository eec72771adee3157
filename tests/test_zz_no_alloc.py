"""cpd_variance_noalloc (the variance entry point that allocates nothing: its
scratch is the library's static per-device array) against cpd_variance with
a caller-owned scratch, through the C ABI: two calls in a row, the second on
a smaller problem, each bit for bit equal to the workspace entry point and
within the oracle's tolerance of the closed form."""

import numpy as np
import pytest

import cpd_inputs as ci
import oracle as O
from parity_util import gpu_decomposition, problem

pytestmark = pytest.mark.gpu


def _noalloc(dec, n, sampler):
    import paper_2103_04081_amd.cpdmi as C
    return C.cpd_variance_noalloc(dec.h, n, sampler)


def _check(dec, X, B, n, sampler):
    ws = dec.variance(n, sampler)
    na = _noalloc(dec, n, sampler)
    assert na == ws, (na, ws)
    ref = O.exact_variance(X, [a.astype(np.float64) for a in dec.factors()], n, sampler, B)
    print(f"mode {n} {sampler}: no-alloc {na[0]:.9e}, workspace {ws[0]:.9e}, oracle {ref:.9e}",
          flush=True)
    assert abs(na[0] - ref) <= 2e-5 * ref


def test_noalloc_variance_two_calls_second_smaller():
    print("CASE noalloc variance", flush=True)
    w = ci.workload(2)   # 300^3, R 10, B 256
    big = gpu_decomposition(w, w["B"], storage="f32", eta=0.5, seed=w["seed"])
    big.step(50)
    _check(big, w["X"], w["B"], 0, "euclidean")
    prob = problem((37, 45, 53), 7)
    small = gpu_decomposition(prob, 30, eta=0.3)
    small.step(20)
    _check(small, prob["X"], 30, 2, "leverage")
    # and the large one again after the small one
    _check(big, w["X"], w["B"], 1, "uniform")
    big.close()
    small.close()
