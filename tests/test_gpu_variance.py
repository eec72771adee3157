"""Exact gradient variance on the GPU (variance theorem of Section 4)
against the FP64 oracle's closed form, for every sampler and mode."""

import numpy as np
import pytest

import cpd_inputs as ci
import oracle as O
from parity_util import gpu_decomposition, problem

pytestmark = pytest.mark.gpu

SAMPLERS = ["uniform", "leverage", "euclidean"]


def _check(dec, X, B, modes, tol=2e-5, label=""):
    A = [a.astype(np.float64) for a in dec.factors()]
    for n in modes:
        for s in SAMPLERS:
            var, T, G2 = dec.variance(n, s)
            ref = O.exact_variance(X, A, n, s, B)
            g = O.full_gradient(X, A, n)
            G2ref = float(np.sum(g * g)) / B
            Tref = ref + G2ref
            print(f"{label} mode {n} {s}: var {var:.6e} (oracle {ref:.6e}, rel "
                  f"{abs(var - ref) / ref:.2e}), T {T:.6e} (rel {abs(T - Tref) / Tref:.2e}), "
                  f"|grad|^2/B {G2:.4e} (rel {abs(G2 - G2ref) / max(G2ref, 1e-300):.2e})",
                  flush=True)
            assert abs(T - Tref) <= tol * Tref
            assert abs(G2 - G2ref) <= tol * G2ref
            assert abs(var - ref) <= tol * ref


@pytest.mark.parametrize("dims,R,storage", [((37, 45, 53), 7, "f32"), ((11, 13, 17, 9), 5, "f32"),
                                            ((40, 33, 70), 20, "bf16"), ((40, 38, 42), 33, "f32")])
def test_variance_matches_oracle(dims, R, storage):
    prob = problem(dims, R, storage=storage)
    B = 30
    dec = gpu_decomposition(prob, B, storage=storage, eta=0.3)
    _check(dec, prob["X"], B, range(len(dims)), label=f"{dims} R{R} {storage} start")
    dec.step(150)
    _check(dec, prob["X"], B, range(len(dims)), label=f"{dims} R{R} {storage} t=150")
    dec.close()


def test_variance_full_300cube():
    w = ci.workload(2)
    dec = gpu_decomposition(w, w["B"], storage="f32", eta=5.0, seed=w["seed"])
    dec.step(100)
    _check(dec, w["X"], w["B"], [0], label="300^3 t=100")
    dec.close()


def test_importance_beats_uniform_on_skewed_factors():
    """The paper's observation: on factors with large maximal leverage scores
    the importance samplers' variance is far below uniform sampling's."""
    w = ci.workload(2)   # 10 % of the rows of every factor scaled by 20
    dec = gpu_decomposition(w, w["B"], storage="f32", eta=5.0, seed=w["seed"])
    dec.step(200)
    v = {s: dec.variance(0, s)[0] for s in SAMPLERS}
    print(v)
    assert v["euclidean"] < 0.5 * v["uniform"] and v["leverage"] < 0.5 * v["uniform"]
    dec.close()
