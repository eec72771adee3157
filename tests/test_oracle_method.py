"""Pins of the oracle's unfolding, gradient, update and fit.

Checked against brute force (explicit index loops, enumeration of every
sampled row), textbook identities (Kronecker-based Khatri-Rao product, the
CP unfolding identity X_(n) = A^(n) Z^(n)T), closed forms (the variance
theorem, AdaGrad's first step) and exact-rank recovery.
"""

import itertools
import math

import numpy as np
import pytest

import cpd_inputs as ci
import oracle as O
from helpers import factor_match_score, rel_err


def _tiny(dims=(3, 4, 5), R=2, seed=0, noise=True):
    rng = np.random.default_rng(seed)
    As = [rng.standard_normal((I, R)) for I in dims]
    X = ci.cp_full(As)
    if noise:
        X = X + 0.3 * rng.standard_normal(X.shape)
    return X, As


# ------------------------------------------------------- index map, KRP ----

@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 4, 5)])
def test_unfolding_index_map_round_trip(dims):
    rng = np.random.default_rng(1)
    X = rng.standard_normal(dims)
    for n in range(len(dims)):
        Xn = O.unfold(X, n)
        assert Xn.shape == (dims[n], int(np.prod(dims)) // dims[n])
        for multi in itertools.product(*[range(d) for d in dims]):
            j = O.column_index(multi, dims, n)
            assert Xn[multi[n], j] == X[multi]
            back = O.multi_index(j, dims, n)
            assert all(back[k] == multi[k] for k in range(len(dims)) if k != n)


def test_generator_fortran_order():
    # the dense tensor is mode-1 fastest: flat index i_1 + I_1 (i_2 + I_2 i_3)
    _, As = _tiny()
    X = ci.cp_full(As)
    flat = X.ravel(order="K")
    assert X.flags.f_contiguous
    for (a, b, c) in [(0, 0, 0), (2, 1, 3), (1, 3, 4)]:
        assert flat[a + 3 * (b + 4 * c)] == X[a, b, c]


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_krp_textbook_kronecker(n):
    rng = np.random.default_rng(2)
    As = [rng.standard_normal((I, 3)) for I in (2, 3, 4, 2)]
    Z = O.krp(As, n)
    # column r of A^(N) (.) ... (.) A^(1) (skipping n) is kron(a^(N)_r, ..., a^(1)_r)
    others = [As[k] for k in reversed(range(4)) if k != n]
    for r in range(3):
        col = others[0][:, r]
        for A in others[1:]:
            col = np.kron(col, A[:, r])
        assert np.allclose(Z[:, r], col, rtol=1e-15, atol=0)
    assert np.array_equal(Z, O.krp_fast(As, n))


def test_cp_unfolding_identity():
    _, As = _tiny((3, 4, 5, 2), R=3, noise=False)
    X = ci.cp_full(As)
    assert np.allclose(X, O.reconstruct(As), rtol=1e-13, atol=1e-13)
    for n in range(4):
        assert np.allclose(O.unfold(X, n), As[n] @ O.krp(As, n).T, rtol=1e-12, atol=1e-12)


def test_sampled_rows_and_fibres_brute_force():
    X, As = _tiny((3, 4, 5, 2), R=3)
    dims = [3, 4, 5, 2]
    rng = np.random.default_rng(3)
    for n in range(4):
        others = [k for k in range(4) if k != n]
        idx = np.stack([rng.integers(0, dims[k], 6) for k in others], axis=1)
        H = O.sampled_krp_rows(As, n, idx)
        Xs = O.gather_fibres(X, n, idx)
        Z = O.krp(As, n)
        Xn = O.unfold(X, n)
        for f in range(6):
            multi = [0] * 4
            for s, k in enumerate(others):
                multi[k] = int(idx[f, s])
            j = O.column_index(multi, dims, n)
            assert np.array_equal(H[f], Z[j])
            assert np.array_equal(Xs[f], Xn[:, j])


# ------------------------------------------------------------- gradient ----

def _grad_at(o, n, idx):
    p = o.probabilities_at(n, idx)
    return o.gradient(n, idx, p), p


@pytest.mark.parametrize("sampler", [O.UNIFORM, O.EUCLIDEAN, O.LEVERAGE])
@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 4, 3)])
def test_unbiased_by_enumeration(sampler, dims):
    # unbiasedness theorem: sum_j p_j G(j) with B = 1 equals the full gradient
    X, As = _tiny(dims, R=2, seed=4)
    o = O.Oracle(X, As, B=1, sampler=sampler)
    for n in range(len(dims)):
        others = [k for k in range(len(dims)) if k != n]
        acc = np.zeros_like(As[n])
        ptot = 0.0
        for multi in itertools.product(*[range(dims[k]) for k in others]):
            idx = np.array([multi])
            G, p = _grad_at(o, n, idx)
            acc += p[0] * G
            ptot += p[0]
        full = O.full_gradient(X, As, n)
        assert math.isclose(ptot, 1.0, rel_tol=1e-12)
        assert rel_err(acc, full) < 1e-12


def test_full_gradient_finite_difference():
    X, As = _tiny((3, 4, 5), R=2, seed=5)
    n = 1
    G = O.full_gradient(X, As, n)

    def f(A):
        Bs = list(As)
        Bs[n] = A
        D = X - O.reconstruct(Bs)
        return 0.5 * float(np.sum(D * D))

    h = 1e-6
    for (i, r) in [(0, 0), (3, 1), (2, 0)]:
        Ap = As[n].copy()
        Am = As[n].copy()
        Ap[i, r] += h
        Am[i, r] -= h
        assert math.isclose((f(Ap) - f(Am)) / (2 * h), G[i, r], rel_tol=1e-6, abs_tol=1e-8)


def _columns(idx, dims, n):
    """Unfolding columns of the sampled multi-indices (index map)."""
    others = [k for k in range(len(dims)) if k != n]
    cols = []
    for f in range(idx.shape[0]):
        multi = [0] * len(dims)
        for s, k in enumerate(others):
            multi[k] = int(idx[f, s])
        cols.append(O.column_index(multi, dims, n))
    return cols


def test_uniform_is_Jn_times_brascpd():
    # under uniform p the weighted gradient is J_n times Algorithm 2's
    # (1/B)(A Z_F^T Z_F - X^F Z_F), with Z_F taken from the explicit KRP
    X, As = _tiny((3, 4, 5), R=2, seed=6)
    o = O.Oracle(X, As, B=7, sampler=O.UNIFORM, seed=9)
    n, idx, p = o.sample(0)
    G = o.gradient(n, idx, p)
    cols = _columns(idx, [3, 4, 5], n)
    ZF = O.krp(As, n)[cols]
    XF = O.unfold(X, n)[:, cols]
    Jn = 60 // [3, 4, 5][n]
    bras = (As[n] @ ZF.T @ ZF - XF @ ZF) / 7
    assert rel_err(G, Jn * bras) < 1e-13


def test_gradient_vanishes_at_exact_solution():
    _, As = _tiny((4, 5, 6), R=3, noise=False, seed=7)
    X = ci.cp_full(As)
    o = O.Oracle(X, As, B=5, sampler=O.EUCLIDEAN, seed=1)
    for t in range(6):
        n, idx, p = o.sample(t)
        G = o.gradient(n, idx, p)
        assert np.max(np.abs(G)) < 1e-10 * max(1.0, np.max(np.abs(X)))


# ------------------------------------------------------------- variance ----

@pytest.mark.parametrize("sampler", [O.UNIFORM, O.EUCLIDEAN, O.LEVERAGE])
def test_variance_theorem_by_enumeration(sampler):
    X, As = _tiny((3, 4, 5), R=2, seed=8)
    o = O.Oracle(X, As, B=1, sampler=sampler)
    n = 2
    full = O.full_gradient(X, As, n)
    var1 = 0.0
    for a in range(3):
        for b in range(4):
            G, p = _grad_at(o, n, np.array([[a, b]]))
            var1 += p[0] * float(np.sum((G - full) ** 2))
    assert math.isclose(O.exact_variance(X, As, n, sampler, 1), var1, rel_tol=1e-10)
    # batch of two independent draws: enumerate all ordered pairs
    o2 = O.Oracle(X, As, B=2, sampler=sampler)
    rows = [(a, b) for a in range(3) for b in range(4)]
    var2 = 0.0
    for r1 in rows:
        for r2 in rows:
            G, p = _grad_at(o2, n, np.array([r1, r2]))
            var2 += p[0] * p[1] * float(np.sum((G - full) ** 2))
    assert math.isclose(O.exact_variance(X, As, n, sampler, 2), var2, rel_tol=1e-10)


@pytest.mark.parametrize("sampler", [O.UNIFORM, O.EUCLIDEAN, O.LEVERAGE])
def test_variance_table1_forms(sampler):
    X, As = _tiny((5, 6, 4), R=3, seed=9)
    for n in range(3):
        a = O.exact_variance(X, As, n, sampler, 4)
        b = O.variance_table1(X, As, n, sampler, 4)
        assert math.isclose(a, b, rel_tol=1e-9)


def test_variance_monte_carlo():
    X, As = _tiny((5, 6, 4), R=2, seed=10)
    o = O.Oracle(X, As, B=8, sampler=O.EUCLIDEAN, seed=21)
    n_target = 1
    full = O.full_gradient(X, As, n_target)
    devs = []
    t = 0
    while len(devs) < 1500:
        n, idx, p = o.sample(t)
        t += 1
        if n != n_target:
            continue
        G = o.gradient(n, idx, p)
        devs.append(float(np.sum((G - full) ** 2)))
    devs = np.array(devs)
    exact = O.exact_variance(X, As, n_target, O.EUCLIDEAN, 8)
    se = devs.std() / math.sqrt(len(devs))
    assert abs(devs.mean() - exact) < 5 * se


# --------------------------------------------------------------- update ----

def test_adagrad_first_step_is_sign_step():
    X, As = _tiny((4, 5, 6), R=3, seed=11)
    o = O.Oracle(X, As, B=6, sampler=O.LEVERAGE, rule=O.ADAGRAD, eta=0.25, b=0.0, seed=2)
    n, idx, p = o.sample(0)
    G = o.gradient(n, idx, p)
    A_before = o.A[n].copy()
    o.step()
    assert np.allclose(o.A[n], A_before - 0.25 * np.sign(G), rtol=0, atol=1e-15)
    for k in range(3):
        if k != n:
            assert np.array_equal(o.A[k], As[k])


def test_fixed_and_decreasing_steps():
    X, As = _tiny((4, 5, 6), R=3, seed=12)
    o = O.Oracle(X, As, B=6, sampler=O.EUCLIDEAN, rule=O.FIXED, alpha=1e-3, seed=3)
    n, idx, p = o.sample(0)
    G = o.gradient(n, idx, p)
    o.step()
    assert np.allclose(o.A[n], As[n] - 1e-3 * G, rtol=0, atol=1e-15)
    o = O.Oracle(X, As, B=6, sampler=O.EUCLIDEAN, rule=O.DECREASING, beta=0.5,
                 gamma=10.0, seed=3)
    o.step()
    o2 = O.Oracle(X, As, B=6, sampler=O.EUCLIDEAN, rule=O.DECREASING, beta=0.5,
                  gamma=10.0, seed=3)
    n, idx, p = o2.sample(0)
    assert np.allclose(o.A[n], As[n] - 0.05 * o2.gradient(n, idx, p), rtol=0, atol=1e-15)


def test_adagrad_zero_gradient_entries_stay():
    # b = 0 and G = 0 at an entry: the update is 0 there, not NaN
    X, As = _tiny((4, 5, 6), R=3, seed=13)
    As = [a.copy() for a in As]
    As[0][:, 2] = 0.0
    As[1][:, 2] = 0.0
    As[2][:, 2] = 0.0
    o = O.Oracle(X, As, B=4, sampler=O.EUCLIDEAN, rule=O.ADAGRAD, eta=0.5, b=0.0, seed=5)
    o.run(5)
    for A in o.A:
        assert np.all(np.isfinite(A))
        assert np.all(A[:, 2] == 0.0)


def test_nonneg_projection():
    X, As = _tiny((4, 5, 6), R=3, seed=14)
    o = O.Oracle(np.abs(X), [np.abs(a) for a in As], B=4, sampler=O.EUCLIDEAN,
                 rule=O.ADAGRAD, eta=0.5, seed=6, nonneg=True)
    o.run(20)
    assert all(np.all(A >= 0) for A in o.A)


# ------------------------------------------------------------------ fit ----

def test_fit_explicit_vs_gram_identity():
    X, As = _tiny((4, 5, 6), R=3, seed=15)
    Xh = O.reconstruct(As)
    x2 = float(np.sum(X * X))
    inner = float(np.sum(X * Xh))
    gram = 1.0 - (x2 - 2 * inner + O.gram_hadamard_norm2(As)) / x2
    assert math.isclose(O.fit_explicit(X, As), gram, rel_tol=1e-12)
    assert math.isclose(O.gram_hadamard_norm2(As), float(np.sum(Xh * Xh)), rel_tol=1e-12)


def test_fit_at_truth_is_noise_level():
    p = ci.make_problem((20, 21, 22), 4, data_seed=3, init_seed=4, snr_db=30.0)
    X = p["X64"]
    fit = O.fit_explicit(X, p["A_true"])
    Xt = ci.cp_full(p["A_true"])
    expect = 1.0 - float(np.sum((X - Xt) ** 2)) / float(np.sum(X * X))
    assert math.isclose(fit, expect, rel_tol=1e-12)
    # 30 dB: ||noise||^2 / ||X_true||^2 = 1e-3
    assert 0.998 < fit < 0.9995


# -------------------------------------------------------- whole method -----

@pytest.mark.parametrize("sampler", [O.EUCLIDEAN, O.LEVERAGE])
def test_noiseless_exact_rank_recovery(sampler):
    p = ci.make_problem((30, 30, 30), 5, data_seed=1001, init_seed=2001, snr_db=None)
    o = O.Oracle(p["X"], p["A0"], B=18, sampler=sampler, rule=O.ADAGRAD, eta=1.0,
                 b=0.0, seed=3001)
    o.run(1500)
    assert o.fit() > 1 - 1e-8
    assert factor_match_score(o.A, p["A_true"]) > 0.99


def test_iterates_stay_at_truth_noiseless():
    p = ci.make_problem((10, 11, 12), 3, data_seed=5, init_seed=6)
    # fixed step: at the exact solution every sampled gradient is zero up to
    # rounding, so the iterates stay put.  (AdaGrad with b = 0 would not: it
    # normalises rounding-level gradients to steps of size eta.)
    o = O.Oracle(p["X64"], p["A_true"], B=8, sampler=O.EUCLIDEAN, rule=O.FIXED,
                 alpha=1e-3, seed=7)
    o.run(50)
    for A, At in zip(o.A, p["A_true"]):
        assert rel_err(A, At) < 1e-9


# ----------------------------------------- planted mistakes are caught -----

def test_planted_unweighted_gradient_is_biased(monkeypatch):
    """Dropping the 1/p reweighting (a plausible mistake) breaks the
    enumeration pin, so the pin can see it."""
    X, As = _tiny((3, 4, 5), R=2, seed=4)
    o = O.Oracle(X, As, B=1, sampler=O.EUCLIDEAN)
    orig = O.Oracle.gradient

    def wrong(self, n, idx, p):
        return orig(self, n, idx, np.ones_like(p) / 20.0)

    monkeypatch.setattr(O.Oracle, "gradient", wrong)
    n = 0
    acc = np.zeros_like(As[n])
    for b in range(4):
        for c in range(5):
            idx = np.array([[b, c]])
            p = o.probabilities_at(n, idx)
            acc += p[0] * o.gradient(n, idx, p)
    assert rel_err(acc, O.full_gradient(X, As, n)) > 1e-3


def test_planted_transposed_unfolding_is_caught():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((3, 4, 5))
    wrong = np.reshape(np.moveaxis(X, 1, 0), (4, -1), order="C")  # upper modes fastest
    j = O.column_index((2, 0, 3), [3, 4, 5], 1)
    assert wrong[0, j] != X[2, 0, 3]


# ------------------------------------------------------------- rescaling ----

def test_rescale_keeps_the_model_and_balances_norms():
    """Reading R10 against what the mathematics fixes: the CP model is the
    same tensor (compared through a brute-force reconstruction loop), every
    component's columns end with equal norms equal to the geometric mean of
    the old ones (computed as exp of the mean log), a second rescale changes
    nothing, and leverage scores (invariant under column scaling) stay."""
    rng = np.random.default_rng(3)
    dims, R = (5, 4, 6), 3
    As = [rng.standard_normal((I, R)) * rng.uniform(0.01, 50.0, size=R) for I in dims]
    Bs = O.rescale_columns(As)
    Xa = np.zeros(dims)
    Xb = np.zeros(dims)
    for i, j, k in itertools.product(*(range(I) for I in dims)):
        for r in range(R):
            Xa[i, j, k] += As[0][i, r] * As[1][j, r] * As[2][k, r]
            Xb[i, j, k] += Bs[0][i, r] * Bs[1][j, r] * Bs[2][k, r]
    assert rel_err(Xb, Xa) < 1e-13
    for r in range(R):
        old = [np.linalg.norm(A[:, r]) for A in As]
        new = [np.linalg.norm(B[:, r]) for B in Bs]
        g = math.exp(sum(math.log(v) for v in old) / len(old))
        assert all(abs(v - g) <= 1e-12 * g for v in new)
        # each column keeps its direction
        for A, B in zip(As, Bs):
            c = A[:, r] @ B[:, r] / (np.linalg.norm(A[:, r]) * np.linalg.norm(B[:, r]))
            assert abs(c - 1.0) < 1e-14
    Cs = O.rescale_columns(Bs)
    assert all(rel_err(C, B) < 1e-14 for B, C in zip(Bs, Cs))
    for A, B in zip(As, Bs):
        assert np.allclose(O.leverage_scores(A), O.leverage_scores(B), rtol=1e-10, atol=1e-14)


def test_rescale_leaves_degenerate_components():
    """A component with a zero column keeps all of its columns as they were;
    the other components are still balanced."""
    rng = np.random.default_rng(4)
    As = [rng.standard_normal((I, 2)) for I in (3, 4, 5)]
    As[1][:, 0] = 0.0
    Bs = O.rescale_columns(As)
    for A, B in zip(As, Bs):
        assert np.array_equal(A[:, 0], B[:, 0])
    n1 = [np.linalg.norm(B[:, 1]) for B in Bs]
    assert max(n1) - min(n1) <= 1e-12 * max(n1)


def test_oracle_rescale_every_matches_manual_rescaling():
    """rescale_every = k rescales after steps k, 2k, ...: the same draws
    replayed into a plain oracle that is rescaled by hand at those steps
    give the same iterates."""
    X, As = _tiny(dims=(6, 5, 7), R=2, seed=5)
    a = O.Oracle(X, As, B=6, sampler="euclidean", eta=0.2, seed=9, rescale_every=3)
    b = O.Oracle(X, As, B=6, sampler="euclidean", eta=0.2, seed=9)
    for t in range(9):
        n, idx, _ = a.step()
        b.step(replay=(n, idx))
        if (t + 1) % 3 == 0:
            b.A = O.rescale_columns(b.A)
        assert all(rel_err(p, q) < 1e-13 for p, q in zip(a.A, b.A)), t
    assert a.t == 9
