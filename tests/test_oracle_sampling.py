"""Pins of the oracle's random stream, distributions and sampler.

Every check here compares the oracle with something other than itself: an
independent Philox implementation and published known answers, brute force,
textbook identities and chi-squared goodness of fit.
"""

import math
import os

import numpy as np
import pytest
from scipy import stats

import cpd_inputs as ci
import oracle as O
from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox ----

def _numpy_block(ctr, key):
    """One Philox4x64-10 block from numpy's implementation.  numpy bumps the
    128..256-bit counter before it generates, so start one below."""
    c = [int(x) for x in ctr]
    for i in range(4):  # decrement with borrow
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = 2**64 - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    return [int(v) for v in bg.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (3002, 0)),
    ((12345, 7, 0, 0), (3002, 63)),
    ((2**64 - 1, 2**63, 5, 9), (2**64 - 1, 17)),
])
def test_philox_matches_numpy(ctr, key):
    assert list(philox.philox4x64(ctr, key)) == _numpy_block(ctr, key)


def test_philox_known_answers():
    path = os.path.join(GOLDEN, "philox4x64_10_kat.txt")
    n = 0
    for line in open(path):
        if not line.strip() or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        assert list(philox.philox4x64(w[0:4], w[4:6])) == w[6:10]
        n += 1
    assert n == 3


def test_draw_layout():
    # draw d of step t is word d % 4 of counter (t, d // 4, 0, 0)
    words = philox.draw_words(11, 3, 9, 10)
    for d in range(10):
        assert words[d] == philox.philox4x64((9, d // 4, 0, 0), (11, 3))[d % 4]
        assert words[d] == philox.draw_word(11, 3, 9, d)


def test_mulhi64():
    rng = np.random.default_rng(0)
    for _ in range(200):
        u = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        n = int(rng.integers(1, 2**53))
        assert philox.mulhi64(u, n) == (u * n) // 2**64
        assert 0 <= philox.mulhi64(u, n) < n


# ------------------------------------------------------- distributions -----

def test_euclidean_weights_closed_form():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((17, 6)).astype(np.float32).astype(np.float64)
    w = O.euclidean_weights(A)
    assert np.array_equal(w, np.array([math.fsum(A[i] ** 2) for i in range(17)])) or \
        np.allclose(w, [math.fsum(A[i] ** 2) for i in range(17)], rtol=1e-15)


def test_euclidean_product_normalisation():
    # sum over all multi-indices of prod_k ||A^(k)(i_k,:)||^2 = prod_k ||A^(k)||_F^2
    rng = np.random.default_rng(2)
    As = [rng.standard_normal((I, 3)) for I in (4, 5, 6)]
    ws = [O.euclidean_weights(A) for A in As]
    total = sum(ws[0][a] * ws[1][b] * ws[2][c]
                for a in range(4) for b in range(5) for c in range(6))
    assert math.isclose(total, np.prod([np.sum(A * A) for A in As]), rel_tol=1e-12)


def test_leverage_properties():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((40, 7))
    ell = O.leverage_scores(A)
    assert math.isclose(float(np.sum(ell)), 7.0, rel_tol=1e-12)
    assert np.all(ell >= 0) and np.all(ell <= 1 + 1e-12)
    # any orthonormal basis gives the same scores: SVD basis and the hat matrix
    U, _, _ = np.linalg.svd(A, full_matrices=False)
    assert np.allclose(ell, np.sum(U * U, axis=1), rtol=1e-10, atol=1e-14)
    hat = np.diag(A @ np.linalg.solve(A.T @ A, A.T))
    assert np.allclose(ell, hat, rtol=1e-10, atol=1e-14)
    # square full-rank factor: every row has leverage 1
    Sq = rng.standard_normal((7, 7))
    assert np.allclose(O.leverage_scores(Sq), 1.0, atol=1e-12)


def test_leverage_rank_deficient():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((20, 4))
    A[:, 3] = A[:, 1]
    with pytest.raises(O.RankDeficient):
        O.leverage_scores(A)
    with pytest.raises(O.RankDeficient):
        O.leverage_scores(rng.standard_normal((3, 5)))


def test_lemma1_krp_leverage_bound():
    # leverage of a row of the explicit KRP <= product of factor leverages (I_k > R)
    rng = np.random.default_rng(5)
    As = [rng.standard_normal((I, 3)) for I in (5, 6, 4)]
    n = 1
    Z = O.krp(As, n)
    lz = O.leverage_scores(Z)
    la = [O.leverage_scores(A) for k, A in enumerate(As) if k != n]
    for j in range(Z.shape[0]):
        mi = O.multi_index(j, [5, 6, 4], n)
        bound = la[0][mi[0]] * la[1][mi[2]]
        assert lz[j] <= bound * (1 + 1e-10) + 1e-15


def test_lemma3_krp_row_norm_bound():
    rng = np.random.default_rng(6)
    for R in (1, 4):
        As = [rng.standard_normal((I, R)) for I in (3, 4, 5)]
        n = 0
        Z = O.krp(As, n)
        for j in range(Z.shape[0]):
            mi = O.multi_index(j, [3, 4, 5], n)
            prod = np.sum(As[1][mi[1]] ** 2) * np.sum(As[2][mi[2]] ** 2)
            z2 = np.sum(Z[j] ** 2)
            assert z2 <= prod * (1 + 1e-12)
            if R == 1:
                assert math.isclose(z2, prod, rel_tol=1e-12)


def test_quantize_integer_cdf():
    rng = np.random.default_rng(7)
    for I in (1, 2, 3, 17, 300, 512):
        w = rng.random(I) ** 3
        w[rng.integers(0, I)] = 0.0 if I > 1 else 1.0
        q, C, Q = O.quantize(w)
        assert np.all(q == np.floor(q)) and np.all(q >= 0)
        assert Q < 2**53
        # zero weights never drawn, non-zero weights always reachable
        assert np.all((q == 0) == (w == 0))
        # exact integer prefix sums: independent of the order of summation
        assert C[-1] == math.fsum(q) == float(sum(int(v) for v in q[::-1]))
        assert np.array_equal(C, np.array([float(sum(int(v) for v in q[:i + 1]))
                                           for i in range(I)]))
        # q / Q close to w / sum(w)
        assert np.allclose(q / Q, w / w.sum(), rtol=0, atol=I * 2.0**-48)


def test_quantize_degenerate():
    with pytest.raises(O.Degenerate):
        O.quantize(np.zeros(5))
    with pytest.raises(O.Degenerate):
        O.quantize(np.array([1.0, np.nan]))


def test_inverse_cdf_brute_force():
    rng = np.random.default_rng(8)
    w = rng.random(23)
    w[[3, 4, 10]] = 0.0
    q, C, Q = O.quantize(w)
    Ci = [int(c) for c in C]
    for _ in range(2000):
        u = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        target = (u * int(Q)) >> 64
        expect = next(i for i, c in enumerate(Ci) if c > target)
        assert O.inverse_cdf(C, Q, u) == expect
    # extremes of the 64-bit word
    assert O.inverse_cdf(C, Q, 0) == next(i for i in range(23) if q[i] > 0)
    assert O.inverse_cdf(C, Q, 2**64 - 1) == max(i for i in range(23) if q[i] > 0)


def test_product_probabilities_sum_to_one():
    rng = np.random.default_rng(9)
    As = [rng.standard_normal((I, 3)) for I in (4, 5, 6, 3)]
    for sampler in (O.UNIFORM, O.EUCLIDEAN, O.LEVERAGE):
        for n in range(4):
            P = O.row_probabilities(As, n, sampler)
            assert P.shape == (int(np.prod([d for k, d in enumerate((4, 5, 6, 3)) if k != n])),)
            assert math.isclose(float(np.sum(P)), 1.0, rel_tol=1e-12)


# --------------------------------------------------------- chi-squared -----

def _oracle_for(As, B, sampler, seed=77):
    dims = [A.shape[0] for A in As]
    X = np.zeros(dims)
    return O.Oracle(X, As, B=B, sampler=sampler, seed=seed)


@pytest.mark.parametrize("sampler", [O.EUCLIDEAN, O.LEVERAGE, O.UNIFORM])
def test_chi2_joint_multi_index(sampler):
    # Lemmas 2/4: independent per-mode draws give the product distribution
    rng = np.random.default_rng(10)
    As = [rng.standard_normal((I, 2)) * rng.random((I, 1)) * 3 for I in (4, 5, 3)]
    o = _oracle_for(As, B=64, sampler=sampler)
    counts = {}
    for t in range(400):
        n, idx, p = o.sample(t)
        for f in range(idx.shape[0]):
            key = (n,) + tuple(int(v) for v in idx[f])
            counts[key] = counts.get(key, 0) + 1
    for n in range(3):
        P = O.row_probabilities(As, n, sampler)
        dims = [4, 5, 3]
        obs = np.zeros(P.shape[0])
        for key, c in counts.items():
            if key[0] != n:
                continue
            multi = [0, 0, 0]
            s = 0
            for k in range(3):
                if k != n:
                    multi[k] = key[1 + s]
                    s += 1
            obs[O.column_index(multi, dims, n)] += c
        tot = obs.sum()
        assert tot > 3000
        keep = P * tot >= 5
        exp = P[keep] * tot
        o_k = obs[keep]
        chi = stats.chisquare(o_k, exp * o_k.sum() / exp.sum())
        assert chi.pvalue > 1e-3, (n, chi)


def test_chi2_mode_draw():
    counts = np.zeros(4)
    for t in range(4000):
        counts[O.mode_draw(5, 1, t, 4)] += 1
    assert stats.chisquare(counts).pvalue > 1e-3


def test_chi2_marginal_large():
    # one factor, many draws: marginal frequencies follow q / Q
    rng = np.random.default_rng(11)
    A = rng.standard_normal((50, 4))
    A[:5] *= 20.0
    q, C, Q = O.distribution(A, O.EUCLIDEAN)
    words = []
    for t in range(500):
        words.extend(philox.draw_words(123, 0, t, 200))
    obs = np.bincount([O.inverse_cdf(C, Q, u) for u in words], minlength=50)
    exp = q / Q * len(words)
    keep = exp >= 5
    chi = stats.chisquare(obs[keep], exp[keep] * obs[keep].sum() / exp[keep].sum())
    assert chi.pvalue > 1e-3


def test_sample_probabilities_match_distribution():
    p = ci.make_problem((6, 7, 5), 3, data_seed=1, init_seed=2)
    o = O.Oracle(p["X"], p["A0"], B=9, sampler=O.EUCLIDEAN, seed=4)
    n, idx, pf = o.sample(3)
    assert np.allclose(pf, o.probabilities_at(n, idx), rtol=0, atol=0)
    P = O.row_probabilities(o.A, n, O.EUCLIDEAN)
    dims = o.dims
    for f in range(9):
        multi = [0] * 3
        s = 0
        for k in range(3):
            if k != n:
                multi[k] = int(idx[f, s])
                s += 1
        assert math.isclose(pf[f], P[O.column_index(multi, dims, n)], rel_tol=1e-14)
