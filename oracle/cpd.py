"""FP64 CPU oracle of block-randomized SGD with importance sampling for CP.

TEST INFRASTRUCTURE.  Only the test-suite, the package's smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the HIP library and never calls it.

Everything here is plain numpy in float64, written in the order of the
paper's algorithms so it can be read against them:

* unfolding and index map ......... Section 1, the mode-n unfolding map
* Khatri-Rao rows .................. Section 2, Hadamard form of KRP rows
* fibre gather (SKRP-ST) ........... Section 2, Algorithm 1
* per-mode distributions ........... Section 3.1, the leverage-score and
                                     Euclidean-norm definitions and the
                                     product lemmas (Lemmas 2 and 4)
* SKRP-ST-I ....................... Section 3.1, Algorithm 3
* reweighted gradient / update ..... Section 3.2, the weighted stochastic
                                     gradient, fixed-step update and the
                                     AdaGrad step (Algorithms 4 and 5)
* relative error Tol ............... Section 5.2
* full gradient, variance .......... Section 4 (Theorem on unbiasedness,
                                     variance theorem and Table 1)

Readings taken where the paper is silent or inconsistent (each is argued in
the design notes):

R1  Gradient scale.  The weight of sampled fibre f is w_f = 1 / (B p_f), so
    that E[G] equals the gradient of f = 1/2 ||X - [[A]]||^2 exactly (the
    unbiasedness theorem).  The printed prefactor 1/(B J_n) of the weighted
    gradient would give J_n times less; under uniform p this reading is J_n
    times the BrasCPD gradient.
R2  Operand placement.  G = A^(n) (H^T W H) - X_s^T W H with H = Z_F (B x R),
    X_s the gathered fibres stored B x I_n, W = diag(w).
R3  Randsample.  Philox4x64-10 counter stream (oracle.philox) and inverse
    CDF sampling on an integer-valued float64 CDF: with w the row weights,
    q_i = ceil(w_i * 2^E) where 2^E * max(w) * 2^ceil(log2 I) < 2^53 is the
    largest such power of two computed from the exponent of max(w), so every
    prefix sum is an exact integer.  A 64-bit word u selects the first i with
    C_i > floor(u * Q / 2^64).  The probability used in D is q_i / Q, which is
    exactly the sampling probability (up to 2^-64).
R4  AdaGrad.  Per-mode accumulator S += G*G before the step, start S = 0,
    update -eta * G / sqrt(b + S) and 0 where b + S == 0.
R5  Leverage scores come from a Householder QR; a factor whose QR diagonal
    has R_jj^2 <= 1e-12 * ||a_j||^2 is rank deficient (error).
R6  Probabilities are recomputed from the current factors at every step.
R7  fit = 1 - Tol with Tol the squared relative error of Section 5.2.
R8  Nonnegative variant: project the updated factor onto A >= 0.
R9  Decreasing step alpha_t = beta / (t + gamma) (Theorem 9).
R10 Rescaling (the remark after the fixed-step error bound, Section 4.2,
    which names no formula): rank component r is rescaled so that its N
    columns all get the geometric mean of their norms, which leaves [[A]]
    unchanged; a component with a zero or non-finite column norm is left as
    it is.  The AdaGrad accumulators are not touched.  With rescaling every
    k steps it follows the update of every k-th step, and the next draws use
    the distributions of the rescaled factors (R6).
"""

import math

import numpy as np

from . import philox

UNIFORM, LEVERAGE, EUCLIDEAN = "uniform", "leverage", "euclidean"
FIXED, ADAGRAD, DECREASING = "fixed", "adagrad", "decreasing"

RANK_TOL = 1e-12


class RankDeficient(ValueError):
    """A leverage-score distribution was asked of a rank-deficient factor."""


class Degenerate(ValueError):
    """All weights of a distribution are zero (or not finite)."""


# ----------------------------------------------------------------------------
# Unfolding, Khatri-Rao rows, fibres (Sections 1 and 2)
# ----------------------------------------------------------------------------

def unfold(X, n):
    """Mode-n unfolding X_(n) (I_n x J_n); column j follows the index map
    j = sum_{k != n} i_k J'_k with J'_k the product of the lower mode sizes
    (Section 1), i.e. lower modes vary fastest."""
    return np.reshape(np.moveaxis(X, n, 0), (X.shape[n], -1), order="F")


def column_index(multi, dims, n):
    """0-based unfolding column of the multi-index ``multi`` (all modes; the
    entry at mode n is ignored), by the Section 1 index map."""
    j, stride = 0, 1
    for k, I in enumerate(dims):
        if k == n:
            continue
        j += int(multi[k]) * stride
        stride *= int(I)
    return j


def multi_index(j, dims, n):
    """Inverse of :func:`column_index` (mode n set to 0)."""
    out = [0] * len(dims)
    for k, I in enumerate(dims):
        if k == n:
            continue
        out[k] = j % int(I)
        j //= int(I)
    return out


def krp(factors, n):
    """Z^(n) = A^(N) (.) ... (.) A^(n+1) (.) A^(n-1) (.) ... (.) A^(1), formed
    explicitly (J_n x R): row j is the Hadamard product of the factor rows at
    the multi-index of column j (Section 2)."""
    dims = [A.shape[0] for A in factors]
    R = factors[0].shape[1]
    Jn = int(np.prod([d for k, d in enumerate(dims) if k != n]))
    Z = np.ones((Jn, R))
    for j in range(Jn):
        mi = multi_index(j, dims, n)
        for k, A in enumerate(factors):
            if k != n:
                Z[j, :] *= A[mi[k], :]
    return Z


def krp_fast(factors, n):
    """Same matrix as :func:`krp`, built by broadcasting (for larger sizes)."""
    others = [A for k, A in enumerate(factors) if k != n]
    R = factors[0].shape[1]
    Z = others[0]
    for A in others[1:]:
        Z = (A[:, None, :] * Z[None, :, :]).reshape(-1, R)
    return Z


def sampled_krp_rows(factors, n, idx):
    """Rows of Z^(n) at the sampled multi-indices: H(f,:) = product over
    k != n (ascending) of A^(k)(idx[f, s_k], :) (Algorithm 1)."""
    B = idx.shape[0]
    R = factors[0].shape[1]
    H = np.ones((B, R))
    s = 0
    for k, A in enumerate(factors):
        if k == n:
            continue
        H = H * A[idx[:, s], :]
        s += 1
    return H


def gather_fibres(X, n, idx):
    """Mode-n fibres of X at the sampled multi-indices, read by direct N-d
    indexing (Algorithm 1); returned as B x I_n (row f = fibre f)."""
    B = idx.shape[0]
    N = X.ndim
    out = np.empty((B, X.shape[n]))
    for f in range(B):
        key = []
        s = 0
        for k in range(N):
            if k == n:
                key.append(slice(None))
            else:
                key.append(int(idx[f, s]))
                s += 1
        out[f, :] = X[tuple(key)]
    return out


# ----------------------------------------------------------------------------
# Per-mode distributions (Section 3.1)
# ----------------------------------------------------------------------------

def euclidean_weights(A):
    """Squared row norms ||A(i,:)||^2, summed over r in ascending order."""
    A = np.asarray(A, dtype=np.float64)
    w = np.zeros(A.shape[0])
    for r in range(A.shape[1]):
        w = w + A[:, r] * A[:, r]
    return w


def leverage_scores(A):
    """l_i(A) = ||Q(i,:)||^2 with Q an orthonormal basis of range(A)
    (leverage-score definition, Section 3.1), from a Householder QR."""
    A = np.asarray(A, dtype=np.float64)
    Q, Rf = np.linalg.qr(A, mode="reduced")
    col2 = np.sum(A * A, axis=0)
    d2 = np.diag(Rf) ** 2
    if A.shape[0] < A.shape[1] or np.any(~np.isfinite(d2)) or np.any(d2 <= RANK_TOL * col2):
        raise RankDeficient("factor is rank deficient; leverage scores undefined")
    return np.sum(Q * Q, axis=1)


def row_weights(A, sampler):
    """Unnormalised sampling weights of the rows of one factor."""
    if sampler == UNIFORM:
        return np.ones(A.shape[0])
    if sampler == EUCLIDEAN:
        return euclidean_weights(A)
    if sampler == LEVERAGE:
        return leverage_scores(A)
    raise ValueError(f"unknown sampler {sampler!r}")


def quantize(w):
    """Integer-valued float64 weights q and CDF C (reading R3).

    Returns (q, C, Q) with C the inclusive prefix sums and Q = C[-1].
    """
    w = np.asarray(w, dtype=np.float64)
    I = w.shape[0]
    wmax = float(np.max(w)) if I else 0.0
    if not (wmax > 0.0 and math.isfinite(wmax)) or np.any(w < 0) or np.any(~np.isfinite(w)):
        raise Degenerate("sampling weights are all zero or not finite")
    _, ex = math.frexp(wmax)          # wmax = m * 2**ex, 0.5 <= m < 1
    c = (I - 1).bit_length()          # 2**c >= I
    E = 52 - ex - c
    q = np.ceil(np.ldexp(w, E))
    C = np.cumsum(q)
    return q, C, float(C[-1])


def distribution(A, sampler):
    """(q, C, Q) of one factor for the given sampler."""
    return quantize(row_weights(A, sampler))


def inverse_cdf(C, Q, u):
    """First i with C_i > floor(u * Q / 2^64) (sampling with replacement)."""
    target = philox.mulhi64(u, int(Q))
    return int(np.searchsorted(C, float(target), side="right"))


# ----------------------------------------------------------------------------
# The method (Section 3.2, Algorithms 3-5)
# ----------------------------------------------------------------------------

def mode_draw(seed, stream_id, t, N):
    """Mode of step t: n = floor(u_0 * N / 2^64) (uniform over the N modes)."""
    return philox.mulhi64(philox.draw_word(seed, stream_id, t, 0), N)


class Oracle:
    """The whole iteration, one step at a time, in float64.

    ``X`` is a dense numpy array (any memory order) of shape dims.
    ``A0`` the initial factors.  ``rule`` is FIXED (step ``alpha``),
    DECREASING (alpha_t = beta/(t+gamma)) or ADAGRAD (``eta``, ``b``).
    """

    def __init__(self, X, A0, *, B, sampler=EUCLIDEAN, rule=ADAGRAD, alpha=0.0,
                 eta=1.0, b=0.0, beta=0.0, gamma=1.0, seed=0, stream_id=0,
                 nonneg=False, rescale_every=0):
        self.X = np.asarray(X, dtype=np.float64)
        self.dims = list(self.X.shape)
        self.N = len(self.dims)
        self.A = [np.array(a, dtype=np.float64, copy=True) for a in A0]
        self.R = self.A[0].shape[1]
        self.S = [np.zeros_like(a) for a in self.A]
        self.B = int(B)
        self.sampler = sampler
        self.rule = rule
        self.alpha, self.eta, self.b = float(alpha), float(eta), float(b)
        self.beta, self.gamma = float(beta), float(gamma)
        self.seed, self.stream_id = int(seed), int(stream_id)
        self.nonneg = bool(nonneg)
        self.rescale_every = int(rescale_every)
        self.t = 0
        self.xnorm2 = float(np.sum(self.X * self.X))

    # -- Algorithm 3 (SKRP-ST-I): sampling of one mini-batch ----------------
    def sample(self, t=None):
        """(n, idx, p) for step t with the current factors.

        idx is B x (N-1) (columns: modes k != n ascending), p the product
        probabilities p_{j_f} = prod_k q_{i_k} / Q_k (Lemmas 2 and 4)."""
        t = self.t if t is None else int(t)
        n = mode_draw(self.seed, self.stream_id, t, self.N)
        B = self.B
        words = philox.draw_words(self.seed, self.stream_id, t, 1 + (self.N - 1) * B)
        idx = np.zeros((B, self.N - 1), dtype=np.int64)
        p = np.ones(B)
        s = 0
        for k in range(self.N):
            if k == n:
                continue
            q, C, Q = distribution(self.A[k], self.sampler)
            for f in range(B):
                i = inverse_cdf(C, Q, words[1 + s * B + f])
                idx[f, s] = i
                p[f] = p[f] * (q[i] / Q)
            s += 1
        return n, idx, p

    def probabilities_at(self, n, idx):
        """p_{j_f} of given multi-indices under the current factors."""
        B = idx.shape[0]
        p = np.ones(B)
        s = 0
        for k in range(self.N):
            if k == n:
                continue
            q, _, Q = distribution(self.A[k], self.sampler)
            p = p * (q[idx[:, s]] / Q)
            s += 1
        return p

    # -- weighted stochastic gradient (Section 3.2) -------------------------
    def gradient(self, n, idx, p):
        """G = A^(n) (H^T W H) - X_s^T W H with w_f = 1/(B p_f) (R1, R2)."""
        H = sampled_krp_rows(self.A, n, idx)
        Xs = gather_fibres(self.X, n, idx)
        w = 1.0 / (idx.shape[0] * p)
        WH = w[:, None] * H
        return self.A[n] @ (H.T @ WH) - Xs.T @ WH

    def step_size(self, t):
        if self.rule == FIXED:
            return self.alpha
        if self.rule == DECREASING:
            return self.beta / (t + self.gamma)
        raise ValueError(self.rule)

    def apply_update(self, n, G):
        """Fixed/decreasing step (Algorithm 4) or AdaGrad (Algorithm 5)."""
        if self.rule == ADAGRAD:
            self.S[n] = self.S[n] + G * G
            den = np.sqrt(self.b + self.S[n])
            upd = np.zeros_like(G)
            nz = den > 0
            upd[nz] = self.eta * G[nz] / den[nz]
            self.A[n] = self.A[n] - upd
        else:
            self.A[n] = self.A[n] - self.step_size(self.t) * G
        if self.nonneg:
            self.A[n] = np.maximum(self.A[n], 0.0)

    def step(self, replay=None):
        """One iteration.  ``replay=(n, idx)`` uses the given draw instead of
        the oracle's own (the probabilities still come from this state).
        Returns (n, idx, p)."""
        if replay is None:
            n, idx, p = self.sample()
        else:
            n, idx = int(replay[0]), np.asarray(replay[1], dtype=np.int64)
            p = self.probabilities_at(n, idx)
        G = self.gradient(n, idx, p)
        self.apply_update(n, G)
        self.t += 1
        if self.rescale_every > 0 and self.t % self.rescale_every == 0:
            self.A = rescale_columns(self.A)  # R10
        return n, idx, p

    def run(self, steps):
        for _ in range(steps):
            self.step()

    # -- diagnostics ---------------------------------------------------------
    def reconstruct(self):
        return reconstruct(self.A)

    def fit(self):
        """1 - Tol with Tol = ||[[A]] - X||^2 / ||X||^2 (Section 5.2), by
        explicit reconstruction."""
        return fit_explicit(self.X, self.A)

    def full_gradient(self, n):
        return full_gradient(self.X, self.A, n)


def rescale_columns(factors):
    """Reading R10: for every rank component r with column norms
    nu_k = ||A^(k)(:, r)|| (all positive and finite), scale column r of
    factor k by g / nu_k, where g = (prod_k nu_k)^(1/N) is their geometric
    mean.  The products of the scales are one, so [[A]] is unchanged."""
    A = [np.array(a, dtype=np.float64, copy=True) for a in factors]
    N, R = len(A), A[0].shape[1]
    for r in range(R):
        nu = [math.sqrt(float(np.sum(A[k][:, r] * A[k][:, r]))) for k in range(N)]
        if not all(math.isfinite(v) and v > 0.0 for v in nu):
            continue
        g = math.prod(nu) ** (1.0 / N)
        for k in range(N):
            A[k][:, r] = A[k][:, r] * (g / nu[k])
    return A


def reconstruct(factors):
    """[[A^(1), ..., A^(N)]] as a dense FP64 array (shape dims)."""
    letters = "abcdefghij"
    N = len(factors)
    spec = ",".join(f"{letters[k]}z" for k in range(N)) + "->" + letters[:N]
    return np.einsum(spec, *[np.asarray(a, dtype=np.float64) for a in factors],
                     optimize=True)


def fit_explicit(X, factors, chunk=None):
    """1 - ||X - [[A]]||^2 / ||X||^2, reconstructing slice by slice along the
    last mode so memory stays bounded."""
    X = np.asarray(X, dtype=np.float64)
    N = X.ndim
    last = factors[-1]
    num = 0.0
    den = 0.0
    letters = "abcdefghij"
    spec = ",".join(f"{letters[k]}z" for k in range(N - 1)) + ",z->" + letters[:N - 1]
    for i in range(X.shape[-1]):
        sl = np.einsum(spec, *[np.asarray(a, dtype=np.float64) for a in factors[:-1]],
                       last[i, :], optimize=True)
        xs = X[..., i]
        d = xs - sl
        num += float(np.sum(d * d))
        den += float(np.sum(xs * xs))
    return 1.0 - num / den


def full_gradient(X, factors, n):
    """Gradient of f = 1/2 ||X - [[A]]||^2 w.r.t. A^(n):
    A^(n) (hadamard_{k != n} A^(k)T A^(k)) - X_(n) Z^(n)."""
    R = factors[0].shape[1]
    V = np.ones((R, R))
    for k, A in enumerate(factors):
        if k != n:
            V = V * (A.T @ A)
    Z = krp_fast(factors, n)
    return factors[n] @ V - unfold(np.asarray(X, dtype=np.float64), n) @ Z


def row_probabilities(factors, n, sampler):
    """p_j for every row j of Z^(n) (product of per-mode q/Q, Lemmas 2/4),
    as a vector in unfolding-column order."""
    others = [k for k in range(len(factors)) if k != n]
    P = None
    for k in others:
        q, _, Q = distribution(factors[k], sampler)
        pk = q / Q
        P = pk if P is None else (pk[:, None] * P[None, :]).reshape(-1)
    return P


def exact_variance(X, factors, n, sampler, B):
    """E||G - grad f||_F^2 for one mini-batch of size B (variance theorem):
    (1/B) (sum_j ||Rs(:,j)||^2 ||Z(j,:)||^2 / p_j - ||grad f||^2)
    with Rs = A^(n) Z^T - X_(n) the residual."""
    Z = krp_fast(factors, n)
    Rs = factors[n] @ Z.T - unfold(np.asarray(X, dtype=np.float64), n)
    p = row_probabilities(factors, n, sampler)
    g = full_gradient(X, factors, n)
    r2 = np.sum(Rs * Rs, axis=0)
    z2 = np.sum(Z * Z, axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        terms = np.where(p > 0, r2 * z2 / np.where(p > 0, p, 1.0), 0.0)
    return (float(np.sum(terms)) - float(np.sum(g * g))) / B


def variance_table1(X, factors, n, sampler, B):
    """The same variance written as in Table 1 for the exact (unquantised)
    distributions: uniform J_n * sum, leverage R^{N-1} * sum / prod l,
    Euclidean prod ||A^(k)||_F^2 * sum / prod ||A^(k)(i_k,:)||^2."""
    Z = krp_fast(factors, n)
    Rs = factors[n] @ Z.T - unfold(np.asarray(X, dtype=np.float64), n)
    g = full_gradient(X, factors, n)
    r2 = np.sum(Rs * Rs, axis=0)
    z2 = np.sum(Z * Z, axis=1)
    N = len(factors)
    others = [k for k in range(N) if k != n]
    Jn = Z.shape[0]
    if sampler == UNIFORM:
        s = Jn * float(np.sum(r2 * z2))
    else:
        den = None
        for k in others:
            v = leverage_scores(factors[k]) if sampler == LEVERAGE else euclidean_weights(factors[k])
            den = v if den is None else (v[:, None] * den[None, :]).reshape(-1)
        if sampler == LEVERAGE:
            const = float(factors[0].shape[1]) ** (N - 1)
        else:
            const = float(np.prod([np.sum(factors[k] ** 2) for k in others]))
        s = const * float(np.sum(r2 * z2 / den))
    return (s - float(np.sum(g * g))) / B


def gram_hadamard_norm2(factors):
    """||[[A]]||^2 = 1^T (hadamard_k A^(k)T A^(k)) 1 (used only as a test pin)."""
    R = factors[0].shape[1]
    V = np.ones((R, R))
    for A in factors:
        V = V * (A.T @ A)
    return float(np.sum(V))
