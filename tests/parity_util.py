"""Shared set-up of the GPU parity tests: one seeded problem handed to both
the HIP library and the FP64 oracle."""

import numpy as np

import cpd_inputs as ci
import oracle as O
from oracle import philox


def problem(dims, R, *, data_seed=11, init_seed=12, snr_db=30.0, storage="f32", skew=None,
            rho=None, nonneg=False):
    dt = "bf16" if storage == "bf16" else np.float32
    return ci.make_problem(dims, R, data_seed=data_seed, init_seed=init_seed, snr_db=snr_db,
                           dtype=dt, skew=skew, rho=rho, nonneg=nonneg)


def gpu_decomposition(prob, B, *, sampler="euclidean", rule="adagrad", eta=0.5, alpha=0.0, b=0.0,
                      beta=0.0, gamma=1.0, storage="f32", seed=5, stream_id=0, nonneg=False,
                      device_input=False, path="auto"):
    """The HIP library on the same tensor (FP32 values, rounded to BF16 by the
    library when storage is BF16) and initial factors."""
    import torch

    import paper_2103_04081_amd as P
    X32 = np.asfortranarray(prob["X"].astype(np.float32))
    if device_input:
        # mode-1-fastest memory: a C-contiguous tensor of shape dims[::-1]
        X = torch.as_tensor(X32.ravel(order="F").copy(), device="cuda")
        X = X.reshape(tuple(prob["dims"][::-1]))
    else:
        X = X32
    return P.Decomposition(X, prob["A0"], B=B, sampler=sampler, rule=rule, eta=eta, alpha=alpha,
                           b=b, beta=beta, gamma=gamma, storage=storage, seed=seed,
                           stream_id=stream_id, nonneg=nonneg, dims=prob["dims"], path=path)


def oracle_for(prob, B, *, sampler="euclidean", rule="adagrad", eta=0.5, alpha=0.0, b=0.0,
               beta=0.0, gamma=1.0, seed=5, stream_id=0, nonneg=False, factors=None):
    """The FP64 oracle on the stored (rounded) tensor, with its FP32-storage
    shadow (Tracked)."""
    return Tracked(O.Oracle(prob["X"], prob["A0"] if factors is None else factors, B=B,
                            sampler=sampler, rule=rule, eta=eta, alpha=alpha, b=b, beta=beta,
                            gamma=gamma, seed=seed, stream_id=stream_id, nonneg=nonneg))


def sample_from_cdfs(cdfs, seed, stream_id, t, B):
    """The oracle's sampling rule applied to given integer CDFs (one per mode)."""
    N = len(cdfs)
    n = O.mode_draw(seed, stream_id, t, N)
    words = philox.draw_words(seed, stream_id, t, 1 + (N - 1) * B)
    idx = np.zeros((B, N - 1), dtype=np.int64)
    p = np.ones(B)
    s = 0
    for k in range(N):
        if k == n:
            continue
        C = cdfs[k]
        Q = float(C[-1])
        q = np.diff(np.concatenate([[0.0], C]))
        for f in range(B):
            i = O.inverse_cdf(C, Q, words[1 + s * B + f])
            idx[f, s] = i
            p[f] = p[f] * (q[i] / Q)
        s += 1
    return n, idx, p


def rel(a, b):
    """Frobenius-norm relative difference (reported beside elem_err)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def elem_err(a, b):
    """Element-wise relative difference of an iterate a against the oracle's b:
    max_ij |a_ij - b_ij| / (|b_ij| + 1e-3 max|b|).  Every entry is held to the
    tolerance on its own scale; the floor 1e-3 max|b| keeps entries that pass
    through zero from dividing by nothing."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if b.size == 0:
        return 0.0
    floor = 1e-3 * float(np.max(np.abs(b)))
    return float(np.max(np.abs(a - b) / (np.abs(b) + max(floor, 1e-300))))


def factor_errs(A, B):
    """(max element-wise error, max Frobenius error) over the factors."""
    return (max(elem_err(a, b) for a, b in zip(A, B)), max(rel(a, b) for a, b in zip(A, B)))


# Element-wise bound of an FP32-storage iterate, as a multiple of what FP32
# storage alone does to the same trajectory (see StorageFloor).  An FP32
# implementation also rounds inside every sum of the step (over the B fibres
# and the R ranks): the CPU pins measure a plain FP32 implementation of the
# step (BLAS summation order) at up to 7x the floor, and over the 136 GPU
# comparisons the device's matrix-core summation order lands at 2.3x the
# floor (median), 5.3x (90th percentile) and 17.5x (largest: six AdaGrad
# steps of size 1.5, where every update is nearly a sign step).  A defect
# (a wrong update, a dropped term) gives element-wise errors of order one.
FLOOR_FACTOR = 32.0


def _r32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


class StorageFloor:
    """An FP64 oracle whose stored quantities are rounded to FP32 where the
    product stores them in FP32: the factors and AdaGrad accumulators after
    every update, and within a step the KRP rows H, the weights w_f, WH,
    H^T W H, X_s^T W H and the gradient.  Every value is computed exactly (in
    FP64) and then rounded; only the rounding inside the sums is left out.
    Stepped with the same draws as the reference oracle, its element-wise
    departure from it is what the FP32 storage of the product alone does to
    this trajectory: AdaGrad with b = 0 takes near-sign steps while an
    accumulator is small, so a rounding of 2^-24 in one entry can grow by
    orders of magnitude over 100 steps (the CPU pins measure up to ~1e-4
    element-wise).  No FP32-storage implementation can be held closer than
    that element by element; the device is held to FLOOR_FACTOR times it
    (its own arithmetic also rounds inside every sum), and to the tolerance
    itself when that is larger."""

    def __init__(self, orc):
        import copy
        self.o = copy.copy(orc)  # shares the tensor; the iterate is its own
        self.o.A = [a.copy() for a in orc.A]
        self.o.S = [s.copy() for s in orc.S]
        o = self.o

        def gradient(n, idx, p):
            H = _r32(O.sampled_krp_rows(o.A, n, idx))
            Xs = O.gather_fibres(o.X, n, idx)
            w = _r32(1.0 / (idx.shape[0] * p))
            WH = _r32(w[:, None] * H)
            return _r32(o.A[n] @ _r32(H.T @ WH) - _r32(Xs.T @ WH))

        o.gradient = gradient
        self._round()

    def _round(self):
        self.o.A = [_r32(a) for a in self.o.A]
        self.o.S = [_r32(s) for s in self.o.S]

    def step(self, replay):
        self.o.step(replay=replay)
        self._round()


class Tracked:
    """A reference oracle stepped together with its StorageFloor shadow
    (every other attribute is the reference oracle's)."""

    def __init__(self, orc):
        self.ref = orc
        self.floor = StorageFloor(orc)

    def step(self, replay=None):
        assert replay is not None, "the shadow follows replayed draws only"
        out = self.ref.step(replay=replay)
        self.floor.step(replay)
        return out

    def __getattr__(self, name):
        return getattr(self.ref, name)


def check_iterates(A, orc, tol, label="", floor_of=None):
    """Device factors A against the reference oracle (a Tracked): norm-wise
    within tol per factor, element-wise within max(tol, FLOOR_FACTOR * the
    storage floor).  floor_of: a Tracked whose shadow measures the floor
    instead (for comparisons against an oracle on other data).
    Returns (element-wise, Frobenius, floor)."""
    err, err_f = factor_errs(A, orc.A)
    src = orc if floor_of is None else floor_of
    fl = factor_errs(src.floor.o.A, orc.A)[0]
    bound = max(tol, FLOOR_FACTOR * fl)
    print(f"{label}: vs oracle element-wise {err:.3e} (bound {bound:.3e}; FP32-storage floor "
          f"{fl:.3e}), Frobenius {err_f:.3e} (tol {tol:g})", flush=True)
    assert err_f <= tol, (label, err_f)
    assert err <= bound, (label, err, fl)
    return err, err_f, fl
