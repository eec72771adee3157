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
    return O.Oracle(prob["X"], prob["A0"] if factors is None else factors, B=B, sampler=sampler,
                    rule=rule, eta=eta, alpha=alpha, b=b, beta=beta, gamma=gamma, seed=seed,
                    stream_id=stream_id, nonneg=nonneg)


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
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
