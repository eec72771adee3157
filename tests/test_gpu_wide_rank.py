"""Ranks 65..128 on the grid step (the paper's Pavia University scene is
decomposed at R = 100, Section 5, Tables 6 and 7): the grid kernels compiled
for eight rank tiles, the distribution refresh reading factor rows from
global memory when they do not fit in LDS, the fit in two passes of 64
ranks; against the FP64 oracle, and the refusals of the paths that take
R <= 64."""

import numpy as np
import pytest

import cpd_inputs as ci
import oracle as O
from parity_util import Tracked, check_iterates, gpu_decomposition, problem, sample_from_cdfs

pytestmark = pytest.mark.gpu


def _announce(*what):
    print("CASE", *what, flush=True)


# dims, R, B, sampler, storage
CASES = [
    ((40, 33, 29), 70, 60, "euclidean", "f32"),
    ((30, 25, 20, 18), 100, 40, "uniform", "f32"),
    ((37, 45, 53), 128, 150, "euclidean", "bf16"),
    ((300, 20, 17), 97, 20, "euclidean", "f32"),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{'x'.join(map(str, c[0]))}-R{c[1]}-B{c[2]}-{c[3]}-"
                                             f"{c[4]}" for c in CASES])
def test_wide_rank_replay_against_oracle(case):
    dims, R, B, sampler, storage = case
    _announce("wide rank replay", case)
    prob = problem(dims, R, storage=storage)
    dec = gpu_decomposition(prob, B, sampler=sampler, storage=storage, eta=0.3)
    orc = Tracked(O.Oracle(prob["X"], prob["A0"], B=B, sampler=sampler, eta=0.3, seed=5))
    N = len(dims)
    for t in range(40):
        cdfs = [dec.cdf(k) for k in range(N)]
        n, idx, p = dec.sample(t)
        n2, idx2, p2 = sample_from_cdfs(cdfs, 5, 0, t, B)
        assert n == n2 and np.array_equal(idx, idx2) and np.array_equal(p, p2), t
        if sampler == "euclidean":
            A = dec.factors()
            for k in range(N):
                _, C_ref, _ = O.distribution(A[k].astype(np.float64), sampler)
                assert np.array_equal(cdfs[k], C_ref), (t, k)
        orc.step(replay=(n, idx))
        dec.step(1)
    check_iterates(dec.factors(), orc, 1e-5, f"{dims} R{R} B{B} {sampler} {storage}, 40 steps")
    f = dec.fit()
    f_ref = O.fit_explicit(prob["X"], [a.astype(np.float64) for a in dec.factors()])
    print(f"fit {f:.9f} (explicit {f_ref:.9f})", flush=True)
    assert abs(f - f_ref) <= 1e-6
    dec.close()


def test_pavia_shaped_100_steps():
    """610 x 340 x 103 at R = 100, B = 20 (the shape and rank of the paper's
    Pavia University scene; a seeded Gaussian stand-in, SNR 30 dB): 100
    steps, draws bit for bit, the oracle replaying them."""
    dims, R, B = (610, 340, 103), 100, 20
    _announce("pavia-shaped R100")
    prob = ci.make_problem(dims, R, data_seed=1110, init_seed=1210, snr_db=30.0,
                           dtype=np.float32)
    dec = gpu_decomposition(prob, B, sampler="euclidean", eta=0.3, seed=1310)
    orc = Tracked(O.Oracle(prob["X"], prob["A0"], B=B, sampler="euclidean", eta=0.3, seed=1310))
    for t in range(100):
        cdfs = [dec.cdf(k) for k in range(3)]
        n, idx, p = dec.sample(t)
        n2, idx2, p2 = sample_from_cdfs(cdfs, 1310, 0, t, B)
        assert n == n2 and np.array_equal(idx, idx2) and np.array_equal(p, p2), t
        orc.step(replay=(n, idx))
        dec.step(1)
    check_iterates(dec.factors(), orc, 1e-5, "610x340x103 R100 B20, 100 steps")
    dec.close()


def test_wide_rank_refusals():
    import paper_2103_04081_amd as P
    import paper_2103_04081_amd.cpdmi as C
    _announce("wide rank refusals")
    prob = problem((20, 21, 22), 70)
    with pytest.raises(P.CpdError) as e:
        gpu_decomposition(prob, 10, sampler="leverage")
    assert e.value.status == C.CPD_E_INVALID
    with pytest.raises(P.CpdError) as e:
        gpu_decomposition(prob, 10, sampler="euclidean", path="persistent")
    assert e.value.status == C.CPD_E_INVALID
    dec = gpu_decomposition(prob, 10, sampler="euclidean")
    with pytest.raises(P.CpdError) as e:
        dec.variance(0, "euclidean")
    assert e.value.status == C.CPD_E_INVALID
    with pytest.raises(P.CpdError):
        C.cpd_variance_noalloc(dec.h, 0, "euclidean")
    dec.close()
    X = np.asfortranarray(prob["X"].astype(np.float32))
    with pytest.raises(P.CpdError):
        P.Batch([dict(X=X, A0=prob["A0"], B=10, sampler="euclidean", fit_every=10,
                      max_steps=20)], tune=False)
