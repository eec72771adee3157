"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes are small enough for the oracle and still span several 16-wide MFMA
tiles, ragged tails in every dimension (I_n, R and B not multiples of the
tile sizes), 3- and 4-way tensors, one, two and three 16-row rank tiles,
modes short enough to split the contraction over waves and long enough that
each wave owns several row tiles, and both storage types.
"""

import math

import numpy as np
import pytest

import oracle as O
from helpers import factor_match_score
from parity_util import (Tracked, check_iterates, gpu_decomposition, oracle_for, problem,
                         sample_from_cdfs)

pytestmark = pytest.mark.gpu

# dims, R, B, sampler, storage
CASES = [
    ((37, 45, 53), 7, 30, "euclidean", "f32"),
    ((37, 45, 53), 7, 30, "leverage", "f32"),
    ((37, 45, 53), 7, 30, "uniform", "f32"),
    ((11, 13, 17, 9), 5, 21, "euclidean", "f32"),
    ((40, 33, 70), 20, 64, "leverage", "f32"),
    ((64, 48, 50), 40, 17, "euclidean", "f32"),
    ((37, 45, 53), 7, 30, "euclidean", "bf16"),
    ((20, 24, 22, 18), 12, 40, "leverage", "bf16"),
    # long modes: waves own several row tiles each (the unsplit contraction)
    ((300, 20, 17), 6, 40, "euclidean", "f32"),
    ((530, 12, 10), 5, 30, "leverage", "bf16"),
    # three rank tiles with more than 96 fibres: every chunk of the fibre
    # range is a power-of-two number of K-steps
    ((64, 48, 50), 40, 200, "euclidean", "f32"),
    ((64, 48, 50), 40, 200, "euclidean", "bf16"),
]
IDS = [f"{'x'.join(map(str, c[0]))}-R{c[1]}-B{c[2]}-{c[3]}-{c[4]}" for c in CASES]


def _announce(*what):
    print("CASE", *what, flush=True)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_initial_cdfs(case):
    dims, R, B, sampler, storage = case
    _announce("initial_cdfs", case)
    prob = problem(dims, R, storage=storage)
    dec = gpu_decomposition(prob, B, sampler=sampler, storage=storage)
    for n in range(len(dims)):
        C = dec.cdf(n)
        q_ref, C_ref, Q_ref = O.distribution(prob["A0"][n], sampler)
        if sampler == "leverage":
            # Cholesky (device) vs Householder QR (oracle): equal up to rounding
            q = np.diff(np.concatenate([[0.0], C]))
            assert np.all(np.abs(q - q_ref) <= np.maximum(2.0, 1e-11 * q_ref))
        else:
            assert np.array_equal(C, C_ref)
    dec.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_sample_bit_exact(case):
    dims, R, B, sampler, storage = case
    _announce("sample_bit_exact", case)
    prob = problem(dims, R, storage=storage)
    dec = gpu_decomposition(prob, B, sampler=sampler, storage=storage, seed=77, stream_id=3)
    cdfs = [dec.cdf(n) for n in range(len(dims))]
    orc = oracle_for(prob, B, sampler=sampler, seed=77, stream_id=3)
    for t in list(range(12)) + [2**40 + 5]:
        n, idx, p = dec.sample(t)
        n2, idx2, p2 = sample_from_cdfs(cdfs, 77, 3, t, B)
        assert n == n2
        assert np.array_equal(idx, idx2)
        assert np.array_equal(p, p2)
        if sampler != "leverage":
            n3, idx3, p3 = orc.sample(t)
            assert n == n3 and np.array_equal(idx, idx3) and np.array_equal(p, p3)
    dec.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_replay_100_steps(case):
    """The oracle replays the device's draws; iterates agree after 100 steps."""
    dims, R, B, sampler, storage = case
    _announce("replay_100_steps", case)
    prob = problem(dims, R, storage=storage)
    dec = gpu_decomposition(prob, B, sampler=sampler, storage=storage, eta=0.3)
    orc = oracle_for(prob, B, sampler=sampler, eta=0.3)
    own_mismatch = 0
    for t in range(100):
        n, idx, p = dec.sample(t)
        n_o, idx_o, _ = orc.sample(t)
        if n_o != n or not np.array_equal(idx_o, idx):
            own_mismatch += 1
        orc.step(replay=(n, idx))
        dec.step(1)
    dec.sync()
    assert dec.t == 100
    check_iterates(dec.factors(), orc, 1e-5, f"100 steps, own-draw mismatches {own_mismatch}")
    # draws differ from the oracle's own only where FP32 vs FP64 iterates move
    # a CDF boundary: rare
    assert own_mismatch <= 10
    dec.close()


def _safe_alpha(factors, frac=0.1):
    """frac / max_n lambda_max(Z^(n)T Z^(n)), from the Gram-Hadamard identity."""
    lam = 0.0
    for n in range(len(factors)):
        V = np.ones((factors[0].shape[1],) * 2)
        for k, A in enumerate(factors):
            if k != n:
                V = V * (A.T @ A)
        lam = max(lam, float(np.linalg.eigvalsh(V)[-1]))
    return frac / lam


@pytest.mark.parametrize("dims,R,B,sampler", [((37, 45, 53), 7, 30, "euclidean"),
                                              ((20, 24, 22, 18), 12, 40, "leverage")])
def test_bf16_storage_error_vs_fp64_oracle(dims, R, B, sampler):
    """BF16 storage against the FP64 oracle on the unrounded tensor.

    With the fixed step (smooth in the data) iterates stay within 2e-2 over
    100 steps.  AdaGrad with b = 0 takes sign steps of size eta while an
    entry's accumulator is small, so a rounding-level change of the data can
    flip a step; there only the fit is compared."""
    _announce("bf16_vs_fp64", dims, R, B, sampler)
    prob = problem(dims, R, storage="bf16")
    alpha = _safe_alpha(prob["A0"])
    dec = gpu_decomposition(prob, B, sampler=sampler, storage="bf16", rule="fixed", alpha=alpha)
    orc64 = Tracked(O.Oracle(prob["X64"], prob["A0"], B=B, sampler=sampler, rule="fixed",
                             alpha=alpha, seed=5))
    # the storage floor here: the oracle on the BF16-rounded tensor, its
    # iterate rounded to FP32
    orc_r = oracle_for(prob, B, sampler=sampler, rule="fixed", alpha=alpha)
    for t in range(100):
        n, idx, _ = dec.sample(t)
        orc64.step(replay=(n, idx))
        orc_r.step(replay=(n, idx))
        dec.step(1)
    check_iterates(dec.factors(), orc64, 2e-2, "BF16 storage, fixed step, vs FP64 oracle on the "
                   "unrounded tensor", floor_of=orc_r)
    dec.close()
    dec = gpu_decomposition(prob, B, sampler=sampler, storage="bf16", eta=0.3)
    orc64 = O.Oracle(prob["X64"], prob["A0"], B=B, sampler=sampler, eta=0.3, seed=5)
    for t in range(100):
        n, idx, _ = dec.sample(t)
        orc64.step(replay=(n, idx))
        dec.step(1)
    A = [a.astype(np.float64) for a in dec.factors()]
    f_gpu = O.fit_explicit(prob["X64"], A)
    f_ora = orc64.fit()
    print(f"BF16 storage, AdaGrad: fit {f_gpu:.5f} vs FP64 oracle {f_ora:.5f}")
    assert abs(f_gpu - f_ora) <= 2e-2
    dec.close()


@pytest.mark.parametrize("rule,kw", [("fixed", dict(alpha=2e-5)),
                                     ("decreasing", dict(beta=2e-3, gamma=100.0))])
def test_fixed_and_decreasing_rules(rule, kw):
    _announce("rules", rule)
    prob = problem((30, 31, 29), 6)
    dec = gpu_decomposition(prob, 24, sampler="euclidean", rule=rule, **kw)
    orc = oracle_for(prob, 24, sampler="euclidean", rule=rule, **kw)
    for t in range(60):
        n, idx, _ = dec.sample(t)
        orc.step(replay=(n, idx))
        dec.step(1)
    check_iterates(dec.factors(), orc, 1e-5, f"{rule} rule, 60 steps")
    dec.close()


def test_nonneg_projection():
    _announce("nonneg")
    prob = problem((30, 31, 29), 6, nonneg=True)
    dec = gpu_decomposition(prob, 24, sampler="euclidean", nonneg=True, eta=0.3)
    orc = oracle_for(prob, 24, sampler="euclidean", nonneg=True, eta=0.3)
    for t in range(60):
        n, idx, _ = dec.sample(t)
        orc.step(replay=(n, idx))
        dec.step(1)
    A = dec.factors()
    assert all(np.all(a >= 0) for a in A)
    check_iterates(A, orc, 1e-5, "nonnegative projection, 60 steps")
    dec.close()


FIT_CASES = [
    ((37, 45, 53), 7, "f32"),
    ((37, 45, 53), 7, "bf16"),
    ((130, 21, 19), 33, "f32"),     # three rank tiles, ragged 64-column tail
    ((520, 9, 8), 20, "bf16"),      # A^(1) too large for LDS: read from global
    ((9, 7, 6, 5), 3, "f32"),       # 4-way, short fibres
    ((1, 40, 30), 2, "f32"),        # fibres of length one
]


@pytest.mark.parametrize("dims,R,storage", FIT_CASES)
def test_fit_matches_explicit_reconstruction(dims, R, storage):
    _announce("fit", dims, R, storage)
    prob = problem(dims, R, storage=storage)
    dec = gpu_decomposition(prob, 30, storage=storage, eta=0.3)
    f0 = dec.fit()
    assert math.isclose(f0, O.fit_explicit(prob["X"], prob["A0"]), rel_tol=1e-6, abs_tol=1e-6)
    dec.step(200)
    f = dec.fit()
    A = [a.astype(np.float64) for a in dec.factors()]
    assert abs(f - O.fit_explicit(prob["X"], A)) <= 1e-6
    dec.close()


@pytest.mark.parametrize("sampler", ["euclidean", "leverage"])
def test_noiseless_exact_rank_recovery(sampler):
    _announce("recovery", sampler)
    prob = problem((30, 30, 30), 5, data_seed=1001, init_seed=2001, snr_db=None)
    dec = gpu_decomposition(prob, 18, sampler=sampler, eta=1.0, seed=3001)
    dec.step(2000)
    f = dec.fit()
    A = dec.factors()
    print(f"fit {f:.9f}")
    assert f > 1 - 1e-5
    assert factor_match_score([a.astype(np.float64) for a in A], prob["A_true"]) > 0.99
    dec.close()


def test_state_resume_is_bit_exact():
    _announce("resume")
    prob = problem((37, 45, 53), 7)
    dec = gpu_decomposition(prob, 30, sampler="leverage", eta=0.3)
    dec.step(17)
    blob = dec.state()
    dec.step(40)
    A1 = dec.factors()
    dec.load_state(blob)
    assert dec.t == 17
    dec.step(40)
    A2 = dec.factors()
    assert all(np.array_equal(a, b) for a, b in zip(A1, A2))
    dec.close()


def test_device_input_matches_host_input():
    _announce("device_input")
    prob = problem((23, 40, 31), 9)
    a = gpu_decomposition(prob, 25, device_input=False)
    b = gpu_decomposition(prob, 25, device_input=True)
    a.step(30)
    b.step(30)
    assert all(np.array_equal(x, y) for x, y in zip(a.factors(), b.factors()))
    assert a.fit() == b.fit()
    a.close()
    b.close()


@pytest.mark.parametrize("dims,R,B", [((5, 4), 1, 1), ((1, 9, 8), 2, 3), ((64, 2, 3), 2, 4),
                                      ((16, 16, 16), 16, 4), ((3, 3, 3, 3, 3), 2, 5)])
def test_edge_shapes(dims, R, B):
    """Degenerate shapes: a matrix (N = 2), a mode of size 1, R = 1, B = 1,
    exact tile multiples and a 5-way tensor."""
    _announce("edge", dims, R, B)
    prob = problem(dims, R)
    dec = gpu_decomposition(prob, B, sampler="euclidean", eta=0.2)
    orc = oracle_for(prob, B, sampler="euclidean", eta=0.2)
    for t in range(20):
        n, idx, p = dec.sample(t)
        n_o, idx_o, p_o = orc.sample(t)
        assert n == n_o and np.array_equal(idx, idx_o)
        orc.step(replay=(n, idx))
        dec.step(1)
    check_iterates(dec.factors(), orc, 1e-5, f"edge shape {dims} R{R} B{B}, 20 steps")
    dec.close()


def test_error_paths():
    import paper_2103_04081_amd as P
    _announce("errors")
    prob = problem((20, 21, 22), 4)
    bad = [a.copy() for a in prob["A0"]]
    bad[1][:, 3] = bad[1][:, 0]
    prob_bad = dict(prob, A0=bad)
    with pytest.raises(P.CpdError) as e:
        gpu_decomposition(prob_bad, 8, sampler="leverage")
    assert e.value.status == P.cpdmi.CPD_E_RANK_DEFICIENT
    zero = [a.copy() for a in prob["A0"]]
    zero[2][:] = 0.0
    with pytest.raises(P.CpdError) as e:
        gpu_decomposition(dict(prob, A0=zero), 8, sampler="euclidean")
    assert e.value.status == P.cpdmi.CPD_E_DEGENERATE
    dec = gpu_decomposition(prob, 8, sampler="euclidean", rule="fixed", alpha=1e30)
    dec.step(20)
    with pytest.raises(P.CpdError) as e:
        dec.sync()
    assert e.value.status == P.cpdmi.CPD_E_DIVERGED
    # the handle stays failed: further steps are no-ops that report the error
    with pytest.raises(P.CpdError):
        dec.fit()
    dec.close()


def test_persistent_largest_batch_and_grid_beyond():
    """24x20x16, R 6: B = 1280 is the largest batch whose step fits the
    persistent kernel's LDS, and B = 1281 (padded to 1408 fibres) is run by
    the grid step instead.  Both draw bit for bit what the oracle's sampler
    draws from the device's CDFs and follow the oracle over 10 replayed
    steps."""
    import paper_2103_04081_amd as P
    import paper_2103_04081_amd.cpdmi as C
    _announce("persistent_largest_batch")
    dims, R = (24, 20, 16), 6
    prob = problem(dims, R)
    P.cpd_workspace_size(P.make_problem(list(dims), R, 1280), C.make_options(path="persistent"))
    with pytest.raises(Exception):
        P.cpd_workspace_size(P.make_problem(list(dims), R, 1281),
                             C.make_options(path="persistent"))
    for B, path in ((1280, "persistent"), (1281, "grid")):
        dec = gpu_decomposition(prob, B, sampler="euclidean", eta=0.3, path=path)
        orc = oracle_for(prob, B, sampler="euclidean", eta=0.3)
        for t in range(10):
            cdfs = [dec.cdf(k) for k in range(3)]
            n, idx, p = dec.sample(t)
            n2, idx2, p2 = sample_from_cdfs(cdfs, 5, 0, t, B)
            assert n == n2 and np.array_equal(idx, idx2) and np.array_equal(p, p2), (B, t)
            orc.step(replay=(n, idx))
            dec.step(1)
        check_iterates(dec.factors(), orc, 1e-5, f"B = {B} ({path}), 10 steps")
        dec.close()
