"""The grid-wide step (CPD_PATH_GRID) on the GPU, through the C ABI.

The grid path splits the sampled fibres of one step over many blocks, sums
the block parts of the gradient in a fixed order, then updates and refreshes
the CDF of the mode.  It must draw exactly the persistent kernel's indices
(same Philox words, same integer CDFs) and follow the FP64 oracle's iterates
when it replays them.  Batches span several gather blocks with a ragged last
block (down to one fibre), 3- and 4-way tensors, one to three 16-row rank
tiles, both storage types and all three samplers.
"""

import numpy as np
import pytest

import oracle as O
from oracle import philox
from parity_util import (FLOOR_FACTOR, check_iterates, factor_errs, gpu_decomposition,
                         oracle_for, problem, sample_from_cdfs)

pytestmark = pytest.mark.gpu

# dims, R, B, sampler, storage
CASES = [
    ((37, 45, 53), 7, 300, "euclidean", "f32"),
    ((37, 45, 53), 7, 300, "leverage", "f32"),
    ((37, 45, 53), 7, 200, "uniform", "f32"),
    ((11, 13, 17, 9), 5, 257, "euclidean", "f32"),
    ((40, 33, 70), 20, 300, "leverage", "f32"),
    ((64, 48, 50), 40, 300, "euclidean", "f32"),
    ((37, 45, 53), 7, 300, "euclidean", "bf16"),
    ((20, 24, 22, 18), 12, 260, "leverage", "bf16"),
    ((300, 20, 17), 6, 400, "euclidean", "f32"),
    ((530, 12, 10), 5, 300, "leverage", "bf16"),
]
IDS = [f"{'x'.join(map(str, c[0]))}-R{c[1]}-B{c[2]}-{c[3]}-{c[4]}" for c in CASES]


def _announce(*what):
    print("CASE", *what, flush=True)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_grid_draws_equal_persistent_draws(case):
    dims, R, B, sampler, storage = case
    _announce("grid_draws", case)
    prob = problem(dims, R, storage=storage)
    g = gpu_decomposition(prob, B, sampler=sampler, storage=storage, seed=77, stream_id=3,
                          path="grid")
    p = gpu_decomposition(prob, B, sampler=sampler, storage=storage, seed=77, stream_id=3,
                          path="persistent")
    cdfs = [g.cdf(n) for n in range(len(dims))]
    for n in range(len(dims)):
        assert np.array_equal(cdfs[n], p.cdf(n))
    for t in [0, 1, 2, 3, 17, 2**40 + 5]:
        n, idx, pr = g.sample(t)
        n2, idx2, pr2 = p.sample(t)
        assert n == n2 and np.array_equal(idx, idx2) and np.array_equal(pr, pr2)
    n, idx, pr = g.sample(5)
    n3, idx3, pr3 = sample_from_cdfs(cdfs, 77, 3, 5, B)
    assert n == n3 and np.array_equal(idx, idx3) and np.array_equal(pr, pr3)
    g.close()
    p.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_grid_replay_against_oracle(case):
    """The oracle replays the grid path's draws; iterates agree after 40
    steps, and the persistent path fed the same draws agrees as well."""
    dims, R, B, sampler, storage = case
    _announce("grid_replay", case)
    prob = problem(dims, R, storage=storage)
    g = gpu_decomposition(prob, B, sampler=sampler, storage=storage, eta=0.3, path="grid")
    p = gpu_decomposition(prob, B, sampler=sampler, storage=storage, eta=0.3, path="persistent")
    orc = oracle_for(prob, B, sampler=sampler, eta=0.3)
    for t in range(40):
        n, idx, _ = g.sample(t)
        orc.step(replay=(n, idx))
        p.step_replay(n, idx)
        g.step(1)
    g.sync()
    assert g.t == 40 and p.t == 40
    A, Ap = g.factors(), p.factors()
    _, _, fl = check_iterates(A, orc, 1e-5, "grid path, 40 steps")
    check_iterates(Ap, orc, 1e-5, "persistent path fed the same draws, 40 steps")
    # the two FP32 paths differ in summation order only: each is within the
    # bound of the oracle, so their distance is within twice it
    err_p, err_pf = factor_errs(A, Ap)
    print(f"grid vs persistent: element-wise {err_p:.3e}, Frobenius {err_pf:.3e}")
    assert err_pf <= 2e-5
    assert err_p <= 2 * max(1e-5, FLOOR_FACTOR * fl)
    g.close()
    p.close()


def test_grid_large_batch():
    """B = 5000 (40 gather blocks, beyond the persistent kernel's LDS): draws
    against the oracle's sampler and 12 replayed steps against the oracle."""
    _announce("grid_large_batch")
    dims, R, B = (60, 50, 40), 10, 5000
    prob = problem(dims, R, skew=(0.1, 20.0), rho=0.6)
    g = gpu_decomposition(prob, B, sampler="euclidean", eta=0.3)  # AUTO picks the grid path
    cdfs = [g.cdf(n) for n in range(len(dims))]
    n, idx, pr = g.sample(0)
    n2, idx2, pr2 = sample_from_cdfs(cdfs, 5, 0, 0, B)
    assert n == n2 and np.array_equal(idx, idx2) and np.array_equal(pr, pr2)
    orc = oracle_for(prob, B, sampler="euclidean", eta=0.3)
    for t in range(12):
        n, idx, _ = g.sample(t)
        orc.step(replay=(n, idx))
        g.step(1)
    check_iterates(g.factors(), orc, 1e-5, "B = 5000, 12 steps")
    assert abs(g.fit() - orc.fit()) <= 1e-6
    g.close()


@pytest.mark.parametrize("rule,kw", [("fixed", dict(alpha=2e-6)),
                                     ("decreasing", dict(beta=2e-4, gamma=100.0))])
def test_grid_fixed_decreasing_nonneg(rule, kw):
    _announce("grid_rules", rule)
    prob = problem((30, 31, 29), 6, nonneg=True)
    g = gpu_decomposition(prob, 300, sampler="euclidean", rule=rule, nonneg=True, path="grid",
                          **kw)
    orc = oracle_for(prob, 300, sampler="euclidean", rule=rule, nonneg=True, **kw)
    for t in range(30):
        n, idx, _ = g.sample(t)
        orc.step(replay=(n, idx))
        g.step(1)
    A = g.factors()
    assert all(np.all(a >= 0) for a in A)
    check_iterates(A, orc, 1e-5, f"grid {rule} rule with projection, 30 steps")
    g.close()


def test_grid_variance_and_state_round_trip():
    import paper_2103_04081_amd as P
    _announce("grid_variance_state")
    prob = problem((37, 45, 53), 7)
    g = gpu_decomposition(prob, 300, sampler="leverage", path="grid")
    p = gpu_decomposition(prob, 300, sampler="leverage", path="persistent")
    for n in range(3):
        for s in ("uniform", "leverage", "euclidean"):
            assert g.variance(n, s) == p.variance(n, s)
    g.step(7)
    blob = g.state()
    A7 = g.factors()
    g.step(5)
    g.load_state(blob)
    assert g.t == 7
    for a, b in zip(g.factors(), A7):
        np.testing.assert_array_equal(a, b)
    g.step(5)
    g2 = gpu_decomposition(prob, 300, sampler="leverage", path="grid")
    g2.step(12)
    for a, b in zip(g.factors(), g2.factors()):
        np.testing.assert_array_equal(a, b)
    # a replayed index outside its mode is reported at the next sync
    bad = np.zeros((300, 2), dtype=np.int32)
    bad[299, 1] = 10_000
    with pytest.raises(P.CpdError) as e:
        g.step_replay(0, bad)
    assert e.value.status == P.cpdmi.CPD_E_INVALID
    g.close()
    g2.close()
    p.close()


def test_grid_graph_replay_equals_single_launches():
    """cpd_step with 16 or more steps replays a captured graph of 16 steps;
    the iterates are those of the same steps launched one by one."""
    _announce("grid_graph")
    prob = problem((37, 45, 53), 7)
    for sampler in ("euclidean", "uniform"):
        g = gpu_decomposition(prob, 300, sampler=sampler, path="grid")
        h = gpu_decomposition(prob, 300, sampler=sampler, path="grid")
        g.step(40)
        g.step(17)
        for _ in range(57):
            h.step(1)
        assert g.t == 57 and h.t == 57
        for a, b in zip(g.factors(), h.factors()):
            np.testing.assert_array_equal(a, b)
        g.close()
        h.close()


@pytest.mark.parametrize("dims,R,sampler,storage", [((20, 24, 22, 18), 12, "leverage", "bf16"),
                                                    ((30, 31, 29), 6, "euclidean", "f32")])
def test_grid_short_modes_split_fibre_range(dims, R, sampler, storage):
    """Modes with fewer 16-row tiles than waves split each block's fibres
    over the waves (several parts per block); B = 38405 makes slices of
    256 fibres with a last block of 5, whose later parts are empty."""
    _announce("grid_short_modes", dims, R, sampler, storage)
    B = 38405
    prob = problem(dims, R, storage=storage)
    g = gpu_decomposition(prob, B, sampler=sampler, storage=storage, eta=0.3, path="grid")
    orc = oracle_for(prob, B, sampler=sampler, eta=0.3)
    for t in range(6):
        n, idx, _ = g.sample(t)
        orc.step(replay=(n, idx))
        g.step(1)
    check_iterates(g.factors(), orc, 1e-5, f"short modes, B = {B}, 6 steps")
    g.close()


def test_grid_max_batch():
    """B = 2^20 (the library's largest batch, 2048 gather blocks), 24x20x16,
    R 6.  Draws bit for bit against the oracle's Philox words and inverse CDF
    at sampled fibres (the first and last 64, the ends of the first gather
    blocks and the middle, where draw numbers reach 1 + 2 B); the
    probabilities of all 2^20 fibres against the product of the CDF ratios;
    the row counts of each mode within 6 sigma of B q_i / Q; then two
    replayed steps against the oracle."""
    import paper_2103_04081_amd.cpdmi as C
    _announce("grid_max_batch")
    dims, R, B, seed = (24, 20, 16), 6, C.MAX_BATCH, 9
    prob = problem(dims, R)
    g = gpu_decomposition(prob, B, sampler="euclidean", eta=0.3, seed=seed)
    cdfs = [g.cdf(k) for k in range(3)]
    n, idx, pr = g.sample(0)
    assert n == O.mode_draw(seed, 0, 0, 3)
    assert idx.shape == (B, 2)
    modes = [k for k in range(3) if k != n]
    p_all = np.ones(B)
    for s, k in enumerate(modes):
        Ck = cdfs[k]
        Q = float(Ck[-1])
        q = np.diff(np.concatenate([[0.0], Ck]))
        assert idx[:, s].min() >= 0 and idx[:, s].max() < dims[k]
        p_all = p_all * (q[idx[:, s]] / Q)
        counts = np.bincount(idx[:, s], minlength=dims[k])
        mean = B * q / Q
        assert np.all(np.abs(counts - mean) <= 6.0 * np.sqrt(mean * (1 - q / Q)) + 1.0), k
    assert np.array_equal(pr, p_all)
    fibres = (list(range(64)) + [511, 512, 513, 1023, 1024, B // 2 - 1, B // 2]
              + list(range(B - 64, B)))
    for f in fibres:
        for s, k in enumerate(modes):
            u = philox.draw_word(seed, 0, 0, 1 + s * B + f)
            assert idx[f, s] == O.inverse_cdf(cdfs[k], float(cdfs[k][-1]), u), (f, s)
    orc = oracle_for(prob, B, sampler="euclidean", eta=0.3, seed=seed)
    for t in range(2):
        n, idx, _ = g.sample(t)
        orc.step(replay=(n, idx))
        g.step(1)
    check_iterates(g.factors(), orc, 1e-5, "B = 2^20, 2 steps")
    g.close()
