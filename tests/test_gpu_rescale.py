"""Column rescaling between steps (cpd_rescale, cpd_options.rescale_every)
on the GPU, through the C ABI, against the oracle's reading of the
bounded-iterate remark (Section 4.2): every rank component's columns get
the geometric mean of their norms, the CP model is unchanged, and the next
draws use the distributions of the rescaled factors."""

import numpy as np
import pytest

import oracle as O
from parity_util import Tracked, check_iterates, elem_err, gpu_decomposition, problem, sample_from_cdfs

pytestmark = pytest.mark.gpu


def _unbalanced(dims, R, storage="f32", seed=11):
    """A seeded problem whose initial factor columns have very different
    norms across the modes (so a rescale moves every column); each
    component's scales multiply to one, so the model is the problem's own."""
    prob = problem(dims, R, storage=storage, data_seed=seed)
    rng = np.random.default_rng(seed + 100)
    logs = [rng.uniform(-2.5, 2.5, size=R) for _ in dims[:-1]]
    logs.append(-np.sum(logs, axis=0))
    scales = [np.exp(l) for l in logs]
    # FP32-representable, so both sides start from the same values
    prob["A0"] = [(np.asarray(A, dtype=np.float64) * s).astype(np.float32).astype(np.float64)
                  for A, s in zip(prob["A0"], scales)]
    return prob


@pytest.mark.parametrize("path", ["persistent", "grid"])
def test_rescale_call_matches_oracle(path):
    print("CASE rescale_call", path, flush=True)
    dims, R = (37, 45, 53), 7
    prob = _unbalanced(dims, R)
    dec = gpu_decomposition(prob, 300 if path == "grid" else 40, sampler="euclidean", eta=0.3,
                            path=path)
    dec.step(3)
    before = [a.astype(np.float64) for a in dec.factors()]
    fit0 = dec.fit()
    dec.rescale()
    after = dec.factors()
    want = O.rescale_columns(before)
    err = max(elem_err(after[k], want[k]) for k in range(3))
    print(f"{path}: rescale vs oracle {err:.3e}, fit {fit0:.9f} -> {dec.fit():.9f}", flush=True)
    assert err <= 1e-6
    assert abs(dec.fit() - fit0) <= 1e-6
    for r in range(R):
        nu = [np.linalg.norm(after[k][:, r].astype(np.float64)) for k in range(3)]
        assert max(nu) - min(nu) <= 1e-5 * max(nu)
    # the distributions were rebuilt from the rescaled factors
    for k in range(3):
        _, C_ref, _ = O.distribution(after[k].astype(np.float64), "euclidean")
        assert np.array_equal(dec.cdf(k), C_ref), k
    dec.close()


CASES = [((37, 45, 53), 7, 40, "euclidean", "f32", 1, "persistent"),
         ((37, 45, 53), 7, 40, "leverage", "f32", 3, "persistent"),
         ((11, 13, 17, 9), 5, 21, "euclidean", "f32", 1, "persistent"),
         ((37, 45, 53), 7, 300, "euclidean", "f32", 2, "grid"),
         ((20, 24, 22, 18), 12, 260, "uniform", "bf16", 1, "grid")]
IDS = [f"{'x'.join(map(str, c[0]))}-R{c[1]}-B{c[2]}-{c[3]}-{c[4]}-every{c[5]}-{c[6]}"
       for c in CASES]


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_rescale_every_replay_against_oracle(case):
    """20 steps with rescale_every = k: draws bit for bit against the
    oracle's sampler on the device's CDFs, the oracle (rescaling after the
    same steps) replays them, and the iterates and the fit agree."""
    dims, R, B, sampler, storage, every, path = case
    print("CASE rescale_every", case, flush=True)
    prob = _unbalanced(dims, R, storage=storage)
    import paper_2103_04081_amd as P
    X32 = np.asfortranarray(prob["X"].astype(np.float32))
    dec = P.Decomposition(X32, prob["A0"], B=B, sampler=sampler, eta=0.3, storage=storage,
                          seed=5, path=path, rescale_every=every)
    orc = Tracked(O.Oracle(prob["X"], prob["A0"], B=B, sampler=sampler, eta=0.3, seed=5,
                           rescale_every=every))
    N = len(dims)
    for t in range(20):
        cdfs = [dec.cdf(k) for k in range(N)]
        n, idx, p = dec.sample(t)
        n2, idx2, p2 = sample_from_cdfs(cdfs, 5, 0, t, B)
        assert n == n2 and np.array_equal(idx, idx2) and np.array_equal(p, p2), t
        orc.step(replay=(n, idx))
        dec.step(1)
    check_iterates(dec.factors(), orc, 1e-5, f"20 steps, rescale every {every}")
    assert abs(dec.fit() - orc.fit()) <= 1e-5
    assert dec.t == 20
    dec.close()


@pytest.mark.parametrize("path,B,every,total,cut", [("persistent", 40, 3, 20, 7),
                                                    ("grid", 300, 17, 40, 7)])
def test_rescale_schedule_across_calls_and_state(path, B, every, total, cut):
    """The rescaling points depend on the step counter only: all steps in
    one cpd_step call (stretches of `every` steps between rescales; on the
    grid path a 17-step stretch is a 16-step graph replay plus one direct
    step), single-step calls, and `cut` steps saved and resumed by a fresh
    handle for the rest all give the same factors, bit for bit."""
    import paper_2103_04081_amd as P
    print("CASE rescale_schedule", path, every, flush=True)
    dims, R = (37, 45, 53), 7
    prob = _unbalanced(dims, R)
    X32 = np.asfortranarray(prob["X"].astype(np.float32))

    def make():
        return P.Decomposition(X32, prob["A0"], B=B, sampler="euclidean", eta=0.3, seed=5,
                               path=path, rescale_every=every)

    a = make()
    a.step(total)
    b = make()
    for _ in range(total):
        b.step(1)
    c = make()
    c.step(cut)
    blob = c.state()
    c.close()
    d = make()
    d.load_state(blob)
    d.step(total - cut)
    A, Bf, D = a.factors(), b.factors(), d.factors()
    assert a.t == b.t == d.t == total
    for k in range(3):
        assert np.array_equal(A[k], Bf[k]), k
        assert np.array_equal(A[k], D[k]), k
    for h in (a, b, d):
        h.close()
