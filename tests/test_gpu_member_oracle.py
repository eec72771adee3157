"""Batch members, served requests and every K-split of the step contraction
against the FP64 oracle.

Each of them must compute the reweighted stochastic gradient step of its
own decomposition (Section 3.2, Algorithm 5).  The K-split (how many parts
a row tile's fibre range is cut into across waves, summed in a fixed order
through LDS) only changes the FP32 summation order, so every legal value is
replayed against the oracle.  A batch member or a served request has no
replay entry of its own; it is tied to the oracle through a single handle
with the same problem, options and K-split: that handle replays its own
draws into the oracle step by step (iterates within 1e-5, element by
element), and its factors after the same steps equal the member's bit for
bit, so the member's draws and iterates are the replayed ones."""

import numpy as np
import pytest

import cpd_inputs as ci
import oracle as O
from parity_util import Tracked, check_iterates, problem

pytestmark = pytest.mark.gpu

STEPS = 100


def _announce(*what):
    print("CASE", *what, flush=True)


def _replayed_handle(prob, B, *, sampler, storage, eta, seed, stream_id, ksplit, label,
                     steps=STEPS):
    """A single handle stepped one step at a time while the oracle replays its
    draws; the iterates are checked against the oracle (norm-wise within
    1e-5, element-wise within the FP32-storage bound); returns the factors."""
    import paper_2103_04081_amd as P
    dec = P.Decomposition(np.asfortranarray(prob["X"].astype(np.float32)), prob["A0"], B=B,
                          sampler=sampler, rule="adagrad", eta=eta, storage=storage, seed=seed,
                          stream_id=stream_id, ksplit=ksplit, path="persistent")
    orc = Tracked(O.Oracle(prob["X"], prob["A0"], B=B, sampler=sampler, eta=eta, seed=seed,
                           stream_id=stream_id))
    for t in range(steps):
        n, idx, _ = dec.sample(t)
        orc.step(replay=(n, idx))
        dec.step(1)
    A = dec.factors()
    dec.close()
    check_iterates(A, orc, 1e-5, f"{label}, {steps} steps")
    return A


def _max_ksplit(I, storage, B, R):
    """The largest K-split of a mode (every part needs a wave of its own and
    at least one chunk of fibres): 8 waves over the mode's 16*VW-row tiles,
    capped by the chunks of the padded fibre range."""
    vw = 2 if storage == "bf16" else 1
    nst = -(-I // (16 * vw))
    rt = -(-R // 16)
    u = 32
    while u > 4 and u * vw * rt > 32:
        u //= 2
    chunks = (-(-B // 128) * 128) // 4 // u
    return max(1, min(8 // nst, chunks))


# every mode short (one or two row tiles), so K-splits up to 8 are legal
KSPLIT_CASES = [
    ((12, 14, 16), 20, 512, "f32"),
    ((12, 14, 16), 20, 512, "bf16"),
    ((12, 14, 16), 40, 300, "f32"),     # three rank tiles, ragged B
    ((30, 9, 13, 11), 7, 1000, "f32"),  # 4-way, one rank tile, a two-tile mode, ragged B
]


@pytest.mark.parametrize("case", KSPLIT_CASES,
                         ids=[f"{'x'.join(map(str, c[0]))}-R{c[1]}-B{c[2]}-{c[3]}"
                              for c in KSPLIT_CASES])
def test_every_ksplit_replayed_against_oracle(case):
    dims, R, B, storage = case
    prob = problem(dims, R, storage=storage, data_seed=31, init_seed=32)
    mx = [_max_ksplit(I, storage, B, R) for I in dims]
    assert max(mx) == 8
    seen = set()
    for ks in range(1, 9):
        ksplit = [min(ks, m) for m in mx]
        if tuple(ksplit) in seen:
            continue
        seen.add(tuple(ksplit))
        _announce("ksplit", case, ksplit)
        _replayed_handle(prob, B, sampler="euclidean", storage=storage, eta=0.3, seed=41,
                         stream_id=ks, ksplit=ksplit, label=f"ksplit {ksplit}")


# one member per rank-tile class (R 1-16, 17-32, 33-48, 49-64), the batch
# recipe's BF16 storage and B = 128, short modes so the tuner weighs K-splits
# of up to 8
BATCH_MEMBERS = [
    ((28, 45, 60), 7, "euclidean"),
    ((24, 70, 33), 20, "leverage"),
    ((30, 26, 50), 40, "euclidean"),
    ((20, 31, 44), 60, "uniform"),
    ((20, 24, 22, 18), 12, "euclidean"),
]


def test_batch_members_replayed_against_oracle():
    import paper_2103_04081_amd as P
    _announce("batch members vs oracle")
    members, probs = [], []
    for i, (dims, R, sampler) in enumerate(BATCH_MEMBERS):
        prob = problem(dims, R, storage="bf16", data_seed=51 + i, init_seed=61 + i)
        probs.append(prob)
        members.append(dict(X=np.asfortranarray(prob["X"].astype(np.float32)), A0=prob["A0"],
                            B=128, sampler=sampler, rule="adagrad", eta=0.5, storage="bf16",
                            fit_every=25, fit_target=2.0, max_steps=STEPS, seed=71,
                            stream_id=i))
    b = P.Batch(members, tune=True)
    assert b.run(max_rounds=10) == 0
    for i, (m, prob) in enumerate(zip(members, probs)):
        info = b.info(i)
        assert info["status"] == 0 and info["t"] == STEPS
        A = _replayed_handle(prob, 128, sampler=m["sampler"], storage="bf16", eta=0.5, seed=71,
                             stream_id=i, ksplit=info["ksplit"],
                             label=f"member {i} {BATCH_MEMBERS[i]} ksplit {info['ksplit']}")
        for a, g in zip(A, b.factors(i)):
            np.testing.assert_array_equal(a, g)
    b.close()


def test_served_requests_replayed_against_oracle():
    import time

    import paper_2103_04081_amd as P
    _announce("served requests vs oracle")
    reqs = [((40, 52, 37), 8, "bf16"), ((24, 20, 18, 22), 12, "bf16"), ((64, 30, 45), 20, "f32")]
    probs = [problem(d, R, storage=s, data_seed=81 + i, init_seed=91 + i)
             for i, (d, R, s) in enumerate(reqs)]
    s = P.Server(256 << 20, max_slots=3, round_steps=25)
    tickets = [s.submit(np.asfortranarray(p["X"].astype(np.float32)), p["A0"], B=64,
                        storage=st, seed=101, stream_id=i, eta=0.5, fit_target=2.0,
                        max_steps=STEPS)
               for i, (p, (_, _, st)) in enumerate(zip(probs, reqs))]
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for tk in tickets:
            if tk not in res:
                r = s.poll(tk)
                if r is not None:
                    res[tk] = r
        assert time.time() - t0 < 120, "requests did not finish"
        time.sleep(0.002)
    s.close()
    for i, (tk, p, (dims, R, st)) in enumerate(zip(tickets, probs, reqs)):
        r = res[tk]
        assert r["status"] == 0 and r["steps"] == STEPS
        A = _replayed_handle(p, 64, sampler="euclidean", storage=st, eta=0.5, seed=101,
                             stream_id=i, ksplit=None, label=f"request {i} {reqs[i]}")
        for a, g in zip(A, r["factors"]):
            np.testing.assert_array_equal(a, g)
