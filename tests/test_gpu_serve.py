"""The request server on the GPU: continuous batching gives every request
the result it gets alone (bit for bit), admission respects the arena, and
errors stay with their request."""

import time

import numpy as np
import pytest

import cpd_inputs as ci

pytestmark = pytest.mark.gpu

# dims, R, storage: 3- and 4-way, two rank-tile classes, both storage types
REQS = [
    ((40, 52, 37), 8, "bf16"),
    ((24, 20, 18, 22), 12, "bf16"),
    ((64, 30, 45), 20, "f32"),
    ((33, 41, 29), 5, "f32"),
    ((50, 50, 50), 26, "bf16"),
    ((18, 16, 20, 15), 9, "f32"),
    ((70, 35, 28), 11, "bf16"),
    ((45, 38, 60), 17, "bf16"),
]


def _problems():
    out = []
    for i, (dims, R, storage) in enumerate(REQS):
        dt = "bf16" if storage == "bf16" else np.float32
        prob = ci.make_problem(dims, R, data_seed=1500 + i, init_seed=1600 + i, snr_db=30.0,
                               dtype=dt)
        out.append(dict(X=np.asfortranarray(prob["X"].astype(np.float32)), A0=prob["A0"], B=64,
                        storage=storage, seed=1700, stream_id=i, eta=1.5, fit_target=0.99,
                        max_steps=1500))
    return out


def _wait(server, tickets, timeout=120.0):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = server.poll(t)
                if r is not None:
                    res[t] = r
        assert time.time() - t0 < timeout, "requests did not finish"
        time.sleep(0.002)
    return [res[t] for t in tickets]


def _arena(problems, n):
    import paper_2103_04081_amd as P
    sizes = []
    for p in problems:
        dims = list(p["X"].shape)
        sizes.append(P.cpd_workspace_size(P.make_problem(dims, p["A0"][0].shape[1], p["B"]),
                                          P.make_options(storage=p["storage"])))
    return sorted(sizes)[-n:], sum(sorted(sizes)[-n:])


def test_each_request_same_alone_and_in_the_mix():
    import paper_2103_04081_amd as P
    probs = _problems()
    _, two_largest = _arena(probs, 2)
    alone = []
    s = P.Server(two_largest + (8 << 20), max_slots=4, round_steps=20)
    for p in probs:
        t = s.submit(**p)
        alone.append(_wait(s, [t])[0])
    s.close()
    # all at once: at most 3 on the device at a time (slots), and the arena
    # holds only a few workspaces, so requests are admitted as others leave
    s = P.Server(two_largest + (8 << 20), max_slots=3, round_steps=20)
    tickets = [s.submit(**p) for p in probs]
    mixed = _wait(s, tickets)
    s.close()
    for i, (a, m) in enumerate(zip(alone, mixed)):
        print(f"request {i} {REQS[i]}: steps {m['steps']} fit {m['fit']:.5f} "
              f"queued {m['seconds_queued']:.4f}s to-fit {m['seconds_to_fit']:.4f}s", flush=True)
        assert a["status"] == m["status"] == 0
        assert a["steps"] == m["steps"] and a["fit"] == m["fit"]
        for x, y in zip(a["factors"], m["factors"]):
            np.testing.assert_array_equal(x, y)
    assert sum(m["reached"] for m in mixed) >= len(probs) - 2


def test_served_request_equals_single_handle_in_rounds():
    import paper_2103_04081_amd as P
    p = _problems()[2]
    s = P.Server(1 << 30, max_slots=2, round_steps=20)
    r = _wait(s, [s.submit(**p)])[0]
    s.close()
    d = P.Decomposition(p["X"], p["A0"], B=p["B"], eta=p["eta"], storage=p["storage"],
                        seed=p["seed"], stream_id=p["stream_id"])
    t = 0
    while True:
        k = min(20, p["max_steps"] - t)
        d.step(k)
        t += k
        fit = d.fit()
        if fit >= p["fit_target"] or t >= p["max_steps"]:
            break
    assert t == r["steps"] and fit == r["fit"]
    for x, y in zip(d.factors(), r["factors"]):
        np.testing.assert_array_equal(x, y)
    d.close()


def test_submit_errors_and_request_errors():
    import paper_2103_04081_amd as P
    probs = _problems()
    s = P.Server(4 << 20, max_slots=2, queue_capacity=2, round_steps=10)
    # a workspace larger than the arena can never be admitted
    big = ci.make_problem((200, 200, 100), 8, data_seed=1, init_seed=2, snr_db=30.0)
    with pytest.raises(P.CpdError) as e:
        s.submit(X=big["X"], A0=big["A0"], B=64)
    assert e.value.status == P.cpdmi.CPD_E_OOM
    # a served request must be bounded
    with pytest.raises(P.CpdError) as e:
        s.submit(**dict(probs[3], max_steps=0))
    assert e.value.status == P.cpdmi.CPD_E_INVALID
    with pytest.raises(P.CpdError) as e:
        s.poll(12345)
    assert e.value.status == P.cpdmi.CPD_E_NOT_FOUND
    s.close()
    # leverage scores of a rank-deficient factor: that request fails alone
    s = P.Server(64 << 20, max_slots=2, queue_capacity=8, round_steps=10)
    bad = dict(probs[3])
    A0 = [a.copy() for a in bad["A0"]]
    A0[1][:, 1] = A0[1][:, 0]
    bad.update(A0=A0, sampler="leverage")
    tb = s.submit(**bad)
    tg = s.submit(**probs[3])
    rb, rg = _wait(s, [tb, tg])
    assert rb["status"] == P.cpdmi.CPD_E_RANK_DEFICIENT
    assert rg["status"] == 0 and rg["steps"] > 0
    s.close()


def test_queue_capacity():
    import paper_2103_04081_amd as P
    probs = _problems()
    s = P.Server(64 << 20, max_slots=1, queue_capacity=2, round_steps=10)
    tickets, refused = [], 0
    for p in probs:
        try:
            tickets.append(s.submit(**dict(p, max_steps=400)))
        except P.CpdError as e:
            assert e.status == P.cpdmi.CPD_E_QUEUE_FULL
            refused += 1
    assert refused >= 1
    res = _wait(s, tickets)
    assert all(r["status"] == 0 for r in res)
    s.close()
