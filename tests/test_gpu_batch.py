"""Batched path on the GPU: every member of a batch computes exactly what a
single handle with the same problem, options and tile choice computes; the
graph-replayed rounds equal the same rounds launched one by one; members stop
on their own at the target fit or the step limit."""

import numpy as np
import pytest

import cpd_inputs as ci

pytestmark = pytest.mark.gpu

# (dims, R, B, sampler): three rank-tile classes, 3- and 4-way, all samplers
SPECS = [
    ((37, 45, 53), 7, 64, "euclidean"),
    ((20, 24, 22, 18), 12, 40, "leverage"),
    ((64, 48, 50), 20, 64, "euclidean"),
    ((40, 33, 70), 40, 64, "uniform"),
    ((30, 30, 30), 5, 18, "euclidean"),
    ((90, 17, 26), 9, 128, "leverage"),
]


def _members(storage="f32", fit_target=0.97, max_steps=400, fit_every=20, eta=0.5, specs=SPECS):
    dt = "bf16" if storage == "bf16" else np.float32
    out = []
    for i, (dims, R, B, sampler) in enumerate(specs):
        prob = ci.make_problem(dims, R, data_seed=700 + i, init_seed=800 + i, snr_db=30.0, dtype=dt)
        out.append(dict(X=np.asfortranarray(prob["X"].astype(np.float32)), A0=prob["A0"], B=B,
                        sampler=sampler, rule="adagrad", eta=eta, storage=storage,
                        fit_every=fit_every, fit_target=fit_target, max_steps=max_steps,
                        seed=900, stream_id=i))
    return out


def _alone(m, ksplit):
    """A single handle run the way a batch member runs: rounds of fit_every
    steps (capped at max_steps), a fit check after each, stop at the target."""
    import paper_2103_04081_amd as P
    d = P.Decomposition(m["X"], m["A0"], B=m["B"], sampler=m["sampler"], rule=m["rule"],
                        eta=m["eta"], storage=m["storage"], seed=m["seed"],
                        stream_id=m["stream_id"], ksplit=ksplit)
    t = 0
    while True:
        k = min(m["fit_every"], m["max_steps"] - t)
        d.step(k)
        t += k
        fit = d.fit()
        if fit >= m["fit_target"] or t >= m["max_steps"]:
            break
    out = (t, fit, d.factors())
    d.close()
    return out


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_batch_member_equals_single_handle(storage):
    import paper_2103_04081_amd as P
    members = _members(storage)
    b = P.Batch(members, tune=True)
    left = b.run(max_rounds=100)
    assert left == 0
    for i, m in enumerate(members):
        info = b.info(i)
        print(f"member {i} dims {SPECS[i][0]} R {SPECS[i][1]} t_done {info['t_done']} "
              f"fit {info['fit']:.5f} ksplit {info['ksplit']}", flush=True)
        assert info["done"] and info["status"] == 0
        t, fit, F = _alone(m, info["ksplit"])
        assert t == info["t_done"] == info["t"]
        assert fit == info["fit"]
        for a, g in zip(F, b.factors(i)):
            np.testing.assert_array_equal(a, g)
    b.close()


def test_graph_rounds_equal_launched_rounds():
    """Replays of the captured round graph (with host reads between them)
    give the same members as the same rounds launched directly."""
    import paper_2103_04081_amd as P
    members = _members("f32", fit_target=2.0, max_steps=10_000)  # target never reached
    g = P.Batch(members, tune=False)
    d = P.Batch(members, tune=False)
    for r in range(6):
        assert g.run(max_rounds=1) == len(members)
        d.step(members[0]["fit_every"])
        fits = d.fits()
        for i in range(len(members)):
            gi = g.info(i)
            assert gi["t"] == (r + 1) * members[0]["fit_every"]
            assert gi["fit"] == fits[i]
            for a, c in zip(g.factors(i), d.factors(i)):
                np.testing.assert_array_equal(a, c)
    g.close()
    d.close()


def test_members_stop_at_step_limit_and_target():
    import paper_2103_04081_amd as P
    members = _members("f32", fit_target=0.9, max_steps=50, fit_every=20)
    members[0]["fit_target"] = 2.0   # unreachable: stops at the limit (50 = 20 + 20 + 10)
    members[1]["max_steps"] = 10_000
    members[1]["fit_target"] = 0.5
    b = P.Batch(members, tune=False)
    assert b.run(max_rounds=50) == 0
    i0, i1 = b.info(0), b.info(1)
    assert i0["done"] and i0["t"] == 50 and i0["t_done"] == 50
    assert i1["done"] and i1["fit"] >= 0.5 and i1["t"] % 20 == 0
    assert i1["seconds_done"] > 0
    # further rounds do not move stopped members
    F = b.factors(0)
    b.step(20)
    b.sync()
    assert b.info(0)["t"] == 50
    for a, c in zip(F, b.factors(0)):
        np.testing.assert_array_equal(a, c)
    b.close()


def test_batch_workload_recipe_small_reaches_fit():
    """The batch recipe (uneven dims, ranks 5-32, B 128, BF16) at capped dims:
    every member reaches fit 0.99."""
    import paper_2103_04081_amd as P
    specs = ci.batch_workload(count=12, max_dims=80)
    members = []
    for s in specs:
        prob = ci.make_problem(s["dims"], s["R"], data_seed=s["data_seed"],
                               init_seed=s["init_seed"], snr_db=s["snr_db"], dtype="bf16")
        members.append(dict(X=np.asfortranarray(prob["X"].astype(np.float32)), A0=prob["A0"],
                            B=s["B"], sampler="euclidean", rule="adagrad", eta=1.5,
                            storage="bf16", fit_every=25, fit_target=0.99, max_steps=5000,
                            seed=s["seed"], stream_id=s["stream_id"]))
    b = P.Batch(members, tune=True)
    assert b.run(max_rounds=400) == 0
    for i in range(len(members)):
        info = b.info(i)
        print(f"member {i} dims {specs[i]['dims']} R {specs[i]['R']} t {info['t_done']} "
              f"fit {info['fit']:.5f}", flush=True)
        assert info["status"] == 0 and info["fit"] >= 0.99
    b.close()
