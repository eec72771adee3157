"""The seeded input generators (CPU): layouts and noise level."""

import numpy as np

import cpd_inputs as ci


def test_device_problem_layout_matches_host_recipe():
    import torch
    spec = dict(dims=[5, 4, 3, 2], R=3, data_seed=7, init_seed=8, snr_db=None)
    X, A0 = ci.device_problem(spec, device="cpu")
    assert X.dtype == torch.float32 and list(X.shape) == [2, 3, 4, 5]
    A = ci.gaussian_factors([5, 4, 3, 2], 3, ci.rng_for(7))
    ref = ci.cp_full(A)
    # C order of shape dims[::-1] is Fortran order of shape dims
    np.testing.assert_allclose(X.numpy().ravel(), ref.ravel(order="F"), rtol=1e-5, atol=1e-5)
    for a, b in zip(A0, ci.init_factors([5, 4, 3, 2], 3, 8)):
        np.testing.assert_array_equal(a, b)


def test_device_problem_noise_level():
    spec = dict(dims=[30, 20, 10], R=4, data_seed=3, init_seed=4, snr_db=20.0)
    X, _ = ci.device_problem(spec, device="cpu")
    Xt, _ = ci.device_problem(dict(spec, snr_db=None), device="cpu")
    x, xt = X.numpy().astype(np.float64), Xt.numpy().astype(np.float64)
    snr = 20 * np.log10(np.linalg.norm(xt) / np.linalg.norm(x - xt))
    assert abs(snr - 20.0) < 1e-3


def test_request_trace_recipe():
    tr = ci.request_trace(400)
    gaps = np.diff([0.0] + [r["arrival"] for r in tr])
    assert abs(gaps.mean() - 1 / 50.0) < 0.004          # Poisson at 50 req/s
    three = [r for r in tr if len(r["dims"]) == 3]
    four = [r for r in tr if len(r["dims"]) == 4]
    assert 0.4 < len(three) / len(tr) < 0.6
    assert all(64 <= d <= 512 for r in three for d in r["dims"])
    assert all(32 <= d <= 128 for r in four for d in r["dims"])
    assert all(8 <= r["R"] <= 32 and r["R"] <= min(r["dims"]) for r in tr)


def test_batch_workload_recipe():
    specs = ci.batch_workload(count=64)
    assert len(specs) == 64
    assert all(50 <= d <= 400 for s in specs for d in s["dims"])
    assert all(5 <= s["R"] <= 32 and s["B"] == 128 for s in specs)
