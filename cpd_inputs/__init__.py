"""Seeded synthetic inputs for the CP decomposition workloads.

This module only *makes data*: factor matrices, CP tensors with noise, the
initial factors and request traces.  It holds none of the stochastic-gradient
method's arithmetic, and both the FP64 oracle and the HIP path consume what
it produces.

Data model (paper, Section 5.2 "Synthetic data"): a true tensor built from
Gaussian factor matrices, plus Gaussian noise scaled so that
    X = X_true + noise * (||X_true|| / ||N||) * N,   N iid N(0, 1).
A signal-to-noise ratio of s dB corresponds to noise = 10**(-s/20).

The paper's own generator for its skewed factors is not specified, so the
skew is produced here by two explicit recipes instead: columns with a fixed
pairwise cosine (column congruence) and a subset of rows scaled up.

Tensors are returned as FP64 numpy arrays of shape ``dims`` in Fortran order,
i.e. mode 1 varies fastest in memory, which is the order in which the mode-1
unfolding of the paper's index map enumerates entries.
"""

import math

import numpy as np

__all__ = [
    "rng_for",
    "gaussian_factors",
    "congruent_factors",
    "skew_rows",
    "cp_full",
    "add_noise",
    "init_factors",
    "make_problem",
    "workload",
    "batch_workload",
    "request_trace",
    "round_bf16",
    "device_problem",
    "variance_data",
]


def rng_for(seed):
    """A numpy Generator on PCG64 for a fixed integer seed."""
    return np.random.Generator(np.random.PCG64(int(seed)))


def gaussian_factors(dims, R, rng):
    """Factor matrices with iid N(0,1) entries, one I_k x R matrix per mode."""
    return [rng.standard_normal((int(I), int(R))) for I in dims]


def congruent_factors(dims, R, rho, rng):
    """Factors whose columns have pairwise cosine exactly ``rho``.

    U has orthonormal columns (QR of a Gaussian matrix); with C the R x R
    matrix of ones off the diagonal scaled by rho and ones on it, and
    C = L L^T, the factor sqrt(I) * U * L^T has Gram I * C.
    """
    C = rho * np.ones((R, R)) + (1.0 - rho) * np.eye(R)
    L = np.linalg.cholesky(C)
    out = []
    for I in dims:
        U, _ = np.linalg.qr(rng.standard_normal((int(I), int(R))))
        out.append(math.sqrt(I) * U @ L.T)
    return out


def skew_rows(factors, frac, scale, rng):
    """Scale a random subset of ceil(frac * I_k) rows of every factor by ``scale``."""
    out = []
    for A in factors:
        A = np.array(A, dtype=np.float64, copy=True)
        I = A.shape[0]
        k = int(math.ceil(frac * I))
        rows = rng.choice(I, size=k, replace=False)
        A[rows, :] *= scale
        out.append(A)
    return out


def cp_full(factors):
    """Dense tensor sum_r a^(1)_r o ... o a^(N)_r (FP64, Fortran order)."""
    factors = [np.asarray(A, dtype=np.float64) for A in factors]
    dims = [A.shape[0] for A in factors]
    R = factors[0].shape[1]
    # rows of T enumerate (i_1, ..., i_{N-1}) with i_1 fastest
    T = factors[0]
    for A in factors[1:-1]:
        T = (A[:, None, :] * T[None, :, :]).reshape(-1, R)
    flat = factors[-1] @ T.T  # (I_N, J) row-major: i_N slowest
    return flat.reshape(dims[::-1]).transpose()


def add_noise(X, snr_db, rng):
    """X + sigma * N with sigma = ||X|| / (||N|| * 10**(snr/20)); None = no noise."""
    if snr_db is None:
        return np.asfortranarray(X)
    Nz = rng.standard_normal(X.shape[::-1]).transpose()  # Fortran order like X
    sigma = np.linalg.norm(X.ravel(order="K")) / (
        np.linalg.norm(Nz.ravel(order="K")) * 10.0 ** (snr_db / 20.0))
    out = X + sigma * Nz
    return np.asfortranarray(out)


def init_factors(dims, R, seed):
    """Initial factors: N(0,1) drawn in FP64 on the host, rounded to FP32."""
    rng = rng_for(seed)
    return [rng.standard_normal((int(I), int(R))).astype(np.float32).astype(np.float64)
            for I in dims]


def round_bf16(a):
    """Round FP32 values to bfloat16 (round to nearest, ties to even), as FP32."""
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32)
    out = np.where(nan, a, out)
    return out


def make_problem(dims, R, *, data_seed, init_seed, snr_db=None, rho=None,
                 skew=None, R_true=None, dtype=np.float32, nonneg=False):
    """One synthetic problem: tensor, true factors and initial factors.

    ``dtype`` is the storage type the HIP path will hold; the returned ``X``
    is the FP64 tensor rounded to that type (and widened back to FP64), so
    that both sides see identical values.  ``X64`` keeps the unrounded one.
    """
    rng = rng_for(data_seed)
    Rt = R if R_true is None else R_true
    if rho is not None:
        A = congruent_factors(dims, Rt, rho, rng)
    else:
        A = gaussian_factors(dims, Rt, rng)
    if skew is not None:
        A = skew_rows(A, skew[0], skew[1], rng)
    if nonneg:
        A = [np.abs(a) for a in A]
    X64 = add_noise(cp_full(A), snr_db, rng)
    if dtype == "bf16":
        Xs = round_bf16(X64.ravel(order="F").astype(np.float32)).astype(np.float64)
        Xs = Xs.reshape(X64.shape, order="F")
    else:
        Xs = np.asfortranarray(X64.astype(dtype).astype(np.float64))
    A0 = init_factors(dims, R, init_seed)
    if nonneg:
        A0 = [np.abs(a) for a in A0]
    return {"dims": list(map(int, dims)), "R": int(R), "X": Xs, "X64": X64,
            "A_true": A, "A0": A0}


# The five workloads.  Seeds: data 1000 + c, init 2000 + c, Philox key (3000 + c, id).
_WORKLOADS = {
    # the 30^3 tensor is built in FP64; the device stores it in FP32
    1: dict(name="dense 30x30x30 R5 B18 SNR40", dims=(30, 30, 30), R=5, B=18,
            snr_db=40.0, dtype=np.float32),
    2: dict(name="300x300x300 R10 B256 FP32, rho0.6, 10% rows x20, SNR30",
            dims=(300, 300, 300), R=10, B=256, snr_db=30.0, rho=0.6,
            skew=(0.1, 20.0), dtype=np.float32),
    3: dict(name="120^4 R20 B512 SNR30", dims=(120, 120, 120, 120), R=20, B=512,
            snr_db=30.0, dtype=np.float32),
}


def workload(c, *, dims=None, dtype=None, with_problem=True):
    """Problem dict for workload ``c`` (1, 2 or 3), optionally at other dims.

    Returns the problem plus ``B``, ``seed`` and ``stream_id``.
    """
    spec = dict(_WORKLOADS[c])
    if dims is not None:
        spec["dims"] = tuple(dims)
    if dtype is not None:
        spec["dtype"] = dtype
    out = {"name": spec["name"], "B": spec["B"], "seed": 3000 + c, "stream_id": 0,
           "dims": list(spec["dims"]), "R": spec["R"]}
    if with_problem:
        out.update(make_problem(spec["dims"], spec["R"], data_seed=1000 + c,
                                init_seed=2000 + c, snr_db=spec.get("snr_db"),
                                rho=spec.get("rho"), skew=spec.get("skew"),
                                dtype=spec["dtype"]))
    return out


def batch_workload(count=64, *, dim_range=(50, 400), rank_range=(5, 32), B=128,
                   snr_db=30.0, dtype="bf16", seed=1004, max_dims=None):
    """Many independent 3-way problems with uneven dims and ranks.

    dims ~ U{dim_range} per mode, R ~ U{rank_range}.  ``max_dims`` caps the
    dims (for small test versions of the same recipe).
    """
    rng = rng_for(seed)
    specs = []
    for i in range(count):
        dims = [int(d) for d in rng.integers(dim_range[0], dim_range[1] + 1, size=3)]
        if max_dims is not None:
            dims = [min(d, max_dims) for d in dims]
        R = int(rng.integers(rank_range[0], rank_range[1] + 1))
        specs.append(dict(dims=dims, R=R, B=B, data_seed=seed * 1000 + i,
                          init_seed=seed * 1000 + 500 + i, snr_db=snr_db, dtype=dtype,
                          seed=3004, stream_id=i))
    return specs


def request_trace(count, *, rate=50.0, seed=1005, B=128, snr_db=30.0, dtype="bf16",
                  dim3=(64, 512), dim4=(32, 128), rank_range=(8, 32)):
    """Poisson arrivals of decomposition requests (3-way / 4-way mix, 50/50)."""
    rng = rng_for(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.random() < 0.5:
            dims = [int(d) for d in rng.integers(dim3[0], dim3[1] + 1, size=3)]
        else:
            dims = [int(d) for d in rng.integers(dim4[0], dim4[1] + 1, size=4)]
        R = int(rng.integers(rank_range[0], rank_range[1] + 1))
        R = min(R, min(dims))
        out.append(dict(arrival=t, dims=dims, R=R, B=B, data_seed=seed * 1000 + i,
                        init_seed=seed * 1000 + 500 + i, snr_db=snr_db, dtype=dtype,
                        seed=3005, stream_id=i))
    return out


def device_problem(spec, device="cuda"):
    """The recipe of :func:`make_problem` (Gaussian factors, no skew) with the
    tensor formed on the device, for workloads too large to build on the host
    at their arrival rate.

    The true factors and the initial factors come from PCG64 on the host as in
    :func:`make_problem`; X_true = [[A]] is one FP32 GEMM on the device and
    the noise comes from torch's device generator seeded with the data seed.
    Returns (X, A0) with X a C-contiguous FP32 device tensor of shape
    dims[::-1] (mode 1 fastest in memory).
    """
    import torch

    dims, R = [int(d) for d in spec["dims"]], int(spec["R"])
    rng = rng_for(spec["data_seed"])
    A = gaussian_factors(dims, R, rng)
    A0 = init_factors(dims, R, spec["init_seed"])
    F = [torch.as_tensor(a, dtype=torch.float32, device=device) for a in A]
    # rows of T enumerate (i_2, ..., i_N) with i_2 fastest
    T = F[1]
    for a in F[2:]:
        T = (a[:, None, :] * T[None, :, :]).reshape(-1, R)
    X = T @ F[0].T  # (J_1, I_1) row-major: i_1 fastest in memory
    if spec.get("snr_db") is not None:
        g = torch.Generator(device=device)
        g.manual_seed(int(spec["data_seed"]))
        Nz = torch.randn(X.shape, generator=g, device=device, dtype=torch.float32)
        sigma = torch.linalg.vector_norm(X) / (torch.linalg.vector_norm(Nz)
                                               * 10.0 ** (spec["snr_db"] / 20.0))
        X.add_(Nz, alpha=float(sigma))
        del Nz
    return X.reshape(dims[::-1]).contiguous(), A0


def variance_data(which, *, seed=1010, I=300, R=10):
    """The tensors of the paper's variance comparison (Section 5): Data II is
    built from three I x R factors with iid N(0,1) entries; Data III is Data
    II with one uniformly chosen entry of each factor set to 20.  No noise.
    Returns a problem dict like :func:`make_problem` (FP32 storage)."""
    rng = rng_for(seed)
    A = gaussian_factors([I, I, I], R, rng)
    if which == 3:
        for a in A:
            a[int(rng.integers(0, a.shape[0])), int(rng.integers(0, a.shape[1]))] = 20.0
    elif which != 2:
        raise ValueError("which must be 2 or 3")
    X64 = cp_full(A)
    X = np.asfortranarray(X64.astype(np.float32).astype(np.float64))
    A0 = init_factors([I, I, I], R, seed + 1)
    return {"dims": [I, I, I], "R": R, "X": X, "X64": X64, "A_true": A, "A0": A0}
