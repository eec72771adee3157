"""ctypes binding of libcpdmi (the C ABI declared in include/cpd.h).

The functions here carry the C names and only marshal arguments: every step
of the method runs in the library's HIP kernels.  PyTorch supplies device
memory (the caller-owned workspace) and the HIP stream.
"""

import ctypes
import os

import numpy as np

import torch  # noqa: F401  (load torch's HIP runtime before the library)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpdmi.so")

MAX_MODES = 8
MAX_RANK = 128

CPD_OK, CPD_PENDING = 0, 1
CPD_E_INVALID, CPD_E_OOM, CPD_E_HIP = -1, -2, -3
CPD_E_RANK_DEFICIENT, CPD_E_DEGENERATE, CPD_E_DIVERGED = -4, -5, -6
CPD_E_QUEUE_FULL, CPD_E_NOT_FOUND, CPD_E_CANCELLED = -7, -8, -9

SAMPLER = {"uniform": 0, "leverage": 1, "euclidean": 2}
RULE = {"fixed": 0, "adagrad": 1, "decreasing": 2}
CPD_F32, CPD_BF16, CPD_F64 = 0, 1, 2
CPD_HOST, CPD_DEVICE = 0, 1
CPD_PATH_AUTO, CPD_PATH_PERSISTENT, CPD_PATH_GRID = 0, 1, 2
PATH = {"auto": CPD_PATH_AUTO, "persistent": CPD_PATH_PERSISTENT, "grid": CPD_PATH_GRID}
MAX_PERSISTENT_BATCH = 4096
MAX_BATCH = 1 << 20
STORAGE = {"f32": CPD_F32, "fp32": CPD_F32, "float32": CPD_F32, "bf16": CPD_BF16,
           "bfloat16": CPD_BF16}


class CpdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"cpd status {status}: {msg}")
        self.status = status


class cpd_problem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("dims", ctypes.c_int32 * MAX_MODES),
                ("R", ctypes.c_int32), ("B", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint64)]


class cpd_options(ctypes.Structure):
    _fields_ = [("sampler", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("eta", ctypes.c_double), ("b", ctypes.c_double),
                ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("storage", ctypes.c_int32), ("nonneg", ctypes.c_int32),
                ("fit_every", ctypes.c_int32), ("fit_target", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("ksplit", ctypes.c_int32 * MAX_MODES),
                ("path", ctypes.c_int32), ("rescale_every", ctypes.c_int32)]


class cpd_member_info(ctypes.Structure):
    _fields_ = [("t", ctypes.c_int64), ("fit", ctypes.c_double), ("done", ctypes.c_int32),
                ("status", ctypes.c_int32), ("t_done", ctypes.c_int64),
                ("seconds_done", ctypes.c_double), ("ksplit", ctypes.c_int32 * MAX_MODES)]


class cpd_server_config(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("queue_capacity", ctypes.c_int32),
                ("round_steps", ctypes.c_int32), ("pad", ctypes.c_int32)]


class cpd_request(ctypes.Structure):
    _fields_ = [("problem", cpd_problem), ("options", cpd_options), ("X", ctypes.c_void_p),
                ("x_dtype", ctypes.c_int32), ("x_space", ctypes.c_int32),
                ("A0", ctypes.c_void_p * MAX_MODES), ("out", ctypes.c_void_p * MAX_MODES)]


class cpd_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("reached", ctypes.c_int32), ("fit", ctypes.c_double),
                ("steps", ctypes.c_int64), ("seconds_queued", ctypes.c_double),
                ("seconds_admit", ctypes.c_double), ("seconds_to_fit", ctypes.c_double),
                ("seconds_total", ctypes.c_double)]


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2103_04081_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        H = ctypes.c_void_p
        P = ctypes.POINTER
        st = ctypes.c_int32
        sig = {
            "cpd_last_error": (ctypes.c_char_p, []),
            "cpd_version": (ctypes.c_char_p, []),
            "cpd_workspace_size": (st, [P(cpd_problem), P(cpd_options), P(ctypes.c_size_t)]),
            "cpd_init": (st, [P(cpd_problem), P(cpd_options), ctypes.c_void_p, ctypes.c_int32,
                              ctypes.c_int32, P(ctypes.c_void_p), ctypes.c_void_p,
                              ctypes.c_size_t, ctypes.c_void_p, P(H)]),
            "cpd_sample": (st, [H, ctypes.c_uint64, P(ctypes.c_int32), ctypes.c_void_p,
                                ctypes.c_void_p]),
            "cpd_step": (st, [H, ctypes.c_int64]),
            "cpd_step_replay": (st, [H, ctypes.c_int32, ctypes.c_void_p]),
            "cpd_rescale": (st, [H]),
            "cpd_sync": (st, [H]),
            "cpd_fit": (st, [H, P(ctypes.c_double)]),
            "cpd_get_step": (st, [H, P(ctypes.c_int64)]),
            "cpd_read_factors": (st, [H, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32]),
            "cpd_read_cdf": (st, [H, ctypes.c_int32, ctypes.c_void_p]),
            "cpd_read_state": (st, [H, ctypes.c_void_p, P(ctypes.c_size_t)]),
            "cpd_write_state": (st, [H, ctypes.c_void_p, ctypes.c_size_t]),
            "cpd_destroy": (st, [H]),
            "cpd_variance_workspace_size": (st, [H, ctypes.c_int32, P(ctypes.c_size_t)]),
            "cpd_variance": (st, [H, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_size_t, P(ctypes.c_double)]),
            "cpd_variance_noalloc": (st, [H, ctypes.c_int32, ctypes.c_int32, P(ctypes.c_double)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _extra_signatures(L)
        _lib = L
    return _lib


def _extra_signatures(L):
    """Signatures of the batched and serving entry points (if present)."""
    H = ctypes.c_void_p
    P = ctypes.POINTER
    st = ctypes.c_int32
    vp = ctypes.c_void_p
    extra = {
        "cpd_batch_workspace_size": (st, [P(cpd_problem), P(cpd_options), ctypes.c_int32,
                                          P(ctypes.c_size_t)]),
        "cpd_batch_create": (st, [P(cpd_problem), P(cpd_options), ctypes.c_int32, P(vp),
                                  ctypes.c_int32, ctypes.c_int32, P(vp), vp, ctypes.c_size_t, vp,
                                  ctypes.c_int32, P(H)]),
        "cpd_batch_step": (st, [H, ctypes.c_int64]),
        "cpd_batch_fits": (st, [H, P(ctypes.c_double)]),
        "cpd_batch_run": (st, [H, ctypes.c_int64, P(ctypes.c_int32)]),
        "cpd_batch_sync": (st, [H]),
        "cpd_batch_member_info": (st, [H, ctypes.c_int32, P(cpd_member_info)]),
        "cpd_batch_read_factors": (st, [H, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_int32]),
        "cpd_batch_destroy": (st, [H]),
        "cpd_server_create": (st, [P(cpd_server_config), vp, ctypes.c_size_t, P(H)]),
        "cpd_submit": (st, [H, P(cpd_request), P(ctypes.c_uint64)]),
        "cpd_poll": (st, [H, ctypes.c_uint64, P(cpd_result)]),
        "cpd_server_stats": (st, [H, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]),
        "cpd_server_destroy": (st, [H]),
    }
    for name, (res, args) in extra.items():
        if hasattr(L, name):
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args


def last_error():
    return lib().cpd_last_error().decode()


def check(status, what=""):
    if status < 0:
        raise CpdError(status, f"{what}: {last_error()}")
    return status


def make_problem(dims, R, B, seed=0, stream_id=0):
    p = cpd_problem()
    p.N = len(dims)
    for k, d in enumerate(dims):
        p.dims[k] = int(d)
    p.R, p.B = int(R), int(B)
    p.seed, p.stream_id = int(seed), int(stream_id)
    return p


def make_options(sampler="euclidean", rule="adagrad", alpha=0.0, eta=1.0, b=0.0, beta=0.0,
                 gamma=1.0, storage="f32", nonneg=False, fit_every=25, fit_target=0.99,
                 max_steps=0, ksplit=None, path="auto", rescale_every=0):
    o = cpd_options()
    o.sampler = SAMPLER[sampler] if isinstance(sampler, str) else int(sampler)
    o.rule = RULE[rule] if isinstance(rule, str) else int(rule)
    o.alpha, o.eta, o.b, o.beta, o.gamma = float(alpha), float(eta), float(b), float(beta), float(gamma)
    o.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    o.nonneg = int(bool(nonneg))
    o.fit_every = int(fit_every)
    o.fit_target = float(fit_target)
    o.max_steps = int(max_steps)
    for k, v in enumerate(ksplit or []):
        o.ksplit[k] = int(v)
    o.path = PATH[path] if isinstance(path, str) else int(path)
    o.rescale_every = int(rescale_every)
    return o


# --- thin wrappers with the C names ----------------------------------------

def cpd_workspace_size(problem, options):
    n = ctypes.c_size_t()
    check(lib().cpd_workspace_size(ctypes.byref(problem), ctypes.byref(options), ctypes.byref(n)),
          "cpd_workspace_size")
    return n.value


def cpd_init(problem, options, X_ptr, x_dtype, x_space, A0_list, ws_ptr, ws_bytes, stream):
    arr = (ctypes.c_void_p * len(A0_list))(*[a.ctypes.data for a in A0_list])
    h = ctypes.c_void_p()
    check(lib().cpd_init(ctypes.byref(problem), ctypes.byref(options), ctypes.c_void_p(X_ptr),
                         x_dtype, x_space, arr, ctypes.c_void_p(ws_ptr), ws_bytes,
                         ctypes.c_void_p(stream), ctypes.byref(h)), "cpd_init")
    return h


def cpd_sample(h, t, idx_ptr, p_ptr):
    mode = ctypes.c_int32()
    check(lib().cpd_sample(h, int(t), ctypes.byref(mode), ctypes.c_void_p(idx_ptr),
                           ctypes.c_void_p(p_ptr)), "cpd_sample")
    return mode.value


def cpd_step(h, nsteps):
    return check(lib().cpd_step(h, int(nsteps)), "cpd_step")


def cpd_step_replay(h, mode, idx_ptr):
    return check(lib().cpd_step_replay(h, int(mode), ctypes.c_void_p(idx_ptr)), "cpd_step_replay")


def cpd_rescale(h):
    return check(lib().cpd_rescale(h), "cpd_rescale")


def cpd_sync(h):
    return check(lib().cpd_sync(h), "cpd_sync")


def cpd_fit(h):
    f = ctypes.c_double()
    check(lib().cpd_fit(h, ctypes.byref(f)), "cpd_fit")
    return f.value


def cpd_get_step(h):
    t = ctypes.c_int64()
    check(lib().cpd_get_step(h, ctypes.byref(t)), "cpd_get_step")
    return t.value


def cpd_read_factors(h, n, dst_ptr, space):
    return check(lib().cpd_read_factors(h, int(n), ctypes.c_void_p(dst_ptr), space),
                 "cpd_read_factors")


def cpd_read_cdf(h, n, dst_ptr):
    return check(lib().cpd_read_cdf(h, int(n), ctypes.c_void_p(dst_ptr)), "cpd_read_cdf")


def cpd_read_state(h):
    n = ctypes.c_size_t()
    check(lib().cpd_read_state(h, None, ctypes.byref(n)), "cpd_read_state")
    buf = ctypes.create_string_buffer(n.value)
    check(lib().cpd_read_state(h, buf, ctypes.byref(n)), "cpd_read_state")
    return bytes(buf.raw[:n.value])


def cpd_write_state(h, blob):
    buf = ctypes.create_string_buffer(blob, len(blob))
    return check(lib().cpd_write_state(h, buf, len(blob)), "cpd_write_state")


def cpd_variance_workspace_size(h, n):
    out = ctypes.c_size_t()
    check(lib().cpd_variance_workspace_size(h, int(n), ctypes.byref(out)),
          "cpd_variance_workspace_size")
    return out.value


def cpd_variance(h, n, sampler, ws_ptr, ws_bytes):
    """(variance, (1/B) sum of the terms, (1/B) ||grad f||^2) for mode n."""
    out = (ctypes.c_double * 3)()
    s = SAMPLER[sampler] if isinstance(sampler, str) else int(sampler)
    check(lib().cpd_variance(h, int(n), s, ctypes.c_void_p(ws_ptr), ctypes.c_size_t(ws_bytes),
                             out), "cpd_variance")
    return out[0], out[1], out[2]


def cpd_variance_noalloc(h, n, sampler):
    """cpd_variance with the library's static scratch (allocates nothing)."""
    out = (ctypes.c_double * 3)()
    s = SAMPLER[sampler] if isinstance(sampler, str) else int(sampler)
    check(lib().cpd_variance_noalloc(h, int(n), s, out), "cpd_variance_noalloc")
    return out[0], out[1], out[2]


def cpd_destroy(h):
    return check(lib().cpd_destroy(h), "cpd_destroy")


def cpd_batch_workspace_size(problems, options):
    n = len(problems)
    P = (cpd_problem * n)(*problems)
    O = (cpd_options * n)(*options)
    out = ctypes.c_size_t()
    check(lib().cpd_batch_workspace_size(P, O, n, ctypes.byref(out)), "cpd_batch_workspace_size")
    return out.value


def cpd_batch_create(problems, options, X_ptrs, x_dtype, x_space, A0_ptrs, ws_ptr, ws_bytes,
                     stream, tune):
    """A0_ptrs: per member a list of N host addresses (padded to MAX_MODES here)."""
    n = len(problems)
    P = (cpd_problem * n)(*problems)
    O = (cpd_options * n)(*options)
    xs = (ctypes.c_void_p * n)(*X_ptrs)
    flat = []
    for ptrs in A0_ptrs:
        flat.extend(list(ptrs) + [None] * (MAX_MODES - len(ptrs)))
    a0 = (ctypes.c_void_p * len(flat))(*flat)
    h = ctypes.c_void_p()
    check(lib().cpd_batch_create(P, O, n, xs, x_dtype, x_space, a0, ctypes.c_void_p(ws_ptr),
                                 ws_bytes, ctypes.c_void_p(stream), int(tune), ctypes.byref(h)),
          "cpd_batch_create")
    return h


def cpd_batch_step(b, nsteps):
    return check(lib().cpd_batch_step(b, int(nsteps)), "cpd_batch_step")


def cpd_batch_fits(b, count):
    out = (ctypes.c_double * count)()
    check(lib().cpd_batch_fits(b, out), "cpd_batch_fits")
    return list(out)


def cpd_batch_run(b, max_rounds):
    left = ctypes.c_int32()
    check(lib().cpd_batch_run(b, int(max_rounds), ctypes.byref(left)), "cpd_batch_run")
    return left.value


def cpd_batch_sync(b):
    return check(lib().cpd_batch_sync(b), "cpd_batch_sync")


def cpd_batch_member_info(b, i):
    info = cpd_member_info()
    check(lib().cpd_batch_member_info(b, int(i), ctypes.byref(info)), "cpd_batch_member_info")
    return info


def cpd_batch_read_factors(b, i, n, dst_ptr, space):
    return check(lib().cpd_batch_read_factors(b, int(i), int(n), ctypes.c_void_p(dst_ptr), space),
                 "cpd_batch_read_factors")


def cpd_batch_destroy(b):
    return check(lib().cpd_batch_destroy(b), "cpd_batch_destroy")


def cpd_server_create(max_slots, queue_capacity, round_steps, arena_ptr, arena_bytes):
    cfg = cpd_server_config(int(max_slots), int(queue_capacity), int(round_steps), 0)
    h = ctypes.c_void_p()
    check(lib().cpd_server_create(ctypes.byref(cfg), ctypes.c_void_p(arena_ptr), arena_bytes,
                                  ctypes.byref(h)), "cpd_server_create")
    return h


def cpd_submit(s, request):
    t = ctypes.c_uint64()
    check(lib().cpd_submit(s, ctypes.byref(request), ctypes.byref(t)), "cpd_submit")
    return t.value


def cpd_poll(s, ticket):
    """None while pending, else the cpd_result."""
    r = cpd_result()
    st = check(lib().cpd_poll(s, int(ticket), ctypes.byref(r)), "cpd_poll")
    return None if st == CPD_PENDING else r


def cpd_server_stats(s):
    w, r, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    check(lib().cpd_server_stats(s, ctypes.byref(w), ctypes.byref(r), ctypes.byref(f)),
          "cpd_server_stats")
    return w.value, r.value, f.value


def cpd_server_destroy(s):
    return check(lib().cpd_server_destroy(s), "cpd_server_destroy")


# --- convenience objects ----------------------------------------------------

def _host_tensor(X):
    Xn = np.asarray(X)
    x_dtype = CPD_F64 if Xn.dtype == np.float64 else CPD_F32
    Xf = np.asfortranarray(Xn.astype(np.float64 if x_dtype == CPD_F64 else np.float32, copy=False))
    return Xf, x_dtype


def _workspace(nbytes, device):
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    return ws, (ws.data_ptr() + 255) // 256 * 256


class Batch:
    """Many decompositions advanced together (one persistent launch).

    ``members``: list of dicts with keys X (numpy tensor), A0 (list of
    factors), B, and any option of :func:`make_options` plus seed and
    stream_id.  All members share ``storage`` and ``fit_every``.
    """

    def __init__(self, members, *, tune=True, device="cuda"):
        self.device = torch.device(device)
        self.members = []
        problems, options, xs, a0s, keep = [], [], [], [], []
        x_dtype = None
        opt_keys = ("sampler", "rule", "alpha", "eta", "b", "beta", "gamma", "storage", "nonneg",
                    "fit_every", "fit_target", "max_steps", "ksplit")
        for m in members:
            Xf, xd = _host_tensor(m["X"])
            if x_dtype is None:
                x_dtype = xd
            if xd != x_dtype:
                Xf, xd = Xf.astype(np.float64 if x_dtype == CPD_F64 else np.float32), x_dtype
                Xf = np.asfortranarray(Xf)
            A0 = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in m["A0"]]
            dims = list(Xf.shape)
            R = A0[0].shape[1]
            problems.append(make_problem(dims, R, m["B"], m.get("seed", 0), m.get("stream_id", 0)))
            options.append(make_options(**{k: m[k] for k in opt_keys if k in m}))
            xs.append(Xf.ctypes.data)
            a0s.append([a.ctypes.data for a in A0])
            keep.append((Xf, A0))
            self.members.append({"dims": dims, "R": R})
        self.count = len(problems)
        self.ws_bytes = cpd_batch_workspace_size(problems, options)
        self.ws, self.ws_ptr = _workspace(self.ws_bytes, self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = cpd_batch_create(problems, options, xs, x_dtype, CPD_HOST, a0s, self.ws_ptr,
                                  self.ws_bytes, self.stream.cuda_stream, tune)
        del keep

    def step(self, nsteps):
        cpd_batch_step(self.h, nsteps)

    def fits(self):
        return cpd_batch_fits(self.h, self.count)

    def run(self, max_rounds):
        return cpd_batch_run(self.h, max_rounds)

    def sync(self):
        cpd_batch_sync(self.h)

    def info(self, i):
        inf = cpd_batch_member_info(self.h, i)
        N = len(self.members[i]["dims"])
        return {"t": inf.t, "fit": inf.fit, "done": bool(inf.done), "status": inf.status,
                "t_done": inf.t_done, "seconds_done": inf.seconds_done,
                "ksplit": [inf.ksplit[k] for k in range(N)]}

    def factors(self, i):
        m = self.members[i]
        out = []
        for k, I in enumerate(m["dims"]):
            a = np.empty((I, m["R"]), dtype=np.float32)
            cpd_batch_read_factors(self.h, i, k, a.ctypes.data, CPD_HOST)
            out.append(a)
        return out

    def close(self):
        if getattr(self, "h", None) is not None:
            cpd_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Decomposition:
    """One decomposition bound to a torch-allocated device workspace.

    ``X``: numpy array (any order; taken as the tensor of shape dims) or a
    CUDA torch tensor whose memory is mode-1-fastest (shape dims[::-1],
    C-contiguous).  ``A0``: list of dims[k] x R arrays.
    """

    def __init__(self, X, A0, *, B, R=None, sampler="euclidean", rule="adagrad", alpha=0.0,
                 eta=1.0, b=0.0, beta=0.0, gamma=1.0, storage="f32", nonneg=False, seed=0,
                 stream_id=0, device="cuda", dims=None, ksplit=None, path="auto",
                 rescale_every=0):
        self.device = torch.device(device)
        if isinstance(X, torch.Tensor):
            assert X.is_cuda and X.is_contiguous()
            dims = list(dims) if dims is not None else list(X.shape[::-1])
            x_ptr, x_space = X.data_ptr(), CPD_DEVICE
            x_dtype = CPD_F64 if X.dtype == torch.float64 else CPD_F32
            self._x_keep = X
        else:
            Xn = np.asarray(X)
            dims = list(Xn.shape)
            x_dtype = CPD_F64 if Xn.dtype == np.float64 else CPD_F32
            Xf = np.asfortranarray(Xn.astype(np.float64 if x_dtype == CPD_F64 else np.float32,
                                             copy=False))
            x_ptr, x_space = Xf.ctypes.data, CPD_HOST
            self._x_keep = Xf
        self.A0 = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in A0]
        R = self.A0[0].shape[1] if R is None else int(R)
        self.dims, self.R, self.B = dims, R, int(B)
        self.problem = make_problem(dims, R, B, seed, stream_id)
        self.options = make_options(sampler, rule, alpha, eta, b, beta, gamma, storage, nonneg,
                                    ksplit=ksplit, path=path, rescale_every=rescale_every)
        self.ws_bytes = cpd_workspace_size(self.problem, self.options)
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = torch.cuda.current_stream(self.device)
        self.h = cpd_init(self.problem, self.options, x_ptr, x_dtype, x_space, self.A0,
                          self.ws_ptr, self.ws_bytes, self.stream.cuda_stream)
        self._x_keep = None

    # calls -------------------------------------------------------------------
    def step(self, nsteps=1):
        cpd_step(self.h, nsteps)

    def sync(self):
        cpd_sync(self.h)

    def fit(self):
        return cpd_fit(self.h)

    @property
    def t(self):
        return cpd_get_step(self.h)

    def factors(self):
        out = []
        for k, I in enumerate(self.dims):
            a = np.empty((I, self.R), dtype=np.float32)
            cpd_read_factors(self.h, k, a.ctypes.data, CPD_HOST)
            out.append(a)
        return out

    def cdf(self, n):
        c = np.empty(self.dims[n], dtype=np.float64)
        cpd_read_cdf(self.h, n, c.ctypes.data)
        return c

    def sample(self, t):
        """(mode, idx (B x N-1 int32 numpy), p (B float64 numpy))."""
        N = len(self.dims)
        idx = torch.empty((self.B, N - 1), dtype=torch.int32, device=self.device)
        p = torch.empty(self.B, dtype=torch.float64, device=self.device)
        mode = cpd_sample(self.h, t, idx.data_ptr(), p.data_ptr())
        return mode, idx.cpu().numpy(), p.cpu().numpy()

    def step_replay(self, mode, idx):
        idx_t = torch.as_tensor(np.ascontiguousarray(idx, dtype=np.int32), device=self.device)
        cpd_step_replay(self.h, mode, idx_t.data_ptr())
        self.sync()

    def rescale(self):
        """Balance every rank component's column norms across the modes
        (the CP model is unchanged) and rebuild the distributions."""
        cpd_rescale(self.h)

    def variance(self, n, sampler):
        """Exact variance of the sampled gradient of mode n under ``sampler``
        (the scratch comes from torch's allocator, kept for later calls)."""
        need = cpd_variance_workspace_size(self.h, n)
        if getattr(self, "_var_ws", None) is None or self._var_ws[1] < need:
            self._var_ws = _workspace(need, self.device)[0], need
        ws = self._var_ws[0]
        ptr = (ws.data_ptr() + 255) // 256 * 256
        return cpd_variance(self.h, n, sampler, ptr, need)

    def state(self):
        return cpd_read_state(self.h)

    def load_state(self, blob):
        cpd_write_state(self.h, blob)

    def close(self):
        if getattr(self, "h", None) is not None:
            cpd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """A request server on one device with a torch-allocated arena.

    ``submit`` takes a numpy tensor (host) or a CUDA torch tensor laid out
    mode-1-fastest (shape dims[::-1], C-contiguous) plus the initial factors;
    ``poll`` returns None while the request is pending, else a dict with the
    result fields and the final factors.
    """

    def __init__(self, arena_bytes, *, max_slots=64, queue_capacity=4096, round_steps=25,
                 device="cuda"):
        self.device = torch.device(device)
        self.arena, self.arena_ptr = _workspace(int(arena_bytes), self.device)
        self.arena_bytes = int(arena_bytes)
        self.round_steps = int(round_steps)
        self.h = cpd_server_create(max_slots, queue_capacity, round_steps, self.arena_ptr,
                                   self.arena_bytes)
        self._keep = {}

    def submit(self, X, A0, *, B, dims=None, seed=0, stream_id=0, sampler="euclidean",
               rule="adagrad", eta=1.0, alpha=0.0, b=0.0, beta=0.0, gamma=1.0, storage="bf16",
               nonneg=False, fit_target=0.99, max_steps=5000, ksplit=None):
        if isinstance(X, torch.Tensor):
            assert X.is_cuda and X.is_contiguous()
            dims = list(dims) if dims is not None else list(X.shape[::-1])
            x_ptr, x_space = X.data_ptr(), CPD_DEVICE
            x_dtype = CPD_F64 if X.dtype == torch.float64 else CPD_F32
            Xk = X
            # admission reads X on the server's own stream: the work that
            # writes X on the caller's stream must be complete first
            torch.cuda.current_stream(X.device).synchronize()
        else:
            Xk, x_dtype = _host_tensor(X)
            dims = list(Xk.shape)
            x_ptr, x_space = Xk.ctypes.data, CPD_HOST
        A0 = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in A0]
        R = A0[0].shape[1]
        out = [np.empty((I, R), dtype=np.float32) for I in dims]
        req = cpd_request()
        req.problem = make_problem(dims, R, B, seed, stream_id)
        req.options = make_options(sampler, rule, alpha, eta, b, beta, gamma, storage, nonneg,
                                   fit_every=self.round_steps, fit_target=fit_target,
                                   max_steps=max_steps, ksplit=ksplit)
        req.X = x_ptr
        req.x_dtype, req.x_space = x_dtype, x_space
        for k in range(len(dims)):
            req.A0[k] = A0[k].ctypes.data
            req.out[k] = out[k].ctypes.data
        ticket = cpd_submit(self.h, req)
        self._keep[ticket] = (Xk, A0, out)
        return ticket

    def poll(self, ticket):
        r = cpd_poll(self.h, ticket)
        if r is None:
            return None
        _, _, out = self._keep.pop(ticket)
        return {"status": r.status, "reached": bool(r.reached), "fit": r.fit, "steps": r.steps,
                "seconds_queued": r.seconds_queued, "seconds_admit": r.seconds_admit,
                "seconds_to_fit": r.seconds_to_fit, "seconds_total": r.seconds_total,
                "factors": out}

    def stats(self):
        return cpd_server_stats(self.h)

    def close(self):
        if getattr(self, "h", None) is not None:
            cpd_server_destroy(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
