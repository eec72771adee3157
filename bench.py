"""Benchmark: SGD steps/s and HBM GB/s of the sampled-gradient step.

Workload (default): the 300 x 300 x 300 FP32 tensor, R = 10, B = 256,
factors N(0,1) with column congruence 0.6 and 10% of rows scaled x20, noise
at 30 dB SNR, AdaGrad with the Euclidean importance sampler (EAdawsCPD).
One "step" is one full pass of the method's hot path (mode draw, per-mode
CDFs, sampling, fibre gather, KRP rows, reweighted gradient, update); the
timed region is K consecutive steps of one persistent launch, inputs already
resident in HBM.

Prints ONE JSON line (rank 0).  Extra fields: the HBM roofline of the step
kernel, the FP64 oracle timed on a bounded sample on the host, and
steps-to-fit / time-to-fit 0.99 for the importance and uniform samplers.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SGD steps/s + HBM GB/s (sampled gradient); solves/s & p99 time-to-fit 0.99"
HBM_PEAK_GBPS = 8000.0
ETA = 5.0

# HBM traffic of the step kernel on this workload, from FETCH_SIZE and WRITE_SIZE counter runs
# scaled by a 256 MiB device copy (FETCH x2.000, WRITE x1.000), 5000-step dispatch.  Valid only
# for the kernel sources it was taken on: reported as null once any hash differs.
MEASURED_TRAFFIC = {
    "bytes_per_step": (262144 / 131088.0625 * 63626.6875 + 1574.78125) * 1024 / 5000,
    "sources": {
        "paper_2103_04081_amd/csrc/step_kernel.hip":
            "22a49e85e29ed80ebcb870d321dee071f8dd2c8ed1302571a11c786d536af934",
        "paper_2103_04081_amd/csrc/step_common.hpp":
            "b7f5c0d7bd54d0a13089887f76d715fe4966bf2634695e342d8e77116b1f72d4",
        "paper_2103_04081_amd/csrc/cpd_internal.hpp":
            "3b3cb343dd3761dd30721b34db95d3ff3373c49eaf4d875c49722fd6c1fe2087",
    },
    "profile": "profiles/chain_kernel_300cube_R10_B256_f32.md",
}


def measured_traffic_per_step():
    """Counter-measured HBM bytes per step, or None if the kernel changed since."""
    import hashlib
    for rel, want in MEASURED_TRAFFIC["sources"].items():
        with open(os.path.join(ROOT, rel), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != want:
                return None
    return MEASURED_TRAFFIC["bytes_per_step"]


def step_bytes(dims, R, B, elem):
    """Algorithmic HBM bytes of one step, averaged over the uniform mode draw:
    fibres B*I_n*s, gathered factor rows min(B, I_k)*R*4 for k != n, factor
    and AdaGrad accumulator read+write 2*2*I_n*R*4, CDF rewrite 8*I_n."""
    N = len(dims)
    tot = 0.0
    for n in range(N):
        b = B * dims[n] * elem
        b += sum(min(B, dims[k]) * R * 4 for k in range(N) if k != n)
        b += 4 * dims[n] * R * 4
        b += 8 * dims[n]
        tot += b
    return tot / N


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--sampler", default="euclidean")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fit", action="store_true", help="skip the time-to-fit runs")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve section")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched-solve section (profiling)")
    ap.add_argument("--no-seq", action="store_true",
                    help="skip the per-tensor FP32 comparison of the batched section")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving section")
    ap.add_argument("--no-variance", action="store_true", help="skip the variance study")
    ap.add_argument("--serve-only", action="store_true",
                    help="run only the serving section (profiling)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--no-grid", action="store_true", help="skip the large-batch grid sweep")
    ap.add_argument("--no-rescale", action="store_true", help="skip the rescaling-cost section")
    ap.add_argument("--rescale-only", action="store_true",
                    help="run only the rescaling-cost section (profiling)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed steps of the main workload (and the CPU baseline unless "
                         "--no-cpu-baseline): the form the profiles are taken on")
    ap.add_argument("--fit-only", action="store_true",
                    help="only time the fit check (300^3 FP32 and 120^4 BF16, 40 fits each)")
    ap.add_argument("--grid-only", action="store_true",
                    help="run only the large-batch grid sweep (profiling)")
    ap.add_argument("--scenes-only", action="store_true",
                    help="run only the scene-shaped workloads (profiling)")
    ap.add_argument("--grid-b", default="4096,16384,65536,131072,262144",
                    help="mini-batch sizes of the grid sweep")
    ap.add_argument("--grid-steps", type=int, default=100)
    ap.add_argument("--no-oracle-extra", action="store_true",
                    help="skip the oracle timings of the small, 4-way and batch workloads")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the timed region, one device copy of this many MiB (a "
                         "known-size kernel to scale hardware byte counters)")
    return ap.parse_args()


_T0 = time.perf_counter()


def progress(what):
    """One line per finished section on stderr (the JSON line stays alone on stdout)."""
    print(f"bench: {what} done at {time.perf_counter() - _T0:.1f} s", file=sys.stderr, flush=True)


def calib_copy(mb):
    """One device copy of mb MiB (a known-size kernel that scales the
    hardware byte counters of a profiled run); nothing when mb is 0."""
    if not mb:
        return
    import torch
    nbytes = mb << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()


def _oracle_batch_member(spec, budget):
    """One member of the 64-tensor recipe solved by the FP64 oracle (in a
    worker process): AdaGrad steps with the explicit-reconstruction fit every
    25 steps, until fit 0.99, 5000 steps or the time budget."""
    import cpd_inputs as ci
    import oracle as O
    t0 = time.perf_counter()
    prob = ci.make_problem(spec["dims"], spec["R"], data_seed=spec["data_seed"],
                           init_seed=spec["init_seed"], snr_db=spec["snr_db"], dtype="bf16")
    orc = O.Oracle(prob["X"], prob["A0"], B=spec["B"], sampler="euclidean", rule="adagrad",
                   eta=BATCH_ETA, seed=spec["seed"], stream_id=spec["stream_id"])
    t1 = time.perf_counter()
    steps, fit = 0, -1.0
    while steps < 5000 and time.perf_counter() - t0 < budget:
        for _ in range(25):
            orc.step()
        steps += 25
        fit = orc.fit()
        if fit >= 0.99:
            break
    return {"steps": steps, "fit": fit, "reached": fit >= 0.99,
            "solve_seconds": time.perf_counter() - t1}


def oracle_beside(budget=25.0):
    """The FP64 oracle beside the other workloads, on bounded samples: the
    small 30^3 workload (its 2000 steps, one core), the 120^4 workload (a
    few steps, one core), the 64-tensor batch recipe and the serving trace
    (their first members / requests, one per worker process, each to fit
    0.99 within the time budget)."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor

    import cpd_inputs as ci
    import oracle as O
    out = {}
    w1 = ci.workload(1)
    orc = O.Oracle(w1["X"], w1["A0"], B=w1["B"], sampler="euclidean", rule="adagrad", eta=1.0,
                   seed=w1["seed"])
    t0 = time.perf_counter()
    for _ in range(2000):
        orc.step()
    el = time.perf_counter() - t0
    out["small_workload"] = {"value": 2000 / el, "unit": "steps/s", "cores": 1, "kind": "oracle",
                             "sample": "all 2000 steps of the 30^3 workload (Euclidean)",
                             "fit_after": orc.fit()}
    w3 = ci.workload(3)
    orc = O.Oracle(w3["X"], w3["A0"], B=w3["B"], sampler="euclidean", rule="adagrad", eta=1.5,
                   seed=w3["seed"])
    t0 = time.perf_counter()
    n = 0
    while n < 200 and time.perf_counter() - t0 < 10.0:
        orc.step()
        n += 1
    el = time.perf_counter() - t0
    out["four_way"] = {"value": n / el, "unit": "steps/s", "cores": 1, "kind": "oracle",
                       "sample": f"first {n} steps of the 120^4 R20 B512 workload (FP32 data)"}
    del orc, w3
    workers = max(1, min(16, os.cpu_count() or 1))
    specs = ci.batch_workload(count=64)[:workers]
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers,
                             mp_context=multiprocessing.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_batch_member, specs, [budget] * len(specs)))
    wall = time.perf_counter() - t0
    reached = sum(r["reached"] for r in res)
    out["batch"] = {"value": reached / wall, "unit": "solves/s", "cores": workers,
                    "kind": "oracle",
                    "sample": f"first {len(specs)} members of the 64-tensor recipe, one per process, "
                              f"each to fit 0.99 (explicit fit every 25 steps) within {budget:.0f} s",
                    "reached": reached, "wall_seconds": wall,
                    "steps": [r["steps"] for r in res]}
    # the serving trace: its first requests, one per process, all submitted
    # at once (the CPU pool is far behind the 50/s arrivals)
    reqs = ci.request_trace(workers)
    t0 = time.perf_counter()
    with ProcessPoolExecutor(max_workers=workers,
                             mp_context=multiprocessing.get_context("spawn")) as ex:
        res = list(ex.map(_oracle_serve_request, reqs, [budget] * len(reqs)))
    wall = time.perf_counter() - t0
    reached = sum(r["reached"] for r in res)
    out["serve"] = {"value": reached / wall, "unit": "solves/s", "cores": workers,
                    "kind": "oracle",
                    "sample": f"first {len(reqs)} requests of the serving trace (host-built "
                              "tensors of the same recipe), one per process, each to fit 0.99 "
                              f"(explicit fit every 25 steps) within {budget:.0f} s",
                    "reached": reached, "wall_seconds": wall,
                    "steps": [r["steps"] for r in res],
                    "dims": [q["dims"] for q in reqs]}
    return out


def cpu_baseline(w, seconds):
    """The FP64 oracle as it stands, single core, on a bounded sample of the
    same workload (a fixed number of its steps)."""
    import oracle as O
    orc = O.Oracle(w["X"], w["A0"], B=w["B"], sampler="euclidean", rule="adagrad", eta=ETA,
                   seed=w["seed"])
    t0 = time.perf_counter()
    n = 0
    while True:
        orc.step()
        n += 1
        el = time.perf_counter() - t0
        if el >= seconds or n >= 100000:
            break
    return {"value": n / el, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} steps of the same 300^3 problem ({el:.1f} s, numpy FP64, "
                      "pure-Python Philox)"}


def main():
    args = parse()
    if args.headline_only:
        args.no_fit = args.no_batch = args.no_rescale = args.no_grid = True
        args.no_variance = args.no_serve = args.no_oracle_extra = True
    if args.gpus != 1:
        print("bench.py: measures a single GPU (no multi-GPU path); --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import cpd_inputs as ci
    import paper_2103_04081_amd as P

    torch.cuda.set_device(0)
    if args.batch_only:
        print(json.dumps({"batch": batch_bench(args.batch_count, seq=not args.no_seq)}),
              flush=True)
        return
    if args.serve_only:
        print(json.dumps({"serve": serve_bench(args.serve_requests),
                          "serve_saturated": serve_bench(args.serve_requests, saturate=True)}),
              flush=True)
        return
    if args.scenes_only:
        print(json.dumps({"scenes": scenes()}), flush=True)
        return
    w = ci.workload(2)
    dims, R, B = w["dims"], w["R"], w["B"]
    X32 = np.asfortranarray(w["X"].astype(np.float32))
    if args.rescale_only:
        print(json.dumps({"rescale": rescale_cost(w, X32)}), flush=True)
        return
    if args.fit_only:
        print(json.dumps({"fit_cost": fit_cost(w, X32)}), flush=True)
        return
    if args.grid_only:
        out = {"grid_sweep": grid_sweep(w, X32, args)}
        calib_copy(args.calib_copy_mb)
        print(json.dumps(out), flush=True)
        return

    def make(sampler, seed=w["seed"]):
        return P.Decomposition(X32, w["A0"], B=B, sampler=sampler, rule="adagrad", eta=ETA,
                               storage="f32", seed=seed)

    dec = make(args.sampler)
    stream = dec.stream
    dec.step(args.warmup)
    dec.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    dec.step(args.steps)
    ev1.record(stream)
    ev1.synchronize()
    torch.cuda.synchronize()
    dec.sync()
    ms = ev0.elapsed_time(ev1)
    sec = ms / 1e3
    steps_per_s = args.steps / sec
    sb = step_bytes(dims, R, B, 4)
    achieved = sb * args.steps / sec / 1e9
    fit_after = dec.fit()
    dec.close()
    progress("timed steps")
    calib_copy(args.calib_copy_mb)

    traffic = measured_traffic_per_step()
    extra = {}
    if not args.no_fit:
        extra["time_to_fit"] = time_to_fit(make, target=0.99, every=25, max_steps=40000)
        extra["time_to_fit"]["euclidean_device_rounds"] = time_to_fit_rounds(
            X32, w, B, target=0.99, every=25, max_steps=40000)
        progress("time_to_fit")
    if not args.no_batch:
        extra["batch"] = batch_bench(args.batch_count, seq=not args.no_seq)
        progress("batch")
    if not args.headline_only:
        extra["small_workload"] = small_workload()
        progress("small_workload")
        extra["four_way"] = four_way()
        progress("four_way")
        extra["scenes"] = scenes()
        progress("scenes")
    if not args.no_rescale:
        extra["rescale"] = rescale_cost(w, X32)
        progress("rescale")
    if not args.no_grid:
        extra["grid_sweep"] = grid_sweep(w, X32, args)
        progress("grid_sweep")
    if not args.no_variance:
        extra["variance"] = variance_study()
        progress("variance")
    if not args.no_serve:
        extra["serve"] = serve_bench(args.serve_requests)
        progress("serve")
        extra["serve_saturated"] = serve_bench(args.serve_requests, saturate=True)
        progress("serve_saturated")

    out = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "300x300x300 FP32 tensor, R=10, B=256, rho=0.6, 10% rows x20, "
                               f"SNR 30 dB; EAdawsCPD (Euclidean sampler, AdaGrad eta={ETA}, b=0)",
                   "sampler": args.sampler, "global_batch": B, "rank": R,
                   "parallelism": "single GPU, one persistent workgroup per decomposition"},
        "alg_gbps": achieved,  # algorithmic bytes per second (not counter-measured)
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": (None if traffic is None else traffic * args.steps),
                     "traffic_per_step": traffic, "bytes_per_step": sb,
                     "steps_per_launch": args.steps, "kernel": "chain_kernel<1>",
                     "counters": MEASURED_TRAFFIC["profile"],
                     "note": "one decomposition's steps form a dependent chain (the CDF of step "
                             "t's mode feeds the draws of step t+1), run by one workgroup: "
                             "latency-bound; grid_sweep and batch carry the bandwidth-bound "
                             "forms of the same step"},
        "fit_after_timed_steps": fit_after,
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        if not args.no_oracle_extra:
            out["oracle_beside"] = oracle_beside()
    print(json.dumps(out), flush=True)


BATCH_ETA = 1.5


def batch_members(count, storage):
    import numpy as np

    import cpd_inputs as ci
    out = []
    for s in ci.batch_workload(count=count):
        prob = ci.make_problem(s["dims"], s["R"], data_seed=s["data_seed"],
                               init_seed=s["init_seed"], snr_db=s["snr_db"], dtype="bf16")
        out.append(dict(X=np.asfortranarray(prob["X"].astype(np.float32)), A0=prob["A0"],
                        B=s["B"], sampler="euclidean", rule="adagrad", eta=BATCH_ETA,
                        storage=storage, fit_every=25, fit_target=0.99, max_steps=5000,
                        seed=s["seed"], stream_id=s["stream_id"], dims=s["dims"], R=s["R"]))
    return out


def per_tensor_fp32(members):
    """Each tensor alone through the plain FP32 single-handle path, to fit 0.99."""
    import torch

    import paper_2103_04081_amd as P
    secs, reached = 0.0, 0
    for m in members:
        d = P.Decomposition(m["X"], m["A0"], B=m["B"], sampler="euclidean", rule="adagrad",
                            eta=BATCH_ETA, storage="f32", seed=m["seed"],
                            stream_id=m["stream_id"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        t, fit = 0, d.fit()
        while fit < 0.99 and t < 5000:
            d.step(25)
            t += 25
            fit = d.fit()
        secs += time.perf_counter() - t1
        reached += fit >= 0.99
        d.close()
    return {"solves_per_s": len(members) / secs, "seconds": secs, "reached": int(reached)}


def batch_bench(count=64, seq=True):
    """64 uneven BF16 decompositions in one batch (persistent launches replayed
    from a HIP graph) run to fit 0.99, against the same tensors solved one by
    one with the plain per-tensor FP32 path."""
    import numpy as np
    import torch

    import paper_2103_04081_amd as P
    t0 = time.perf_counter()
    members = batch_members(count, "bf16")
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    b = P.Batch([{k: v for k, v in m.items() if k not in ("dims", "R")} for m in members],
                tune=True)
    create_s = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    left = b.run(max_rounds=400)
    run_s = time.perf_counter() - t0
    infos = [b.info(i) for i in range(count)]
    b.close()
    steps = np.array([i["t_done"] for i in infos], dtype=np.float64)
    secs = np.array([i["seconds_done"] for i in infos])
    reached = sum(1 for i in infos if i["fit"] >= 0.99)
    alg = sum(i["t_done"] * step_bytes(m["dims"], m["R"], m["B"], 2) for i, m in zip(infos, members))
    rounds = int(max(steps) // 25 + (1 if max(steps) % 25 else 0))
    fit_bytes = sum(2.0 * np.prod(m["dims"]) * (i["t_done"] / 25) for i, m in zip(infos, members))

    # the same tensors, one plain FP32 handle at a time
    seq = per_tensor_fp32(members) if seq else None
    return {
        "workload": f"{count} 3-way tensors, dims U{{50..400}}, R U{{5..32}}, B 128, BF16 "
                    f"storage, SNR 30 dB; Euclidean sampler, AdaGrad eta={BATCH_ETA}; fit check "
                    "every 25 steps; each run to fit 0.99 or 5000 steps",
        "solves_per_s": count / run_s, "seconds": run_s, "reached": reached,
        "remaining": left, "rounds": rounds, "ms_per_round": run_s / max(rounds, 1) * 1e3,
        "steps_to_fit_p50": float(np.percentile(steps, 50)),
        "steps_to_fit_p99": float(np.percentile(steps, 99)),
        "device_seconds_to_fit_p50": float(np.percentile(secs, 50)),
        "device_seconds_to_fit_p99": float(np.percentile(secs, 99)),
        "member_steps_per_s": float(steps.sum() / run_s),
        "step_gbps": alg / run_s / 1e9, "fit_gbps": fit_bytes / run_s / 1e9,
        "alg_bw_frac": (alg + fit_bytes) / run_s / 1e9 / HBM_PEAK_GBPS,
        "tune_and_create_seconds": create_s, "host_generation_seconds": gen_s,
        "per_tensor_fp32_sequential": seq,
        "speedup_vs_per_tensor_fp32": None if seq is None else seq["seconds"] / run_s,
    }


SERVE_ETA = 1.0


def _oracle_serve_request(spec, budget):
    """One request of the serving trace solved by the FP64 oracle (in a worker
    process): the request's shape, rank, seeds and B, its tensor from the
    host recipe (the server's is formed on the device, whose noise draws
    differ), AdaGrad with the explicit-reconstruction fit every 25 steps,
    until fit 0.99, 5000 steps or the time budget."""
    import cpd_inputs as ci
    import oracle as O
    t0 = time.perf_counter()
    prob = ci.make_problem(spec["dims"], spec["R"], data_seed=spec["data_seed"],
                           init_seed=spec["init_seed"], snr_db=spec["snr_db"], dtype="bf16")
    orc = O.Oracle(prob["X"], prob["A0"], B=spec["B"], sampler="euclidean", rule="adagrad",
                   eta=SERVE_ETA, seed=spec["seed"], stream_id=spec["stream_id"])
    t1 = time.perf_counter()
    steps, fit = 0, -1.0
    while steps < 5000 and time.perf_counter() - t0 < budget:
        for _ in range(25):
            orc.step()
        steps += 25
        fit = orc.fit()
        if fit >= 0.99:
            break
    return {"steps": steps, "fit": fit, "reached": fit >= 0.99,
            "solve_seconds": time.perf_counter() - t1,
            "setup_seconds": t1 - t0}


def serve_bench(n_requests=200, rate=50.0, saturate=False):
    """Poisson arrivals (50 req/s) of 3-way / 4-way BF16 requests into the
    server, each run to fit 0.99 or 5000 steps.  Tensors are built on the
    device before the clock starts (seeded recipe); the server stages them
    (layout, BF16 rounding) at admission, inside the measured time."""
    import numpy as np
    import torch

    import cpd_inputs as ci
    import paper_2103_04081_amd as P
    trace = ci.request_trace(n_requests, rate=rate)
    t0 = time.perf_counter()
    data = [ci.device_problem(r) for r in trace]
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    arena = 64 << 30
    srv = P.Server(arena, max_slots=128, queue_capacity=4096, round_steps=25)
    pending, done = {}, []
    start = time.perf_counter()
    nxt = 0
    while nxt < len(trace) or pending:
        now = time.perf_counter() - start
        while nxt < len(trace) and (saturate or trace[nxt]["arrival"] <= now):
            r = trace[nxt]
            X, A0 = data[nxt]
            tk = srv.submit(X, A0, B=r["B"], seed=r["seed"], stream_id=r["stream_id"],
                            sampler="euclidean", eta=SERVE_ETA, storage="bf16",
                            fit_target=0.99, max_steps=5000)
            pending[tk] = (nxt, time.perf_counter() - start)
            nxt += 1
        for tk in list(pending):
            res = srv.poll(tk)
            if res is not None:
                i, t_sub = pending.pop(tk)
                res["arrival"] = t_sub
                res["finish"] = time.perf_counter() - start
                res["index"] = i
                res.pop("factors")
                done.append(res)
        time.sleep(0.0005)
    makespan = max(d["finish"] for d in done)
    srv.close()
    del data
    ok = [d for d in done if d["status"] == 0]
    reached = [d for d in ok if d["reached"]]
    fit_t = np.array([d["seconds_admit"] + d["seconds_to_fit"] for d in reached])
    tot_t = np.array([d["seconds_total"] for d in reached])
    pct = lambda a, q: float(np.percentile(a, q)) if len(a) else None  # noqa: E731
    return {
        "workload": f"{n_requests} requests, Poisson arrivals at {rate:g}/s"
                    f"{' (all submitted at once)' if saturate else ''}; 50/50 3-way dims "
                    "U{64..512} and 4-way dims U{32..128}, R U{8..32}, B 128, BF16 storage, "
                    f"SNR 30 dB; Euclidean sampler, AdaGrad eta={SERVE_ETA}; fit check every 25 "
                    "steps; each to fit 0.99 or 5000 steps",
        "solves_per_s": len(reached) / makespan, "completed": len(done), "reached": len(reached),
        "errors": len(done) - len(ok), "makespan_s": makespan,
        "time_to_fit_from_admission_p50": pct(fit_t, 50),
        "time_to_fit_from_admission_p99": pct(fit_t, 99),
        "time_to_fit_from_arrival_p50": pct(tot_t, 50),
        "time_to_fit_from_arrival_p99": pct(tot_t, 99),
        "queued_p99": pct(np.array([d["seconds_queued"] for d in done]), 99),
        "steps_p50": pct(np.array([d["steps"] for d in done]), 50),
        "device_generation_seconds": gen_s,
        "missed": [{"index": d["index"], "dims": trace[d["index"]]["dims"],
                    "R": trace[d["index"]]["R"], "steps": d["steps"], "fit": d["fit"]}
                   for d in sorted(ok, key=lambda d: d["index"]) if not d["reached"]],
    }


def variance_study(steps=1000, every=100, B=18):
    """The variance of the sampled gradient (mode 1, variance theorem) for the
    three samplers along an EAdawsCPD run on the paper's Data II and Data III,
    and the wall time of one evaluation (scratch allocation, the sampler's
    CDFs and one pass over copy 1)."""
    import numpy as np
    import torch

    import cpd_inputs as ci
    import paper_2103_04081_amd as P
    out = {"setting": f"300^3 from 300x10 Gaussian factors (Data II; Data III = one entry per "
                      f"factor set to 20), no noise, B={B}, Euclidean sampler + AdaGrad eta=1 "
                      f"driving the run; mode 1 variances at every {every} steps"}
    for which in (2, 3):
        w = ci.variance_data(which)
        dec = P.Decomposition(np.asfortranarray(w["X"].astype(np.float32)), w["A0"], B=B,
                              sampler="euclidean", eta=1.0, seed=3010 + which)
        rows = []
        for t in range(0, steps + 1, every):
            if t:
                dec.step(every)
            v = {s: dec.variance(0, s)[0] for s in ("uniform", "leverage", "euclidean")}
            rows.append({"t": t, **v})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dec.variance(0, "euclidean")
        el = (time.perf_counter() - t0) / 5
        nbytes = 300 * 320 * 300 * 4  # one pass over copy 1 (rows padded to 320)
        out[f"data_{'ii' if which == 2 else 'iii'}"] = rows
        out[f"data_{'ii' if which == 2 else 'iii'}_eval_seconds"] = el
        out[f"data_{'ii' if which == 2 else 'iii'}_eval_gbps"] = nbytes / el / 1e9
        dec.close()
    return out


def four_way(steps=2000):
    """The 4-way workload: 120^4 (207M entries), R = 20, B = 512, SNR 30 dB
    (tensor built on the device), FP32 vs BF16 storage, persistent step,
    Euclidean sampler, AdaGrad eta = 1.5; steps/s and algorithmic GB/s."""
    import torch

    import cpd_inputs as ci
    import paper_2103_04081_amd as P
    spec = {"dims": (120, 120, 120, 120), "R": 20, "data_seed": 1003, "init_seed": 2003,
            "snr_db": 30.0}
    X, A0 = ci.device_problem(spec, "cuda")
    out = {"workload": "120x120x120x120 tensor, R=20, B=512, N(0,1) factors, SNR 30 dB; "
                       "Euclidean sampler, AdaGrad eta=1.5; persistent step"}
    for storage, elem in (("f32", 4), ("bf16", 2)):
        dec = P.Decomposition(X, A0, B=512, sampler="euclidean", rule="adagrad", eta=1.5,
                              storage=storage, seed=3003)
        dec.step(200)
        dec.sync()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(dec.stream)
        dec.step(steps)
        ev1.record(dec.stream)
        ev1.synchronize()
        dec.sync()
        ms = ev0.elapsed_time(ev1) / steps
        sb = step_bytes(list(spec["dims"]), spec["R"], 512, elem)
        out[storage] = {"steps_per_s": 1e3 / ms, "us_per_step": ms * 1e3, "bytes_per_step": sb,
                        "gbps": sb / ms / 1e6, "alg_bw_frac": sb / ms / 1e6 / 8000.0,
                        "fit_after": dec.fit()}
        dec.close()
    del X
    return out


def rescale_cost(w, X32, steps=2000):
    """Column rescaling between steps on the main 300^3 workload (persistent
    step): steps/s without it, rescaling after every step and after every
    25th, the fit after the run, and the cost of one cpd_rescale (the
    rescale kernel plus the rebuild of every mode's CDF)."""
    import torch

    import paper_2103_04081_amd as P
    out = {"workload": "300x300x300 FP32 tensor of the main workload, R=10, B=256, Euclidean "
                       f"sampler, AdaGrad eta={ETA}; {steps} steps from the initial factors"}

    def timed(dec, fn):
        dec.sync()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(dec.stream)
        fn()
        ev1.record(dec.stream)
        ev1.synchronize()
        return ev0.elapsed_time(ev1)

    for every in (0, 25, 1):
        dec = P.Decomposition(X32, w["A0"], B=256, sampler="euclidean", rule="adagrad", eta=ETA,
                              storage="f32", seed=w["seed"], rescale_every=every)
        ms = timed(dec, lambda: dec.step(steps)) / steps
        out[f"every_{every}"] = {"steps_per_s": 1e3 / ms, "us_per_step": ms * 1e3,
                                 "fit_after": dec.fit()}
        if every == 0:
            n = 200
            out["us_per_rescale"] = timed(dec, lambda: [dec.rescale() for _ in range(n)]) * 1e3 / n
        dec.close()
    return out


def scenes(steps=2000):
    """Stand-ins of the paper's hyperspectral scenes (Section 5, Tables 6 and
    7; the data are not available here): seeded Gaussian tensors of the
    same shapes and ranks, SNR 30 dB, built on the device; B = 20, Euclidean
    sampler, AdaGrad eta = 0.5.  The R = 10 scenes run on the persistent step,
    the R = 100 one on the grid step (ranks beyond 64).  Steps/s, the
    algorithmic bandwidth, and the time of the paper's run length at that
    rate."""
    import torch

    import cpd_inputs as ci
    import paper_2103_04081_amd as P
    out = {"setting": "B=20, Euclidean sampler, AdaGrad eta=0.5, FP32 storage; seeded Gaussian "
                      "stand-ins (SNR 30 dB) of the scene shapes"}
    for name, dims, R, iters, seed in (("salinas_a", (83, 86, 224), 10, 20000, 1121),
                                       ("indian_pines", (145, 145, 220), 10, 20000, 1122),
                                       ("pavia_university", (610, 340, 103), 100, 30000, 1123)):
        spec = {"dims": dims, "R": R, "data_seed": seed, "init_seed": seed + 100, "snr_db": 30.0}
        X, A0 = ci.device_problem(spec, "cuda")
        dec = P.Decomposition(X, A0, B=20, sampler="euclidean", rule="adagrad", eta=0.5,
                              storage="f32", seed=seed + 200, dims=list(dims))
        n = steps if R <= 64 else steps // 4
        dec.step(200)
        dec.sync()
        torch.cuda.synchronize()
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(dec.stream)
        dec.step(n)
        ev1.record(dec.stream)
        ev1.synchronize()
        dec.sync()
        ms = ev0.elapsed_time(ev1) / n
        sb = step_bytes(list(dims), R, 20, 4)
        out[name] = {"dims": list(dims), "R": R, "path": "grid" if R > 64 else "persistent",
                     "steps_per_s": 1e3 / ms, "us_per_step": ms * 1e3, "bytes_per_step": sb,
                     "gbps": sb / ms / 1e6, "alg_bw_frac": sb / ms / 1e6 / 8000.0,
                     "paper_iterations": iters, "seconds_for_paper_iterations": iters * ms / 1e3,
                     "fit_after": dec.fit(), "steps_timed": n}
        dec.close()
        del X
    return out


def small_workload(steps=2000):
    """The 30x30x30 workload (R 5, B 18, SNR 40 dB, FP32 storage): its 2000
    steps in one persistent launch per importance sampler, with the fit
    after them."""
    import numpy as np
    import torch

    import cpd_inputs as ci
    import paper_2103_04081_amd as P
    w = ci.workload(1)
    out = {"workload": "30x30x30 tensor, R=5 (true rank 5), B=18, SNR 40 dB, FP32 storage, "
                       f"AdaGrad eta=1.0, {steps} steps"}
    for sampler in ("euclidean", "leverage"):
        dec = P.Decomposition(np.asfortranarray(w["X"].astype(np.float32)), w["A0"], B=w["B"],
                              sampler=sampler, rule="adagrad", eta=1.0, storage="f32",
                              seed=w["seed"])
        dec.step(50)
        dec.sync()
        t0 = dec.t
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(dec.stream)
        dec.step(steps)
        ev1.record(dec.stream)
        ev1.synchronize()
        dec.sync()
        ms = ev0.elapsed_time(ev1)
        out[sampler] = {"steps_per_s": steps / (ms / 1e3), "us_per_step": ms * 1e3 / steps,
                        "fit_after": dec.fit(), "t": dec.t - t0}
        dec.close()
    return out


def fit_cost(w, X32, reps=40):
    """The explicit fit check (a8) on the main workload (300^3 FP32) and on
    the 120^4 BF16 tensor: host wall time per fit (launches of the partial
    and final kernels plus the state read-back), and the algorithmic bytes
    of its stream (one copy of the tensor)."""
    import numpy as np

    import cpd_inputs as ci
    import paper_2103_04081_amd as P

    out = {}
    cases = [("300^3 FP32, R=10", lambda: P.Decomposition(X32, w["A0"], B=w["B"], eta=ETA,
                                                           storage="f32", seed=w["seed"]),
              w["dims"], 4)]
    spec = {"dims": (120, 120, 120, 120), "R": 20, "data_seed": 1003, "init_seed": 2003,
            "snr_db": 30.0}
    X4, A04 = ci.device_problem(spec, "cuda")
    cases.append(("120^4 BF16, R=20", lambda: P.Decomposition(X4, A04, B=512, eta=1.5,
                                                              storage="bf16", seed=3003),
                  spec["dims"], 2))
    for name, make, dims, s in cases:
        dec = make()
        dec.step(10)
        dec.sync()
        for _ in range(5):
            dec.fit()
        t0 = time.perf_counter()
        for _ in range(reps):
            f = dec.fit()
        dt = (time.perf_counter() - t0) / reps
        ld0 = (dims[0] + 63) // 64 * 64
        nbytes = int(np.prod(dims[1:])) * ld0 * s
        out[name] = {"host_us_per_fit": dt * 1e6, "stream_bytes": nbytes, "fit": f}
        dec.close()
    return out


def grid_sweep(w, X32, args):
    """The same 300^3 FP32 tensor and R, with mini-batches far beyond one
    workgroup: the grid step (three launches per step over the whole GPU),
    timed with HIP events on the handle's stream, K steps after 19 warm-up
    steps.  Uniform sampling reads fibres spread over the whole copy;
    Euclidean sampling of this skewed tensor concentrates on few fibres.
    GB/s are algorithmic bytes per step (fibres, sampled factor rows, A and
    S read and write, CDF) over the step time."""
    import torch

    import paper_2103_04081_amd as P
    dims, R = w["dims"], w["R"]
    rows = []
    for sampler in ("uniform", "euclidean"):
        for B in [int(b) for b in args.grid_b.split(",") if b]:
            dec = P.Decomposition(X32, w["A0"], B=B, sampler=sampler, rule="adagrad", eta=ETA,
                                  storage="f32", seed=w["seed"], path="grid")
            dec.step(19)  # builds and replays the 16-step graph once
            dec.sync()
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(dec.stream)
            dec.step(args.grid_steps)
            ev1.record(dec.stream)
            ev1.synchronize()
            dec.sync()
            ms = ev0.elapsed_time(ev1) / args.grid_steps
            sb = step_bytes(dims, R, B, 4)
            rows.append({"sampler": sampler, "B": B, "ms_per_step": ms,
                         "steps_per_s": 1e3 / ms, "fibres_per_s": B * 1e3 / ms,
                         "bytes_per_step": sb, "gbps": sb / ms / 1e6,
                         "alg_bw_frac": sb / ms / 1e6 / 8000.0, "fit_after": dec.fit()})
            dec.close()
    # the 4-way workload in BF16 storage: 120^4 (207M entries), R = 20, SNR 30 dB,
    # built on the device; 8-row output tiles per mode split each block's
    # fibre range over two wave groups
    import cpd_inputs as ci
    spec4 = {"dims": (120, 120, 120, 120), "R": 20, "data_seed": 1003, "init_seed": 2003,
             "snr_db": 30.0}
    X4, A04 = ci.device_problem(spec4, "cuda")
    rows4 = []
    for sampler in ("uniform", "euclidean"):
        for B in (65536, 262144):
            dec = P.Decomposition(X4, A04, B=B, sampler=sampler, rule="adagrad", eta=1.0,
                                  storage="bf16", seed=3003, path="grid")
            dec.step(19)
            dec.sync()
            torch.cuda.synchronize()
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(dec.stream)
            dec.step(args.grid_steps)
            ev1.record(dec.stream)
            ev1.synchronize()
            dec.sync()
            ms = ev0.elapsed_time(ev1) / args.grid_steps
            sb = step_bytes(list(spec4["dims"]), spec4["R"], B, 2)
            rows4.append({"sampler": sampler, "B": B, "ms_per_step": ms, "steps_per_s": 1e3 / ms,
                          "bytes_per_step": sb, "gbps": sb / ms / 1e6,
                          "alg_bw_frac": sb / ms / 1e6 / 8000.0})
            dec.close()
    del X4
    return {"workload": "300x300x300 FP32 tensor of the main workload, R=10, AdaGrad "
                        f"eta={ETA}; grid step (CPD_PATH_GRID), {args.grid_steps} timed steps",
            "rows": rows,
            "workload_4way_bf16": "120^4 tensor (N(0,1) factors, SNR 30 dB, built on the device) "
                                  "stored in BF16, R=20, AdaGrad eta=1.0; grid step",
            "rows_4way_bf16": rows4,
            "fields": "gbps / alg_bw_frac: algorithmic bytes per step (every sampled fibre "
                      "counted, including rows the importance samplers draw again and the "
                      "caches serve) over the step time, and that rate over the 8 TB/s HBM "
                      "peak; it is not the HBM traffic fraction. The counter-measured HBM bytes "
                      "are in profiles/wide_gather_300cube_R10_B262144_f32.md"}


def time_to_fit(make, target, every, max_steps):
    """Steps and wall time to the first fit check >= target, per sampler."""
    import torch
    res = {}
    for sampler in ("euclidean", "leverage", "uniform"):
        dec = make(sampler)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        fit = dec.fit()
        while fit < target and steps < max_steps:
            dec.step(every)
            steps += every
            fit = dec.fit()
        el = time.perf_counter() - t0
        res[sampler] = {"steps": steps, "seconds": el, "fit": fit, "reached": fit >= target}
        dec.close()
    res["check_every"] = every
    res["target"] = target
    return res


def time_to_fit_rounds(X32, w, B, target, every, max_steps):
    """The same Euclidean run as a batch of one: rounds of `every` steps and a
    fit check replayed from a HIP graph, the stop decided on the device (no
    host round trip per check).  Same draws and arithmetic as the single
    handle, so the same steps to fit."""
    import torch

    import paper_2103_04081_amd as P
    b = P.Batch([dict(X=X32, A0=w["A0"], B=B, sampler="euclidean", rule="adagrad", eta=ETA,
                      storage="f32", fit_every=every, fit_target=target, max_steps=max_steps,
                      seed=w["seed"])], tune=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(max_rounds=max_steps // every + 1)
    el = time.perf_counter() - t0
    inf = b.info(0)
    b.close()
    return {"steps": inf["t_done"], "seconds": el, "device_seconds": inf["seconds_done"],
            "fit": inf["fit"], "reached": inf["fit"] >= target}


if __name__ == "__main__":
    main()
