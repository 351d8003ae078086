#!/usr/bin/env python3
"""Throughput of batched ensemble fidelity+gradient evaluation on one MI355X.

Workload: parallel CNOT on N = 50 qubits (25 pairs), chi = 64, M = 200 slices,
K = 128 crosstalk samples x R = 8 random product inputs, complex128, seeded
synthetic controls/crosstalk/inputs.  One step = one grape_fidelity_grad call:
forward TEBD of all 1024 trajectories with checkpoints, the adjoint sweep with
recomputation and the ensemble reduction, all in one persistent launch.

Prints one JSON line (stdout); progress goes to stderr.
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "noise-sample fidelity+grad evals/sec at N=50 chi=64 vs plain GPU; p50/p99 latency"
FP64_PEAK_TFLOPS = 78.6   # MI355X fp64 vector (= fp64 matrix) peak


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


CPU_SCRIPT = r"""
import os, sys, time, json
sys.path.insert(0, {root!r})
import workloads as W
from oracle import grape
p = W.make_problem({name!r}, xt_model={xt!r})
t0 = time.perf_counter()
for r in range({n}):
    grape.trajectory(p, 0, r)
dt = time.perf_counter() - t0
print(json.dumps(dict(seconds=dt)))
"""


TASKS = {"x": "parallel X gate", "cnot": "parallel CNOT", "ghz": "GHZ state preparation",
         "heisenberg": "Heisenberg ground-state preparation"}


def cpu_baseline(name, n_traj, R, xt_model="zz"):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    code = CPU_SCRIPT.format(root=ROOT, name=name, n=n_traj, xt=xt_model)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=900)
    if out.returncode != 0:
        log(out.stderr)
        return None
    secs = json.loads(out.stdout.strip().splitlines()[-1])["seconds"]
    samples = n_traj / R
    return {"value": samples / secs, "unit": "noise-samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_traj} of the {R} trajectories of noise sample k=0 (forward + adjoint "
                      f"over all slices), one process, 1 BLAS thread: {secs:.2f} s",
            "seconds": secs}


def sources_sha256():
    """Hash of the sources compiled into device code (the kernels, their
    headers and the launching host file; not the host-only serving runtime),
    to match stored counter runs to the compiled library."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(f for f in glob.glob(os.path.join(ROOT, "paper_2603_03639_amd", "csrc", "*"))
                   if not f.endswith(".cpp"))
    for f in files + [os.path.join(ROOT, "include", "tnrg.h")]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(workload, ckpt_stride):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE runs, or
    None when the kernel sources or the checkpoint stride changed since those
    counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_grape_{workload}_hbm.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ok = rec.get("sources_sha256") == sources_sha256() and rec.get("ckpt_stride") == ckpt_stride
    return rec["bytes_per_launch"] if ok else None


def _request_pool(P, W, dev, n, seed=4):
    """Device-resident requests of the serving mix (distinct problems)."""
    f = lambda a: torch_mod().as_tensor(a, dtype=torch_mod().float64, device=dev)
    pool = []
    for spec in W.serving_mix(n, seed=seed):
        p = W.make_problem(**spec)
        inputs = P.MPSBatch.from_product(p.inputs, device=dev)
        tcap = max(max(A.shape[0] for A in T) for T in p.targets)
        targets = P.MPSBatch.from_mps(p.targets, dcap=max(1, tcap), device=dev)
        pool.append((spec, P.Model.from_problem(p), f(p.ux), f(p.uy), f(p.uzz), f(p.J),
                     inputs, targets))
    return pool


def torch_mod():
    import torch
    return torch


def serving_leg(P, W, dev, seconds, open_loop_seconds, pool_size, arena_gib, streams,
                max_dcap):
    """Continuous-batching serving of the request mix (Poisson arrivals).

    1. every pool request once alone, back to back through a one-stream
       server: service times, bucket plan warm-up;
    2. every servable pool request at once on all streams: the capacity
       (requests/s) with the GPU shared;
    3. a window at 0.7 x that capacity: p50/p99 latency and throughput of
       completed requests;
    4. an open-loop window at 200 requests/s: what was admitted, completed,
       left queued (then cancelled) and how the queue grew.
    Requests whose bonds outgrow the largest capacity bucket the server
    admits (max_dcap) fail with their status and are counted, not hidden.
    """
    import numpy as np
    torch = torch_mod()
    S = P.serve
    pool = _request_pool(P, W, dev, pool_size)
    mk = lambda i: S.Request(*pool[i][1:])
    arena = int(arena_gib * (1 << 30))

    # 1. alone, back to back
    service, fails, ok_idx, alone = [], {}, [], []
    with S.Server(arena, n_streams=1, max_dcap=max_dcap) as srv:
        for i in range(len(pool)):
            srv.submit(mk(i))
            c = srv.drain()[0]
            sp = pool[i][0]
            alone.append({"task": sp["task"], "N": sp["N"], "chi": sp["chi"], "K": sp["K"],
                          "R": sp["R"], "M": sp["M"], "status": c["status"], "dcap": c["dcap"],
                          "launches": c["launches"], "ms": round(c["total_ms"], 1)})
            log(f"  alone {i}: {alone[-1]}")
            if c["status"] == 0:
                service.append(c["total_ms"])
                ok_idx.append(i)
            else:
                key = f"{sp['task']}/N{sp['N']}/chi{sp['chi']}"
                fails[key] = c["status"]
    mean_service = float(np.mean(service)) if service else float("nan")
    log(f"serving: {len(service)} of {len(pool)} pool requests served alone, mean "
        f"{mean_service:.1f} ms, failures {fails}")

    def window(rate, secs, seed, cancel_at_end):
        rng = np.random.default_rng(seed)
        lat, statuses, qmax = [], {}, 0
        sub = 0
        with S.Server(arena, n_streams=streams, max_dcap=max_dcap) as srv:
            t0 = time.perf_counter()
            next_t = rng.exponential(1.0 / rate)
            while True:
                now = time.perf_counter() - t0
                if now >= secs:
                    break
                while next_t <= now:
                    srv.submit(mk(int(rng.choice(ok_idx))))
                    sub += 1
                    next_t += rng.exponential(1.0 / rate)
                for c in srv.progress():
                    statuses[c["status"]] = statuses.get(c["status"], 0) + 1
                    if c["status"] == 0:
                        lat.append(c["total_ms"])
                qmax = max(qmax, srv.info()["queued"])
                time.sleep(0.0005)
            info_end = srv.info()
            cancelled = srv.cancel_queued() if cancel_at_end else []
            t_close = time.perf_counter() - t0
            for c in srv.drain():
                statuses[c["status"]] = statuses.get(c["status"], 0) + 1
                if c["status"] == 0:
                    lat.append(c["total_ms"])
            elapsed = time.perf_counter() - t0
            info = srv.info()
        out = {"offered_rate": rate, "window_s": secs, "submitted": sub,
               "completed_ok": len(lat), "status_counts": {str(k): v for k, v in statuses.items()},
               "max_queue": qmax, "queued_at_window_end": info_end["queued"],
               "running_at_window_end": info_end["running"], "cancelled": len(cancelled),
               "elapsed_s": elapsed, "drain_s": elapsed - t_close,
               "throughput_req_s": len(lat) / elapsed if elapsed > 0 else None,
               "admitted": info["admitted"], "regrown": info["regrown"]}
        if lat:
            out["latency_ms"] = {"p50": percentile(lat, 50), "p99": percentile(lat, 99),
                                 "mean": float(np.mean(lat))}
        return out

    # capacity with the GPU shared: every servable pool request at once
    burst_s, burst_ok = None, 0
    if ok_idx:
        with S.Server(arena, n_streams=streams, max_dcap=max_dcap) as srv:
            t0 = time.perf_counter()
            for i in ok_idx:
                srv.submit(mk(i))
            burst_ok = sum(c["status"] == 0 for c in srv.drain())
            burst_s = time.perf_counter() - t0
    capacity = burst_ok / burst_s if burst_s else 0.0
    log(f"serving: burst of {len(ok_idx)} requests on {streams} streams in {burst_s} s "
        f"-> capacity {capacity:.2f} req/s")
    sustainable = window(0.7 * capacity, seconds, 41, cancel_at_end=False) if capacity else None
    if sustainable:
        log(f"serving at {0.7 * capacity:.2f} req/s: {sustainable}")
    open_loop = window(200.0, open_loop_seconds, 42, cancel_at_end=True)
    log(f"serving open loop at 200 req/s: {open_loop}")
    return {"mix": "N in {10,20,30,50}, chi in {16,32,64,128}, K in {8,32,128}, M in 100..300, "
                   "task in {X, CNOT, GHZ, Heisenberg N=20}",
            "pool_requests": len(pool), "streams": streams, "arena_gib": arena_gib,
            "max_dcap": max_dcap,
            "alone": {"served": len(service), "failed": fails, "requests": alone,
                      "mean_service_ms": mean_service,
                      "p50_service_ms": percentile(service, 50) if service else None,
                      "max_service_ms": max(service) if service else None},
            "burst": {"requests": len(ok_idx), "completed_ok": burst_ok, "seconds": burst_s,
                      "capacity_req_s": capacity},
            "sustainable": sustainable, "open_loop": open_loop}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cnot_n50")
    ap.add_argument("--cpu-sample", type=int, default=4,
                    help="trajectories of the oracle timed on the host (0 disables)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--profile", action="store_true",
                    help="one extra call with in-kernel phase timers")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the sustainable-rate serving window (0 disables serving)")
    ap.add_argument("--serve-open-loop", type=float, default=3.0,
                    help="length of the open-loop serving window at 200 requests/s")
    ap.add_argument("--serve-max-dcap", type=int, default=32,
                    help="largest capacity bucket a served request may grow to (32: LDS path)")
    ap.add_argument("--serve-pool", type=int, default=24,
                    help="distinct requests drawn from the serving mix")
    ap.add_argument("--ckpt-stride", type=int, default=None,
                    help="checkpoint stride of the adjoint sweep (0: ceil(sqrt(M)); "
                         "default: the smallest that fits 60%% of the free HBM)")
    ap.add_argument("--xt-model", choices=("zz", "heisenberg"), default="zz",
                    help="crosstalk: the workload's J ZZ (default), or the paper's "
                         "J^x XX + J^y YY + J^z ZZ, uniform in [-0.05, 0.05], on every bond")
    ap.add_argument("--K", type=int, default=0,
                    help="noise samples: the first K of the workload's (0: all of them)")
    ap.add_argument("--threads", type=int, default=None,
                    help="threads per trajectory (workgroup size) instead of the autotuner's choice")
    ap.add_argument("--plain", type=int, default=8,
                    help="trajectories run one at a time for the plain GPU path (0 disables)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the trajectory batch "
              "would be split across GPUs with one all-reduce of [F, grad], which this library "
              "does not implement.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "_tnrg_build", os.path.join(ROOT, "paper_2603_03639_amd", "build.py"))
    B = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(B)
    if not os.path.exists(B.LIB_PATH):
        B.build()
    import paper_2603_03639_amd as P
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    p = W.make_problem(args.workload, xt_model=args.xt_model)
    heis = args.xt_model == "heisenberg"
    wname = args.workload + ("_heisenberg" if heis else "")
    if args.K and args.K < p.K:
        p = p.subset(ks=range(args.K))
        wname += f"_K{args.K}"

    log(f"workload {wname}: N={p.N} M={p.M} chi={p.chi} K={p.K} R={p.R}")
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float64), device=dev)
    ux, uy, uzz, J = f(p.ux), f(p.uy), f(p.uzz), f(p.J)
    inputs = P.MPSBatch.from_product(p.inputs, device=dev)
    tcap = max(max(A.shape[0] for A in T) for T in p.targets)
    targets = P.MPSBatch.from_mps(p.targets, dcap=max(1, tcap), device=dev)
    model = P.Model.from_problem(p)

    # plan: grow the capacity bucket until no bond overflows (untimed)
    t0 = time.perf_counter()
    plan = P.grape_fidelity_grad(model, ux, uy, uzz, J, inputs, targets)
    torch.cuda.synchronize()
    log(f"plan: dcap={plan['dcap']} max_dim={plan['info']['max_dim']} "
        f"({time.perf_counter() - t0:.2f} s incl. bucket search)")
    from paper_2603_03639_amd import tune
    if args.threads is None:
        tuned = tune.autotune(model, ux, uy, uzz, J, inputs, targets, plan["dcap"])
    else:
        tune.set_threads(plan["dcap"], args.threads)
        tuned = {"threads": args.threads, "forced": True}
    log(f"autotune: {tuned}")
    # checkpoint stride: keep as many forward states as 60% of the free HBM
    # holds (stride 1 recomputes nothing); --ckpt-stride forces one
    if args.ckpt_stride is None:
        torch.cuda.empty_cache()
        ck = tune.ckpt_stride(model, p.K, p.R, plan["dcap"])
    else:
        ck = {"stride": args.ckpt_stride,
              "workspace_bytes": P.tnrg.grape_workspace_bytes(model, p.K, p.R, plan["dcap"],
                                                              args.ckpt_stride)}
    log(f"checkpoint stride {ck['stride']} (workspace {ck['workspace_bytes'] / 2**30:.1f} GiB)")
    call = P.GrapeCall(model, p.K, p.R, inputs, targets, plan["dcap"], ckpt_stride=ck["stride"],
                       device=dev)
    stream = torch.cuda.current_stream()

    for i in range(args.warmup):
        call.run(ux, uy, uzz, J)
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        call.run(ux, uy, uzz, J)
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
        log(f"step {i + 1}/{args.steps}: {lat[-1]:.1f} ms")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    info = call.check()
    ms = 1000.0 * wall / args.steps
    value = p.K / (ms / 1000.0)
    F = float(call.F.cpu())
    del call  # its workspace (up to a third of the HBM) is not needed any more
    torch.cuda.empty_cache()

    flops = info["jacobi_flops"] + info["contraction_flops"]
    kern_ms = sum(lat) / len(lat)
    achieved = flops / (kern_ms / 1000.0) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                "traffic": stored_traffic(wname, ck["stride"]),
                "kernel": "k_grape", "flops_per_launch": flops,
                "jacobi_flops_per_launch": info["jacobi_flops"],
                "contraction_flops_per_launch": info["contraction_flops"],
                "avg_launch_ms": kern_ms}

    if args.copy_calib:
        # a plain device copy of known size: the HBM counters of the profiled
        # run are scaled by what they read for this kernel
        src = torch.empty(args.copy_calib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calib} MiB device-to-device")
        del src, dst

    phases = None
    if args.profile:
        import dataclasses
        mprof = dataclasses.replace(model, profile=True)
        pc = P.GrapeCall(mprof, p.K, p.R, inputs, targets, plan["dcap"],
                         ckpt_stride=ck["stride"], device=dev)
        pc.run(ux, uy, uzz, J)
        pinfo = pc.check()
        ticks = pinfo["phase_ticks"]
        tot = max(ticks["total"], 1)
        phases = {k: v / tot for k, v in ticks.items() if k != "total"}
        phases["per_workgroup_total_s"] = tot / P.tnrg.CLOCK_HZ / (p.K * p.R)
        ns = 1e9 / P.tnrg.CLOCK_HZ
        phases["ns_per_jacobi_round"] = ticks["jacobi"] * ns / max(pinfo["jacobi_rounds"], 1)
        phases["ns_per_lq_step"] = ticks["lq"] * ns / max(pinfo["lq_steps"], 1)
        phases["ns_per_svd"] = (ticks["theta"] + ticks["lq"] + ticks["jacobi"] + ticks["finish"]) * ns / max(pinfo["n_svd"], 1)
        phases["ns_per_jacobi_round_loop"] = pinfo["jacobi_round_ticks"] * ns / max(pinfo["jacobi_rounds"], 1)
        phases["jacobi_sweep_end_share"] = pinfo["jacobi_sweep_end_ticks"] / max(ticks["jacobi"], 1)
        phases["rounds_per_svd"] = pinfo["jacobi_rounds"] / max(pinfo["n_svd"], 1)
        phases["lq_steps_per_svd"] = pinfo["lq_steps"] / max(pinfo["n_svd"], 1)
        log("phase fractions of the persistent kernel: " +
            ", ".join(f"{k} {v:.3f}" for k, v in phases.items()))
        del pc

    plain = None
    if args.plain > 0:
        n = min(args.plain, p.R)
        sub_in = P.MPSBatch.from_product(p.inputs[:n], device=dev)
        sub_tg = P.MPSBatch.from_mps(p.targets[:n], dcap=max(1, tcap), device=dev)
        one_in = [P.MPSBatch(p.N, 1, 1, dev, sub_in.data[r:r + 1], sub_in.dims[r:r + 1])
                  for r in range(n)]
        one_tg = [P.MPSBatch(p.N, 1, sub_tg.dcap, dev, sub_tg.data[r:r + 1], sub_tg.dims[r:r + 1])
                  for r in range(n)]
        calls = [P.GrapeCall(model, 1, 1, one_in[r], one_tg[r], plan["dcap"],
                             ckpt_stride=ck["stride"], device=dev)
                 for r in range(n)]
        Jk = J[0:1].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r in range(n):
            calls[r].run(ux, uy, uzz, Jk)
            torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        plain = {"value": (n / p.R) / secs, "unit": "noise-samples/s",
                 "sample": f"{n} trajectories of noise sample k=0, one trajectory per launch",
                 "seconds": secs}
        log(f"plain one-trajectory-at-a-time path: {secs:.2f} s for {n} trajectories")

    serving = None
    if args.serve_seconds > 0:
        try:
            serving = serving_leg(P, W, dev, args.serve_seconds, args.serve_open_loop,
                                  args.serve_pool, arena_gib=64.0, streams=4,
                                  max_dcap=args.serve_max_dcap)
        except Exception as exc:  # the headline line is printed regardless
            serving = {"error": f"{type(exc).__name__}: {exc}"}
            log(f"serving leg failed: {serving['error']}")

    cpu = None
    if args.cpu_sample > 0:
        log("timing the CPU oracle ...")
        cpu = cpu_baseline(args.workload, min(args.cpu_sample, p.R), p.R, args.xt_model)

    out = {
        "metric": METRIC, "value": value, "unit": "noise-samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{wname}: {TASKS.get(p.task, p.task)}, N={p.N}, chi={p.chi}, "
                               f"M={p.M}, K={p.K} noise samples x R={p.R} inputs, T={p.T:.4g}, "
                               + ("Heisenberg crosstalk J^x XX + J^y YY + J^z ZZ, uniform in "
                                  "[-0.05, 0.05], every bond" if heis else
                                  "ZZ crosstalk Normal(0, sigma)"),
                   "N": p.N, "chi": p.chi, "M": p.M, "K": p.K, "R": p.R,
                   "dcap": plan["dcap"], "max_bond_dim": info["max_dim"],
                   "ckpt_stride": ck["stride"], "workspace_gib": ck["workspace_bytes"] / 2**30,
                   "threads_per_trajectory": tune.threads(plan["dcap"])},
        "autotune": tuned,
        "trajectories_per_s": value * p.R,
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "plain_gpu": plain,
        "batched_vs_plain": (value / plain["value"]) if plain else None,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "fidelity": F,
        "phases": phases,
        "jacobi": {"svds": info["n_svd"], "total_sweeps": info["total_sweeps"],
                   "max_sweeps": info["max_sweeps"]},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
