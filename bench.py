"""Benchmark of the dynamic-circuit state-vector path on one MI355X.

A step is one library call that runs the whole hot path over one batch of the
workload. Default workload (--workload c2): 28 qubits, complex128, 40 U3 + CX
brickwork layers, a 4-qubit mid-circuit measurement, a multi-bit predicate
block, an if/else on one bit and a final measure-all; one step is one
qsv_run_shots call of 16 shots (4 GiB of state per shot, all resident in HBM).
Other workloads: c1 (10 qubits, 1000 shots), c3 (batching: 4096 shots of a
16-qubit repeat-until-success circuit and 256 distinct 12-18-qubit circuits),
c4 (energy + adjoint gradient, 20 qubits, 64 parameter vectors), c5 (serving).

Prints one JSON line. `value` is the workload's throughput over the timed
steps. `roofline` describes the dominant kernel, timed with HIP events that
the library records on its stream around every launch in the timed steps;
`achieved` is the kernel's algorithmic bytes (the method's reads and writes,
not what the hardware moved) per launch over its average launch time.
`cpu_baseline` times the CPU oracle, as it stands, on a bounded sample of the
same workload, spread over the host's cores.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload c2|c1|c3|c4|c5]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "shots/s + achieved HBM GB/s on 16q/28q dynamic circuits; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CUs x 128 FP64 flops/clock x 2.4 GHz (vector and matrix cores alike)
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 matrix-core peak of the MI355X
COPY_BYTES = 4 << 30
MAX_CPU_WORKERS = 16  # oracle worker processes at most (the host cores one GPU's jobs may use)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Host facts and the CPU oracle leg (the only part of this file that runs the
# oracle; workers are fresh processes that never touch the GPU)
# ---------------------------------------------------------------------------
def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = None
    try:
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemAvailable"):
                    avail = int(line.split()[1]) * 1024
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    usable = max(1, min(usable, MAX_CPU_WORKERS))
    return {"cpu_count": os.cpu_count(), "usable_cpus": usable, "cpu_model": model,
            "mem_available_gib": None if avail is None else round(avail / (1 << 30), 1)}


def _one_thread():
    # every BLAS flavour to one thread before numpy loads its library (the
    # environment may ask for more), then once more through threadpoolctl
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        os.environ[v] = "1"
    try:
        import numpy  # noqa: F401
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass


def _w_gates(job):
    """Applies gate statements gates[idx] of the program, in order, to a fresh
    state with the oracle's own interpreter; returns (ops, seconds)."""
    src, idx = job
    from oracle import sim
    prog = sim.Program(src)
    gates = [st for st in prog.body if st[0] == "gate"]
    it = sim.Interpreter(prog)
    t0 = time.perf_counter()
    it.eng = sim.TensorEngine(prog.n_qubits)
    it.cbits, it.gate_count, it.tape, it.shift = [0] * prog.n_clbits, 0, None, {}
    for k in idx:
        it.exec_stmt(gates[k], {})
    return len(idx), time.perf_counter() - t0


def _w_shots(job):
    """Runs whole oracle shots (source, theta, seed, shot) until the list or
    the time budget ends; returns (shots, seconds)."""
    items, budget = job
    from oracle import sim
    progs = {}
    t0 = time.perf_counter()
    done = 0
    for src, theta, seed, shot in items:
        if src not in progs:
            progs[src] = sim.Program(src)
        sim.run_shot(progs[src], theta, seed=seed, shot=shot)
        done += 1
        if time.perf_counter() - t0 > budget:
            break
    return done, time.perf_counter() - t0


def _w_adjoint(job):
    src, theta, coeffs, codes = job
    from oracle import sim
    t0 = time.perf_counter()
    sim.grad_adjoint(src, theta, coeffs, codes)
    return 1, time.perf_counter() - t0


def _w_lower(srcs):
    """Host-side lowering of OpenQASM sources (front end only, no GPU)."""
    from paper_2604_11599_amd.lower import lower
    return [lower(s) for s in srcs]


def _pool_map(fn, jobs, workers):
    import multiprocessing as mp
    out = []
    with mp.get_context("spawn").Pool(workers, initializer=_one_thread) as pool:
        for k, r in enumerate(pool.imap(fn, jobs, chunksize=1)):
            out.append(r)
            log(f"  cpu worker {k + 1}/{len(jobs)} done: {r[0]} units in {r[1]:.1f} s")
    return out


def _rate(results):
    """Aggregate rate of workers that ran side by side: sum of their own rates."""
    return sum(n / t for n, t in results if t > 0)


def cpu_c2(src, budget_s):
    """The first two brickwork layers of the 28-qubit program, their gates dealt
    round-robin to W workers that each evolve their own 28-qubit state
    (independent shots, as the GPU's 16 shots are); the aggregate operation rate
    is extrapolated to whole shots (gates + measurement operations)."""
    from oracle import sim
    info = host_info()
    prog = sim.Program(src)
    n = prog.n_qubits
    gates = [st for st in prog.body if st[0] == "gate"]
    per_layer = n + (n - 1) // 2 if n > 1 else 1
    sample = min(len(gates), 2 * per_layer + 1)  # layer 0 has n//2 CX, layer 1 (n-1)//2
    ops_per_shot = len(gates) + n
    for st in prog.body:
        if st[0] == "measure" and st[1][2] is not None:
            ops_per_shot += 1
    mem = info["mem_available_gib"] or 64.0
    workers = max(1, min(info["usable_cpus"], int(mem // 24), 4))
    jobs = [(src, list(range(w, sample, workers))) for w in range(workers)]
    log(f"cpu baseline: {sample} gates of two layers over {workers} workers ({n} qubits each)")
    res = _pool_map(_w_gates, jobs, workers)
    ops_s = _rate(res)
    secs = max(t for _, t in res)
    return {"value": ops_s / ops_per_shot, "unit": "shots/s", "cores": workers, "kind": "oracle",
            "sample": f"the first two layers ({sample} of {ops_per_shot} state operations of a shot), dealt "
                      f"round-robin to {workers} single-threaded workers, each with its own {n}-qubit state; "
                      f"{secs:.1f} s wall; operation rate extrapolated to whole shots",
            "extrapolated": True, "host": info}


def cpu_shots(items, budget_s, unit="shots/s", what=""):
    info = host_info()
    workers = max(1, info["usable_cpus"])
    jobs = [(items[w::workers], budget_s) for w in range(workers)]
    log(f"cpu baseline: {len(items)} shots over {workers} workers, {budget_s:.0f} s budget")
    res = _pool_map(_w_shots, jobs, workers)
    done = sum(n for n, _ in res)
    return {"value": _rate(res), "unit": unit, "cores": workers, "kind": "oracle",
            "sample": f"{done} of the step's {len(items)} shots{what}, dealt round-robin to {workers} "
                      f"single-threaded workers with a {budget_s:.0f} s budget each",
            "extrapolated": done < len(items), "host": info}


def cpu_c4(src, thetas, coeffs, codes):
    info = host_info()
    workers = max(1, min(info["usable_cpus"], len(thetas)))
    jobs = [(src, thetas[w], coeffs, codes) for w in range(workers)]
    log(f"cpu baseline: oracle adjoint of {workers} parameter vectors over {workers} workers")
    res = _pool_map(_w_adjoint, jobs, workers)
    return {"value": _rate(res), "unit": "parameter vectors/s (energy + 240-entry gradient)", "cores": workers,
            "kind": "oracle",
            "sample": f"the oracle's plain adjoint of {workers} of the 64 parameter vectors, one per "
                      f"single-threaded worker, side by side ({max(t for _, t in res):.1f} s wall)",
            "extrapolated": False, "host": info}


# ---------------------------------------------------------------------------
# GPU helpers
# ---------------------------------------------------------------------------
def copy_ceiling(reps=5):
    """A plain 4 GiB device-to-device copy kernel of the library, timed with
    HIP events on the stream it runs on: the bandwidth a streaming kernel
    reaches on this device (reads + writes)."""
    import ctypes as C

    import torch

    from paper_2604_11599_amd import Context
    from paper_2604_11599_amd import _abi as A
    stream = torch.cuda.current_stream()
    ctx = Context(0, stream=stream)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        ctx.check(A.lib().qsv_diag_copy(ctx.handle, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                        COPY_BYTES))
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    ctx.close()
    del src, dst
    torch.cuda.empty_cache()
    t = sorted(times)[len(times) // 2]
    gbs = 2 * COPY_BYTES / t / 1e9
    return {"kernel": "k_copy", "bytes_per_launch": 2 * COPY_BYTES, "median_launch_ms": 1e3 * t,
            "achieved": gbs, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}


def traffic_from_profiles(name):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"tile_pass_{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    from traffic_summary import kernel_hash
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def c4_traffic():
    """HBM bytes per launch of the energy + gradient kernels from committed
    counter runs taken on the current kernel source, by kernel name."""
    path = os.path.join(ROOT, "profiles", "c4_20q_traffic.json")
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        d = json.load(f)
    from traffic_summary import ADJOINT_SOURCES, kernel_hash
    if d.get("kernel_hash") != kernel_hash(ADJOINT_SOURCES):
        return {}
    return {k: v["bytes_per_launch"] for k, v in d.get("kernels", {}).items()}


def hbm_roof(kernel, launches, ms, nbytes, ceiling=None, traffic=None, bytes_note=""):
    t = ms / 1e3
    gbs = nbytes / t / 1e9 if t else 0.0
    out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
           "traffic": traffic, "kernel": kernel, "launches": launches,
           "avg_launch_ms": ms / launches if launches else 0.0,
           "algorithmic_bytes_per_launch": nbytes / launches if launches else 0.0,
           "algorithmic_bytes": bytes_note}
    if ceiling:
        out["copy_ceiling"] = ceiling
        out["frac_of_copy_ceiling"] = gbs / ceiling["achieved"] if ceiling["achieved"] else None
    return out


def timed(fn, steps, warmup, on_step=None):
    import torch
    for w in range(warmup):
        fn(1000 + w)
        log(f"warmup {w} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        fn(s)
        if on_step:
            on_step(s)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def base_line(args, value, unit, dt, cfg, dtype="f64"):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": cfg}


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def workload(name):
    import workloads as W
    if name == "c2":
        return (W.c2_program(seed=2, n=28, layers=40), 16,
                {"workload": "28-qubit complex128 dynamic circuit: 40 U3+CX brickwork layers, "
                             "4-qubit mid-circuit measurement, if (c == 0b1010) 3-gate block, "
                             "if/else rx/rz on c[0], measure-all; 16 shots per step",
                 "qubits": 28, "layers": 40, "shots_per_step": 16})
    if name == "c1":
        return (W.c1_program(seed=1), 1000,
                {"workload": "10-qubit complex128 dynamic circuit: 20 U3+CX layers with 3 "
                             "measure/if/reset sites, measure-all; 1000 shots per step",
                 "qubits": 10, "layers": 20, "shots_per_step": 1000})
    raise SystemExit(f"unknown workload {name}")


def bench_shots(args):
    """c2 / c1: one qsv_run_shots call of the workload's shots per step."""
    import torch

    from paper_2604_11599_amd import Context
    src, shots, cfg = workload(args.workload)
    log("workload", args.workload, cfg["workload"])
    ceiling = copy_ceiling() if args.workload == "c2" else None
    if ceiling:
        log(f"copy ceiling {ceiling['achieved']:.0f} GB/s")
    # the timed steps run in a context without profiling events; the same
    # steps are then repeated in a profiling context for the roofline figures
    ctx = Context(0)
    prog = ctx.load(src)
    log(f"planned {prog.info.n_passes} passes, {prog.info.n_sites} measurement sub-sites")
    for w in range(args.warmup):
        prog.run_shots(shots, seed=1000 + w)
        log(f"warmup {w} done")
    dt = timed(lambda s: prog.run_shots(shots, seed=s), args.steps, 0, lambda s: log(f"step {s} done"))
    pctx = Context(0, profile=True)
    pprog = pctx.load(src)
    pprog.run_shots(shots, seed=999)
    pctx.profile_reset()
    dt_prof = timed(lambda s: pprog.run_shots(shots, seed=s), args.steps, 0)
    prof = pctx.profile()
    log("profiled steps done")
    out = base_line(args, shots * args.steps / dt, "shots/s", dt, cfg)
    out["profiled_ms_per_step"] = 1e3 * dt_prof / args.steps
    launches = prof["pass_uncond_launches"]
    roof = hbm_roof("k_tile_pass_d8" if args.workload == "c2" else "k_tile_pass_d8, k_tile_pass_r", launches,
                    prof["pass_uncond_ms"], prof["pass_uncond_bytes"], ceiling,
                    traffic_from_profiles(args.workload),
                    "32 B per amplitude per tile pass (read + write of a complex128), 16 B for the pass "
                    "that also prepares |0...0>; passes without guarded gates only")
    t = prof["pass_uncond_ms"] / 1e3
    tfl = prof["pass_uncond_flops"] / t / 1e12 if t else 0.0
    roof["fp64"] = {"achieved": tfl, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tfl / FP64_PEAK_TFLOPS,
                    "flops": "14 per amplitude per dense one-qubit gate (the complex 2x2 product's real "
                             "multiplies and adds), 0 for CX"}
    roof["fp64_at_8_flops"] = {"achieved": tfl * 8 / 14, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                               "frac": tfl * 8 / 14 / FP64_PEAK_TFLOPS,
                               "flops": "8 per amplitude per dense one-qubit gate, 0 for CX (every gate "
                                        "of the counted passes is a U3 or a CX)"}
    roof["time_share"] = {"tile_pass_ms": prof["pass_ms"], "site_ms": prof["site_ms"],
                          "other_ms": prof["other_ms"], "wall_ms": 1e3 * dt}
    out["roofline"] = roof
    out["passes_per_shot"] = prog.info.n_passes

    if args.workload == "c1":
        # the same steps as one captured launch sequence replayed per call
        prog.run_shots(shots, seed=999, graph=True)
        dt_g = timed(lambda s: prog.run_shots(shots, seed=s, graph=True), args.steps, 0)
        out["graph"] = {"value": shots * args.steps / dt_g, "unit": "shots/s", "ms_per_step": 1e3 * dt_g / args.steps,
                        "note": "same shots, QSV_RUN_GRAPH: the call's launches captured once in a HIP graph and "
                                "replayed (bit-identical results)"}
        log("graph steps done")
        # the same shots under depolarizing noise (rate 1e-3 per qubit after every gate)
        noisy = ctx.load(src, noise=True)
        noisy.run_shots(shots, seed=998, depolarizing=1e-3)
        dt_n = timed(lambda s: noisy.run_shots(shots, seed=s, depolarizing=1e-3), args.steps, 0)
        out["depolarizing"] = {"value": shots * args.steps / dt_n, "unit": "shots/s",
                               "ms_per_step": 1e3 * dt_n / args.steps, "rate": 1e-3,
                               "passes_per_shot": noisy.info.n_passes,
                               "note": "same program loaded with depolarizing slots: after every gate each of "
                                       "its qubits takes X, Y or Z with probability 1e-3/3; each shot binds its own "
                                       "matrices and composes the dense phases in which it draws a Pauli"}
        log("depolarizing steps done")
    if args.workload == "c2":
        # the same steps with trajectory sharing (shots with equal measurement histories share one state)
        dt_sp = timed(lambda s: prog.run_shots(shots, seed=s, share=True), args.steps, 0)
        out["shared_trajectories"] = {
            "value": shots * args.steps / dt_sp, "unit": "shots/s", "ms_per_step": 1e3 * dt_sp / args.steps,
            "note": "same shots, bit-identical results; shots with equal measurement histories share one "
                    "state (gate passes once per distinct history)"}
        log("shared-trajectory steps done")
        # the same steps with a complex64 state
        prog.run_shots(shots, seed=1000, complex64=True)
        dt_c64 = timed(lambda s: prog.run_shots(shots, seed=s, complex64=True), args.steps, 0)
        pprog.run_shots(shots, seed=1000, complex64=True)
        pctx.profile_reset()
        timed(lambda s: pprog.run_shots(shots, seed=s, complex64=True), args.steps, 0)
        p64 = pctx.profile()
        r64 = hbm_roof("k_tile_pass_d8", p64["pass_uncond_launches"], p64["pass_uncond_ms"],
                       p64["pass_uncond_bytes"], ceiling, traffic_from_profiles("c2_c64"),
                       "16 B per amplitude per tile pass (read + write of a complex64)")
        t64 = p64["pass_uncond_ms"] / 1e3
        tf32 = p64["pass_uncond_flops"] / t64 / 1e12 if t64 else 0.0
        r64["fp32_mfma"] = {"achieved": tf32, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                            "frac": tf32 / FP32_MFMA_PEAK_TFLOPS}
        out["complex64"] = {"value": shots * args.steps / dt_c64, "unit": "shots/s",
                            "ms_per_step": 1e3 * dt_c64 / args.steps, "dtype": "c64", "roofline": r64,
                            "note": "same shots with a complex64 state (the precision of the paper's GPU runs)"}
        log("complex64 steps done")
    pctx.close()
    ctx.close()
    if not args.no_cpu_baseline:
        if args.workload == "c2":
            out["cpu_baseline"] = cpu_c2(src, args.cpu_budget)
        else:
            items = [(src, None, 0, s) for s in range(shots)]
            out["cpu_baseline"] = cpu_shots(items, args.cpu_budget)
    print(json.dumps(out))


def bench_batching(args):
    """c3: 4096 shots of the 16-qubit RUS circuit plus 256 distinct 12..18-qubit
    circuits of the same structure (16 shots each) in one qsv_run_batch call per
    step. The 256-circuit mix runs as work items of one persistent launch; the
    4096-shot request (13..20 qubits, at least 64 shots) and the 18-qubit
    circuits of the mix run on the tile passes with shared trajectories, on the
    context's batch forks from host threads of their own while the persistent
    launch runs, as qsv_run_batch routes them."""
    import workloads as W
    from paper_2604_11599_amd import Context
    # the timed steps run in a context without profiling events; the same
    # batches are then repeated in a profiling context for the roofline figures
    ctx = Context(0)
    main_src = W.c3_program(seed=3, n=16)
    mix_src = W.c3_mix(seed=33, count=256)
    main_prog = ctx.load(main_src)
    mix = [ctx.load(src) for src in mix_src]
    reqs = [{"prog": main_prog, "shots": 4096, "seed": 1}]
    reqs += [{"prog": p, "shots": 16, "seed": 100 + k} for k, p in enumerate(mix)]
    shots = sum(r["shots"] for r in reqs)
    log(f"batching workload: {len(reqs)} requests, {shots} shots")
    for _ in range(args.warmup):
        ctx.run_batch(reqs)
    dt = timed(lambda s: ctx.run_batch(reqs), args.steps, 0)
    log("batched steps done")
    pctx = Context(0, profile=True)
    preqs = [dict(r, prog=pctx.load(src)) for r, src in zip(reqs, [main_src] + list(mix_src))]
    pctx.run_batch(preqs)
    pctx.profile_reset()
    dt_prof = timed(lambda s: pctx.run_batch(preqs), args.steps, 0)
    prof = pctx.profile()
    pctx.close()
    log("profiled batches done")
    dt_plain = timed(lambda s: [r["prog"].run_shots(r["shots"], seed=r["seed"]) for r in reqs], args.steps, 0)
    dt_plain_sh = timed(lambda s: [r["prog"].run_shots(r["shots"], seed=r["seed"], share=True) for r in reqs],
                        args.steps, 0)
    for r in reqs:
        r["prog"].run_shots(r["shots"], seed=r["seed"], graph=True)  # capture
    dt_plain_g = timed(lambda s: [r["prog"].run_shots(r["shots"], seed=r["seed"], graph=True) for r in reqs],
                       args.steps, 0)
    t_main = timed(lambda s: main_prog.run_shots(4096, seed=1, share=True), args.steps, 0)
    out = base_line(args, shots * args.steps / dt, "shots/s", dt,
                    {"workload": "batching: 4096 shots of a 16-qubit RUS circuit (tile passes, shared "
                                 "trajectories) + 256 distinct 12-18 qubit circuits x 16 shots (one persistent "
                                 "launch; the 18-qubit ones on the tile passes), one qsv_run_batch call per step",
                     "shots_per_step": shots})
    out["profiled_ms_per_step"] = 1e3 * dt_prof / args.steps
    out["roofline"] = hbm_roof(
        "k_persistent", prof["persistent_launches"], prof["persistent_ms"], prof["persistent_bytes"], None, None,
        "32 B per amplitude per pass of every 13-18-qubit state streamed from its HBM slot, 16 B per site "
        "reduction and state preparation, counted on the device; 12-qubit states stay in LDS and count 0")
    out["roofline"]["tile_pass_leg"] = {
        "launches": prof["pass_uncond_launches"], "ms": prof["pass_uncond_ms"],
        "achieved_gbs": (prof["pass_uncond_bytes"] / (prof["pass_uncond_ms"] / 1e3) / 1e9
                         if prof["pass_uncond_ms"] else 0.0)}
    out["plain_per_program"] = {"value": shots * args.steps / dt_plain, "unit": "shots/s",
                                "ms_per_step": 1e3 * dt_plain / args.steps,
                                "note": "same requests through qsv_run_shots, one program at a time, "
                                        "every shot its own state"}
    out["plain_per_program_shared"] = {"value": shots * args.steps / dt_plain_sh, "unit": "shots/s",
                                       "ms_per_step": 1e3 * dt_plain_sh / args.steps,
                                       "note": "same, with trajectory sharing in every call (the gain of "
                                               "batching alone, sharing on both sides)"}
    out["plain_per_program_graph"] = {"value": shots * args.steps / dt_plain_g, "unit": "shots/s",
                                      "ms_per_step": 1e3 * dt_plain_g / args.steps,
                                      "note": "same requests through qsv_run_shots with QSV_RUN_GRAPH: each program's "
                                              "launch sequence captured once and replayed, every shot its own state"}
    out["main_request_alone_ms"] = 1e3 * t_main / args.steps
    ctx.close()
    if not args.no_cpu_baseline:
        items = [(main_src, None, 1, s) for s in range(4096)]
        for k, src in enumerate(mix_src):
            items += [(src, None, 100 + k, s) for s in range(16)]
        # interleave the requests so that every worker's share samples the whole mix
        import random
        random.Random(0).shuffle(items)
        out["cpu_baseline"] = cpu_shots(items, args.cpu_budget, what=" (4096 RUS shots and the 256-circuit mix, "
                                                                     "in seeded random order)")
    print(json.dumps(out))


def bench_vqe(args):
    """c4: energy + full adjoint gradient of the 20-qubit, 240-parameter
    hardware-efficient ansatz with a 60-term Pauli Hamiltonian, batched over 64
    parameter vectors per call."""
    import workloads as W
    from paper_2604_11599_amd import Context
    ctx = Context(0, profile=True)
    src = W.c4_ansatz(20, 6)
    prog = ctx.load(src)
    coeffs, codes = W.c4_hamiltonian(seed=4, n=20, terms=60)
    thetas = W.c4_thetas(seed=44, batch=64, n_params=240)
    for _ in range(args.warmup):
        prog.expval_grad(thetas, coeffs, codes)
    ctx.profile_reset()
    dt = timed(lambda s: prog.expval_grad(thetas, coeffs, codes), args.steps, 0)
    prof = ctx.profile()
    dt_e = timed(lambda s: prog.expval(thetas, coeffs, codes), args.steps, 0)
    out = base_line(args, 64 * args.steps / dt, "parameter vectors/s (energy + 240-entry gradient)", dt,
                    {"workload": "20-qubit HEA, 6 layers RY/RZ + CX ladder, 240 parameters, 60-term "
                                 "2-local Pauli Hamiltonian, batch of 64 parameter vectors per call"})
    tr = c4_traffic()
    out["roofline"] = hbm_roof("k_backward_mfma", prof["sweep_launches"], prof["sweep_ms"], prof["sweep_bytes"],
                               None, tr.get("k_backward_mfma"), "64 B per amplitude per swept pass (psi and "
                                                                "lambda, each read and written, complex128)")
    out["roofline"]["hamiltonian"] = hbm_roof("k_hamiltonian", prof["ham_launches"], prof["ham_ms"],
                                              prof["ham_bytes"], None, tr.get("k_hamiltonian"),
                                              "16 B per amplitude read (psi) + 16 B written (lambda)")
    out["roofline"]["forward_tile_pass"] = hbm_roof("k_tile_pass_d8", prof["pass_uncond_launches"],
                                                    prof["pass_uncond_ms"], prof["pass_uncond_bytes"], None, None,
                                                    "32 B per amplitude per pass")
    out["energy_only"] = {"value": 64 * args.steps / dt_e, "ms_per_step": 1e3 * dt_e / args.steps}
    out["time_share_ms"] = {"forward_tile_pass": prof["pass_ms"], "hamiltonian": prof["ham_ms"],
                            "adjoint_sweep": prof["sweep_ms"], "other": prof["other_ms"], "wall": 1e3 * dt}
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_c4(src, thetas, coeffs, codes)
    print(json.dumps(out))


def bench_serving(args):
    """c5: a Poisson request stream replayed in real time against the serving
    engine; 80% dynamic circuits (12..26 qubits), 20% 20-qubit energy+gradient
    calls. Circuits are lowered and loaded before the replay starts."""
    import numpy as np

    import workloads as W
    from paper_2604_11599_amd import Context
    from paper_2604_11599_amd.serve import replay
    from concurrent.futures import ThreadPoolExecutor
    ctx = Context(0, profile=True)
    log("serving: generating the request trace")
    trace = W.c5_trace(seed=5, rate=args.rate, duration=args.window, pool=args.pool or None)
    vqe = ctx.load(W.c4_ansatz(20, 6))
    # every distinct circuit compiled before the replay: lowered in worker
    # processes, planned and uploaded by forked contexts on host threads
    t_c = time.perf_counter()
    srcs = sorted({r["source"] for r in trace if r["kind"] != "vqe"})
    workers = host_info()["usable_cpus"]
    chunks = [srcs[k::workers] for k in range(workers)]
    log(f"serving: lowering {len(srcs)} distinct circuits over {workers} processes")
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        lowered_chunks = pool.map(_w_lower, chunks)
    forks = [ctx.fork() for _ in range(min(8, workers))]
    jobs = [[] for _ in forks]
    for k, (chunk, lps) in enumerate(zip(chunks, lowered_chunks)):
        jobs[k % len(forks)] += list(zip(chunk, lps))
    log(f"serving: planning and uploading on {len(forks)} forked contexts")
    with ThreadPoolExecutor(len(forks)) as ex:
        parts = list(ex.map(lambda fj: [(s, fj[0].load(lp)) for s, lp in fj[1]], zip(forks, jobs)))
    loaded = {s: p for part in parts for s, p in part}
    compile_s = time.perf_counter() - t_c
    log(f"serving: {len(loaded)} circuits compiled in {compile_s:.1f} s")
    reqs = []
    for r in trace:
        r = dict(r)
        r["prog"] = vqe if r["kind"] == "vqe" else loaded[r["source"]]
        reqs.append(r)
    offered_shots = sum(r.get("shots", 0) for r in reqs)
    log(f"serving: {len(reqs)} requests over {args.window} s ({offered_shots} shots offered)")
    out = replay(ctx, reqs, hbm_budget=int(args.hbm_gib * (1 << 30)), shots_per_tick=args.slice,
                 drain_limit_s=args.drain, log=log, profile=True)
    prof = out["profile"]
    lat = np.array(sorted(out["latency"].values())) if out["latency"] else np.zeros(1)
    res = {"metric": METRIC, "value": out["shots_done"] / out["elapsed"], "unit": "shots/s", "n_gpus": 1,
           "steps": 1, "warmup": 0, "ms_per_step": 1e3 * out["elapsed"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"serving: Poisson {args.rate} req/s for {args.window} s, 80% dynamic "
                                  f"circuits 12-26 qubits (1-1024 shots, "
                                  f"{'distinct circuits' if not args.pool else str(args.pool) + ' circuits'}), "
                                  f"20% 20-qubit energy+gradient", "hbm_budget_gib": args.hbm_gib,
                      "shots_per_tick": args.slice},
           "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
           "offered_req_per_s": len(reqs) / max(out["window"], 1e-9),
           "served_req_per_s": out["completed"] / out["elapsed"],
           "completed": out["completed"], "submitted": out["submitted"], "unfinished": out["unfinished"],
           "backlog_at_window_end": out["backlog_at_window_end"], "ticks": out["ticks"],
           "distinct_circuits": len(loaded), "compile_s_before_replay": compile_s}
    res["roofline"] = hbm_roof("k_tile_pass", prof["pass_uncond_launches"], prof["pass_uncond_ms"],
                               prof["pass_uncond_bytes"], None, None,
                               "32 B per amplitude per tile pass of the wide requests' states")
    res["roofline"]["persistent"] = hbm_roof("k_persistent", prof["persistent_launches"], prof["persistent_ms"],
                                             prof["persistent_bytes"], None, None, "streamed states, counted on "
                                                                                    "the device")
    ctx.close()
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_serving(reqs, args.cpu_budget)
    print(json.dumps(res))


def cpu_serving(reqs, budget_s):
    """The oracle's per-request cost, extrapolated: per-gate times measured at
    every width the trace uses, times each request's operations and shots."""
    info = host_info()
    widths = sorted({r["n"] for r in reqs})
    jobs = []
    for n in widths:
        src = "OPENQASM 3.0;\nqubit[%d] q;\n" % n + "".join(f"U(0.1, 0.2, 0.3) q[{q % n}];\n" for q in range(6))
        jobs.append((src, list(range(6))))
    workers = max(1, min(info["usable_cpus"], len(jobs)))
    log(f"cpu baseline: per-gate oracle time at {len(widths)} widths")
    res = _pool_map(_w_gates, jobs, workers)
    per_gate = {n: t / k for n, (k, t) in zip(widths, res)}
    total = 0.0
    for r in reqs:
        if r["kind"] == "vqe":
            # forward gates, the Hamiltonian's terms, and per gate of the backward
            # sweep the two states' inverse gates and one derivative
            gates = 354 + 60 + 3 * 354
            total += gates * per_gate[r["n"]]
        else:
            ops = 0
            for line in r["source"].splitlines():
                if not line or line.startswith(("OPENQASM", "include", "qubit", "bit", "}")):
                    continue
                ops += r["n"] if line.startswith("f = measure") else 1
            total += r["shots"] * ops * per_gate[r["n"]]
    return {"value": len(reqs) / total * workers, "unit": "requests/s", "cores": workers, "kind": "oracle",
            "sample": f"per-gate oracle times at the trace's {len(widths)} widths, 6 gates each, on {workers} "
                      f"workers; every request's gates x shots summed and spread over the workers",
            "extrapolated": True, "host": info}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--window", type=float, default=60.0)
    ap.add_argument("--drain", type=float, default=60.0)
    ap.add_argument("--slice", type=int, default=256)
    ap.add_argument("--hbm-gib", type=float, default=64.0)
    ap.add_argument("--pool", type=int, default=0, help="0: every circuit request has its own circuit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c3":
        bench_batching(args)
    elif args.workload == "c4":
        bench_vqe(args)
    elif args.workload == "c5":
        bench_serving(args)
    else:
        bench_shots(args)


if __name__ == "__main__":
    main()
