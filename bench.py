"""Benchmark of the dynamic-circuit state-vector path on one MI355X.

A step is one qsv_run_shots call that runs every shot of the workload through
the whole hot path (state init, fused gate passes, mid-circuit measurement,
feed-forward, final measure-all). Default workload: 28 qubits, complex128,
40 U3 + CX brickwork layers, a 4-qubit mid-circuit measurement, a multi-bit
predicate block, an if/else on one bit and a final measure-all; 16 shots per
step (4 GiB of state per shot, all resident in HBM).

Prints one JSON line. `value` is shots/s over the timed steps. `roofline`
describes the dominant kernel (the tile pass), timed with HIP events inside
the library during the timed steps. `cpu_baseline` times the CPU oracle on a
bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload c2|c1|c3]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6   # 256 CUs x 128 FP64 flops/clock x 2.4 GHz (vector and matrix cores alike)
FP32_MFMA_PEAK_TFLOPS = 157.3  # dense FP32 matrix-core peak of the MI355X


def log(*a):
    print(*a, file=sys.stderr, flush=True)


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
    if name == "c3":
        return (W.c3_program(seed=3, n=16), 4096,
                {"workload": "16-qubit complex128: 12 random layers, then a repeat-until-success "
                             "loop of at most 8 iterations; measure-all; 4096 shots per step",
                 "qubits": 16, "layers": 12, "shots_per_step": 4096})
    raise SystemExit(f"unknown workload {name}")


def traffic_from_profiles(name):
    """HBM bytes per tile-pass launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"tile_pass_{name}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    from paper_2604_11599_amd.traffic_summary import kernel_hash
    if d.get("kernel_hash") != kernel_hash():
        return None
    return d.get("bytes_per_launch")


def cpu_baseline(src, budget_s=15.0):
    """The oracle, as it stands, on the first operations of one shot of the workload;
    the per-operation time is extrapolated to a whole shot."""
    import numpy as np

    from oracle import sim
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    prog = sim.Program(src)
    ops_per_shot = 0
    for st in prog.body:
        if st[0] in ("gate",):
            ops_per_shot += 1
        elif st[0] == "measure":
            ops_per_shot += prog.qregs["q"][1] if st[1][2] is None else 1
        elif st[0] == "if":
            ops_per_shot += max(len(st[2]), len(st[3]))
    gates = [st for st in prog.body if st[0] == "gate"]
    it = sim.Interpreter(prog)
    t0 = time.perf_counter()
    it.eng = sim.TensorEngine(prog.n_qubits)
    it.cbits, it.gate_count, it.tape, it.shift = [0] * prog.n_clbits, 0, None, {}
    t_alloc = time.perf_counter() - t0
    done = 0
    t1 = time.perf_counter()
    while done < len(gates) and (done < 2 or time.perf_counter() - t1 < budget_s):
        it.exec_stmt(gates[done], {})
        done += 1
    dt = time.perf_counter() - t1
    per_op = dt / done
    shot_s = per_op * ops_per_shot + t_alloc
    del it
    _ = np
    return {"value": 1.0 / shot_s, "unit": "shots/s", "cores": threads, "kind": "oracle",
            "sample": f"first {done} of {ops_per_shot} state operations of one shot "
                      f"({prog.n_qubits} qubits), {dt:.1f} s; extrapolated linearly to a whole shot"}


def bench_batching(args):
    """The batching workload: 4096 shots of the 16-qubit RUS circuit plus 256 distinct
    12..18-qubit circuits of the same structure (16 shots each), all in one persistent
    launch (qsv_run_batch), against the same shots through qsv_run_shots per program."""
    import torch

    import workloads as W
    from paper_2604_11599_amd import Context
    ctx = Context(0, profile=True)
    main_prog = ctx.load(W.c3_program(seed=3, n=16))
    mix = [ctx.load(src) for src in W.c3_mix(seed=33, count=256)]
    reqs = [{"prog": main_prog, "shots": 4096, "seed": 1}]
    reqs += [{"prog": p, "shots": 16, "seed": 100 + k} for k, p in enumerate(mix)]
    shots = sum(r["shots"] for r in reqs)
    log(f"batching workload: {len(reqs)} requests, {shots} shots")
    for _ in range(args.warmup):
        ctx.run_batch(reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.run_batch(reqs)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("persistent steps done")
    t1 = time.perf_counter()
    for _ in range(args.steps):
        for r in reqs:
            r["prog"].run_shots(r["shots"], seed=r["seed"])
    torch.cuda.synchronize()
    dt_plain = time.perf_counter() - t1
    out = {"metric": "shots/s + achieved HBM GB/s on 16q/28q dynamic circuits; p50/p99 request latency",
           "value": shots * args.steps / dt, "unit": "shots/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "batching: 4096 shots of a 16-qubit RUS circuit + 256 distinct 12-18 "
                                  "qubit circuits x 16 shots, one persistent launch per step",
                      "shots_per_step": shots},
           "plain_per_program": {"value": shots * args.steps / dt_plain, "unit": "shots/s",
                                 "ms_per_step": 1e3 * dt_plain / args.steps,
                                 "note": "same requests through qsv_run_shots, one program at a time"}}
    print(json.dumps(out))


def bench_vqe(args):
    """The differentiation workload: energy + full adjoint gradient of the 20-qubit,
    240-parameter hardware-efficient ansatz with a 60-term Pauli Hamiltonian, batched
    over 64 parameter vectors per call."""
    import torch

    import workloads as W
    from paper_2604_11599_amd import Context
    ctx = Context(0, profile=True)
    prog = ctx.load(W.c4_ansatz(20, 6))
    coeffs, codes = W.c4_hamiltonian(seed=4, n=20, terms=60)
    thetas = W.c4_thetas(seed=44, batch=64, n_params=240)
    for _ in range(args.warmup):
        prog.expval_grad(thetas, coeffs, codes)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prog.expval_grad(thetas, coeffs, codes)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        prog.expval(thetas, coeffs, codes)
    torch.cuda.synchronize()
    dt_e = time.perf_counter() - t1
    out = {"metric": "shots/s + achieved HBM GB/s on 16q/28q dynamic circuits; p50/p99 request latency",
           "value": 64 * args.steps / dt, "unit": "parameter vectors/s (energy + 240-entry gradient)",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * dt / args.steps,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic",
           "config": {"workload": "20-qubit HEA, 6 layers RY/RZ + CX ladder, 240 parameters, 60-term "
                                  "2-local Pauli Hamiltonian, batch of 64 parameter vectors per call"},
           "energy_only": {"value": 64 * args.steps / dt_e, "ms_per_step": 1e3 * dt_e / args.steps},
           "time_share_ms": {"forward_tile_pass": prof["pass_ms"], "other": prof["other_ms"],
                             "wall": 1e3 * dt}}
    print(json.dumps(out))


def bench_serving(args):
    """The serving workload: a Poisson request stream replayed in real time against the
    serving engine; 80% dynamic circuits (12..26 qubits), 20% 20-qubit energy+gradient
    calls. Circuits are lowered and loaded before the replay starts."""
    import numpy as np

    import workloads as W
    from paper_2604_11599_amd import Context
    from paper_2604_11599_amd.serve import replay
    ctx = Context(0)
    trace = W.c5_trace(seed=5, rate=args.rate, duration=args.window, pool=args.pool)
    vqe = ctx.load(W.c4_ansatz(20, 6))
    loaded, reqs = {}, []
    for r in trace:
        r = dict(r)
        if r["kind"] == "vqe":
            r["prog"] = vqe
        else:
            if r["source"] not in loaded:
                loaded[r["source"]] = ctx.load(r["source"])
            r["prog"] = loaded[r["source"]]
        reqs.append(r)
    offered_shots = sum(r.get("shots", 0) for r in reqs)
    log(f"serving: {len(reqs)} requests over {args.window} s ({offered_shots} shots offered)")
    out = replay(ctx, reqs, hbm_budget=int(args.hbm_gib * (1 << 30)), shots_per_tick=args.slice,
                 drain_limit_s=args.drain, log=log)
    lat = np.array(sorted(out["latency"].values())) if out["latency"] else np.zeros(1)
    res = {"metric": "shots/s + achieved HBM GB/s on 16q/28q dynamic circuits; p50/p99 request latency",
           "value": out["shots_done"] / out["elapsed"], "unit": "shots/s", "n_gpus": 1, "steps": 1,
           "warmup": 0, "ms_per_step": 1e3 * out["elapsed"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"serving: Poisson {args.rate} req/s for {args.window} s, 80% dynamic "
                                  f"circuits 12-26 qubits (1-1024 shots, {args.pool} distinct circuits), "
                                  f"20% 20-qubit energy+gradient", "hbm_budget_gib": args.hbm_gib,
                      "shots_per_tick": args.slice},
           "latency_p50_s": float(np.percentile(lat, 50)), "latency_p99_s": float(np.percentile(lat, 99)),
           "offered_req_per_s": len(reqs) / max(out["window"], 1e-9),
           "served_req_per_s": out["completed"] / out["elapsed"],
           "completed": out["completed"], "submitted": out["submitted"], "unfinished": out["unfinished"],
           "backlog_at_window_end": out["backlog_at_window_end"], "ticks": out["ticks"]}
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--window", type=float, default=10.0)
    ap.add_argument("--drain", type=float, default=60.0)
    ap.add_argument("--slice", type=int, default=256)
    ap.add_argument("--hbm-gib", type=float, default=64.0)
    ap.add_argument("--pool", type=int, default=64)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "c3":
        bench_batching(args)
        return
    if args.workload == "c5":
        bench_serving(args)
        return
    if args.workload == "c4":
        bench_vqe(args)
        return

    import torch
    from paper_2604_11599_amd import Context

    src, shots, cfg = workload(args.workload)
    log("workload", args.workload, cfg["workload"])
    ctx = Context(0, profile=True)
    prog = ctx.load(src)
    log(f"planned {prog.info.n_passes} passes, {prog.info.n_sites} measurement sub-sites")
    for w in range(args.warmup):
        prog.run_shots(shots, seed=1000 + w)
        log(f"warmup {w} done")
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        prog.run_shots(shots, seed=s)
        log(f"step {s} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile()
    ms_per_step = 1e3 * dt / args.steps
    value = shots * args.steps / dt

    launches = prof["pass_uncond_launches"]
    t_pass = prof["pass_uncond_ms"] / 1e3
    gbs = prof["pass_uncond_bytes"] / t_pass / 1e9 if t_pass else 0.0
    tfl = prof["pass_uncond_flops"] / t_pass / 1e12 if t_pass else 0.0
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    # gate arithmetic runs on the FP64 matrix cores where the plan has dense
    # phases (the MI355X FP64 matrix and vector peaks are both 78.6 TFLOP/s);
    # achieved counts the gates' algorithmic flops either way
    from paper_2604_11599_amd import lower
    from paper_2604_11599_amd.api import plan_inspect
    dense = plan_inspect(lower(src), 0).n_dense_phases > 0
    alu = {"bound": "mfma" if dense else "alu", "achieved": tfl, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": tfl / FP64_PEAK_TFLOPS}
    roof = dict(hbm if hbm["frac"] >= alu["frac"] else alu)
    per_launch = prof["pass_uncond_bytes"] / launches if launches else 0.0
    tr = traffic_from_profiles(args.workload)
    roof["traffic"] = tr
    roof["kernel"] = "k_tile_pass"
    roof["launches"] = launches
    roof["avg_launch_ms"] = prof["pass_uncond_ms"] / launches if launches else 0.0
    roof["algorithmic_bytes_per_launch"] = per_launch
    roof["other_bound"] = alu if roof["bound"] == "hbm" else hbm
    roof["time_share"] = {"tile_pass_ms": prof["pass_ms"], "site_ms": prof["site_ms"],
                          "other_ms": prof["other_ms"], "wall_ms": 1e3 * dt}

    # the same steps with trajectory sharing (shots with equal measurement histories share one state)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for s in range(args.steps):
        prog.run_shots(shots, seed=s, share=True)
    torch.cuda.synchronize()
    dt_sp = time.perf_counter() - t1
    shared = {"value": shots * args.steps / dt_sp, "unit": "shots/s", "ms_per_step": 1e3 * dt_sp / args.steps,
              "note": "same shots, bit-identical results; shots with equal measurement histories "
                      "share one state (gate passes once per distinct history)"}
    log("shared-trajectory steps done")

    # the same steps with a complex64 state (single-precision amplitudes and
    # matrix-core products; outcomes agree with complex128 except where a draw
    # lies within single-precision error of its threshold)
    prog.run_shots(shots, seed=1000, complex64=True)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for s in range(args.steps):
        prog.run_shots(shots, seed=s, complex64=True)
    torch.cuda.synchronize()
    dt_c64 = time.perf_counter() - t2
    p64 = ctx.profile()
    l64 = p64["pass_uncond_launches"]
    t64 = p64["pass_uncond_ms"] / 1e3
    g64 = p64["pass_uncond_bytes"] / t64 / 1e9 if t64 else 0.0
    tf32 = p64["pass_uncond_flops"] / t64 / 1e12 if t64 else 0.0
    c64 = {"value": shots * args.steps / dt_c64, "unit": "shots/s", "ms_per_step": 1e3 * dt_c64 / args.steps,
           "dtype": "c64",
           "roofline": {"kernel": "k_tile_pass", "launches": l64, "avg_launch_ms": 1e3 * t64 / l64 if l64 else 0.0,
                        "hbm": {"achieved": g64, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": g64 / HBM_PEAK_GBS},
                        "mfma": {"achieved": tf32, "peak": FP32_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": tf32 / FP32_MFMA_PEAK_TFLOPS}},
           "note": "same shots with a complex64 state (the precision of the paper's GPU runs)"}
    c64["roofline"]["traffic"] = traffic_from_profiles("c2_c64")
    log("complex64 steps done")

    out = {"metric": "shots/s + achieved HBM GB/s on 16q/28q dynamic circuits; p50/p99 request latency",
           "value": value, "unit": "shots/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic", "config": cfg, "roofline": roof, "shared_trajectories": shared,
           "complex64": c64}
    ctx.close()
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a sample of the workload")
        out["cpu_baseline"] = cpu_baseline(src)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
