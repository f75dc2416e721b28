"""Turns the two hardware byte-counter runs of traffic_probe.py into HBM bytes per
tile-pass launch.

FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the passes without guarded
gates (the launches bench.py's achieved figure covers) are each scaled by the factor that
maps the same counter on a plain device copy of known size (4 GiB read, 4 GiB
written) to its true byte count. Writes profiles/tile_pass_c2_traffic.json (read
by bench.py while the kernel source hash matches) and a short text summary.

    python traffic_summary.py [--complex64] FETCH_CSV WRITE_CSV PROBE_LOG [COMMAND]

--complex64: the probe ran with a complex64 state; the results go to
profiles/tile_pass_c2_c64_traffic.json and tile_pass_c2_28q_c64_traffic.txt.

PROBE_LOG is the output of the probe run; its kernel_hash line names the kernel
source the counters were taken on.
"""
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 4 << 30
PASS_KERNEL = "k_tile_pass"
COPY_KERNEL = "k_copy"


# device sources of the tile pass and of the energy + gradient kernels
PASS_SOURCES = ("kernels.hip", "device_common.h", "qsv_types.h")
ADJOINT_SOURCES = ("adjoint.hip", "device_common.h", "qsv_types.h")


def kernel_hash(sources=PASS_SOURCES):
    """Hash of the device sources the counted kernels are built from."""
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_2604_11599_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _short(name):
    return name.split("(")[0].split("<")[0].strip().split("::")[-1]


def read_counter(path, counter):
    """[(dispatch id, kernel name, KiB)] in dispatch order."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            key = {k.lower(): k for k in r}
            if r[key["counter_name"]] != counter:
                continue
            rows.append((int(r[key["dispatch_id"]]), _short(r[key["kernel_name"]]), float(r[key["counter_value"]])))
    rows.sort()
    return rows


def probe_hash(log, tag="kernel_hash"):
    with open(log) as f:
        for line in f:
            if line.startswith(tag + "="):
                return line.strip().split("=", 1)[1]
    raise SystemExit(f"no {tag} line in the probe log")


def uncond_mask():
    """Per tile pass of the probed workload, in launch order: True when no gate
    of the pass is guarded (the launches the bench's achieved figure covers)."""
    import workloads as W
    from paper_2604_11599_amd import lower
    from paper_2604_11599_amd.api import plan_inspect
    lp = lower(W.c2_program(seed=2, n=28, layers=40))
    st = plan_inspect(lp, 0)
    order = list(st.gate_instr[:st.n_gates])
    mask, k = [], 0
    for i in range(st.n_steps):
        if st.step_kind[i] != 1:
            continue
        gates = order[k:k + st.step_count[i]]
        k += st.step_count[i]
        mask.append(all(int(lp.instr[g]["guard"]) == 0 for g in gates))
    return mask


def summarize(fetch_csv, write_csv, khash):
    fe = read_counter(fetch_csv, "FETCH_SIZE")
    wr = read_counter(write_csv, "WRITE_SIZE")
    cf = [v for _, k, v in fe if k == COPY_KERNEL]
    cw = [v for _, k, v in wr if k == COPY_KERNEL]
    if len(cf) != 1 or len(cw) != 1:
        raise SystemExit("expected exactly one calibration copy per run")
    f_fac = COPY_BYTES / (cf[0] * 1024.0)
    w_fac = COPY_BYTES / (cw[0] * 1024.0)
    pf = [v for _, k, v in fe if k.startswith(PASS_KERNEL)]
    pw = [v for _, k, v in wr if k.startswith(PASS_KERNEL)]
    if not pf or len(pf) != len(pw):
        raise SystemExit("tile-pass dispatch counts differ between the two runs")
    mask = uncond_mask()
    if len(mask) != len(pf):
        raise SystemExit("tile-pass launches do not match the plan of the workload")
    pf = [v for v, m in zip(pf, mask) if m]
    pw = [v for v, m in zip(pw, mask) if m]
    per = [a * 1024.0 * f_fac + b * 1024.0 * w_fac for a, b in zip(pf, pw)]
    return {
        "kernel_hash": khash,
        "workload": "28 qubits, 40 brickwork layers, 16 shots in one launch per pass",
        "launches": len(per),
        "bytes_per_launch": sum(per) / len(per),
        "fetch_bytes_per_launch": sum(pf) * 1024.0 * f_fac / len(pf),
        "write_bytes_per_launch": sum(pw) * 1024.0 * w_fac / len(pw),
        "calibration": {"copy_bytes_each_way": COPY_BYTES, "copy_fetch_kib": cf[0], "copy_write_kib": cw[0],
                        "fetch_factor": f_fac, "write_factor": w_fac},
        "per_launch_min": min(per), "per_launch_max": max(per),
    }


# the energy + gradient workload: 20 qubits, 64 parameter vectors per call
C4_AMPS = 64 * 2 ** 20
C4_KERNELS = {"k_hamiltonian": 32.0, "k_backward_mfma": 64.0}  # algorithmic B per amplitude per launch


def summarize_kernels(fetch_csv, write_csv, khash, kernels, amps):
    """Scaled HBM bytes per launch of each named kernel (all its launches)."""
    fe = read_counter(fetch_csv, "FETCH_SIZE")
    wr = read_counter(write_csv, "WRITE_SIZE")
    cf = [v for _, k, v in fe if k == COPY_KERNEL]
    cw = [v for _, k, v in wr if k == COPY_KERNEL]
    if len(cf) != 1 or len(cw) != 1:
        raise SystemExit("expected exactly one calibration copy per run")
    f_fac = COPY_BYTES / (cf[0] * 1024.0)
    w_fac = COPY_BYTES / (cw[0] * 1024.0)
    out = {"kernel_hash": khash, "amplitudes_per_launch": amps, "kernels": {},
           "calibration": {"copy_bytes_each_way": COPY_BYTES, "copy_fetch_kib": cf[0], "copy_write_kib": cw[0],
                           "fetch_factor": f_fac, "write_factor": w_fac}}
    for name, alg in kernels.items():
        pf = [v for _, k, v in fe if k == name]
        pw = [v for _, k, v in wr if k == name]
        if not pf or len(pf) != len(pw):
            raise SystemExit(f"{name}: dispatch counts differ between the two runs")
        fetch = sum(pf) * 1024.0 * f_fac / len(pf)
        write = sum(pw) * 1024.0 * w_fac / len(pw)
        out["kernels"][name] = {"launches": len(pf), "bytes_per_launch": fetch + write, "fetch_bytes_per_launch": fetch,
                                "write_bytes_per_launch": write, "bytes_per_amplitude": (fetch + write) / amps,
                                "algorithmic_bytes_per_amplitude": alg}
    return out


def main_c4(args):
    fetch_csv, write_csv, log = args[0], args[1], args[2]
    cmd = args[3] if len(args) > 3 else ""
    d = summarize_kernels(fetch_csv, write_csv, probe_hash(log, "kernel_hash_adjoint"), C4_KERNELS, C4_AMPS)
    d["command"] = cmd
    d["workload"] = "20-qubit ansatz, 64 parameter vectors, one energy + gradient call"
    with open(os.path.join(ROOT, "profiles", "c4_20q_traffic.json"), "w") as f:
        json.dump(d, f, indent=1)
    with open(os.path.join(ROOT, "profiles", "c4_20q_traffic.txt"), "w") as f:
        f.write("HBM traffic of the energy + gradient kernels, 20 qubits x 64 vectors per launch (rocprofv3 --pmc)\n")
        f.write(f"command: {cmd}\n")
        f.write(f"kernel source hash: {d['kernel_hash']}\n")
        c = d["calibration"]
        f.write(f"calibration copy (4 GiB each way): FETCH_SIZE {c['copy_fetch_kib']:.0f} KiB "
                f"(factor {c['fetch_factor']:.4f}), WRITE_SIZE {c['copy_write_kib']:.0f} KiB "
                f"(factor {c['write_factor']:.4f})\n")
        for name, k in d["kernels"].items():
            f.write(f"{name}: {k['launches']} launches, fetch {k['fetch_bytes_per_launch']:.4e} B, write "
                    f"{k['write_bytes_per_launch']:.4e} B per launch = {k['bytes_per_amplitude']:.2f} B per amplitude "
                    f"(algorithmic {k['algorithmic_bytes_per_amplitude']:.0f})\n")
    print(json.dumps(d))


def main():
    if "--workload" in sys.argv:
        i = sys.argv.index("--workload")
        wl = sys.argv[i + 1]
        rest = sys.argv[1:i] + sys.argv[i + 2:]
        if wl == "c4":
            return main_c4(rest)
        if wl != "c2":
            raise SystemExit(f"unknown workload {wl}")
        sys.argv = [sys.argv[0]] + rest
    args = [a for a in sys.argv[1:] if a != "--complex64"]
    c64 = len(args) != len(sys.argv) - 1
    fetch_csv, write_csv, log = args[0], args[1], args[2]
    cmd = args[3] if len(args) > 3 else ""
    d = summarize(fetch_csv, write_csv, probe_hash(log))
    d["command"] = cmd
    d["amplitude"] = "complex64" if c64 else "complex128"
    sfx = "_c64" if c64 else ""
    out = os.path.join(ROOT, "profiles", f"tile_pass_c2{sfx}_traffic.json")
    with open(out, "w") as f:
        json.dump(d, f, indent=1)
    amps = 16 * 2 ** 28
    with open(os.path.join(ROOT, "profiles", f"tile_pass_c2_28q{sfx}_traffic.txt"), "w") as f:
        f.write(f"HBM traffic of the tile pass, 28 qubits x 16 shots per launch, {d['amplitude']} state "
                "(rocprofv3 --pmc)\n")
        f.write(f"command: {cmd}\n")
        f.write(f"kernel source hash: {d['kernel_hash']}\n")
        c = d["calibration"]
        f.write(f"calibration copy (4 GiB each way): FETCH_SIZE {c['copy_fetch_kib']:.0f} KiB "
                f"(factor {c['fetch_factor']:.4f}), WRITE_SIZE {c['copy_write_kib']:.0f} KiB "
                f"(factor {c['write_factor']:.4f})\n")
        f.write(f"tile-pass launches of passes without guarded gates: {d['launches']}\n")
        f.write(f"scaled bytes per launch: fetch {d['fetch_bytes_per_launch']:.4e}, write "
                f"{d['write_bytes_per_launch']:.4e}, total {d['bytes_per_launch']:.4e} "
                f"(min {d['per_launch_min']:.4e}, max {d['per_launch_max']:.4e})\n")
        f.write(f"per amplitude: {d['bytes_per_launch'] / amps:.2f} B (read + write of {d['amplitude']} is "
                f"{16 if c64 else 32} B)\n")
    print(json.dumps(d))


if __name__ == "__main__":
    main()
