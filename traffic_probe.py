"""Workload for the hardware byte-counter runs (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE).

Runs, in one process: one plain device copy of 4 GiB (qsv_diag_copy, the
calibration: it reads and writes exactly 4 GiB), then one step of the 28-qubit
benchmark workload (16 shots) with the same launch configuration as bench.py;
with --complex64 the step holds its state in complex64; with --workload c4 the
step is one energy + gradient call of the 20-qubit ansatz over 64 vectors.

    rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT -o fetch -- python3 traffic_probe.py
"""
import ctypes as C
import os
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

COPY_BYTES = 4 << 30


def main():
    import torch

    import workloads as W
    from paper_2604_11599_amd import Context
    from paper_2604_11599_amd import _abi as A
    from traffic_summary import ADJOINT_SOURCES, kernel_hash
    print(f"kernel_hash={kernel_hash()}", flush=True)
    print(f"kernel_hash_adjoint={kernel_hash(ADJOINT_SOURCES)}", flush=True)
    ctx = Context(0)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ctx.check(A.lib().qsv_diag_copy(ctx.handle, C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()),
                                    COPY_BYTES))
    del src, dst
    torch.cuda.empty_cache()
    print("copy done", flush=True)
    if "c4" in sys.argv[1:]:
        prog = ctx.load(W.c4_ansatz(20, 6))
        coeffs, codes = W.c4_hamiltonian(seed=4, n=20, terms=60)
        prog.expval_grad(W.c4_thetas(seed=44, batch=64, n_params=240), coeffs, codes)
    else:
        prog = ctx.load(W.c2_program(seed=2, n=28, layers=40))
        prog.run_shots(16, seed=0, complex64="--complex64" in sys.argv[1:])
    print("step done", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
