"""Writes the 28-qubit headline-circuit fixtures from the CPU oracle.

    python tests/golden/make_c2_28q.py LAYERS [OUT]

The program is the seeded 28-qubit brickwork workload (U3 on every qubit and
alternating CX pairs per layer, a 4-qubit measurement into ``bit[4] c``, the
``if (c == 0b1010)`` block and the if/else on ``c[0]``) at LAYERS layers,
without the final measure-all, run once by the oracle with a forced record.
The fixture keeps the record's probability, the classical bits, the state's
amplitudes at seeded random indices, its norm and one global checksum
sum_i psi_i conj(w_i) with w_i = exp(2 pi i frac(i * 0.6180339887498949)),
which every amplitude enters. Only the oracle and the input generators run
here; the GPU tests read the JSON.

A 28-qubit complex128 state is 4 GiB and the oracle's tensor reshapes hold
about four of them at once, so this needs ~20 GiB of host memory and a few
seconds per gate (4 layers: minutes; 40 layers: hours).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import sim  # noqa: E402

N = 28
SEED = 2             # circuit generator seed (the benchmark's)
SHOT_SEED = 7        # Philox key of the forced shot (unused draws still advance the stream)
FORCED = [0, 1, 0, 1]  # c[0..3]: c == 0b1010 takes the block, c[0] == 0 takes the rz branch
INDEX_SEED = 20260
N_INDICES = 2048
PHI = 0.6180339887498949
CHUNK = 1 << 24


def checksum(psi):
    """sum_i psi_i * conj(w_i), summed chunk by chunk in index order."""
    acc = 0j
    for s in range(0, psi.size, CHUNK):
        i = np.arange(s, min(psi.size, s + CHUNK), dtype=np.float64)
        w = np.exp(2j * np.pi * np.mod(i * PHI, 1.0))
        acc += complex(np.sum(psi[s:s + i.size] * np.conj(w)))
    return acc


def sample_indices():
    rng = np.random.Generator(np.random.PCG64(INDEX_SEED))
    idx = rng.integers(0, 1 << N, size=N_INDICES, dtype=np.int64)
    return np.concatenate([[0, (1 << N) - 1], idx])


class _Progress(sim.TensorEngine):
    """The oracle's engine, printing a line every 50 gates."""
    count = 0
    t0 = time.time()

    def apply(self, m, qubits):
        super().apply(m, qubits)
        _Progress.count += 1
        if _Progress.count % 50 == 0:
            print(f"  {_Progress.count} gates, {time.time() - _Progress.t0:.0f} s", flush=True)


def main():
    layers = int(sys.argv[1])
    out = sys.argv[2] if len(sys.argv) > 2 else os.path.join(HERE, f"c2_28q_L{layers}_forced.json")
    src = W.c2_program(seed=SEED, n=N, layers=layers, final_measure=False)
    it = sim.run_shot(src, seed=SHOT_SEED, shot=0, forced=FORCED, engine_cls=_Progress)
    assert it.status == sim.STATUS_OK, "the forced record has (near) zero probability"
    psi = it.psi
    idx = sample_indices()
    amps = psi[idx]
    cs = checksum(psi)
    doc = {
        "generator": {"function": "workloads.c2_program", "seed": SEED, "n": N, "layers": layers,
                      "final_measure": False},
        "shot": {"seed": SHOT_SEED, "shot": 0, "forced": FORCED},
        "record": list(it.record),
        "cbits": list(it.cbits),
        "record_prob": it.record_prob,
        "outcome_probs": [e[4] if e[2] == 0 else 1.0 - e[4] for e in it.events],
        "norm": float(np.vdot(psi, psi).real),
        "checksum": {"phi": PHI, "chunk": CHUNK, "value": [cs.real, cs.imag]},
        "index_seed": INDEX_SEED,
        "indices": [int(i) for i in idx],
        "amps": [[float(a.real), float(a.imag)] for a in amps],
        "gates_applied": _Progress.count,
    }
    with open(out, "w") as f:
        json.dump(doc, f, indent=0)
    print(f"wrote {out}: {_Progress.count} gates, record_prob {it.record_prob:.17g}")


if __name__ == "__main__":
    main()
