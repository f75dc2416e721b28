"""Seeded request trace for the serving configuration (C5).

Poisson arrivals at ``rate`` requests/s over ``duration`` seconds. 80% of the
requests are dynamic circuits of the C1 pattern with n ~ U{12..26} qubits,
depth ~ U{10..40} layers, 0..4 measure/feed-forward sites and a log-uniform
shot count round(2^U[0,10]) in [1, 1024]; 20% are single-vector VQE
energy+gradient calls on the 20-qubit ansatz with their own Hamiltonian.
"""
import math

import numpy as np

from .circuits import c1_program, c4_hamiltonian


def c5_trace(seed=5, rate=200.0, duration=60.0, n_lo=12, n_hi=26, vqe_frac=0.2,
             vqe_qubits=20, vqe_layers=6, pool=None):
    """pool=None: every circuit request has its own circuit; pool=k: circuits are drawn
    from k seeded circuits (requests still differ in shots and seeds)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, reqs = 0.0, []
    circuits = None
    if pool:
        circuits = []
        for _ in range(pool):
            n = int(rng.integers(n_lo, n_hi + 1))
            depth = int(rng.integers(10, 41))
            n_sites = int(rng.integers(0, 5))
            sites = tuple(sorted(int(x) for x in rng.choice(np.arange(1, depth + 1), size=n_sites,
                                                               replace=False)))
            circuits.append((n, c1_program(seed=int(rng.integers(1 << 62)), n=n, layers=depth, sites=sites)))
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        rid = len(reqs)
        if rng.random() < vqe_frac:
            coeffs, codes = c4_hamiltonian(seed=int(rng.integers(1 << 62)), n=vqe_qubits)
            theta = rng.uniform(-math.pi, math.pi, size=2 * vqe_qubits * vqe_layers)
            reqs.append({"id": rid, "arrival": t, "kind": "vqe", "n": vqe_qubits,
                         "coeffs": coeffs, "codes": codes, "theta": theta})
        elif circuits is not None:
            n, src = circuits[int(rng.integers(len(circuits)))]
            shots = int(round(2.0 ** rng.uniform(0.0, 10.0)))
            reqs.append({"id": rid, "arrival": t, "kind": "shots", "n": n, "source": src,
                         "shots": shots, "seed": int(rng.integers(1 << 62))})
        else:
            n = int(rng.integers(n_lo, n_hi + 1))
            depth = int(rng.integers(10, 41))
            n_sites = int(rng.integers(0, 5))
            sites = tuple(sorted(int(x) for x in rng.choice(np.arange(1, depth + 1),
                                                               size=n_sites, replace=False)))
            shots = int(round(2.0 ** rng.uniform(0.0, 10.0)))
            src = c1_program(seed=int(rng.integers(1 << 62)), n=n, layers=depth, sites=sites)
            reqs.append({"id": rid, "arrival": t, "kind": "shots", "n": n, "source": src,
                         "shots": shots, "seed": int(rng.integers(1 << 62))})
    return reqs
