"""Seeded synthetic workloads shaped like the paper's dynamic-circuit suites.

This package only *produces inputs*: OpenQASM 3 program text, parameter
vectors, Pauli-sum Hamiltonians and request traces. It contains no simulation
arithmetic, so both the CPU oracle and the GPU library can be fed from it.

Every generator takes a seed and draws from ``numpy.random.Generator(PCG64(seed))``.
Angles are printed with ``repr(float)`` (17 significant digits), which parses
back to the identical double.
"""
from .circuits import (  # noqa: F401
    c1_program, c2_program, c3_program, c3_mix, c4_ansatz, c4_hamiltonian, c4_thetas,
    brickwork_program, separable_brickwork, mirror_program, random_dynamic_program,
    random_clifford_program, qft_program, bv_program, teleport_program,
    conditional_reset_program, if_else_program, multibit_predicate_program, rus_program,
    hea2_program, param_program, modifier_program, logic_program,
)
from .trace import c5_trace  # noqa: F401
