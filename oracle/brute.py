"""Dense brute-force engine (n <= 8): full 2^n x 2^n operators and projectors.

TEST INFRASTRUCTURE ONLY: checks ``oracle.sim.TensorEngine`` by a second,
independent route for the state arithmetic.

  * a one-qubit gate U on qubit q is the Kronecker product
    I_(2^(n-1-q)) (x) U (x) I_(2^q)   (the leftmost factor is the most
    significant index bit, so this realises little-endian qubit order);
  * a k-qubit gate M on operands (q_0, ..., q_{k-1}) is built entry by entry
    from its definition: F[i', i] = M[j(i'), j(i)] when i and i' agree on every
    bit outside the operands, j(i) = sum_m b_{q_m}(i) 2^m;
  * measuring qubit q with outcome m applies the projector
    P_m = I (x) |m><m| (x) I and renormalises: psi <- P_m psi / ||P_m psi||.
"""
import math

import numpy as np

from . import gates as G

MAX_QUBITS = 8


def kron_1q(u, q, n):
    return np.kron(np.kron(np.eye(1 << (n - 1 - q)), u), np.eye(1 << q))


def full_operator(m, qubits, n):
    k = len(qubits)
    if k == 1:
        return kron_1q(m, qubits[0], n)
    dim = 1 << n
    opmask = sum(1 << q for q in qubits)
    f = np.zeros((dim, dim), dtype=np.complex128)
    for i in range(dim):
        j = sum(((i >> q) & 1) << t for t, q in enumerate(qubits))
        rest = i & ~opmask
        for jp in range(1 << k):
            ip = rest | sum(((jp >> t) & 1) << q for t, q in enumerate(qubits))
            f[ip, i] = m[jp, j]
    return f


def projector(q, m, n):
    ket = np.zeros((2, 2), dtype=np.complex128)
    ket[m, m] = 1.0
    return kron_1q(ket, q, n)


class DenseEngine:
    def __init__(self, n):
        if n > MAX_QUBITS:
            raise ValueError("dense brute force is limited to 8 qubits")
        self.n = n
        self.psi = np.zeros(1 << n, dtype=np.complex128)
        self.psi[0] = 1.0

    def apply(self, m, qubits):
        self.psi = full_operator(m, qubits, self.n) @ self.psi

    def probs(self, q):
        p0 = float(np.linalg.norm(projector(q, 0, self.n) @ self.psi) ** 2)
        p1 = float(np.linalg.norm(projector(q, 1, self.n) @ self.psi) ** 2)
        return p0, p1

    def collapse(self, q, m, p_m):
        self.psi = (projector(q, m, self.n) @ self.psi) / math.sqrt(p_m)

    def flip(self, q):
        self.psi = kron_1q(G.X, q, self.n) @ self.psi
