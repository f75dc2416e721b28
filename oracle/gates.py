"""Gate matrices written from their textbook / OpenQASM 3 definitions (complex128).

TEST INFRASTRUCTURE ONLY: part of the CPU oracle.

The paper maps each standard OpenQASM 3 gate one-to-one onto a backend gate
(Methodology, kernel generation via the AST visitor); the matrices below are
the definitions those names stand for.

Conventions (readings where the paper is silent):
  * little-endian amplitudes: index i = sum_q b_q 2^q (qubit 0 is the LSB);
  * a two-qubit matrix acts on the local index j = b_{first operand} + 2 b_{second operand};
  * controlled gates take the control as the first operand;
  * u3 / U carry no extra global phase; rz(t) = exp(-i t Z / 2), not p(t);
  * named Clifford gates (x, y, z, h, s, ...) use their exact matrices.
"""
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
SDG = S.conj().T
T = np.array([[1, 0], [0, np.exp(1j * math.pi / 4)]], dtype=np.complex128)
TDG = T.conj().T
SX = 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128)
SXDG = SX.conj().T

PAULI = {"I": I2, "X": X, "Y": Y, "Z": Z}


def u_gate(theta, phi, lam):
    """OpenQASM 3 built-in U(theta, phi, lambda)."""
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    return np.array(
        [[c, -np.exp(1j * lam) * s],
         [np.exp(1j * phi) * s, np.exp(1j * (phi + lam)) * c]],
        dtype=np.complex128)


def rx(t):
    c, s = math.cos(t / 2.0), math.sin(t / 2.0)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(t):
    c, s = math.cos(t / 2.0), math.sin(t / 2.0)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(t):
    return np.array([[np.exp(-0.5j * t), 0], [0, np.exp(0.5j * t)]], dtype=np.complex128)


def phase(lam):
    return np.array([[1, 0], [0, np.exp(1j * lam)]], dtype=np.complex128)


def controlled(u):
    """4x4 matrix of a 1-qubit gate u on the second operand, controlled by the first."""
    m = np.eye(4, dtype=np.complex128)
    # local index j = b_ctrl + 2 b_tgt; the control-set subspace is j in {1, 3}
    m[1, 1], m[1, 3] = u[0, 0], u[0, 1]
    m[3, 1], m[3, 3] = u[1, 0], u[1, 1]
    return m


SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)

# name -> (number of angle parameters, number of qubits, matrix builder)
ONE_QUBIT = {
    "id": (0, lambda: I2), "x": (0, lambda: X), "y": (0, lambda: Y), "z": (0, lambda: Z),
    "h": (0, lambda: H), "s": (0, lambda: S), "sdg": (0, lambda: SDG), "t": (0, lambda: T),
    "tdg": (0, lambda: TDG), "sx": (0, lambda: SX), "sxdg": (0, lambda: SXDG),
    "rx": (1, rx), "ry": (1, ry), "rz": (1, rz), "p": (1, phase), "phase": (1, phase),
    "u1": (1, phase), "u2": (2, lambda a, b: u_gate(math.pi / 2.0, a, b)),
    "u3": (3, u_gate), "u": (3, u_gate), "U": (3, u_gate),
}
TWO_QUBIT = {
    "cx": (0, lambda: controlled(X)), "CX": (0, lambda: controlled(X)),
    "cy": (0, lambda: controlled(Y)), "cz": (0, lambda: controlled(Z)),
    "ch": (0, lambda: controlled(H)), "swap": (0, lambda: SWAP),
    "cp": (1, lambda a: controlled(phase(a))), "cphase": (1, lambda a: controlled(phase(a))),
    "crx": (1, lambda a: controlled(rx(a))), "cry": (1, lambda a: controlled(ry(a))),
    "crz": (1, lambda a: controlled(rz(a))),
}


def gate_matrix(name, angles):
    """Return (matrix, n_qubits) of a standard gate with numeric angles."""
    if name in ONE_QUBIT:
        npar, fn = ONE_QUBIT[name]
        if len(angles) != npar:
            raise ValueError(f"gate {name} takes {npar} parameters, got {len(angles)}")
        return fn(*angles), 1
    if name in TWO_QUBIT:
        npar, fn = TWO_QUBIT[name]
        if len(angles) != npar:
            raise ValueError(f"gate {name} takes {npar} parameters, got {len(angles)}")
        return fn(*angles), 2
    raise KeyError(name)


def is_standard(name):
    return name in ONE_QUBIT or name in TWO_QUBIT


# ---- derivatives d(matrix)/d(angle_k), by differentiating the definitions above ----

def _d_u(theta, phi, lam, k):
    c, s = math.cos(theta / 2.0), math.sin(theta / 2.0)
    el, ep, epl = np.exp(1j * lam), np.exp(1j * phi), np.exp(1j * (phi + lam))
    if k == 0:
        return np.array([[-s / 2, -el * c / 2], [ep * c / 2, -epl * s / 2]], dtype=np.complex128)
    if k == 1:
        return np.array([[0, 0], [1j * ep * s, 1j * epl * c]], dtype=np.complex128)
    return np.array([[0, -1j * el * s], [0, 1j * epl * c]], dtype=np.complex128)


def gate_derivative(name, angles, k):
    """d/d(angles[k]) of the gate matrix (for the oracle's plain adjoint sweep)."""
    a = angles
    if name == "rx":
        c, s = math.cos(a[0] / 2.0), math.sin(a[0] / 2.0)
        return np.array([[-s / 2, -0.5j * c], [-0.5j * c, -s / 2]], dtype=np.complex128)
    if name == "ry":
        c, s = math.cos(a[0] / 2.0), math.sin(a[0] / 2.0)
        return np.array([[-s / 2, -c / 2], [c / 2, -s / 2]], dtype=np.complex128)
    if name == "rz":
        return np.array([[-0.5j * np.exp(-0.5j * a[0]), 0], [0, 0.5j * np.exp(0.5j * a[0])]],
                        dtype=np.complex128)
    if name in ("p", "phase", "u1"):
        return np.array([[0, 0], [0, 1j * np.exp(1j * a[0])]], dtype=np.complex128)
    if name in ("u3", "u", "U"):
        return _d_u(a[0], a[1], a[2], k)
    if name == "u2":
        return _d_u(math.pi / 2.0, a[0], a[1], k + 1)
    if name in ("cp", "cphase", "crx", "cry", "crz"):
        inner = {"cp": "p", "cphase": "p", "crx": "rx", "cry": "ry", "crz": "rz"}[name]
        d = gate_derivative(inner, a, k)
        m = np.zeros((4, 4), dtype=np.complex128)
        m[1, 1], m[1, 3], m[3, 1], m[3, 3] = d[0, 0], d[0, 1], d[1, 0], d[1, 1]
        return m
    raise KeyError(f"no derivative for gate {name}")
