"""Brute-force circuit unitaries from Kronecker products (test helper).

Independent of the oracle's strided application: every gate is expanded to
a full 2^n x 2^n matrix, with rotation gates from the matrix exponential
exp(-i theta P / 2) computed by scipy.linalg.expm, and the circuit unitary is
their ordered product. Qubit q is bit q of the index, so in a Kronecker
product the factor of qubit n-1 comes first and qubit 0 last.
"""
import numpy as np
from scipy.linalg import expm

from workloads.circuits import OP

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
HAD = np.array([[1, 1], [1, -1]], dtype=complex) / np.sqrt(2)
P0 = np.array([[1, 0], [0, 0]], dtype=complex)
P1 = np.array([[0, 0], [0, 1]], dtype=complex)
GEN = {OP["RX"]: PX, OP["RY"]: PY, OP["RZ"]: PZ}
FIXED = {OP["X"]: PX, OP["Y"]: PY, OP["Z"]: PZ, OP["H"]: HAD}


def kron_all(factors_by_qubit):
    """factors_by_qubit[q] is the 2x2 factor on qubit q."""
    out = np.array([[1.0 + 0j]])
    for q in reversed(range(len(factors_by_qubit))):
        out = np.kron(out, factors_by_qubit[q])
    return out


def embed(n, q, U):
    f = [I2] * n
    f = list(f)
    f[q] = U
    return kron_all(f)


def gate_full(n, gate, theta):
    op = int(gate["op"])
    if op in GEN:
        return embed(n, int(gate["q0"]), expm(-0.5j * theta * GEN[op]))
    if op in FIXED:
        return embed(n, int(gate["q0"]), FIXED[op])
    a, b = int(gate["q0"]), int(gate["q1"])
    f0 = [I2] * n
    f0[a] = P0
    f1 = [I2] * n
    f1[a] = P1
    f1[b] = PX if op == OP["CNOT"] else PZ
    return kron_all(f0) + kron_all(f1)


def angle(gate, params_row, feats_row):
    """theta = scale (w f + bias) for one sample, written out per field."""
    w = params_row[gate["p_w"]] if gate["p_w"] >= 0 else 1.0
    f = feats_row[gate["feat"]] if gate["feat"] >= 0 else 1.0
    b = params_row[gate["p_b"]] if gate["p_b"] >= 0 else 0.0
    return float(gate["scale"]) * (float(w) * float(f) + float(b))


def circuit_full(circuit, params_row, feats_row=None):
    n = circuit.n_qubits
    U = np.eye(1 << n, dtype=complex)
    for gate in circuit.gates:
        U = gate_full(n, gate, angle(gate, params_row, feats_row)) @ U
    return U
