"""Flat gate-list circuit descriptors.

A circuit is an ordered list of gates over ``n_qubits`` qubits. Each gate is
one record of ``GATE_DTYPE`` (32 bytes, the same layout as ``qs_gate`` in
``include/qs.h``):

=======  =====================================================================
op       gate kind (``OP``)
q0, q1   qubits: target of a 1-qubit gate (q1 = -1); control and target of
         CNOT; the two qubits of CZ
p_w      index of the weight parameter, or -1
feat     index of the per-sample input feature, or -1
p_b      index of the bias parameter, or -1
scale    angle multiplier
flags    reserved, 0
=======  =====================================================================

The angle of a rotation on sample ``b`` is
``scale * (w * f + bias)`` with ``w = P[p_w]`` (1 if ``p_w < 0``),
``f = X[b, feat]`` (1 if ``feat < 0``) and ``bias = P[p_b]`` (0 if
``p_b < 0``). A trainable rotation is ``(p_w=k, scale=1)``; a fixed angle is
``scale`` alone; data re-uploading ``RY(w x + b)`` sets all three indices.

This module only lays gates out; it computes nothing about them.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Gate kinds. The numbering is part of the descriptor format. RESET and
# MEASURE are mid-circuit channels on qubit q0: one trajectory, its outcome
# drawn from the uniform X[b, feat] (then reset to |0>, or kept).
OP = {"RX": 0, "RY": 1, "RZ": 2, "X": 3, "Y": 4, "Z": 5, "H": 6,
      "CNOT": 7, "CZ": 8, "RESET": 9, "MEASURE": 10}
CHANNELS = (OP["RESET"], OP["MEASURE"])
OP_NAMES = {v: k for k, v in OP.items()}
ROTATIONS = (OP["RX"], OP["RY"], OP["RZ"])

GATE_DTYPE = np.dtype([
    ("op", "<i4"), ("q0", "<i4"), ("q1", "<i4"), ("p_w", "<i4"),
    ("feat", "<i4"), ("p_b", "<i4"), ("scale", "<f4"), ("flags", "<i4"),
])
assert GATE_DTYPE.itemsize == 32


@dataclass
class Circuit:
    """A gate list plus the sizes that describe its parameter/feature use.

    ``layer_end[l]`` is the index one past the last gate of layer ``l`` (used
    to place state checkpoints every k layers).
    """

    n_qubits: int
    gates: np.ndarray  # structured, GATE_DTYPE
    n_params: int
    n_features: int = 0
    layer_end: list = field(default_factory=list)
    name: str = ""

    @property
    def n_gates(self) -> int:
        return int(self.gates.shape[0])

    def copy(self) -> "Circuit":
        return Circuit(self.n_qubits, self.gates.copy(), self.n_params,
                       self.n_features, list(self.layer_end), self.name)


class _Builder:
    def __init__(self, n: int):
        self.n = n
        self.rows: list[tuple] = []
        self.layer_end: list[int] = []
        self.n_params = 0

    def new_param(self) -> int:
        self.n_params += 1
        return self.n_params - 1

    def rot(self, kind: str, q: int, p_w: int = -1, feat: int = -1,
            p_b: int = -1, scale: float = 1.0):
        self.rows.append((OP[kind], q, -1, p_w, feat, p_b, scale, 0))

    def fixed(self, kind: str, q0: int, q1: int = -1):
        self.rows.append((OP[kind], q0, q1, -1, -1, -1, 0.0, 0))

    def channel(self, kind: str, q: int, feat: int):
        """A mid-circuit RESET or MEASURE of qubit q; its uniform is X[b, feat]."""
        self.rows.append((OP[kind], q, -1, -1, feat, -1, 0.0, 0))

    def end_layer(self):
        self.layer_end.append(len(self.rows))

    def build(self, n_features: int = 0, name: str = "") -> Circuit:
        g = np.array(self.rows, dtype=GATE_DTYPE) if self.rows else \
            np.zeros(0, dtype=GATE_DTYPE)
        return Circuit(self.n, g, self.n_params, n_features,
                       list(self.layer_end), name)


def hea_ry_rz_ring(n: int, layers: int, name: str = "") -> Circuit:
    """Hardware-efficient layers: RY(theta) then RZ(phi) on every qubit, then
    the ring CNOT(i, (i+1) mod n), i = 0..n-1 (chain for n = 2 is one CNOT)."""
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            b.rot("RY", q, p_w=b.new_param())
            b.rot("RZ", q, p_w=b.new_param())
        if n == 2:
            b.fixed("CNOT", 0, 1)
        elif n > 2:
            for i in range(n):
                b.fixed("CNOT", i, (i + 1) % n)
        b.end_layer()
    return b.build(name=name)


def rxyz_cz_ring(n: int, layers: int, name: str = "") -> Circuit:
    """RX, RY, RZ on every qubit, then the CZ ring CZ(i, (i+1) mod n)."""
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            b.rot("RX", q, p_w=b.new_param())
            b.rot("RY", q, p_w=b.new_param())
            b.rot("RZ", q, p_w=b.new_param())
        if n == 2:
            b.fixed("CZ", 0, 1)
        elif n > 2:
            for i in range(n):
                b.fixed("CZ", i, (i + 1) % n)
        b.end_layer()
    return b.build(name=name)


def reupload_ry_rz_chain(n: int, layers: int, n_features: int,
                         name: str = "") -> Circuit:
    """Data re-uploading: per layer RY(w x_{q mod F} + b) on every qubit, then a
    trainable RZ(phi) on every qubit, then the CNOT chain (i, i+1)."""
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            w = b.new_param()
            bias = b.new_param()
            b.rot("RY", q, p_w=w, feat=q % n_features, p_b=bias)
        for q in range(n):
            b.rot("RZ", q, p_w=b.new_param())
        for i in range(n - 1):
            b.fixed("CNOT", i, i + 1)
        b.end_layer()
    return b.build(n_features=n_features, name=name)


def ry_rz_chain(n: int, layers: int, name: str = "") -> Circuit:
    """Encoder layers: RY then RZ on every qubit, then the CNOT chain."""
    b = _Builder(n)
    for _ in range(layers):
        for q in range(n):
            b.rot("RY", q, p_w=b.new_param())
            b.rot("RZ", q, p_w=b.new_param())
        for i in range(n - 1):
            b.fixed("CNOT", i, i + 1)
        b.end_layer()
    return b.build(name=name)


def inverse_structure(c: Circuit) -> Circuit:
    """The gate list of the inverse circuit: gates in reverse order, rotation
    angles negated through ``scale``; X, Y, Z, H, CNOT and CZ are their own
    inverses. Parameter indices are kept, so the inverse is differentiable in
    the same parameters."""
    g = c.gates[::-1].copy()
    rot = np.isin(g["op"], ROTATIONS)
    g["scale"][rot] = -g["scale"][rot]
    ends = []
    total = c.n_gates
    for e in reversed([0] + list(c.layer_end[:-1])):
        ends.append(total - e)
    return Circuit(c.n_qubits, g, c.n_params, c.n_features, ends,
                   (c.name + "^-1") if c.name else "")


def concat(a: Circuit, b: Circuit, shift_b_params: bool = True) -> Circuit:
    """Gates of ``a`` then gates of ``b`` (b's parameter indices shifted past
    a's unless ``shift_b_params`` is False)."""
    assert a.n_qubits == b.n_qubits
    gb = b.gates.copy()
    off = a.n_params if shift_b_params else 0
    for f in ("p_w", "p_b"):
        m = gb[f] >= 0
        gb[f][m] += off
    g = np.concatenate([a.gates, gb])
    ends = list(a.layer_end) + [e + a.n_gates for e in b.layer_end]
    return Circuit(a.n_qubits, g, off + b.n_params,
                   max(a.n_features, b.n_features), ends)


def random_circuit(n: int, n_gates: int, rng: np.random.Generator,
                   n_params: int = 8, n_features: int = 0,
                   kinds=("RX", "RY", "RZ", "X", "Y", "Z", "H", "CNOT", "CZ"),
                   ) -> Circuit:
    """A seeded random gate list using every gate kind, shared parameter
    indices, fixed angles, features and biases: a stress input for parity."""
    b = _Builder(n)
    b.n_params = n_params
    kinds = [k for k in kinds if not (k in ("CNOT", "CZ") and n < 2)]
    for _ in range(n_gates):
        k = kinds[int(rng.integers(len(kinds)))]
        if k in ("CNOT", "CZ"):
            q0, q1 = (int(v) for v in rng.choice(n, size=2, replace=False))
            b.fixed(k, q0, q1)
        elif k in ("RX", "RY", "RZ"):
            q = int(rng.integers(n))
            mode = int(rng.integers(4))
            scale = float(np.float32(rng.uniform(-2.0, 2.0)))
            if mode == 0:      # fixed angle
                b.rot(k, q, scale=scale)
            elif mode == 1 or n_features == 0:  # trainable, maybe shared
                b.rot(k, q, p_w=int(rng.integers(n_params)), scale=scale)
            elif mode == 2:    # weight * feature + bias
                b.rot(k, q, p_w=int(rng.integers(n_params)),
                      feat=int(rng.integers(n_features)),
                      p_b=int(rng.integers(n_params)), scale=scale)
            else:              # plain feature encoding plus bias
                b.rot(k, q, feat=int(rng.integers(n_features)),
                      p_b=int(rng.integers(n_params)), scale=scale)
        else:
            b.fixed(k, int(rng.integers(n)))
    return b.build(n_features=n_features, name=f"random{n}q{n_gates}g")


def with_channels(c: Circuit, where, rng: np.random.Generator,
                  kinds=("RESET", "MEASURE")) -> Circuit:
    """A copy of ``c`` with a channel inserted before each gate index in
    ``where`` (ascending), each on a seeded random qubit, alternating
    ``kinds``; each channel reads its uniform from a new feature column
    appended after the circuit's own (so n_features grows by len(where))."""
    rows = [tuple(r) for r in c.gates.tolist()]
    out, k = [], 0
    for g in range(len(rows) + 1):
        while k < len(where) and where[k] == g:
            q = int(rng.integers(c.n_qubits))
            out.append((OP[kinds[k % len(kinds)]], q, -1, -1, c.n_features + k, -1, 0.0, 0))
            k += 1
        if g < len(rows):
            out.append(rows[g])
    g = np.array(out, dtype=GATE_DTYPE)
    return Circuit(c.n_qubits, g, c.n_params, c.n_features + len(where), [],
                   c.name + "+channels")
