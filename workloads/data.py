"""Seeded synthetic inputs for the six benchmark workloads.

Every draw comes from ``numpy.random.default_rng([seed, stream])`` with a
fixed stream id per quantity (inputs, parameters, labels/upstream weights),
so a reduced batch draws the same parameters as the full one, and the first
``B`` rows of the inputs are a prefix of the full batch's inputs. Values are
drawn in FP64 and rounded to the storage type the GPU reads (float32 for the
complex64 workloads), so the oracle and the GPU see identical bits.

Nothing here simulates a circuit.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .circuits import (Circuit, hea_ry_rz_ring, rxyz_cz_ring,
                       reupload_ry_rz_chain, ry_rz_chain)

STREAM_X, STREAM_P, STREAM_Y, STREAM_P2, STREAM_SPEC, STREAM_U = 1, 2, 3, 4, 5, 6


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([seed, stream])


def amplitude_inputs(B: int, D: int, seed: int = 0, dtype=np.float32,
                     stream: int = STREAM_X) -> np.ndarray:
    """x ~ N(0,1)^D per row; normalisation is the encoder's job."""
    rng = _rng(seed, stream)
    # Row-by-row generation keeps a smaller B a prefix of a larger B.
    x = rng.standard_normal((B, D))
    return x.astype(dtype)


def uniform_features(B: int, F: int, seed: int = 0, dtype=np.float32,
                     lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    return _rng(seed, STREAM_X).uniform(lo, hi, size=(B, F)).astype(dtype)


def uniform_params(P: int, seed: int = 0, dtype=np.float32,
                   stream: int = STREAM_P, rows: int | None = None):
    """Parameters ~ U(-pi, pi): shape [P], or [rows, P] for per-sample sets."""
    shape = (P,) if rows is None else (rows, P)
    return _rng(seed, stream).uniform(-np.pi, np.pi, size=shape).astype(dtype)


def pm1_labels(B: int, seed: int = 0) -> np.ndarray:
    """Labels +-1 with probability 1/2 each (float64)."""
    return np.where(_rng(seed, STREAM_Y).random(B) < 0.5, -1.0, 1.0)


def upstream_weights(n: int, seed: int = 0) -> np.ndarray:
    """Fixed readout weights g_q ~ U(-1, 1) for the loss sum_q g_q <Z_q>."""
    return _rng(seed, STREAM_Y).uniform(-1.0, 1.0, size=n)


@dataclass
class Workload:
    """One benchmark configuration with its seeded inputs.

    ``encoding`` is "amplitude" (``x`` rows are the un-normalised amplitudes)
    or "zero" (start from |0...0>; ``feats`` may carry angle-encoded data).
    ``loss`` names how the upstream gradient is formed: "none" (forward only),
    "mse_z0" (mean (<Z_0> - y)^2), "fidelity_reset" (1 - mean fidelity after
    resetting the trash qubits), "fidelity_postselect" (1 - mean fidelity when
    the trash qubits are measured and only the all-zero outcome is kept,
    renormalised), "fidelity_trajectory" (1 - mean fidelity of one trajectory
    of the reset channel per sample, its measurement outcome drawn from the
    uniforms ``trajectory_uniforms``), "weighted_z" (sum_b sum_q g_q <Z_q>_b).
    """

    name: str
    n_qubits: int
    batch: int
    circuit: Circuit
    dtype: str                    # "c64" or "c128"
    encoding: str
    loss: str
    x: np.ndarray | None = None   # amplitude inputs [B, D]
    feats: np.ndarray | None = None
    params: np.ndarray | None = None
    labels: np.ndarray | None = None
    weights: np.ndarray | None = None
    decoder: Circuit | None = None
    params_dec: np.ndarray | None = None
    n_trash: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def real_dtype(self):
        return np.float32 if self.dtype == "c64" else np.float64

    def updates_per_step(self) -> int:
        """Gate-amplitude updates of one forward + adjoint pass:
        3 * B * 2^n * G (forward sweep, then uncompute and propagate)."""
        G = self.circuit.n_gates + (self.decoder.n_gates if self.decoder else 0)
        passes = 1 if self.loss == "none" else 3
        return passes * self.batch * (1 << self.n_qubits) * G


def _c1(B, seed):
    c = hea_ry_rz_ring(4, 2, name="ryrz-ring n4 L2")
    return Workload("c1_n4_b64_c128_fwd", 4, B, c, "c128", "amplitude", "none",
                    x=amplitude_inputs(B, 16, seed, np.float64),
                    params=uniform_params(c.n_params, seed, np.float64))


def _c2(B, seed):
    c = rxyz_cz_ring(10, 8, name="rxyz-czring n10 L8")
    return Workload("c2_n10_b4096_c64_mse", 10, B, c, "c64", "amplitude",
                    "mse_z0", x=amplitude_inputs(B, 1024, seed),
                    params=uniform_params(c.n_params, seed),
                    labels=pm1_labels(B, seed))


def _c3(B, seed):
    c = reupload_ry_rz_chain(8, 16, 4, name="reupload n8 L16 F4")
    return Workload("c3_n8_b65536_reupload", 8, B, c, "c64", "zero", "mse_z0",
                    feats=uniform_features(B, 4, seed),
                    params=uniform_params(c.n_params, seed),
                    labels=pm1_labels(B, seed))


def _c4(B, seed):
    enc = ry_rz_chain(12, 6, name="ryrz-chain n12 L6")
    return Workload("c4_n12_b1024_autoenc", 12, B, enc, "c64", "amplitude",
                    "fidelity_reset", x=amplitude_inputs(B, 4096, seed),
                    params=uniform_params(enc.n_params, seed),
                    decoder=enc.copy(),
                    params_dec=uniform_params(enc.n_params, seed, stream=STREAM_P2),
                    n_trash=4)


def _c5b(B, seed):
    c = hea_ry_rz_ring(26, 20, name="ryrz-ring n26 L20")
    return Workload("c5b_n26_ryrz_ring_L20", 26, B, c, "c64", "zero",
                    "weighted_z", params=uniform_params(c.n_params, seed),
                    weights=upstream_weights(26, seed),
                    extra={"ckpt_every_layers": 4, "fuse_qubits": 5})


WORKLOADS = {
    "c1": (_c1, 64), "c2": (_c2, 4096), "c3": (_c3, 65536),
    "c4": (_c4, 1024), "c5b": (_c5b, 1),
}


def make_workload(key: str, batch: int | None = None, seed: int = 0) -> Workload:
    fn, full = WORKLOADS[key]
    return fn(full if batch is None else batch, seed)


@dataclass
class UnevenBatch:
    """Circuits of uneven qubit count and depth, grouped into classes of
    identical structure and packed class after class (the layout of the
    packed buffers of the library's uneven-batch calls).

    classes[k] = (n, depth, circuit, idx) where idx are the original circuit
    numbers of the class's circuits, in packed order. x, params and weights
    are packed: x [sum 2^n] float32 (amplitude inputs, N(0,1)), params
    [sum P] float32 (U(-pi, pi)), weights [sum n] float64 (g_q ~ U(-1, 1),
    the loss sum_q g_q <Z_q> per circuit)."""
    classes: list
    x: np.ndarray
    params: np.ndarray
    weights: np.ndarray
    state_off: np.ndarray
    param_off: np.ndarray
    expz_off: np.ndarray
    n_circuits: int

    def circuit_slices(self, k: int, j: int):
        """Packed slices (x/state, params, expz) of circuit j of class k."""
        n, _, c, _ = self.classes[k]
        so = self.state_off[k] + (j << n)
        po = self.param_off[k] + j * c.n_params
        eo = self.expz_off[k] + j * n
        return slice(so, so + (1 << n)), slice(po, po + c.n_params), slice(eo, eo + n)

    def updates_per_step(self) -> int:
        tot = 0
        for n, d, c, idx in self.classes:
            tot += 3 * len(idx) * (1 << n) * c.n_gates
        return tot


def uneven_batch(n_circuits: int = 10000, seed: int = 0, n_lo: int = 6,
                 n_hi: int = 14, d_lo: int = 4, d_hi: int = 32) -> UnevenBatch:
    """The uneven batch: n ~ U{n_lo..n_hi}, depth ~ U{d_lo..d_hi}
    hardware-efficient layers (RY, RZ per qubit + ring CNOT), one amplitude
    input, one parameter set and one readout-weight vector per circuit."""
    n, d = uneven_batch_spec(n_circuits, seed, n_lo, n_hi, d_lo, d_hi)
    keys = sorted(set(zip(n.tolist(), d.tolist())))
    rng_x = _rng(seed, STREAM_X)
    rng_p = _rng(seed, STREAM_P)
    rng_w = _rng(seed, STREAM_Y)
    # per-circuit draws in original circuit order, then packed by class
    xs = [rng_x.standard_normal(1 << int(n[i])).astype(np.float32) for i in range(n_circuits)]
    ps = [rng_p.uniform(-np.pi, np.pi, 2 * int(n[i]) * int(d[i])).astype(np.float32)
          for i in range(n_circuits)]
    ws = [rng_w.uniform(-1.0, 1.0, int(n[i])) for i in range(n_circuits)]
    classes, X, P, W, so, po, eo = [], [], [], [], [], [], []
    s_off = p_off = e_off = 0
    for (nk, dk) in keys:
        idx = np.nonzero((n == nk) & (d == dk))[0]
        c = hea_ry_rz_ring(nk, dk, name=f"ryrz-ring n{nk} L{dk}")
        classes.append((nk, dk, c, idx))
        so.append(s_off); po.append(p_off); eo.append(e_off)
        for i in idx:
            X.append(xs[i]); P.append(ps[i]); W.append(ws[i])
        s_off += len(idx) << nk
        p_off += len(idx) * c.n_params
        e_off += len(idx) * nk
    return UnevenBatch(classes, np.concatenate(X), np.concatenate(P),
                       np.concatenate(W), np.array(so, dtype=np.int64),
                       np.array(po, dtype=np.int64), np.array(eo, dtype=np.int64),
                       n_circuits)


def uneven_batch_spec(n_circuits: int = 10000, seed: int = 0,
                      n_lo: int = 6, n_hi: int = 14, d_lo: int = 4,
                      d_hi: int = 32):
    """The uneven batch: qubit count n ~ U{n_lo..n_hi} and depth ~ U{d_lo..d_hi}
    hardware-efficient layers per circuit. Returns (n[i], depth[i])."""
    rng = _rng(seed, STREAM_SPEC)
    n = rng.integers(n_lo, n_hi + 1, size=n_circuits)
    d = rng.integers(d_lo, d_hi + 1, size=n_circuits)
    return n.astype(np.int64), d.astype(np.int64)


def trajectory_uniforms(B: int, seed: int = 0) -> np.ndarray:
    """Uniforms in [0, 1), one per sample, that draw the measurement outcome
    of a reset-channel trajectory (the random numbers are inputs, so both
    sides of a comparison see the same draw)."""
    return _rng(seed, STREAM_U).random(B)
