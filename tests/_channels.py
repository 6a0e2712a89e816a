"""Inputs for circuits with mid-circuit channels (test helper)."""
import numpy as np

import oracle as O
from workloads import circuits as C


def stable_uniforms(c, params, feats, psi0):
    """Sets each channel's uniform to the middle of the interval of the
    outcome it draws (channels in order), so the drawn outcomes do not depend
    on rounding: the GPU and the oracle then take the same branch, and small
    parameter changes keep every outcome."""
    feats = np.array(feats, dtype=np.float64, copy=True)
    B = psi0.shape[0]
    for g, gate in enumerate(c.gates):
        if int(gate["op"]) not in C.CHANNELS:
            continue
        pre = O.run_circuit(C.Circuit(c.n_qubits, c.gates[:g], c.n_params, c.n_features),
                            params, feats, psi0)
        p = O.channel_probabilities(pre, int(gate["q0"]))
        m = O.trajectory_outcome(p, np.full(B, 0.5))
        lo = np.where(m == 1, p[:, 0], 0.0)
        feats[:, int(gate["feat"])] = (lo + 0.5 * p[np.arange(B), m]) / p.sum(axis=1)
    return feats


def channel_gates(c):
    return [g for g, gate in enumerate(c.gates) if int(gate["op"]) in C.CHANNELS]
