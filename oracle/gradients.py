"""Gradients of circuit outputs, three independent ways (test infrastructure).

Convention for a state cotangent ``lam``: a scalar loss L of the final state
psi changes as dL = 2 Re <lam | d psi>. For a loss of the expectations,
lam = O psi with O = sum_q (dL/d<Z_q>) Z_q.
"""

from __future__ import annotations

import numpy as np

from workloads.circuits import OP

from .statevector import (apply_gate, gate_angles, pauli_of, run_circuit,
                          apply_1q, expz, apply_channel, channel_cotangent)

_ROT = (OP["RX"], OP["RY"], OP["RZ"])
_CHANNELS = (OP["RESET"], OP["MEASURE"])


def observable_cotangent(psi: np.ndarray, dexpz: np.ndarray) -> np.ndarray:
    """lam = sum_q dexpz[b, q] Z_q psi (Z_q diagonal: +1 on bit q = 0)."""
    B, N = psi.shape
    n = N.bit_length() - 1
    idx = np.arange(N)
    diag = np.zeros((B, N))
    for q in range(n):
        zq = 1.0 - 2.0 * ((idx >> q) & 1)
        diag += dexpz[:, q:q + 1] * zq[None, :]
    return diag * psi


def adjoint_vjp(circuit, params, feats, psi0, lam_final=None, dexpz=None):
    """Adjoint method (Jones & Gacon, arXiv:2009.02823, §3).

    Runs the circuit forward, forms lam at the output, then walks the gates
    backwards: at gate g, with psi and lam both taken just after g,
    dL/dtheta_g = Im <lam | P_g | psi> for R_P(theta) = exp(-i theta P / 2);
    then psi <- U_g^dagger psi and lam <- U_g^dagger lam. At a mid-circuit
    channel (one trajectory, outcome held fixed) psi is restored to the state
    the forward saw in front of it and lam goes through ``channel_cotangent``.
    Returns (dL/dtheta [B, G], final state psi_G).
    """
    B = psi0.shape[0]
    channels = [g for g, gate in enumerate(circuit.gates) if int(gate["op"]) in _CHANNELS]
    if channels:
        # A channel cannot be un-applied: keep the state in front of each one.
        pre, psi = {}, psi0.copy()
        for g, gate in enumerate(circuit.gates):
            op = int(gate["op"])
            if op in _CHANNELS:
                pre[g] = psi.copy()
                u = np.asarray(feats, dtype=np.float64)[:, int(gate["feat"])]
                psi = apply_channel(psi, gate, u)[0]
            else:
                th = gate_angles(gate, params, feats, B) if op in _ROT else None
                psi = apply_gate(psi, gate, th)
        psi_G = psi
    else:
        psi_G = run_circuit(circuit, params, feats, psi0)
    lam = observable_cotangent(psi_G, dexpz) if dexpz is not None \
        else np.asarray(lam_final, dtype=np.complex128).copy()
    psi = psi_G.copy()
    gtheta = np.zeros((B, circuit.n_gates))
    for g in range(circuit.n_gates - 1, -1, -1):
        gate = circuit.gates[g]
        if int(gate["op"]) in _CHANNELS:  # outcome held fixed: no gradient here
            u = np.asarray(feats, dtype=np.float64)[:, int(gate["feat"])]
            lam, _ = channel_cotangent(pre[g], gate, u, lam)
            psi = pre[g].copy()
            continue
        theta = None
        if int(gate["op"]) in _ROT:
            theta = gate_angles(gate, params, feats, B)
            Ppsi = apply_1q(psi, int(gate["q0"]), pauli_of(int(gate["op"])))
            gtheta[:, g] = np.imag(np.sum(np.conj(lam) * Ppsi, axis=1))
        psi = apply_gate(psi, gate, theta, inverse=True)
        lam = apply_gate(lam, gate, theta, inverse=True)
    return gtheta, psi_G


def theta_to_param_grads(circuit, params, feats, gtheta):
    """Chain rule through theta = scale (w f + bias):
    dL/dP[p_w] += g scale f,  dL/dP[p_b] += g scale,  dL/dX[b, feat] += g scale w.
    Shared parameters ([P]) sum over the batch; per-sample ones ([B, P]) do not.
    Returns (dparams like params, dfeats [B, F] or None)."""
    p = np.asarray(params, dtype=np.float64)
    B = gtheta.shape[0]
    dp = np.zeros((B, p.shape[-1]))
    df = None if feats is None else np.zeros(np.shape(feats))
    X = None if feats is None else np.asarray(feats, dtype=np.float64)
    for g, gate in enumerate(circuit.gates):
        if int(gate["op"]) not in _ROT:
            continue
        s = float(gate["scale"])
        gt = gtheta[:, g]
        f = X[:, int(gate["feat"])] if gate["feat"] >= 0 else 1.0
        if gate["p_w"] >= 0:
            dp[:, int(gate["p_w"])] += gt * s * f
        if gate["p_b"] >= 0:
            dp[:, int(gate["p_b"])] += gt * s
        if gate["feat"] >= 0:
            w = p[..., int(gate["p_w"])] if gate["p_w"] >= 0 else 1.0
            df[:, int(gate["feat"])] += gt * s * w
    dparams = dp.sum(axis=0) if p.ndim == 1 else dp
    return dparams, df


def param_shift_theta_jacobian(circuit, params, feats, psi0, readout):
    """Parameter-shift rule (Mitarai et al. 2018; Schuld et al. 2019, eq. 12):
    for R_P(theta) = exp(-i theta P / 2) and any observable,
    d<O>/dtheta = (<O>(theta + pi/2) - <O>(theta - pi/2)) / 2, exactly.
    Each gate occurrence is shifted on its own. ``readout(psi_G)`` returns
    [B, K]; the result is J[b, g, k] = d readout_k / d theta_g."""
    B = psi0.shape[0]
    base = readout(run_circuit(circuit, params, feats, psi0))
    J = np.zeros((B, circuit.n_gates, base.shape[1]))
    for g, gate in enumerate(circuit.gates):
        if int(gate["op"]) not in _ROT:
            continue
        th = gate_angles(gate, params, feats, B)
        rp = readout(run_circuit(circuit, params, feats, psi0,
                                 {g: th + np.pi / 2}))
        rm = readout(run_circuit(circuit, params, feats, psi0,
                                 {g: th - np.pi / 2}))
        J[:, g, :] = 0.5 * (rp - rm)
    return J


def finite_difference(fn, x: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """Central differences (fn(x + h e_i) - fn(x - h e_i)) / 2h of a scalar fn."""
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros_like(x)
    flat = x.reshape(-1)
    gf = g.reshape(-1)
    for i in range(flat.size):
        old = flat[i]
        flat[i] = old + h
        fp = fn(x)
        flat[i] = old - h
        fm = fn(x)
        flat[i] = old
        gf[i] = (fp - fm) / (2 * h)
    return g


def loss_and_dexpz(kind: str, z: np.ndarray, labels=None, weights=None):
    """Loss of the expectations and dL/d<Z> [B, n].
    "mse_z0": L = mean_b (<Z_0>_b - y_b)^2;  "weighted_z": L = sum_b sum_q g_q <Z_q>_b."""
    B, n = z.shape
    d = np.zeros_like(z)
    if kind == "mse_z0":
        r = z[:, 0] - np.asarray(labels, dtype=np.float64)
        d[:, 0] = 2.0 * r / B
        return float(np.mean(r * r)), d
    if kind == "weighted_z":
        w = np.asarray(weights, dtype=np.float64)
        d[:] = w[None, :]
        return float(np.sum(z * w[None, :])), d
    raise ValueError(kind)


def expz_readout(psi):
    return expz(psi)
