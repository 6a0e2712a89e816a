"""Plain FP64 state-vector simulation (test infrastructure; see package doc).

Every function works on a batch ``psi[b, i]`` (complex128), qubit q = bit q
of i. Nothing here is blocked, fused or reordered: each gate is applied to
the whole state in descriptor order.
"""

from __future__ import annotations

import numpy as np

from workloads.circuits import OP

_RX, _RY, _RZ = OP["RX"], OP["RY"], OP["RZ"]
_X, _Y, _Z, _H = OP["X"], OP["Y"], OP["Z"], OP["H"]
_CNOT, _CZ = OP["CNOT"], OP["CZ"]
_RESET, _MEASURE = OP["RESET"], OP["MEASURE"]


def gate_matrix(op: int, theta=None) -> np.ndarray:
    """2x2 matrix of a 1-qubit gate; shape [B, 2, 2] for an array ``theta``.

    Rotations are R_P(t) = exp(-i t P / 2) = cos(t/2) I - i sin(t/2) P
    (Nielsen & Chuang §4.2, eqs. 4.4-4.6):
    RX = [[c, -i s], [-i s, c]], RY = [[c, -s], [s, c]],
    RZ = diag(exp(-i t/2), exp(+i t/2)), with c = cos(t/2), s = sin(t/2).
    """
    if op in (_RX, _RY, _RZ):
        t = np.atleast_1d(np.asarray(theta, dtype=np.float64))
        c, s = np.cos(t / 2), np.sin(t / 2)
        m = np.zeros(t.shape + (2, 2), dtype=np.complex128)
        if op == _RX:
            m[..., 0, 0] = c
            m[..., 0, 1] = -1j * s
            m[..., 1, 0] = -1j * s
            m[..., 1, 1] = c
        elif op == _RY:
            m[..., 0, 0] = c
            m[..., 0, 1] = -s
            m[..., 1, 0] = s
            m[..., 1, 1] = c
        else:
            m[..., 0, 0] = np.exp(-0.5j * t)
            m[..., 1, 1] = np.exp(0.5j * t)
        return m
    fixed = {
        _X: [[0, 1], [1, 0]],
        _Y: [[0, -1j], [1j, 0]],
        _Z: [[1, 0], [0, -1]],
        _H: np.array([[1, 1], [1, -1]]) / np.sqrt(2.0),
    }
    return np.asarray(fixed[op], dtype=np.complex128)[None]


def pauli_of(op: int) -> np.ndarray:
    """The Pauli generator P of a rotation gate R_P."""
    return gate_matrix({_RX: _X, _RY: _Y, _RZ: _Z}[op])[0]


def apply_1q(psi: np.ndarray, q: int, U: np.ndarray) -> np.ndarray:
    """psi <- (I (x) U_q (x) I) psi; U is [2,2], [1,2,2] or [B,2,2]."""
    B, N = psi.shape
    v = psi.reshape(B, N >> (q + 1), 2, 1 << q)
    U = np.broadcast_to(U.reshape((-1, 2, 2)), (B, 2, 2))
    out = np.einsum("bij,bhjl->bhil", U, v)
    return out.reshape(B, N)


def apply_cnot(psi: np.ndarray, c: int, t: int) -> np.ndarray:
    """CNOT: flip bit t of the index wherever bit c is 1 (N&C §4.3)."""
    idx = np.arange(psi.shape[1])
    src = np.where((idx >> c) & 1, idx ^ (1 << t), idx)
    return psi[:, src]


def apply_cz(psi: np.ndarray, a: int, b: int) -> np.ndarray:
    """CZ: negate the amplitudes whose bits a and b are both 1."""
    idx = np.arange(psi.shape[1])
    sign = np.where(((idx >> a) & 1) & ((idx >> b) & 1), -1.0, 1.0)
    return psi * sign


def gate_angles(gate, params, feats, B: int) -> np.ndarray:
    """theta[b] = scale * (w * f + bias), the descriptor's angle rule.

    ``params`` is [P] (shared) or [B, P] (one set per sample); ``feats`` is
    [B, F] or None. Computed in FP64 from the stored values.
    """
    p = np.asarray(params, dtype=np.float64)
    scale = float(gate["scale"])
    w = p[..., int(gate["p_w"])] if gate["p_w"] >= 0 else 1.0
    f = (np.asarray(feats, dtype=np.float64)[:, int(gate["feat"])]
         if gate["feat"] >= 0 else 1.0)
    bias = p[..., int(gate["p_b"])] if gate["p_b"] >= 0 else 0.0
    return np.broadcast_to(scale * (w * f + bias), (B,)).astype(np.float64)


def apply_gate(psi: np.ndarray, gate, theta=None, inverse: bool = False):
    """Apply one descriptor gate (its inverse if ``inverse``)."""
    op = int(gate["op"])
    if op == _CNOT:
        return apply_cnot(psi, int(gate["q0"]), int(gate["q1"]))
    if op == _CZ:
        return apply_cz(psi, int(gate["q0"]), int(gate["q1"]))
    if op in (_RX, _RY, _RZ):
        U = gate_matrix(op, -theta if inverse else theta)
    else:
        U = gate_matrix(op)  # X, Y, Z, H are Hermitian and unitary
    return apply_1q(psi, int(gate["q0"]), U)


def encode_amplitude(x: np.ndarray, n: int) -> np.ndarray:
    """|x> = x / ||x||_2 zero-padded to 2^n amplitudes (Schuld & Petruccione
    §5.2). The norm is taken in FP64. Raises on D > 2^n or a zero row."""
    x = np.asarray(x, dtype=np.float64)
    B, D = x.shape
    if D > (1 << n):
        raise ValueError("input dimension exceeds 2^n")
    norm = np.sqrt(np.sum(x * x, axis=1))
    if np.any(norm == 0):
        raise ValueError("zero-norm input row")
    psi = np.zeros((B, 1 << n), dtype=np.complex128)
    psi[:, :D] = x / norm[:, None]
    return psi


def encode_zero(B: int, n: int) -> np.ndarray:
    psi = np.zeros((B, 1 << n), dtype=np.complex128)
    psi[:, 0] = 1.0
    return psi


def channel_probabilities(psi: np.ndarray, q: int) -> np.ndarray:
    """p[b, m] = sum of |psi_bi|^2 over the amplitudes whose bit q is m (FP64)."""
    B, N = psi.shape
    v = psi.reshape(B, N >> (q + 1), 2, 1 << q)
    return np.sum(np.abs(v) ** 2, axis=(1, 3))


def apply_channel(psi: np.ndarray, gate, u: np.ndarray):
    """One trajectory of a mid-circuit measurement of qubit q0 in the Z basis
    (projective-measurement postulate, Nielsen & Chuang sec. 2.2.3): outcome
    m drawn from the Born probabilities p_m by the uniform u (inverse CDF,
    ``trajectory_outcome``), the state projected on bit q0 = m and
    renormalised by sqrt(p_m); RESET then moves it to bit q0 = 0 (the reset
    channel's Kraus operator |0><m|), MEASURE keeps it. A row of zeros gives
    outcome 0 and NaN. Returns (psi' [B, N], m [B], p_m [B])."""
    B, N = psi.shape
    q = int(gate["q0"])
    p = channel_probabilities(psi, q)
    m = trajectory_outcome(p, np.asarray(u, dtype=np.float64))
    rows = np.arange(B)
    v = psi.reshape(B, N >> (q + 1), 2, 1 << q)
    pm = p[rows, m]
    with np.errstate(invalid="ignore", divide="ignore"):
        kept = v[rows, :, m, :] / np.sqrt(pm)[:, None, None]
    out = np.zeros_like(v)
    dst = np.zeros(B, dtype=np.int64) if int(gate["op"]) == _RESET else m
    out[rows, :, dst, :] = kept
    return out.reshape(B, N), m, pm


def channel_cotangent(psi_pre: np.ndarray, gate, u: np.ndarray, lam: np.ndarray):
    """Cotangent before a channel from the cotangent ``lam`` after it, the
    drawn outcome m held fixed (pathwise; convention dL = 2 Re<lam|d psi>).
    With phi = K psi (K = |0><m| or Pi_m on qubit q0), r = ||phi|| =
    sqrt(p_m) and psi' = phi / r: d psi' = d phi / r - psi' Re<psi'|d phi> / r,
    so the cotangent of phi is (lam - Re<lam|psi'> psi') / r and that of psi
    is K^dagger of it. Returns (lam_pre [B, N], psi' [B, N])."""
    B, N = psi_pre.shape
    q = int(gate["q0"])
    post, m, pm = apply_channel(psi_pre, gate, u)
    c = np.real(np.sum(np.conj(lam) * post, axis=1))
    g = (lam - c[:, None] * post) / np.sqrt(pm)[:, None]
    rows = np.arange(B)
    gv = g.reshape(B, N >> (q + 1), 2, 1 << q)
    src = np.zeros(B, dtype=np.int64) if int(gate["op"]) == _RESET else m
    out = np.zeros_like(gv)
    out[rows, :, m, :] = gv[rows, :, src, :]  # K^dagger: slice src of g -> slice m
    return out.reshape(B, N), post


def run_circuit(circuit, params, feats, psi, theta_override=None):
    """psi_G = U_G ... U_1 psi, gates in descriptor order (a channel gate is
    one trajectory, ``apply_channel``, its uniform read from feats).
    ``theta_override`` maps a gate index to a replacement angle array
    (parameter shift)."""
    B = psi.shape[0]
    psi = psi.copy()
    for g, gate in enumerate(circuit.gates):
        op = int(gate["op"])
        if op in (_RESET, _MEASURE):
            u = np.asarray(feats, dtype=np.float64)[:, int(gate["feat"])]
            psi = apply_channel(psi, gate, u)[0]
            continue
        theta = None
        if op in (_RX, _RY, _RZ):
            theta = gate_angles(gate, params, feats, B)
            if theta_override is not None and g in theta_override:
                theta = theta_override[g]
        psi = apply_gate(psi, gate, theta)
    return psi


def expz(psi: np.ndarray) -> np.ndarray:
    """<Z_q>_b = sum_i |psi_bi|^2 (+1 if bit q of i is 0, -1 otherwise)."""
    B, N = psi.shape
    n = N.bit_length() - 1
    prob = np.abs(psi) ** 2
    out = np.empty((B, n))
    for q in range(n):
        v = prob.reshape(B, N >> (q + 1), 2, 1 << q).sum(axis=(1, 3))
        out[:, q] = v[:, 0] - v[:, 1]
    return out


def fidelity_reset(psi: np.ndarray, chi: np.ndarray, n_trash: int):
    """Autoencoder fidelity after resetting the top ``n_trash`` qubits to |0>.

    With psi = U(theta)|x>, the decoder D = V(phi)^dagger and chi = V(phi)|x>,
    the reset channel K_m = |0><m| on the trash qubits gives
    F = <x| D (sum_m K_m |psi><psi| K_m^dagger) D^dagger |x>
      = sum_m |<chi_0 | psi_m>|^2,
    where psi_m is the slice of psi whose trash bits equal m and chi_0 the
    slice of chi whose trash bits are 0. Returns (F [B], c [B, 2^t]).
    """
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    pr = psi.reshape(B, 1 << n_trash, 1 << k)
    chi0 = chi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    c = np.einsum("bj,bmj->bm", np.conj(chi0), pr)
    return np.sum(np.abs(c) ** 2, axis=1), c


def reset_channel_fidelity_cotangents(psi, chi, c, dF, n_trash: int):
    """State cotangents of F (convention dL = 2 Re<lam|d psi>), scaled by
    dF[b] = dL/dF_b:  lam = sum_m c_m |m>|chi_0>,  mu = |0> sum_m conj(c_m) psi_m.
    """
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    chi0 = chi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    pr = psi.reshape(B, 1 << n_trash, 1 << k)
    lam = (c[:, :, None] * chi0[:, None, :]).reshape(B, N)
    mu = np.zeros((B, 1 << n_trash, 1 << k), dtype=np.complex128)
    mu[:, 0, :] = np.einsum("bm,bmj->bj", np.conj(c), pr)
    dF = np.asarray(dF, dtype=np.float64)[:, None]
    return lam * dF, mu.reshape(B, N) * dF


def fidelity_postselect(psi: np.ndarray, chi: np.ndarray, n_trash: int):
    """Autoencoder fidelity when the trash qubits are measured and only the
    all-zero outcome is kept (post-selection), renormalised in FP64.

    The projector Pi_0 = |0><0| on the trash qubits keeps psi_0, the slice of
    psi whose trash bits are 0, with probability p = ||psi_0||^2; the kept
    state is Pi_0 psi / sqrt(p). Its fidelity with |x> after the decoder is
    F' = |<chi_0 | psi_0>|^2 / p  (chi = V|x>, chi_0 its trash-0 slice).
    Rows with p = 0 (nothing survives the post-selection) give NaN.
    Returns (F' [B], c [B] = <chi_0|psi_0>, p [B]).
    """
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    psi0 = psi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    chi0 = chi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    c = np.sum(np.conj(chi0) * psi0, axis=1)
    p = np.sum(np.abs(psi0) ** 2, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        F = np.abs(c) ** 2 / p
    return F, c, p


def postselect_fidelity_cotangents(psi, chi, c, p, dF, n_trash: int):
    """State cotangents of F' = |c|^2 / p (convention dL = 2 Re<lam|d psi>),
    scaled by dF[b] = dL/dF'_b. With dc = <chi_0|d psi_0> and
    dp = 2 Re<psi_0|d psi_0>, dF' = 2 Re(conj(c) dc) / p - |c|^2 dp / p^2, so
        lam = (c / p) chi_0 - (F' / p) psi_0     on the trash-0 slice, 0 elsewhere;
    and with dc = conj(<psi_0|d chi_0>),
        mu = (conj(c) / p) psi_0                  on the trash-0 slice, 0 elsewhere.
    """
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    psi0 = psi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    chi0 = chi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    F = np.abs(c) ** 2 / p
    lam = np.zeros((B, 1 << n_trash, 1 << k), dtype=np.complex128)
    mu = np.zeros_like(lam)
    lam[:, 0, :] = (c / p)[:, None] * chi0 - (F / p)[:, None] * psi0
    mu[:, 0, :] = (np.conj(c) / p)[:, None] * psi0
    dF = np.asarray(dF, dtype=np.float64)[:, None]
    return lam.reshape(B, N) * dF, mu.reshape(B, N) * dF


def trajectory_outcome(p_m: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Outcome of one measurement of the trash qubits, drawn by inverse CDF
    from a uniform u in [0, 1): the smallest m with u * sum_j p_j < sum_{j<=m}
    p_j, the sums running over m = 0, 1, ... in FP64 (m = the last outcome
    with p_m > 0 if rounding leaves none)."""
    B, M = p_m.shape
    out = np.empty(B, dtype=np.int64)
    for b in range(B):
        tot = float(np.sum(p_m[b]))
        acc = 0.0
        pick = -1
        for m in range(M):
            acc += float(p_m[b, m])
            if u[b] * tot < acc:
                pick = m
                break
        if pick < 0:
            nz = np.nonzero(p_m[b] > 0)[0]
            pick = int(nz[-1]) if len(nz) else 0
        out[b] = pick
    return out


def fidelity_trajectory(psi: np.ndarray, chi: np.ndarray, n_trash: int, u: np.ndarray):
    """One quantum trajectory of the reset channel: the trash qubits are
    measured (outcome m with probability p_m = ||psi_m||^2 / ||psi||^2, drawn
    from u by ``trajectory_outcome``) and then reset, so the kept state is
    |0>_t (x) psi_m / sqrt(p_m') with p_m' = ||psi_m||^2, and its fidelity is
        F_traj = |<chi_0 | psi_m>|^2 / ||psi_m||^2.
    Averaged over outcomes (weights p_m) it is the reset-channel fidelity
    sum_m |c_m|^2 (for a normalised psi). Returns (F [B], m [B], c [B], p [B])
    with c = <chi_0|psi_m> and p = ||psi_m||^2 of the drawn outcome.
    """
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    pr = psi.reshape(B, 1 << n_trash, 1 << k)
    chi0 = chi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    p_all = np.sum(np.abs(pr) ** 2, axis=2)
    m = trajectory_outcome(p_all, np.asarray(u, dtype=np.float64))
    psim = pr[np.arange(B), m, :]
    c = np.sum(np.conj(chi0) * psim, axis=1)
    p = p_all[np.arange(B), m]
    with np.errstate(invalid="ignore", divide="ignore"):
        F = np.abs(c) ** 2 / p
    return F, m, c, p


def trajectory_fidelity_cotangents(psi, chi, m, c, p, dF, n_trash: int):
    """State cotangents of F_traj for the drawn (fixed) outcome m, convention
    dL = 2 Re<lam|d psi>, scaled by dF[b]: the post-selection formulas on
    slice m,
        lam = (c/p) |m>|chi_0> - (F/p) |m>|psi_m>   (zero on the other slices),
        mu  = (conj(c)/p) |0>|psi_m>                (zero on the other slices).
    """
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    pr = psi.reshape(B, 1 << n_trash, 1 << k)
    chi0 = chi.reshape(B, 1 << n_trash, 1 << k)[:, 0, :]
    psim = pr[np.arange(B), m, :]
    F = np.abs(c) ** 2 / p
    lam = np.zeros((B, 1 << n_trash, 1 << k), dtype=np.complex128)
    mu = np.zeros_like(lam)
    lam[np.arange(B), m, :] = (c / p)[:, None] * chi0 - (F / p)[:, None] * psim
    mu[:, 0, :] = (np.conj(c) / p)[:, None] * psim
    dF = np.asarray(dF, dtype=np.float64)[:, None]
    return lam.reshape(B, N) * dF, mu.reshape(B, N) * dF


def circuit_unitary(circuit, params, feats_row=None) -> np.ndarray:
    """Full 2^n x 2^n matrix of a circuit for one sample, column j = the
    circuit applied to basis state |j>."""
    n = circuit.n_qubits
    N = 1 << n
    basis = np.eye(N, dtype=np.complex128)
    f = None if feats_row is None else np.repeat(
        np.asarray(feats_row)[None], N, axis=0)
    p = np.asarray(params)
    if p.ndim == 2:
        p = p[0]
    return run_circuit(circuit, p, f, basis).T


def fidelity_reset_direct(x_state, enc, params_enc, dec, params_dec,
                          n_trash: int) -> np.ndarray:
    """The autoencoder fidelity from its definition, with density matrices:
    rho = U|x><x|U^dagger, rho' = sum_m K_m rho K_m^dagger on the trash qubits,
    rho'' = D rho' D^dagger, F = <x|rho''|x>. ``dec`` is the decoder's own gate
    list (D itself). For small n only."""
    B, N = x_state.shape
    n = N.bit_length() - 1
    k = n - n_trash
    U = circuit_unitary(enc, params_enc)
    D = circuit_unitary(dec, params_dec)
    out = np.empty(B)
    for b in range(B):
        x = x_state[b]
        psi = U @ x
        rho = np.outer(psi, np.conj(psi))
        rho_r = np.zeros_like(rho)
        for m in range(1 << n_trash):
            K = np.zeros((N, N), dtype=np.complex128)
            for j in range(1 << k):
                K[j, (m << k) | j] = 1.0    # |0>_t|j> <m|_t<j|
            rho_r += K @ rho @ K.conj().T
        rho2 = D @ rho_r @ D.conj().T
        out[b] = np.real(np.conj(x) @ rho2 @ x)
    return out


def fidelity_postselect_direct(x_state, enc, params_enc, dec, params_dec,
                               n_trash: int) -> np.ndarray:
    """The post-selected autoencoder fidelity from its definition, with
    density matrices: rho = U|x><x|U^dagger, the trash qubits measured with
    outcome 0: rho' = Pi_0 rho Pi_0 / tr(Pi_0 rho) with Pi_0 = |0><0|_t (x) I,
    rho'' = D rho' D^dagger, F' = <x|rho''|x>. For small n only."""
    B, N = x_state.shape
    n = N.bit_length() - 1
    k = n - n_trash
    U = circuit_unitary(enc, params_enc)
    D = circuit_unitary(dec, params_dec)
    Pi = np.zeros((N, N), dtype=np.complex128)
    for j in range(1 << k):
        Pi[j, j] = 1.0          # trash bits (the top n_trash) all zero
    out = np.empty(B)
    for b in range(B):
        x = x_state[b]
        psi = U @ x
        rho = np.outer(psi, np.conj(psi))
        kept = Pi @ rho @ Pi
        rho_p = kept / np.real(np.trace(kept))
        rho2 = D @ rho_p @ D.conj().T
        out[b] = np.real(np.conj(x) @ rho2 @ x)
    return out


def fidelity_trajectory_direct(x_state, enc, params_enc, dec, params_dec,
                               n_trash: int, m: np.ndarray) -> np.ndarray:
    """One trajectory from its definition, for a given outcome m per sample:
    rho = U|x><x|U^dagger; the measurement keeps Pi_m rho Pi_m / tr(Pi_m rho)
    (Pi_m the projector on trash bits = m); the reset K_m = |0><m| then moves
    it to the trash-0 slice; rho'' = D rho' D^dagger, F = <x|rho''|x>. For
    small n only."""
    B, N = x_state.shape
    n = N.bit_length() - 1
    k = n - n_trash
    U = circuit_unitary(enc, params_enc)
    D = circuit_unitary(dec, params_dec)
    out = np.empty(B)
    for b in range(B):
        x = x_state[b]
        psi = U @ x
        rho = np.outer(psi, np.conj(psi))
        K = np.zeros((N, N), dtype=np.complex128)
        for j in range(1 << k):
            K[j, (int(m[b]) << k) | j] = 1.0   # |0>_t|j> <m|_t<j|  (= K_m Pi_m)
        kept = K @ rho @ K.conj().T
        rho_p = kept / np.real(np.trace(kept))
        rho2 = D @ rho_p @ D.conj().T
        out[b] = np.real(np.conj(x) @ rho2 @ x)
    return out
