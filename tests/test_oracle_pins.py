"""Pins of the FP64 oracle against things other than itself.

* hand-derived values from the textbook gate definitions (tests/golden);
* closed forms (<Z> = cos theta after RY/RX, products of cosines, -sin theta);
* brute-force 2^n x 2^n Kronecker products with scipy's matrix exponential
  for n <= 6 (tests/_brute.py), covering every gate kind and qubit position;
* invariants: unitarity, norm preservation, U then U^dagger = identity, the
  CNOT ring as a permutation of basis states, fidelity in [0, 1] and = 1 for
  a mirrored autoencoder without trash qubits;
* the autoencoder's two-pass fidelity against its density-matrix definition,
  for the reset channel and for post-selection on the all-zero trash outcome
  (plus a hand value, its reduction to the reset fidelity when only that
  outcome is populated, scale invariance, Cauchy-Schwarz bounds, and its
  state cotangents against finite differences entry by entry), and for one
  trajectory of the reset channel (hand values of the outcome draw, its
  outcome-weighted average equal to the reset fidelity, outcome 0 equal to
  post-selection, cotangents against finite differences);
* gradients: adjoint = parameter shift (exact) = central finite differences.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle.gradients import observable_cotangent
from oracle.statevector import circuit_unitary
from workloads import circuits as C
from workloads import data as Dt

from _brute import circuit_full, gate_full, angle
from _channels import stable_uniforms

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "hand_values.json")))
OPS = C.OP


def _one(op, q=0, n=1, theta=0.0, q1=-1):
    g = np.array([(OPS[op], q, q1, -1, -1, -1, theta, 0)], dtype=C.GATE_DTYPE)
    return C.Circuit(n, g, 0)


def _run1(op, theta, psi):
    c = _one(op, theta=theta)
    return O.run_circuit(c, np.zeros(0), None, psi)


# ---------------------------------------------------------------- hand values
@pytest.mark.parametrize("key,op,start", [("rx_on_zero", "RX", "zero"),
                                          ("ry_on_zero", "RY", "zero"),
                                          ("rz_on_plus", "RZ", "plus")])
def test_single_qubit_states_hand_values(key, op, start):
    gv = GOLD[key]
    psi = O.encode_zero(1, 1) if start == "zero" else \
        np.array([[1, 1]], dtype=complex) / np.sqrt(2)
    out = _run1(op, gv["theta"], psi)[0]
    np.testing.assert_allclose(out.real, gv["re"], atol=1e-15)
    np.testing.assert_allclose(out.imag, gv["im"], atol=1e-15)


def test_basis_state_expz_bit_order():
    gv = GOLD["basis5_n3_expz"]
    x = np.zeros((1, 8))
    x[0, gv["index"]] = 3.0  # unnormalised on purpose
    z = O.expz(O.encode_amplitude(x, gv["n"]))
    np.testing.assert_array_equal(z[0], gv["expz"])


@pytest.mark.parametrize("key", ["cnot_ring_n3_on_1", "cnot_ring_n3_on_4"])
def test_cnot_ring_permutation(key):
    gv = GOLD[key]
    n = gv["n"]
    rows = [(OPS["CNOT"], i, (i + 1) % n, -1, -1, -1, 0.0, 0) for i in range(n)]
    c = C.Circuit(n, np.array(rows, dtype=C.GATE_DTYPE), 0)
    psi = np.zeros((1, 1 << n), dtype=complex)
    psi[0, gv["input_index"]] = 1
    out = O.run_circuit(c, np.zeros(0), None, psi)
    expect = np.zeros(1 << n)
    expect[gv["output_index"]] = 1
    np.testing.assert_array_equal(out[0], expect)


def test_cz_sign_pattern():
    gv = GOLD["cz_sign_n3"]
    psi = np.ones((1, 8), dtype=complex)
    out = O.apply_cz(psi, gv["a"], gv["b"])
    np.testing.assert_array_equal(out[0].real, gv["sign"])


def test_bell_state():
    gv = GOLD["bell"]
    rows = [(OPS["H"], 0, -1, -1, -1, -1, 0.0, 0),
            (OPS["CNOT"], 0, 1, -1, -1, -1, 0.0, 0)]
    c = C.Circuit(2, np.array(rows, dtype=C.GATE_DTYPE), 0)
    out = O.run_circuit(c, np.zeros(0), None, O.encode_zero(1, 2))
    np.testing.assert_allclose(out[0].real, gv["re"], atol=1e-15)
    np.testing.assert_allclose(out[0].imag, 0, atol=1e-15)
    np.testing.assert_allclose(O.expz(out)[0], gv["expz"], atol=1e-15)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("op", ["RX", "RY"])
def test_expz_cos_theta(op):
    th = np.linspace(-np.pi, np.pi, 17)
    psi = O.encode_zero(th.size, 1)
    g = np.array([(OPS[op], 0, -1, 0, -1, -1, 1.0, 0)], dtype=C.GATE_DTYPE)
    c = C.Circuit(1, g, 1)
    z = np.array([O.expz(O.run_circuit(c, np.array([t]), None, psi[:1]))[0, 0]
                  for t in th])
    np.testing.assert_allclose(z, np.cos(th), atol=1e-15)
    # d<Z>/dtheta = -sin(theta), from the adjoint and from parameter shift
    for t in th:
        gth, _ = O.adjoint_vjp(c, np.array([t]), None, psi[:1],
                               dexpz=np.ones((1, 1)))
        np.testing.assert_allclose(gth[0, 0], -np.sin(t), atol=1e-14)


def test_rz_leaves_z_unchanged_and_product_of_cosines():
    gv = GOLD["ry_then_rx_expz"]
    # angles through FP64 parameters (the descriptor's scale is float32)
    P = np.array([gv["a"], 0.9, gv["b"]])
    rows = [(OPS["RY"], 0, -1, 0, -1, -1, 1.0, 0),
            (OPS["RZ"], 0, -1, 1, -1, -1, 1.0, 0),
            (OPS["RX"], 0, -1, 2, -1, -1, 1.0, 0)]
    # RZ after RY leaves <Z> = cos(a); RY then RX gives cos(a) cos(b).
    c_rz = C.Circuit(1, np.array(rows[:2], dtype=C.GATE_DTYPE), 3)
    z = O.expz(O.run_circuit(c_rz, P, None, O.encode_zero(1, 1)))
    np.testing.assert_allclose(z[0, 0], np.cos(gv["a"]), atol=1e-15)
    c = C.Circuit(1, np.array([rows[0], rows[2]], dtype=C.GATE_DTYPE), 3)
    z = O.expz(O.run_circuit(c, P, None, O.encode_zero(1, 1)))
    np.testing.assert_allclose(z[0, 0], gv["expz"], atol=1e-15)


def test_product_circuit_expz_is_product_of_cosines(rng):
    n = 5
    a = rng.uniform(-np.pi, np.pi, n)
    b = rng.uniform(-np.pi, np.pi, n)
    rows = []
    for q in range(n):
        rows.append((OPS["RY"], q, -1, -1, -1, -1, a[q], 0))
        rows.append((OPS["RX"], q, -1, -1, -1, -1, b[q], 0))
    c = C.Circuit(n, np.array(rows, dtype=C.GATE_DTYPE), 0)
    z = O.expz(O.run_circuit(c, np.zeros(0), None, O.encode_zero(1, n)))[0]
    np.testing.assert_allclose(z, np.cos(a.astype(np.float32).astype(float)) *
                               np.cos(b.astype(np.float32).astype(float)),
                               atol=1e-14)


def test_x_flips_only_its_qubit():
    n = 4
    for q in range(n):
        c = _one("X", q=q, n=n)
        z = O.expz(O.run_circuit(c, np.zeros(0), None, O.encode_zero(1, n)))[0]
        expect = np.ones(n)
        expect[q] = -1
        np.testing.assert_array_equal(z, expect)


# ---------------------------------------------------------------- encodings
def test_amplitude_encoding_pads_and_normalises(rng):
    x = rng.standard_normal((3, 5))
    psi = O.encode_amplitude(x, 3)
    np.testing.assert_allclose(np.linalg.norm(psi, axis=1), 1, atol=1e-15)
    np.testing.assert_allclose(psi[:, :5].real * np.linalg.norm(x, axis=1)[:, None], x,
                               atol=1e-14)
    assert np.all(psi[:, 5:] == 0)
    with pytest.raises(ValueError):
        O.encode_amplitude(np.zeros((1, 4)), 2)
    with pytest.raises(ValueError):
        O.encode_amplitude(np.ones((1, 9)), 3)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_every_gate_kind_every_position_vs_kron(n, rng):
    kinds = ["RX", "RY", "RZ", "X", "Y", "Z", "H"]
    psi = rng.standard_normal((2, 1 << n)) + 1j * rng.standard_normal((2, 1 << n))
    for k in kinds:
        for q in range(n):
            th = float(np.float32(rng.uniform(-4, 4)))
            c = _one(k, q=q, n=n, theta=th)
            U = gate_full(n, c.gates[0], th)
            np.testing.assert_allclose(U.conj().T @ U, np.eye(1 << n), atol=1e-13)
            out = O.run_circuit(c, np.zeros(0), None, psi)
            np.testing.assert_allclose(out, psi @ U.T, atol=1e-13)
    for k in ["CNOT", "CZ"]:
        for a in range(n):
            for b in range(n):
                if a == b:
                    continue
                c = _one(k, q=a, n=n, q1=b)
                U = gate_full(n, c.gates[0], 0.0)
                out = O.run_circuit(c, np.zeros(0), None, psi)
                np.testing.assert_allclose(out, psi @ U.T, atol=1e-13)


@pytest.mark.parametrize("n,G", [(1, 12), (2, 30), (3, 40), (4, 60), (5, 80), (6, 90)])
def test_random_circuits_vs_kron(n, G, rng):
    c = C.random_circuit(n, G, rng, n_params=6, n_features=3)
    B = 3
    params = rng.uniform(-np.pi, np.pi, c.n_params)
    feats = rng.uniform(-1, 1, (B, c.n_features))
    x = rng.standard_normal((B, 1 << n))
    psi0 = O.encode_amplitude(x, n)
    out = O.run_circuit(c, params, feats, psi0)
    for b in range(B):
        U = circuit_full(c, params, feats[b])
        np.testing.assert_allclose(U.conj().T @ U, np.eye(1 << n), atol=1e-12)
        np.testing.assert_allclose(out[b], U @ psi0[b], atol=1e-12)
        np.testing.assert_allclose(np.linalg.norm(out[b]), 1.0, atol=1e-13)


def test_per_sample_params_vs_kron(rng):
    n, B = 3, 4
    c = C.hea_ry_rz_ring(n, 2)
    params = rng.uniform(-np.pi, np.pi, (B, c.n_params))
    psi0 = O.encode_amplitude(rng.standard_normal((B, 8)), n)
    out = O.run_circuit(c, params, None, psi0)
    for b in range(B):
        np.testing.assert_allclose(out[b], circuit_full(c, params[b]) @ psi0[b],
                                   atol=1e-12)


def test_angle_rule_written_out():
    # theta = scale (w f + bias), per field, against the brute helper's rule
    g = np.array([(OPS["RY"], 0, -1, 1, 0, 2, 0.5, 0)], dtype=C.GATE_DTYPE)[0]
    params = np.array([9.0, 2.0, -3.0])
    feats = np.array([[0.25]])
    th = O.gate_angles(g, params, feats, 1)[0]
    assert th == pytest.approx(0.5 * (2.0 * 0.25 - 3.0), abs=0)
    assert th == pytest.approx(angle(g, params, feats[0]), abs=0)


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("key,B", [("c1", 8), ("c2", 4), ("c3", 16), ("c4", 2)])
def test_workload_norm_and_inverse(key, B):
    w = Dt.make_workload(key, B)
    n = w.n_qubits
    psi0 = O.encode_amplitude(w.x, n) if w.encoding == "amplitude" else \
        O.encode_zero(B, n)
    out = O.run_circuit(w.circuit, w.params, w.feats, psi0)
    np.testing.assert_allclose(np.linalg.norm(out, axis=1), 1, atol=1e-12)
    inv = C.inverse_structure(w.circuit)
    back = O.run_circuit(inv, w.params, w.feats, out)
    np.testing.assert_allclose(back, psi0, atol=1e-12)
    z = O.expz(out)
    assert np.all(np.abs(z) <= 1 + 1e-12)


def test_inverse_structure_layer_ends():
    c = C.ry_rz_chain(3, 2)
    inv = C.inverse_structure(c)
    assert c.layer_end == [8, 16]
    assert inv.layer_end == [8, 16]


# ---------------------------------------------------------------- fidelity
@pytest.mark.parametrize("n,t", [(3, 1), (4, 2), (5, 2)])
def test_fidelity_two_pass_equals_density_matrix_definition(n, t, rng):
    enc = C.ry_rz_chain(n, 2)
    B = 3
    th = rng.uniform(-np.pi, np.pi, enc.n_params)
    ph = rng.uniform(-np.pi, np.pi, enc.n_params)
    x = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    psi = O.run_circuit(enc, th, None, x)
    chi = O.run_circuit(enc, ph, None, x)          # chi = V(phi)|x>
    F, _ = O.fidelity_reset(psi, chi, t)
    dec = C.inverse_structure(enc)                 # D = V(phi)^dagger
    Fd = O.fidelity_reset_direct(x, enc, th, dec, ph, t)
    np.testing.assert_allclose(F, Fd, atol=1e-12)
    assert np.all((F >= -1e-12) & (F <= 1 + 1e-12))


def test_fidelity_mirrored_without_trash_is_one(rng):
    n = 4
    enc = C.ry_rz_chain(n, 3)
    th = rng.uniform(-np.pi, np.pi, enc.n_params)
    x = O.encode_amplitude(rng.standard_normal((2, 16)), n)
    psi = O.run_circuit(enc, th, None, x)
    F, _ = O.fidelity_reset(psi, psi.copy(), 0)
    np.testing.assert_allclose(F, 1.0, atol=1e-13)


# ------------------------------------------------ post-selected fidelity
@pytest.mark.parametrize("n,t", [(3, 1), (4, 2), (5, 2), (4, 3)])
def test_postselect_two_pass_equals_density_matrix_definition(n, t, rng):
    enc = C.ry_rz_chain(n, 2)
    B = 3
    th = rng.uniform(-np.pi, np.pi, enc.n_params)
    ph = rng.uniform(-np.pi, np.pi, enc.n_params)
    x = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    psi = O.run_circuit(enc, th, None, x)
    chi = O.run_circuit(enc, ph, None, x)
    F, c, p = O.fidelity_postselect(psi, chi, t)
    Fd = O.fidelity_postselect_direct(x, enc, th, C.inverse_structure(enc), ph, t)
    np.testing.assert_allclose(F, Fd, atol=1e-12)
    # Cauchy-Schwarz: 0 <= F' <= ||chi_0||^2 <= 1
    k = n - t
    chi0 = chi.reshape(B, 1 << t, 1 << k)[:, 0, :]
    assert np.all(F >= -1e-12)
    assert np.all(F <= np.sum(np.abs(chi0) ** 2, axis=1) + 1e-12)
    assert np.all((p > 0) & (p <= 1 + 1e-12))


def test_postselect_hand_value():
    """n = 2, one trash qubit (bit 1): psi = (1, i, 1, 0)/sqrt 3 keeps
    (1, i)/sqrt 3 with probability 2/3; against chi = |00> the overlap is
    1/sqrt 3, so F' = (1/3) / (2/3) = 1/2 (and the reset fidelity is
    |<00|psi>|^2 + |<00|10-slice>|^2 = 1/3 + 1/3)."""
    psi = np.array([[1, 1j, 1, 0]]) / np.sqrt(3)
    chi = np.array([[1, 0, 0, 0]], dtype=np.complex128)
    F, c, p = O.fidelity_postselect(psi, chi, 1)
    np.testing.assert_allclose(F, [0.5], atol=1e-15)
    np.testing.assert_allclose(p, [2 / 3], atol=1e-15)
    np.testing.assert_allclose(c, [1 / np.sqrt(3)], atol=1e-15)
    np.testing.assert_allclose(O.fidelity_reset(psi, chi, 1)[0], [2 / 3], atol=1e-15)


def test_postselect_equals_reset_when_only_trash_zero_is_populated(rng):
    n, t, B = 5, 2, 4
    k = n - t
    psi = np.zeros((B, 1 << n), dtype=np.complex128)
    v = rng.standard_normal((B, 1 << k)) + 1j * rng.standard_normal((B, 1 << k))
    psi[:, :1 << k] = v / np.linalg.norm(v, axis=1, keepdims=True)
    chi = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    F, _, p = O.fidelity_postselect(psi, chi, t)
    np.testing.assert_allclose(p, 1.0, atol=1e-14)
    np.testing.assert_allclose(F, O.fidelity_reset(psi, chi, t)[0], atol=1e-14)


def test_postselect_renormalisation_scale_invariance_and_empty_outcome(rng):
    n, t, B = 4, 2, 3
    psi = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    chi = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    F, _, _ = O.fidelity_postselect(psi, chi, t)
    F2, _, _ = O.fidelity_postselect(psi * (0.3 - 1.7j), chi, t)
    np.testing.assert_allclose(F2, F, rtol=1e-13)
    # nothing in the trash-0 slice: probability 0, fidelity undefined (NaN)
    psi[0, :1 << (n - t)] = 0
    F3, _, p3 = O.fidelity_postselect(psi, chi, t)
    assert p3[0] == 0 and np.isnan(F3[0]) and np.all(np.isfinite(F3[1:]))


def test_postselect_cotangents_match_finite_differences_of_the_states(rng):
    """dF'/d Re psi_i = 2 Re lam_i and dF'/d Im psi_i = 2 Im lam_i (and the
    same for chi with mu), by central differences on every entry."""
    n, t, B = 3, 1, 2
    psi = O.encode_amplitude(rng.standard_normal((B, 8)), n) * (0.8 + 0.3j)
    chi = O.encode_amplitude(rng.standard_normal((B, 8)), n) * np.exp(0.4j)
    F, c, p = O.fidelity_postselect(psi, chi, t)
    lam, mu = O.postselect_fidelity_cotangents(psi, chi, c, p, np.ones(B), t)
    h = 1e-6
    for which, st, cot in (("psi", psi, lam), ("chi", chi, mu)):
        for i in range(8):
            for unit in (1.0, 1j):
                e = np.zeros_like(st)
                e[:, i] = unit * h
                a = (st + e, chi) if which == "psi" else (psi, st + e)
                b_ = (st - e, chi) if which == "psi" else (psi, st - e)
                fd = (O.fidelity_postselect(*a, t)[0] - O.fidelity_postselect(*b_, t)[0]) / (2 * h)
                want = 2 * (cot[:, i].real if unit == 1.0 else cot[:, i].imag)
                np.testing.assert_allclose(fd, want, atol=1e-8)


def test_postselect_parameter_gradients_adjoint_vs_fd(rng):
    n, t, B = 4, 2, 2
    enc = C.ry_rz_chain(n, 2)
    th = rng.uniform(-np.pi, np.pi, enc.n_params)
    ph = rng.uniform(-np.pi, np.pi, enc.n_params)
    x = O.encode_amplitude(rng.standard_normal((B, 16)), n)

    def L(th_, ph_):
        psi = O.run_circuit(enc, th_, None, x)
        chi = O.run_circuit(enc, ph_, None, x)
        return 1.0 - float(np.mean(O.fidelity_postselect(psi, chi, t)[0]))

    psi = O.run_circuit(enc, th, None, x)
    chi = O.run_circuit(enc, ph, None, x)
    F, c, p = O.fidelity_postselect(psi, chi, t)
    lam, mu = O.postselect_fidelity_cotangents(psi, chi, c, p, -np.ones(B) / B, t)
    g1, _ = O.adjoint_vjp(enc, th, None, x, lam_final=lam)
    g2, _ = O.adjoint_vjp(enc, ph, None, x, lam_final=mu)
    d_th, _ = O.theta_to_param_grads(enc, th, None, g1)
    d_ph, _ = O.theta_to_param_grads(enc, ph, None, g2)
    np.testing.assert_allclose(d_th, O.finite_difference(lambda v: L(v, ph), th.copy()),
                               atol=1e-8)
    np.testing.assert_allclose(d_ph, O.finite_difference(lambda v: L(th, v), ph.copy()),
                               atol=1e-8)


# --------------------------------------------- trajectory of the reset channel
def _mid_u(psi, n_trash, m):
    """u in the middle of outcome m's CDF interval (far from any boundary)."""
    B, N = psi.shape
    k = (N.bit_length() - 1) - n_trash
    p = np.sum(np.abs(psi.reshape(B, 1 << n_trash, 1 << k)) ** 2, axis=2)
    cum = np.cumsum(p, axis=1) / p.sum(axis=1, keepdims=True)
    lo = np.where(m > 0, cum[np.arange(B), np.maximum(m - 1, 0)], 0.0)
    return (lo + cum[np.arange(B), m]) / 2


def test_trajectory_outcome_hand_values():
    p = np.array([[0.2, 0.0, 0.5, 0.3]] * 6)
    u = np.array([0.1, 0.2, 0.69, 0.7, 0.999, 0.0])
    np.testing.assert_array_equal(O.trajectory_outcome(p, u), [0, 2, 2, 3, 3, 0])
    # unnormalised probabilities: u scales with their sum
    np.testing.assert_array_equal(O.trajectory_outcome(p * 4, u), [0, 2, 2, 3, 3, 0])


@pytest.mark.parametrize("n,t", [(3, 1), (4, 2), (5, 3)])
def test_trajectory_average_is_the_reset_fidelity(n, t, rng):
    """Sum over outcomes m of p_m F_traj(m) = the reset-channel fidelity."""
    enc = C.ry_rz_chain(n, 2)
    B = 3
    th = rng.uniform(-np.pi, np.pi, enc.n_params)
    ph = rng.uniform(-np.pi, np.pi, enc.n_params)
    x = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    psi = O.run_circuit(enc, th, None, x)
    chi = O.run_circuit(enc, ph, None, x)
    avg = np.zeros(B)
    for m in range(1 << t):
        mm = np.full(B, m)
        F, got, c, p = O.fidelity_trajectory(psi, chi, t, _mid_u(psi, t, mm))
        np.testing.assert_array_equal(got, mm)
        avg += p * F
        np.testing.assert_allclose(
            F, O.fidelity_trajectory_direct(x, enc, th, C.inverse_structure(enc), ph, t, mm),
            atol=1e-12)
    np.testing.assert_allclose(avg, O.fidelity_reset(psi, chi, t)[0], atol=1e-12)
    # outcome 0 is the post-selected fidelity
    F0 = O.fidelity_trajectory(psi, chi, t, _mid_u(psi, t, np.zeros(B, int)))[0]
    np.testing.assert_allclose(F0, O.fidelity_postselect(psi, chi, t)[0], atol=1e-13)


def test_trajectory_cotangents_match_finite_differences(rng):
    n, t, B = 3, 1, 2
    psi = O.encode_amplitude(rng.standard_normal((B, 8)), n) * (0.9 - 0.2j)
    chi = O.encode_amplitude(rng.standard_normal((B, 8)), n) * np.exp(-0.3j)
    m = np.array([1, 0])
    u = _mid_u(psi, t, m)
    F, got, c, p = O.fidelity_trajectory(psi, chi, t, u)
    np.testing.assert_array_equal(got, m)
    lam, mu = O.trajectory_fidelity_cotangents(psi, chi, got, c, p, np.ones(B), t)
    h = 1e-6
    for which, st, cot in (("psi", psi, lam), ("chi", chi, mu)):
        for i in range(8):
            for unit in (1.0, 1j):
                e = np.zeros_like(st)
                e[:, i] = unit * h
                a = (st + e, chi) if which == "psi" else (psi, st + e)
                b_ = (st - e, chi) if which == "psi" else (psi, st - e)
                fd = (O.fidelity_trajectory(*a, t, u)[0] -
                      O.fidelity_trajectory(*b_, t, u)[0]) / (2 * h)
                want = 2 * (cot[:, i].real if unit == 1.0 else cot[:, i].imag)
                np.testing.assert_allclose(fd, want, atol=1e-8)


# ---------------------------------------------------------------- gradients
def _expz_loss_setup(rng, n=3, G=30, B=3, F=2, per_sample=False):
    c = C.random_circuit(n, G, rng, n_params=5, n_features=F)
    params = rng.uniform(-np.pi, np.pi, (B, c.n_params) if per_sample else c.n_params)
    feats = rng.uniform(-1, 1, (B, F))
    psi0 = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    wts = rng.uniform(-1, 1, (B, n))
    return c, params, feats, psi0, wts


@pytest.mark.parametrize("per_sample", [False, True])
def test_adjoint_equals_param_shift_equals_fd(rng, per_sample):
    c, params, feats, psi0, wts = _expz_loss_setup(rng, per_sample=per_sample)

    def loss(p, f):
        return float(np.sum(wts * O.expz(O.run_circuit(c, p, f, psi0))))

    gth, _ = O.adjoint_vjp(c, params, feats, psi0, dexpz=wts)
    dp, df = O.theta_to_param_grads(c, params, feats, gth)
    J = O.param_shift_theta_jacobian(c, params, feats, psi0, O.expz)
    gth_ps = np.einsum("bgk,bk->bg", J, wts)
    np.testing.assert_allclose(gth, gth_ps, atol=1e-12)
    dp_fd = O.finite_difference(lambda p: loss(p, feats), params.copy())
    df_fd = O.finite_difference(lambda f: loss(params, f), feats.copy())
    np.testing.assert_allclose(dp, dp_fd, atol=1e-8)
    np.testing.assert_allclose(df, df_fd, atol=1e-8)


def test_mse_loss_gradient_matches_fd(rng):
    w = Dt.make_workload("c2", 3)
    c = C.rxyz_cz_ring(4, 2)
    params = w.params[:c.n_params].astype(np.float64)
    psi0 = O.encode_amplitude(w.x[:, :16], 4)
    y = w.labels

    def loss(p):
        return O.loss_and_dexpz("mse_z0", O.expz(O.run_circuit(c, p, None, psi0)), y)[0]

    z = O.expz(O.run_circuit(c, params, None, psi0))
    _, dz = O.loss_and_dexpz("mse_z0", z, y)
    gth, _ = O.adjoint_vjp(c, params, None, psi0, dexpz=dz)
    dp, _ = O.theta_to_param_grads(c, params, None, gth)
    np.testing.assert_allclose(dp, O.finite_difference(loss, params.copy()), atol=1e-8)


def test_weighted_z_loss_hand_value_and_gradient():
    """The readout loss of the uneven batch and of the 26-qubit circuit is the
    plain sum L = sum_b sum_q g_q <Z_q>_b (not a mean): two samples, two
    qubits, worked by hand: (2 * 0.5 - 4 * -0.25) + (2 * 1.0 - 4 * 0.0) = 4."""
    z = np.array([[0.5, -0.25], [1.0, 0.0]])
    g = np.array([2.0, -4.0])
    L, d = O.loss_and_dexpz("weighted_z", z, None, g)
    assert L == 4.0
    np.testing.assert_array_equal(d, [[2.0, -4.0], [2.0, -4.0]])
    # dL/dz against central differences of the returned loss
    fd = O.finite_difference(lambda v: O.loss_and_dexpz("weighted_z", v, None, g)[0],
                             z.copy())
    np.testing.assert_allclose(d, fd, atol=1e-9)


def test_weighted_z_gradient_through_the_26_qubit_structure_matches_fd(rng):
    """The 26-qubit workload's structure (RY, RZ on every qubit + ring CNOT)
    at 5 qubits with its weighted readout loss: adjoint = parameter shift =
    central differences of the loss."""
    c = C.hea_ry_rz_ring(5, 3)
    params = rng.uniform(-np.pi, np.pi, c.n_params)
    g = rng.uniform(-1, 1, 5)
    psi0 = O.encode_zero(2, 5)

    def loss(p):
        return O.loss_and_dexpz("weighted_z", O.expz(O.run_circuit(c, p, None, psi0)),
                                None, g)[0]

    z = O.expz(O.run_circuit(c, params, None, psi0))
    _, dz = O.loss_and_dexpz("weighted_z", z, None, g)
    gth, _ = O.adjoint_vjp(c, params, None, psi0, dexpz=dz)
    dp, _ = O.theta_to_param_grads(c, params, None, gth)
    np.testing.assert_allclose(dp, O.finite_difference(loss, params.copy()), atol=1e-8)
    J = O.param_shift_theta_jacobian(c, params, None, psi0, O.expz)
    np.testing.assert_allclose(gth, np.einsum("bgk,k->bg", J, g), atol=1e-12)


# ------------------------------------------------- mid-circuit channels
def _chan_circuit(rows, n, n_params=0, n_features=1):
    return C.Circuit(n, np.array(rows, dtype=C.GATE_DTYPE), n_params, n_features)


def test_channel_hand_values():
    gv = GOLD["channel_plus"]
    for kind in ("reset", "measure"):
        c = _chan_circuit([(OPS["H"], 0, -1, -1, -1, -1, 0.0, 0),
                           (OPS[kind.upper()], 0, -1, -1, 0, -1, 0.0, 0)], 1)
        for u, want in zip(gv["u"], gv[kind]):
            out = O.run_circuit(c, np.zeros(0), np.array([[u]]), O.encode_zero(1, 1))
            np.testing.assert_allclose(out[0], want, atol=1e-12)
    gv = GOLD["channel_ry"]
    c = _chan_circuit([(OPS["RY"], 0, -1, -1, -1, -1, gv["theta"], 0),
                       (OPS["MEASURE"], 0, -1, -1, 0, -1, 0.0, 0)], 1)
    for u, want in zip(gv["u"], gv["measure"]):
        out = O.run_circuit(c, np.zeros(0), np.array([[u]]), O.encode_zero(1, 1))
        np.testing.assert_allclose(out[0], want, atol=1e-12)
    gv = GOLD["channel_bell"]
    for kind, idx in (("MEASURE", gv["measure_index"]), ("RESET", gv["reset_index"])):
        c = _chan_circuit([(OPS["H"], 0, -1, -1, -1, -1, 0.0, 0),
                           (OPS["CNOT"], 0, 1, -1, -1, -1, 0.0, 0),
                           (OPS[kind], 1, -1, -1, 0, -1, 0.0, 0)], 2)
        out = O.run_circuit(c, np.zeros(0), np.array([[gv["u"]]]), O.encode_zero(1, 2))
        want = np.zeros(4)
        want[idx] = 1.0
        np.testing.assert_allclose(out[0], want, atol=1e-12)


@pytest.mark.parametrize("kind", ["RESET", "MEASURE"])
@pytest.mark.parametrize("n,q", [(1, 0), (3, 0), (3, 2), (4, 1)])
def test_channel_trajectories_average_to_the_kraus_channel(n, q, kind, rng):
    """Averaged over outcomes (weights p_m), the trajectory states are the
    channel applied to the density matrix, with Kraus operators |0><m| (reset)
    or |m><m| (measurement) built by Kronecker products."""
    from _brute import embed
    psi = O.encode_amplitude(rng.standard_normal((1, 1 << n)), n)
    psi = psi * np.exp(1j * rng.uniform(0, 2 * np.pi, psi.shape))
    rho = np.outer(psi[0], np.conj(psi[0]))
    ket = [np.array([[1, 0], [0, 0]], complex), np.array([[0, 0], [0, 1]], complex)]
    lower = np.array([[0, 1], [0, 0]], complex)  # |0><1|
    K = [embed(n, q, ket[0]), embed(n, q, lower if kind == "RESET" else ket[1])]
    want = sum(k @ rho @ k.conj().T for k in K)
    g = np.array([(OPS[kind], q, -1, -1, 0, -1, 0.0, 0)], dtype=C.GATE_DTYPE)[0]
    p = np.array([np.real(np.vdot(psi[0], embed(n, q, ket[m]) @ psi[0])) for m in (0, 1)])
    got = np.zeros_like(rho)
    for m in (0, 1):
        if p[m] <= 0:
            continue
        u = (p[:m].sum() + 0.5 * p[m]) / p.sum()  # inside outcome m's interval
        out, mm, pm = O.apply_channel(psi, g, np.array([u]))
        assert mm[0] == m and abs(pm[0] - p[m]) < 1e-12
        got += p[m] * np.outer(out[0], np.conj(out[0]))
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_channel_on_a_qubit_in_zero_is_the_identity(rng):
    n, q = 4, 2
    c = _chan_circuit([(OPS["RESET"], q, -1, -1, 0, -1, 0.0, 0),
                       (OPS["MEASURE"], q, -1, -1, 1, -1, 0.0, 0)], n, n_features=2)
    psi = O.encode_amplitude(rng.standard_normal((3, 1 << n)), n)
    idx = np.arange(1 << n)
    psi[:, (idx >> q) & 1 == 1] = 0
    psi /= np.linalg.norm(psi, axis=1, keepdims=True)
    out = O.run_circuit(c, np.zeros(0), rng.uniform(0, 1, (3, 2)), psi)
    np.testing.assert_allclose(out, psi, atol=1e-13)


@pytest.mark.parametrize("per_sample", [False, True])
def test_channel_gradients_adjoint_vs_fd(rng, per_sample):
    """Rotations before, between and after two channels (one reset, one
    measurement), with features: the adjoint through the channels (outcomes
    held fixed) equals central differences of the loss, for a <Z> loss and for
    a state cotangent."""
    n, B = 4, 3
    base = C.random_circuit(n, 36, rng, n_params=6, n_features=2)
    c = C.with_channels(base, [12, 25], rng)
    P = c.n_params
    params = rng.uniform(-np.pi, np.pi, (B, P) if per_sample else P)
    psi0 = O.encode_amplitude(rng.standard_normal((B, 1 << n)), n)
    feats = np.concatenate([rng.uniform(-1, 1, (B, 2)), np.full((B, 2), 0.5)], axis=1)
    feats = stable_uniforms(c, params, feats, psi0)
    wts = rng.uniform(-1, 1, (B, n))

    def loss(p, f):
        return float(np.sum(wts * O.expz(O.run_circuit(c, p, f, psi0))))

    gth, _ = O.adjoint_vjp(c, params, feats, psi0, dexpz=wts)
    dp, df = O.theta_to_param_grads(c, params, feats, gth)
    np.testing.assert_allclose(dp, O.finite_difference(lambda p: loss(p, feats), params.copy()),
                               atol=1e-7)
    fd_f = O.finite_difference(lambda f: loss(params, f), feats.copy())
    np.testing.assert_allclose(df[:, :2], fd_f[:, :2], atol=1e-7)
    assert np.all(df[:, 2:] == 0)
    # a state cotangent: L = 2 Re <a | psi_G>
    a = rng.standard_normal((B, 1 << n)) + 1j * rng.standard_normal((B, 1 << n))

    def loss2(p):
        return float(2 * np.real(np.sum(np.conj(a) * O.run_circuit(c, p, feats, psi0))))

    gth2, _ = O.adjoint_vjp(c, params, feats, psi0, lam_final=a)
    dp2, _ = O.theta_to_param_grads(c, params, feats, gth2)
    np.testing.assert_allclose(dp2, O.finite_difference(loss2, params.copy()), atol=1e-7)


def test_fidelity_gradients_adjoint_shift_fd(rng):
    n, t, B = 4, 2, 2
    enc = C.ry_rz_chain(n, 2)
    th = rng.uniform(-np.pi, np.pi, enc.n_params)
    ph = rng.uniform(-np.pi, np.pi, enc.n_params)
    x = O.encode_amplitude(rng.standard_normal((B, 16)), n)

    def L(th_, ph_):
        psi = O.run_circuit(enc, th_, None, x)
        chi = O.run_circuit(enc, ph_, None, x)
        return 1.0 - float(np.mean(O.fidelity_reset(psi, chi, t)[0]))

    psi = O.run_circuit(enc, th, None, x)
    chi = O.run_circuit(enc, ph, None, x)
    F, cm = O.fidelity_reset(psi, chi, t)
    dF = -np.ones(B) / B
    lam, mu = O.reset_channel_fidelity_cotangents(psi, chi, cm, dF, t)
    g1, _ = O.adjoint_vjp(enc, th, None, x, lam_final=lam)
    g2, _ = O.adjoint_vjp(enc, ph, None, x, lam_final=mu)
    d_th, _ = O.theta_to_param_grads(enc, th, None, g1)
    d_ph, _ = O.theta_to_param_grads(enc, ph, None, g2)
    np.testing.assert_allclose(d_th, O.finite_difference(lambda v: L(v, ph), th.copy()),
                               atol=1e-8)
    np.testing.assert_allclose(d_ph, O.finite_difference(lambda v: L(th, v), ph.copy()),
                               atol=1e-8)
    # parameter shift through F as an observable of psi (chi fixed)
    J = O.param_shift_theta_jacobian(
        enc, th, None, x, lambda p: O.fidelity_reset(p, chi, t)[0][:, None])
    np.testing.assert_allclose(g1, J[:, :, 0] * dF[:, None], atol=1e-12)


def test_observable_cotangent_is_diagonal_weighting(rng):
    psi = O.encode_amplitude(rng.standard_normal((2, 8)), 3)
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 2.0]])
    lam = observable_cotangent(psi, d)
    # sample 0: Z_0 = diag(+1,-1,+1,-1,...); sample 1: 2 Z_2 = 2 diag(+,+,+,+,-,-,-,-)
    np.testing.assert_allclose(lam[0], psi[0] * np.array([1, -1] * 4))
    np.testing.assert_allclose(lam[1], psi[1] * 2 * np.array([1] * 4 + [-1] * 4))


def test_unitary_helper_matches_kron(rng):
    c = C.random_circuit(3, 20, rng, n_params=4)
    p = rng.uniform(-np.pi, np.pi, c.n_params)
    np.testing.assert_allclose(circuit_unitary(c, p), circuit_full(c, p), atol=1e-12)
